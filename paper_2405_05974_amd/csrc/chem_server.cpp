// chem_server.cpp -- continuous-batching request server of libchem (see the
// serving section of include/chem.h).
//
// Requests (host arrays) wait in arrival order until their state fits in the
// device arena (the HBM budget) and in the pinned staging area; a dispatcher
// thread then copies them in and, whenever a launch stream is free, launches
// everything admitted since the previous launch (grouped by mechanism,
// pressure and tolerances) as one persistent box launch.  Requests that
// arrive while earlier launches run are launched on another stream and
// overlap with them on the device.  Completion is detected with events; the
// results are copied to pinned memory in the same stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/chem.h"
#include "chem_handle.h"
#include "chem_internal.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t start = it->first + bytes, rem = it->second - bytes;
      free_.erase(it);
      if (rem) free_[start] = rem;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Request {
  int64_t id = 0;
  chem_mech* m = nullptr;
  int64_t n = 0;
  double p = 0, dt = 0, rtol = 0, atol = 0;
  std::vector<double> in;        // T[n] then Y[S n], copied at submit
  size_t dev_bytes = 0, pin_bytes = 0, dev_off = 0, pin_off = 0;
  double t_arrival = 0, latency_ms = 0;
  int state = 0;                 // 0 queued, 1 admitted, 2 launched, 3 done
  int status = CHEM_OK;
  std::vector<double> out;       // T then Y
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  chemgpu::BoxDev* dboxes = nullptr;
  chemgpu::BoxDev* hboxes = nullptr;   // pinned staging of the descriptors
  int box_cap = 0;
  chemgpu::BoxJob* djob = nullptr;
  chemgpu::BoxJob* hjob = nullptr;
  unsigned* dhead = nullptr;
  int* dremaining = nullptr;
  int32_t* rec = nullptr;
  int64_t rec_cap = 0;
  unsigned long long* dstats = nullptr;
  std::vector<Request*> reqs;
  std::vector<int64_t> cell_off;       // record column of each request
  bool busy = false;
};

}  // namespace

struct chem_server {
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  int device = 0;
  int n_cu = 256;
  char* arena_dev = nullptr;
  char* arena_pin = nullptr;
  Arena dev_arena, pin_arena;
  int64_t budget = 0;
  std::deque<Request*> queue;
  std::vector<Request*> ready;
  std::unordered_map<int64_t, Request*> reqs;
  std::vector<Slot> slots;
  int64_t next_id = 1;
  chem_server_stats st{};
  std::string err;
};

namespace {

bool ensure_slot(Slot& sl, int nbox, int64_t cells) {
  if (nbox > sl.box_cap) {
    if (sl.dboxes) (void)hipFree(sl.dboxes);
    if (sl.dremaining) (void)hipFree(sl.dremaining);
    if (sl.hboxes) (void)hipHostFree(sl.hboxes);
    sl.dboxes = nullptr;
    sl.dremaining = nullptr;
    sl.hboxes = nullptr;
    sl.box_cap = 0;
    const int cap = std::max(nbox, 64);
    if (hipMalloc(&sl.dboxes, sizeof(chemgpu::BoxDev) * cap) != hipSuccess ||
        hipMalloc(&sl.dremaining, sizeof(int) * cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.hboxes), sizeof(chemgpu::BoxDev) * cap) != hipSuccess)
      return false;
    sl.box_cap = cap;
  }
  if (cells > sl.rec_cap) {
    if (sl.rec) (void)hipFree(sl.rec);
    sl.rec = nullptr;
    sl.rec_cap = 0;
    const int64_t cap = std::max<int64_t>(cells, 4096);
    if (hipMalloc(&sl.rec, sizeof(int32_t) * chemgpu::kRecRows * cap) != hipSuccess) return false;
    sl.rec_cap = cap;
  }
  return true;
}

// Launch one group (same mechanism, pressure and tolerances) on a free slot.
bool launch_group(chem_server* s, Slot& sl, const std::vector<Request*>& group) {
  chem_mech* m = group[0]->m;
  const int S = m->dev.S;
  bool lpc = false;
  if (chem_select_kernel(m, &lpc) != CHEM_OK) return false;
  const int cpw = chem_cells_per_tile(m, lpc);
  int64_t cells = 0;
  for (Request* r : group) cells += r->n;
  if (!ensure_slot(sl, (int)group.size(), cells)) return false;
  // largest boxes first
  std::vector<int> order(group.size());
  for (size_t i = 0; i < group.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return group[a]->n > group[b]->n; });
  sl.cell_off.assign(group.size(), 0);
  int64_t tiles = 0, coff = 0;
  for (size_t i = 0; i < order.size(); ++i) {
    Request* r = group[order[i]];
    double* dT = reinterpret_cast<double*>(s->arena_dev + r->dev_off);
    chemgpu::BoxDev& b = sl.hboxes[i];
    b.T = dT;
    b.Y = dT + r->n;
    b.n = r->n;
    b.dt = r->dt;
    b.cell_off = coff;
    b.tile_pre = tiles;
    b.box_id = order[i];
    b.pad = 0;
    sl.cell_off[order[i]] = coff;
    tiles += (r->n + cpw - 1) / cpw;
    coff += r->n;
  }
  sl.hjob->n_boxes = (int)group.size();
  sl.hjob->total_tiles = (unsigned)tiles;
  sl.hjob->total_cells = cells;
  hipStream_t st = sl.stream;
  for (Request* r : group) {
    const size_t state_bytes = sizeof(double) * (size_t)(S + 1) * r->n;
    if (hipMemcpyAsync(s->arena_dev + r->dev_off, s->arena_pin + r->pin_off, state_bytes, hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return false;
  }
  if (hipMemcpyAsync(sl.dboxes, sl.hboxes, sizeof(chemgpu::BoxDev) * group.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(sl.djob, sl.hjob, sizeof(chemgpu::BoxJob), hipMemcpyHostToDevice, st) != hipSuccess)
    return false;
  const chemgpu::IntParams prm = make_int_params(m, group[0]->p, 0.0, group[0]->rtol, group[0]->atol);
  const int grid = (int)std::min<int64_t>(tiles, (int64_t)m->waves_per_cu * s->n_cu);
  if (chem_launch_box_queue(m, lpc, prm, sl.dboxes, sl.djob, sl.dhead, sl.dremaining, sl.rec, nullptr, grid, st) !=
      hipSuccess)
    return false;
  for (size_t i = 0; i < group.size(); ++i) {
    Request* r = group[i];
    const size_t state_bytes = sizeof(double) * (size_t)(S + 1) * r->n;
    if (hipMemcpyAsync(s->arena_pin + r->pin_off, s->arena_dev + r->dev_off, state_bytes, hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipMemcpyAsync(s->arena_pin + r->pin_off + state_bytes, sl.rec + sl.cell_off[i], sizeof(int32_t) * r->n,
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      return false;
  }
  if (hipEventRecord(sl.done, st) != hipSuccess) return false;
  for (Request* r : group) r->state = 2;
  sl.reqs = group;
  sl.busy = true;
  s->st.launches++;
  return true;
}

void complete_slot(chem_server* s, Slot& sl) {
  const double t = now_ms();
  for (Request* r : sl.reqs) {
    const int S = r->m->dev.S;
    const size_t nd = (size_t)(S + 1) * r->n;
    const double* src = reinterpret_cast<const double*>(s->arena_pin + r->pin_off);
    r->out.assign(src, src + nd);
    const int32_t* stc = reinterpret_cast<const int32_t*>(s->arena_pin + r->pin_off + nd * sizeof(double));
    r->status = CHEM_OK;
    for (int64_t i = 0; i < r->n; ++i)
      if (stc[i] != 0) r->status = CHEM_WARN_CELLS_FAILED;
    s->dev_arena.release(r->dev_off, r->dev_bytes);
    s->pin_arena.release(r->pin_off, r->pin_bytes);
    r->latency_ms = t - r->t_arrival;
    r->state = 3;
    s->st.completed++;
    s->st.cells_completed += r->n;
    s->st.in_flight--;
  }
  sl.reqs.clear();
  sl.busy = false;
}

void dispatcher(chem_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool progress = false;
    for (Slot& sl : s->slots) {
      if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
        complete_slot(s, sl);
        progress = true;
      }
    }
    if (progress) s->cv.notify_all();
    while (!s->queue.empty()) {   // admission in arrival order
      Request* r = s->queue.front();
      size_t doff = 0, poff = 0;
      if (!s->dev_arena.alloc(r->dev_bytes, &doff)) break;
      if (!s->pin_arena.alloc(r->pin_bytes, &poff)) {
        s->dev_arena.release(doff, r->dev_bytes);
        break;
      }
      r->dev_off = doff;
      r->pin_off = poff;
      std::memcpy(s->arena_pin + poff, r->in.data(), sizeof(double) * r->in.size());
      std::vector<double>().swap(r->in);
      r->state = 1;
      s->queue.pop_front();
      s->ready.push_back(r);
      s->st.queued--;
      s->st.bytes_in_use = (int64_t)s->dev_arena.used();
      s->st.bytes_peak = std::max(s->st.bytes_peak, s->st.bytes_in_use);
      progress = true;
    }
    while (!s->ready.empty()) {
      Slot* free_slot = nullptr;
      for (Slot& sl : s->slots)
        if (!sl.busy) {
          free_slot = &sl;
          break;
        }
      if (!free_slot) break;
      Request* first = s->ready.front();
      std::vector<Request*> group, rest;
      for (Request* r : s->ready) {
        if (r->m == first->m && r->p == first->p && r->rtol == first->rtol && r->atol == first->atol)
          group.push_back(r);
        else
          rest.push_back(r);
      }
      s->ready.swap(rest);
      if (!launch_group(s, *free_slot, group)) {
        s->err = "launch failed";
        // copies already queued on the slot's stream may still read or write
        // the requests' arena regions: let them finish before releasing
        (void)hipStreamSynchronize(free_slot->stream);
        for (Request* r : group) {   // report the failure on the requests
          r->status = CHEM_ERR_DEVICE;
          r->state = 3;
          s->dev_arena.release(r->dev_off, r->dev_bytes);
          s->pin_arena.release(r->pin_off, r->pin_bytes);
          s->st.in_flight--;
        }
        s->cv.notify_all();
      }
      progress = true;
    }
    s->st.bytes_in_use = (int64_t)s->dev_arena.used();
    if (!progress) s->cv.wait_for(lk, std::chrono::microseconds(100));
  }
}

}  // namespace

extern "C" {

int chem_server_create(int64_t budget_bytes, int streams, chem_server** out) {
  if (!out || budget_bytes <= 0 || streams < 1 || streams > 8) return CHEM_ERR_ARG;
  *out = nullptr;
  chem_server* s = new (std::nothrow) chem_server();
  if (!s) return CHEM_ERR_OOM;
  s->budget = budget_bytes;
  s->st.budget_bytes = budget_bytes;
  (void)hipGetDevice(&s->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, s->device) == hipSuccess && prop.multiProcessorCount > 0)
    s->n_cu = prop.multiProcessorCount;
  const size_t pin_bytes = (size_t)std::min<int64_t>(budget_bytes + budget_bytes / 8, (int64_t)8 << 30);
  if (hipMalloc(reinterpret_cast<void**>(&s->arena_dev), (size_t)budget_bytes) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->arena_pin), pin_bytes) != hipSuccess) {
    chem_server_destroy(s);
    return CHEM_ERR_OOM;
  }
  s->dev_arena.init((size_t)budget_bytes);
  s->pin_arena.init(pin_bytes);
  s->slots.resize(streams);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&sl.djob, sizeof(chemgpu::BoxJob)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.hjob), sizeof(chemgpu::BoxJob)) != hipSuccess ||
        hipMalloc(&sl.dhead, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&sl.dstats, sizeof(unsigned long long) * chemgpu::kStatCount) != hipSuccess) {
      chem_server_destroy(s);
      return CHEM_ERR_DEVICE;
    }
  }
  s->th = std::thread(dispatcher, s);
  *out = s;
  return CHEM_OK;
}

int chem_server_submit(chem_server* s, chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p,
                       double dt, double rtol, double atol, int64_t* id) {
  if (!s || !m || !id || n_cells < 0 || (n_cells > 0 && (!T || !Y))) return CHEM_ERR_ARG;
  if (!(dt > 0) || !(rtol > 0) || !(atol >= 0) || !(p > 0)) return CHEM_ERR_ARG;
  const int S = m->dev.S;
  Request* r = new (std::nothrow) Request();
  if (!r) return CHEM_ERR_OOM;
  r->m = m;
  r->n = n_cells;
  r->p = p;
  r->dt = dt;
  r->rtol = rtol;
  r->atol = atol;
  r->dev_bytes = sizeof(double) * (size_t)(S + 1) * n_cells;
  r->pin_bytes = r->dev_bytes + sizeof(int32_t) * n_cells;
  if ((int64_t)Arena::round(r->dev_bytes) > s->budget) {
    delete r;
    return CHEM_ERR_OOM;
  }
  r->in.resize((size_t)(S + 1) * n_cells);
  if (n_cells) {
    std::memcpy(r->in.data(), T, sizeof(double) * n_cells);
    std::memcpy(r->in.data() + n_cells, Y, sizeof(double) * (size_t)S * n_cells);
  }
  r->t_arrival = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  *id = r->id;
  s->reqs[r->id] = r;
  s->st.submitted++;
  if (n_cells == 0) {
    r->state = 3;
    s->st.completed++;
  } else {
    s->queue.push_back(r);
    s->st.queued++;
    s->st.in_flight++;
  }
  s->cv.notify_all();
  return CHEM_OK;
}

int chem_server_poll(chem_server* s, int64_t id, double* T_out, double* Y_out, double* latency_ms, int* status) {
  if (!s) return CHEM_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return CHEM_ERR_ARG;
  Request* r = it->second;
  if (r->state != 3) return 0;
  const size_t n = (size_t)r->n;
  // a request that failed before its results came back has no outputs: the
  // caller's arrays are left alone and the status says why
  if (n && r->out.size() == (size_t)(r->m->dev.S + 1) * n) {
    if (T_out) std::memcpy(T_out, r->out.data(), sizeof(double) * n);
    if (Y_out) std::memcpy(Y_out, r->out.data() + n, sizeof(double) * (r->out.size() - n));
  }
  if (latency_ms) *latency_ms = r->latency_ms;
  if (status) *status = r->status;
  s->reqs.erase(it);
  delete r;
  return 1;
}

int chem_server_drain(chem_server* s) {
  if (!s) return CHEM_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->st.in_flight == 0 || s->stop; });
  return CHEM_OK;
}

int chem_server_stats_get(chem_server* s, chem_server_stats* out) {
  if (!s || !out) return CHEM_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return CHEM_OK;
}

void chem_server_destroy(chem_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.dboxes) (void)hipFree(sl.dboxes);
    if (sl.hboxes) (void)hipHostFree(sl.hboxes);
    if (sl.djob) (void)hipFree(sl.djob);
    if (sl.hjob) (void)hipHostFree(sl.hjob);
    if (sl.dhead) (void)hipFree(sl.dhead);
    if (sl.dremaining) (void)hipFree(sl.dremaining);
    if (sl.rec) (void)hipFree(sl.rec);
    if (sl.dstats) (void)hipFree(sl.dstats);
  }
  for (auto& kv : s->reqs) delete kv.second;
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  if (s->arena_pin) (void)hipHostFree(s->arena_pin);
  delete s;
}

}  // extern "C"
