// chem_server.cpp -- continuous-batching request server of libchem (see the
// serving section of include/chem.h).
//
// Requests wait in arrival order until their state and records fit in the
// device arena (the HBM budget).  The dispatcher thread then copies them in
// (through pinned memory) and appends their boxes to the work queue of a
// resident kernel that is already running for the same mechanism, pressure
// and tolerances (a channel): its waves pick the new tiles up as they finish
// the tiles they hold.  The wave that finishes a box's last tile raises a
// host-mapped flag; once every box of a request is done, its state and
// status row are copied back.  The queue protocol is in chem_serve_ring.h.
// The server lock guards only the tables shared with the API calls: no HIP
// call and no bulk copy runs under it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/chem.h"
#include "chem_handle.h"
#include "chem_internal.h"
#include "chem_serve_ring.h"

namespace {

constexpr unsigned kRingSlots = 4096;           // boxes in flight per channel
constexpr unsigned kTileCap = 1u << 20;         // tile table entries per channel (a box has at most a quarter)
constexpr unsigned kTileLimit = 1u << 31;       // rebase the 32-bit tile count before it passes this
constexpr int kIdlePolls = 400;                 // empty polls (about 20 ms with backoff) before a wave leaves
constexpr int64_t kQuantumTicks = 20000000;     // 200 ms of the 100 MHz counter: waves leave between tiles

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
    size_ = size;
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
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, size_ = 0;
};

struct Request {
  int64_t id = 0;
  chem_mech* m = nullptr;
  int64_t n = 0;
  double p = 0, dt = 0, rtol = 0, atol = 0;
  std::vector<double> in;        // T[n] then Y[S n], copied at submit
  std::vector<double> out;       // the same layout, filled at completion
  double t_arrival = 0, latency_ms = 0;
  int status = CHEM_OK;
  bool finished = false;         // results (or an error) ready for poll
  // owned by the dispatcher thread
  int S = 0;
  int cpt = 0;                   // cells per tile of the kernel family
  bool lpc = false;
  std::vector<int64_t> box_n;    // the request's cells split into boxes
  size_t dev_off = 0, dev_bytes = 0, state_bytes = 0;
  size_t pin_off = 0, pin_bytes = 0;
  bool has_dev = false, has_pin = false;
  hipEvent_t ev = nullptr;       // end of the copy in or out
  int boxes_done = 0;
};

// A resident kernel and its queue, for one (mechanism, pressure, tolerances).
struct Channel {
  hipStream_t stream = nullptr;
  hipEvent_t ended = nullptr;   // recorded after every launch
  bool running = false;         // a launch not yet seen to end
  bool keyed = false;
  bool draining = false;        // takes no new requests: another key waits for a channel
  chem_mech* m = nullptr;
  double p = 0, rtol = 0, atol = 0;
  bool lpc = false;
  int cpt = 0, grid = 0;
  char* host_block = nullptr;   // coherent host-mapped queue memory
  chemgpu::ServeBox* boxes = nullptr;
  unsigned* tile_slot = nullptr;
  unsigned* pub = nullptr;
  int* stop = nullptr;
  int* done = nullptr;
  unsigned* head = nullptr;     // device
  int* finished = nullptr;      // device [kRingSlots]
  chemgpu::ServeRing<chemgpu::ServeBox> ring;
  std::vector<std::pair<Request*, int>> owner;    // slot -> (request, box)
  std::deque<std::pair<Request*, int>> pending;   // boxes waiting for room in the ring
};

}  // namespace

struct chem_server {
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::thread th;
  bool stop = false;
  std::atomic<bool> broken{false};  // a device error: every request fails, new ones are refused
  int device = 0;
  int n_cu = 256;
  char* arena_dev = nullptr;
  char* arena_pin = nullptr;
  unsigned* zero_pin = nullptr;     // a pinned zero word, copied over a channel's claim counter
  Arena dev_arena, pin_arena;       // dispatcher thread only
  int64_t budget = 0;
  size_t pin_size = 0;
  hipStream_t copy_stream = nullptr;
  std::deque<Request*> incoming;    // submitted, not yet seen by the dispatcher
  std::unordered_map<int64_t, Request*> reqs;
  std::vector<Channel> ch;
  std::vector<hipEvent_t> event_pool;
  int64_t next_id = 1;
  chem_server_stats st{};
  std::string err;
};

namespace {

void set_broken(chem_server* s, const char* why) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->err.empty()) s->err = why;
  s->broken = true;
}

bool key_matches(const Channel& c, const Request* r) {
  return c.keyed && c.m == r->m && c.p == r->p && c.rtol == r->rtol && c.atol == r->atol;
}

hipEvent_t take_event(chem_server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void give_event(chem_server* s, hipEvent_t& e) {
  if (e) s->event_pool.push_back(e);
  e = nullptr;
}

// Release the request's memory and hand it to poll() with `status`.
void complete(chem_server* s, Request* r, int status) {
  if (r->has_dev) s->dev_arena.release(r->dev_off, r->dev_bytes);
  if (r->has_pin) s->pin_arena.release(r->pin_off, r->pin_bytes);
  r->has_dev = r->has_pin = false;
  give_event(s, r->ev);
  std::vector<double>().swap(r->in);
  const double t = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = status;
  r->latency_ms = t - r->t_arrival;
  r->finished = true;
  if (status == CHEM_OK || status == CHEM_WARN_CELLS_FAILED) {
    s->st.completed++;
    s->st.cells_completed += r->n;
  }
  s->st.in_flight--;
  s->st.bytes_in_use = (int64_t)s->dev_arena.used();
  s->cv_done.notify_all();
}

// Device layout of a request: the states of its boxes (T[nb], Y[S nb] each),
// then their records (kRecRows x nb each).  Offsets of box j in doubles and
// in int32 words from the two region starts.
void box_offsets(const Request* r, int j, size_t* state_dbl, size_t* rec_words, int64_t* first_cell) {
  int64_t a = 0;
  for (int i = 0; i < j; ++i) a += r->box_n[i];
  *first_cell = a;
  *state_dbl = (size_t)(r->S + 1) * (size_t)a;
  *rec_words = (size_t)chemgpu::kRecRows * (size_t)a;
}

// Admission in arrival order: device memory for state and records, pinned
// staging for the state; copy in on the copy stream.  Returns true if any
// request moved on.
bool admit(chem_server* s, std::deque<Request*>& wait, std::vector<Request*>& staging_in) {
  bool progress = false;
  while (!wait.empty()) {
    Request* r = wait.front();
    if (r->cpt == 0) {   // first look: kernel family and box split
      bool lpc = false;
      const int rc = chem_select_kernel(r->m, &lpc);
      if (rc != CHEM_OK) {
        wait.pop_front();
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->st.queued--;
        }
        complete(s, r, rc);
        progress = true;
        continue;
      }
      r->lpc = lpc;
      r->cpt = chem_cells_per_tile(r->m, lpc);
      r->box_n = chemgpu::serve_split(r->n, (int64_t)(kTileCap / 4) * r->cpt);
    }
    size_t doff = 0, poff = 0;
    if (!s->dev_arena.alloc(r->dev_bytes, &doff)) break;
    if (!s->pin_arena.alloc(r->state_bytes, &poff)) {
      s->dev_arena.release(doff, r->dev_bytes);
      break;
    }
    r->dev_off = doff;
    r->pin_off = poff;
    r->pin_bytes = r->state_bytes;
    r->has_dev = r->has_pin = true;
    chemgpu::serve_pack(r->in.data(), r->n, r->S, r->box_n, reinterpret_cast<double*>(s->arena_pin + poff));
    std::vector<double>().swap(r->in);
    r->ev = take_event(s);
    if (!r->ev ||
        hipMemcpyAsync(s->arena_dev + doff, s->arena_pin + poff, r->state_bytes, hipMemcpyHostToDevice,
                       s->copy_stream) != hipSuccess ||
        hipEventRecord(r->ev, s->copy_stream) != hipSuccess) {
      set_broken(s, "copy to the device failed");
      return true;
    }
    wait.pop_front();
    staging_in.push_back(r);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.queued--;
      s->st.bytes_in_use = (int64_t)s->dev_arena.used();
      s->st.bytes_peak = std::max(s->st.bytes_peak, s->st.bytes_in_use);
    }
    progress = true;
  }
  return progress;
}

// Copies that have landed: staging released, request ready for a channel.
bool finish_copy_in(chem_server* s, std::vector<Request*>& staging_in, std::deque<Request*>& ready) {
  bool progress = false;
  size_t keep = 0;
  for (size_t i = 0; i < staging_in.size(); ++i) {
    Request* r = staging_in[i];
    const hipError_t e = hipEventQuery(r->ev);
    if (e == hipErrorNotReady) {
      staging_in[keep++] = r;
      continue;
    }
    if (e != hipSuccess) {
      set_broken(s, "copy to the device failed");
    }
    s->pin_arena.release(r->pin_off, r->pin_bytes);
    r->has_pin = false;
    give_event(s, r->ev);
    ready.push_back(r);
    progress = true;
  }
  staging_in.resize(keep);
  return progress;
}

bool key_channel(chem_server* s, Channel& c, Request* r) {
  c.keyed = true;
  c.draining = false;
  c.m = r->m;
  c.p = r->p;
  c.rtol = r->rtol;
  c.atol = r->atol;
  c.lpc = r->lpc;
  c.cpt = r->cpt;
  const int waves = c.lpc ? chemgpu::lpc_serve_waves_per_cu(c.m->lpc_serve)
                          : chemgpu::serve_waves_per_cu(c.m->dev, c.m->lu_fp32 != 0, c.m->ir_max);
  c.grid = std::max(1, waves) * s->n_cu;
  // a fresh tile count: the claim counter back to zero (SDMA copy of a pinned
  // zero, ordered before the next launch on this stream)
  if (c.ring.published() != 0) {
    if (hipMemcpyAsync(c.head, s->zero_pin, sizeof(unsigned), hipMemcpyHostToDevice, c.stream) != hipSuccess)
      return false;
    c.ring.rebase();
  }
  return true;
}

// Ready requests to channels of their key; a request with no such channel
// takes an idle one (stopping its kernel first) or marks the least busy one
// draining so that it frees up.
bool assign(chem_server* s, std::deque<Request*>& ready) {
  bool progress = false;
  for (size_t i = 0; i < ready.size();) {
    Request* r = ready[i];
    Channel* home = nullptr;
    for (Channel& c : s->ch)
      if (key_matches(c, r) && !c.draining) home = &c;
    if (!home) {
      Channel* idle = nullptr;
      for (Channel& c : s->ch)
        if (!c.keyed || (c.ring.idle() && c.pending.empty() && !key_matches(c, r))) {
          idle = &c;
          break;
        }
      if (idle && idle->running) {   // ask its kernel to leave; take it once it has
        __atomic_store_n(idle->stop, 1, __ATOMIC_RELEASE);
        ++i;
        continue;
      }
      if (idle) {
        if (!key_channel(s, *idle, r)) {
          set_broken(s, "channel reset failed");
          return true;
        }
        home = idle;
      } else {
        bool someone_draining = false;
        for (Channel& c : s->ch) someone_draining |= c.draining;
        if (!someone_draining) {
          Channel* least = nullptr;
          size_t best = ~(size_t)0;
          for (Channel& c : s->ch) {
            const size_t load = c.ring.live() + c.pending.size();
            if (load < best) {
              best = load;
              least = &c;
            }
          }
          if (least) least->draining = true;
        }
        ++i;
        continue;
      }
    }
    for (int j = 0; j < (int)r->box_n.size(); ++j) home->pending.emplace_back(r, j);
    ready.erase(ready.begin() + (std::ptrdiff_t)i);
    progress = true;
  }
  return progress;
}

// One channel: notice a finished launch, collect done boxes, publish
// waiting boxes, relaunch while boxes are live.
bool service(chem_server* s, Channel& c, std::vector<Request*>& to_out) {
  bool progress = false;
  if (c.running) {
    const hipError_t e = hipEventQuery(c.ended);
    if (e == hipSuccess) {
      c.running = false;
      __atomic_store_n(c.stop, 0, __ATOMIC_RELEASE);
      progress = true;
    } else if (e != hipErrorNotReady) {
      set_broken(s, "serving kernel failed");
      return true;
    }
  }
  if (!c.keyed) return progress;
  if (c.ring.collect([&](unsigned slot) {
        Request* r = c.owner[slot].first;
        c.owner[slot] = {nullptr, -1};
        if (++r->boxes_done == (int)r->box_n.size()) to_out.push_back(r);
      }) > 0)
    progress = true;
  if (c.draining && c.ring.idle() && c.pending.empty()) {
    c.keyed = false;   // free for the key that waits
    c.draining = false;
    return true;
  }
  while (!c.pending.empty()) {
    Request* r = c.pending.front().first;
    const int j = c.pending.front().second;
    const int64_t nb = r->box_n[(size_t)j];
    const unsigned tiles = (unsigned)((nb + c.cpt - 1) / c.cpt);
    if (c.ring.needs_rebase(tiles)) {
      if (!c.ring.idle() || c.running) break;
      if (hipMemcpyAsync(c.head, s->zero_pin, sizeof(unsigned), hipMemcpyHostToDevice, c.stream) != hipSuccess) {
        set_broken(s, "channel reset failed");
        return true;
      }
      c.ring.rebase();
    }
    if (!c.ring.can_append(tiles)) break;
    size_t so = 0, ro = 0;
    int64_t a = 0;
    box_offsets(r, j, &so, &ro, &a);
    double* state = reinterpret_cast<double*>(s->arena_dev + r->dev_off) + so;
    int32_t* recs = reinterpret_cast<int32_t*>(s->arena_dev + r->dev_off + r->state_bytes) + ro;
    chemgpu::ServeBox b;
    b.T = state;
    b.Y = state + nb;
    b.rec = recs;
    b.n = nb;
    b.dt = r->dt;
    b.tile_pre = 0;
    const int slot = c.ring.append(b, tiles);
    c.owner[(size_t)slot] = {r, j};
    c.pending.pop_front();
    progress = true;
  }
  if (!c.running && !c.ring.idle()) {
    chemgpu::ServeQueue q;
    q.boxes = c.boxes;
    q.tile_slot = c.tile_slot;
    q.pub = c.pub;
    q.stop = c.stop;
    q.head = c.head;
    q.finished = c.finished;
    q.done = c.done;
    q.tile_mask = kTileCap - 1;
    q.idle_polls = kIdlePolls;
    q.quantum = kQuantumTicks;
    const chemgpu::IntParams prm = make_int_params(c.m, c.p, 0.0, c.rtol, c.atol);
    const hipError_t e = c.lpc ? chemgpu::launch_lpc_serve(c.m->lpc_serve, prm, q, c.grid, c.stream)
                               : chemgpu::launch_serve(c.m->dev, prm, q, c.grid, c.stream);
    if (e != hipSuccess || hipEventRecord(c.ended, c.stream) != hipSuccess) {
      set_broken(s, "serving kernel launch failed");
      return true;
    }
    c.running = true;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.launches++;
    }
    progress = true;
  }
  return progress;
}

// Requests whose boxes are all done: state and records back to pinned memory.
bool copy_out(chem_server* s, std::vector<Request*>& to_out, std::vector<Request*>& staging_out) {
  bool progress = false;
  size_t keep = 0;
  for (size_t i = 0; i < to_out.size(); ++i) {
    Request* r = to_out[i];
    size_t poff = 0;
    if (!s->pin_arena.alloc(r->dev_bytes, &poff)) {
      to_out[keep++] = r;
      continue;
    }
    r->pin_off = poff;
    r->pin_bytes = r->dev_bytes;
    r->has_pin = true;
    r->ev = take_event(s);
    if (!r->ev ||
        hipMemcpyAsync(s->arena_pin + poff, s->arena_dev + r->dev_off, r->dev_bytes, hipMemcpyDeviceToHost,
                       s->copy_stream) != hipSuccess ||
        hipEventRecord(r->ev, s->copy_stream) != hipSuccess) {
      set_broken(s, "copy to the host failed");
      return true;
    }
    staging_out.push_back(r);
    progress = true;
  }
  to_out.resize(keep);
  return progress;
}

bool finish_copy_out(chem_server* s, std::vector<Request*>& staging_out) {
  bool progress = false;
  size_t keep = 0;
  for (size_t i = 0; i < staging_out.size(); ++i) {
    Request* r = staging_out[i];
    const hipError_t e = hipEventQuery(r->ev);
    if (e == hipErrorNotReady) {
      staging_out[keep++] = r;
      continue;
    }
    if (e != hipSuccess) {
      set_broken(s, "copy to the host failed");
      staging_out[keep++] = r;
      continue;
    }
    const int64_t n = r->n;
    r->out.assign((size_t)(r->S + 1) * (size_t)n, 0.0);
    chemgpu::serve_unpack(reinterpret_cast<const double*>(s->arena_pin + r->pin_off), n, r->S, r->box_n,
                          r->out.data());
    // status row (row 0 of each box's records)
    const int32_t* rec = reinterpret_cast<const int32_t*>(s->arena_pin + r->pin_off + r->state_bytes);
    int status = CHEM_OK;
    for (size_t j = 0; j < r->box_n.size(); ++j) {
      size_t so = 0, ro = 0;
      int64_t a = 0;
      box_offsets(r, (int)j, &so, &ro, &a);
      for (int64_t c = 0; c < r->box_n[j]; ++c)
        if (rec[ro + (size_t)c] != 0) status = CHEM_WARN_CELLS_FAILED;
    }
    complete(s, r, status);
    progress = true;
  }
  staging_out.resize(keep);
  return progress;
}

// After a device error: stop every kernel, wait for the streams, and fail
// every request the dispatcher holds.
void fail_all(chem_server* s, std::deque<Request*>& wait, std::vector<Request*>& staging_in,
              std::deque<Request*>& ready, std::vector<Request*>& to_out, std::vector<Request*>& staging_out) {
  for (Channel& c : s->ch) __atomic_store_n(c.stop, 1, __ATOMIC_RELEASE);
  for (Channel& c : s->ch) (void)hipStreamSynchronize(c.stream);
  (void)hipStreamSynchronize(s->copy_stream);
  std::vector<Request*> all;
  for (Request* r : wait) all.push_back(r);
  for (Request* r : staging_in) all.push_back(r);
  for (Request* r : ready) all.push_back(r);
  for (Request* r : to_out) all.push_back(r);
  for (Request* r : staging_out) all.push_back(r);
  for (Channel& c : s->ch) {
    for (auto& o : c.owner)
      if (o.first && std::find(all.begin(), all.end(), o.first) == all.end()) all.push_back(o.first);
    for (auto& p : c.pending)
      if (std::find(all.begin(), all.end(), p.first) == all.end()) all.push_back(p.first);
    c.owner.assign(kRingSlots, {nullptr, -1});
    c.pending.clear();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.queued -= (int64_t)wait.size();
  }
  for (Request* r : all) complete(s, r, CHEM_ERR_DEVICE);
  wait.clear();
  staging_in.clear();
  ready.clear();
  to_out.clear();
  staging_out.clear();
}

void dispatcher(chem_server* s) {
  (void)hipSetDevice(s->device);
  std::deque<Request*> wait, ready;
  std::vector<Request*> staging_in, to_out, staging_out;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop) break;
      while (!s->incoming.empty()) {
        wait.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
    }
    bool progress = false;
    if (!s->broken) progress |= admit(s, wait, staging_in);
    if (!s->broken) progress |= finish_copy_in(s, staging_in, ready);
    if (!s->broken) progress |= assign(s, ready);
    for (Channel& c : s->ch)
      if (!s->broken) progress |= service(s, c, to_out);
    if (!s->broken) progress |= copy_out(s, to_out, staging_out);
    if (!s->broken) progress |= finish_copy_out(s, staging_out);
    if (s->broken) fail_all(s, wait, staging_in, ready, to_out, staging_out);
    if (!progress) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return s->stop || !s->incoming.empty(); });
    }
  }
  // shutdown: every kernel leaves at its next claim
  for (Channel& c : s->ch)
    if (c.stop) __atomic_store_n(c.stop, 1, __ATOMIC_RELEASE);
  for (Channel& c : s->ch)
    if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
}

bool init_channel(Channel& c) {
  const size_t boxes_b = sizeof(chemgpu::ServeBox) * kRingSlots;
  const size_t table_b = sizeof(unsigned) * kTileCap;
  const size_t done_b = sizeof(int) * kRingSlots;
  const size_t total = boxes_b + table_b + done_b + 256;
  if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c.ended, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c.host_block), total, hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipMalloc(&c.head, sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&c.finished, sizeof(int) * kRingSlots) != hipSuccess)
    return false;
  std::memset(c.host_block, 0, total);
  c.boxes = reinterpret_cast<chemgpu::ServeBox*>(c.host_block);
  c.tile_slot = reinterpret_cast<unsigned*>(c.host_block + boxes_b);
  c.done = reinterpret_cast<int*>(c.host_block + boxes_b + table_b);
  c.pub = reinterpret_cast<unsigned*>(c.host_block + boxes_b + table_b + done_b);
  c.stop = reinterpret_cast<int*>(c.host_block + boxes_b + table_b + done_b + 64);
  c.ring.init(c.boxes, c.tile_slot, c.pub, c.done, kRingSlots, kTileCap, kTileLimit);
  c.owner.assign(kRingSlots, {nullptr, -1});
  if (chemgpu::launch_zero_u32(c.head, 1, c.stream) != hipSuccess ||
      chemgpu::launch_zero_u32(reinterpret_cast<unsigned*>(c.finished), (int)kRingSlots, c.stream) != hipSuccess ||
      hipStreamSynchronize(c.stream) != hipSuccess)
    return false;
  return true;
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
  s->pin_size = (size_t)std::min<int64_t>(budget_bytes / 4 + ((int64_t)64 << 20), (int64_t)8 << 30);
  if (hipMalloc(reinterpret_cast<void**>(&s->arena_dev), (size_t)budget_bytes) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->arena_pin), s->pin_size) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->zero_pin), 256) != hipSuccess) {
    chem_server_destroy(s);
    return CHEM_ERR_OOM;
  }
  std::memset(s->zero_pin, 0, 256);
  s->dev_arena.init((size_t)budget_bytes);
  s->pin_arena.init(s->pin_size);
  if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    chem_server_destroy(s);
    return CHEM_ERR_DEVICE;
  }
  s->ch.resize((size_t)streams);
  for (Channel& c : s->ch)
    if (!init_channel(c)) {
      chem_server_destroy(s);
      return CHEM_ERR_DEVICE;
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
  r->S = S;
  r->p = p;
  r->dt = dt;
  r->rtol = rtol;
  r->atol = atol;
  r->state_bytes = sizeof(double) * (size_t)(S + 1) * (size_t)n_cells;
  r->dev_bytes = r->state_bytes + sizeof(int32_t) * chemgpu::kRecRows * (size_t)n_cells;
  if ((int64_t)Arena::round(r->dev_bytes) > s->budget || Arena::round(r->dev_bytes) > s->pin_size) {
    delete r;
    return CHEM_ERR_OOM;
  }
  try {
    r->in.resize((size_t)(S + 1) * (size_t)n_cells);
  } catch (...) {
    delete r;
    return CHEM_ERR_OOM;
  }
  if (n_cells) {
    std::memcpy(r->in.data(), T, sizeof(double) * (size_t)n_cells);
    std::memcpy(r->in.data() + n_cells, Y, sizeof(double) * (size_t)S * (size_t)n_cells);
  }
  r->t_arrival = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->broken) {
    delete r;
    return CHEM_ERR_DEVICE;
  }
  r->id = s->next_id++;
  *id = r->id;
  s->reqs[r->id] = r;
  s->st.submitted++;
  if (n_cells == 0) {
    r->finished = true;
    s->st.completed++;
  } else {
    s->incoming.push_back(r);
    s->st.queued++;
    s->st.in_flight++;
    s->cv_work.notify_one();
  }
  return CHEM_OK;
}

int chem_server_poll(chem_server* s, int64_t id, double* T_out, double* Y_out, double* latency_ms, int* status) {
  if (!s) return CHEM_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return CHEM_ERR_ARG;
  Request* r = it->second;
  if (!r->finished) return 0;
  const size_t n = (size_t)r->n;
  // a request that failed before its results came back has no outputs: the
  // caller's arrays are left alone and the status says why
  if (n && r->out.size() == (size_t)(r->S + 1) * n) {
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
  s->cv_done.wait(lk, [&] { return s->st.in_flight == 0 || s->stop; });
  return s->broken ? CHEM_ERR_DEVICE : CHEM_OK;
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
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  if (s->th.joinable()) s->th.join();
  for (Channel& c : s->ch) {
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    if (c.ended) (void)hipEventDestroy(c.ended);
    if (c.host_block) (void)hipHostFree(c.host_block);
    if (c.head) (void)hipFree(c.head);
    if (c.finished) (void)hipFree(c.finished);
  }
  if (s->copy_stream) {
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipStreamDestroy(s->copy_stream);
  }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (auto& kv : s->reqs) {
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    delete kv.second;
  }
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  if (s->arena_pin) (void)hipHostFree(s->arena_pin);
  if (s->zero_pin) (void)hipHostFree(s->zero_pin);
  delete s;
}

}  // extern "C"
