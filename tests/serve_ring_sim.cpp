// CPU model of the serving queue: the server's producer half
// (chem_serve_ring.h) against threads that follow the device half of the
// protocol step by step (claim by compare-and-swap below the published count,
// slot from the tile table, per-slot finished counter reset by the last
// tile, done flag), with the dispatcher's launch rules: a "launch" is a set of
// consumer threads that leave after a bounded number of empty polls, after a
// quantum of tiles, or at the stop flag; the producer relaunches while boxes
// are live and rebases the 32-bit tile count once drained.
//
// Small ring, small tile table and a low tile limit make every path run:
// full ring, table entries reused, rebase, idle exits, quantum exits, stop.
// Checks: every cell of every box is processed exactly once, by a consumer
// that found the box the tile belongs to; every box completes once.  Also
// the split of a request into boxes and its per-box layout (pack, unpack).
// Usage: serve_ring_sim <seed> <boxes>; exit status 0 on success.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../paper_2405_05974_amd/csrc/chem_serve_ring.h"

namespace {

struct Box {
  int64_t id;        // request-level box number
  int64_t n;         // cells
  int64_t tile_pre;
};

constexpr int kCpt = 4;             // cells per tile
constexpr unsigned kCap = 8;        // ring slots
constexpr unsigned kTileCap = 64;   // tile table entries
constexpr unsigned kTileLimit = 600;

struct Shared {
  Box boxes[kCap];
  unsigned tile_slot[kTileCap];
  unsigned pub = 0;
  int stop = 0;
  unsigned head = 0;
  int finished[kCap] = {};
  int done[kCap] = {};
};

std::atomic<int> g_errors{0};

void fail(const char* what, long long a, long long b) {
  if (g_errors.fetch_add(1) < 10) std::fprintf(stderr, "error: %s (%lld, %lld)\n", what, a, b);
}

// One consumer ("wave") of a launch: the device half of the protocol.
void consumer(Shared* q, std::vector<std::vector<std::atomic<int>>>* hits, int idle_polls, int quantum,
              unsigned seed) {
  std::mt19937 rng(seed);
  int tiles_done = 0;
  for (;;) {
    unsigned item = 0;
    bool got = false;
    int polls = 0;
    while (polls < idle_polls) {
      if (__atomic_load_n(&q->stop, __ATOMIC_RELAXED)) break;
      const unsigned pub = __atomic_load_n(&q->pub, __ATOMIC_RELAXED);
      unsigned h = __atomic_load_n(&q->head, __ATOMIC_RELAXED);
      if (h < pub) {
        if (__atomic_compare_exchange_n(&q->head, &h, h + 1u, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
          __atomic_thread_fence(__ATOMIC_ACQUIRE);
          item = h;
          got = true;
          break;
        }
        continue;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      ++polls;
    }
    if (!got) return;
    const unsigned s = q->tile_slot[item & (kTileCap - 1)];
    if (s >= kCap) {
      fail("slot out of range", item, s);
      return;
    }
    const Box bx = q->boxes[s];
    const int64_t tiles = (bx.n + kCpt - 1) / kCpt;
    const int64_t t = (int64_t)item - bx.tile_pre;
    if (t < 0 || t >= tiles) fail("tile outside the box found for it", item, bx.id);
    else
      for (int g = 0; g < kCpt; ++g) {
        const int64_t c = t * kCpt + g;
        if (c < bx.n) (*hits)[bx.id][c].fetch_add(1, std::memory_order_relaxed);
      }
    if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
    const int fin = __atomic_add_fetch(&q->finished[s], 1, __ATOMIC_ACQ_REL);
    if (fin == tiles) {
      __atomic_store_n(&q->finished[s], 0, __ATOMIC_RELAXED);
      __atomic_store_n(&q->done[s], 1, __ATOMIC_RELEASE);
    }
    if (quantum > 0 && ++tiles_done >= quantum) return;
  }
}

// Request split into boxes and the per-box layout: every box holds its own
// cells, T first, and unpacking restores the request exactly.
void check_layout(std::mt19937& rng) {
  for (int trial = 0; trial < 200; ++trial) {
    const int64_t n = 1 + (int64_t)(rng() % 500);
    const int S = 1 + (int)(rng() % 7);
    const int64_t max_cells = 1 + (int64_t)(rng() % 120);
    const std::vector<int64_t> box_n = chemgpu::serve_split(n, max_cells);
    int64_t total = 0, lo = n, hi = 0;
    for (int64_t nb : box_n) {
      total += nb;
      lo = std::min(lo, nb);
      hi = std::max(hi, nb);
      if (nb > max_cells) fail("box larger than the limit", nb, max_cells);
    }
    if (total != n || hi - lo > 1 || (int64_t)box_n.size() != (n + max_cells - 1) / max_cells)
      fail("split", n, max_cells);
    std::vector<double> in((size_t)(S + 1) * n), packed(in.size()), back(in.size(), -1.0);
    for (int64_t c = 0; c < n; ++c)
      for (int k = 0; k <= S; ++k) in[(size_t)k * n + c] = 1000.0 * k + c;   // row 0 is T
    chemgpu::serve_pack(in.data(), n, S, box_n, packed.data());
    int64_t a = 0;
    const double* b = packed.data();
    for (int64_t nb : box_n) {
      for (int k = 0; k <= S; ++k)
        for (int64_t c = 0; c < nb; ++c)
          if (b[(size_t)k * nb + c] != 1000.0 * k + (a + c)) fail("packed value", a + c, k);
      b += (size_t)(S + 1) * nb;
      a += nb;
    }
    chemgpu::serve_unpack(packed.data(), n, S, box_n, back.data());
    if (back != in) fail("unpack", n, S);
  }
}

struct Launch {
  std::vector<std::thread> th;
  bool running() const { return !th.empty(); }
  void join() {
    for (auto& t : th) t.join();
    th.clear();
  }
};

}  // namespace

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  const int n_boxes = argc > 2 ? std::atoi(argv[2]) : 400;
  std::mt19937 rng(seed);
  check_layout(rng);
  Shared* q = new Shared();
  chemgpu::ServeRing<Box> ring;
  ring.init(q->boxes, q->tile_slot, &q->pub, q->done, kCap, kTileCap, kTileLimit);
  std::vector<int64_t> sizes(n_boxes);
  for (auto& n : sizes) n = 1 + (int64_t)(rng() % (ring.max_box_tiles() * kCpt));
  std::vector<std::vector<std::atomic<int>>> hits(n_boxes);
  for (int b = 0; b < n_boxes; ++b) hits[b] = std::vector<std::atomic<int>>(sizes[b]);
  std::vector<int> completions(n_boxes, 0);
  std::vector<int64_t> slot_box(kCap, -1);

  Launch launch;
  int next = 0, collected = 0, launches = 0, rebases = 0;
  bool launch_done = true;   // the running launch's threads have all returned
  std::atomic<int> alive{0};
  const auto t0 = std::chrono::steady_clock::now();
  while (collected < n_boxes) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
      fail("timeout", collected, n_boxes);
      __atomic_store_n(&q->stop, 1, __ATOMIC_RELAXED);
      break;
    }
    // arrivals: a few boxes at a time, with pauses that let launches go idle
    if (next < n_boxes && rng() % 3 != 0) {
      const unsigned tiles = (unsigned)((sizes[next] + kCpt - 1) / kCpt);
      if (ring.needs_rebase(tiles)) {
        if (ring.idle() && !launch.running()) {   // drained and nobody claiming: start from tile 0
          q->head = 0;
          ring.rebase();
          ++rebases;
        }
      } else {
        const int s = ring.append(Box{next, sizes[next], 0}, tiles);
        if (s >= 0) {
          slot_box[s] = next;
          ++next;
        }
      }
    } else if (rng() % 50 == 0) {
      std::this_thread::sleep_for(std::chrono::milliseconds(3));
    }
    collected += ring.collect([&](unsigned s) {
      const int64_t b = slot_box[s];
      if (b < 0) fail("done flag on an empty slot", s, 0);
      else ++completions[b];
      slot_box[s] = -1;
    });
    if (launch.running() && alive.load() == 0) {
      launch.join();
      launch_done = true;
    }
    if (!launch.running() && !ring.idle()) {   // relaunch while boxes are live
      const int waves = 1 + (int)(rng() % 6);
      const int quantum = (rng() % 2) ? 0 : 1 + (int)(rng() % 8);
      alive.store(waves);
      for (int w = 0; w < waves; ++w)
        launch.th.emplace_back([&, w, quantum] {
          consumer(q, &hits, 40, quantum, seed * 131u + (unsigned)launches * 7u + (unsigned)w);
          alive.fetch_sub(1);
        });
      ++launches;
      launch_done = false;
    }
  }
  __atomic_store_n(&q->stop, 1, __ATOMIC_RELAXED);
  launch.join();
  (void)launch_done;
  int64_t cells = 0;
  for (int b = 0; b < n_boxes; ++b) {
    if (completions[b] != 1) fail("box completions", b, completions[b]);
    for (int64_t c = 0; c < sizes[b]; ++c) {
      const int h = hits[b][c].load();
      if (h != 1) fail("cell processed", b * 100000 + c, h);
    }
    cells += sizes[b];
  }
  std::printf("boxes %d cells %lld launches %d rebases %d errors %d\n", n_boxes, (long long)cells, launches, rebases,
              g_errors.load());
  delete q;
  return g_errors.load() == 0 ? 0 : 1;
}
