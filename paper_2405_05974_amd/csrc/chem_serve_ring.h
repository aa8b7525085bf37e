// chem_serve_ring.h -- host half of the serving queue protocol (plain C++,
// no HIP: the request server uses it, and a CPU test drives it against
// threads that follow the device half).
//
// Protocol.  A producer (the server's dispatcher thread) appends boxes of
// tiles while consumers (the waves of a resident kernel) claim tiles:
//   producer, per box of k tiles taking tiles [P, P + k):
//     boxes[s] = box (tile_pre = P)            s: a free ring slot
//     tile_slot[t & (tile_cap - 1)] = s         for t in [P, P + k)
//     *pub = P + k                              release store
//   consumer, per tile:
//     h = *head; if h < *pub (acquire): claim h by compare-and-swap on *head
//     s = tile_slot[h & (tile_cap - 1)]; tile h - boxes[s].tile_pre of box s
//     ... work ...
//     if ++finished[s] == k (acq_rel): finished[s] = 0; done[s] = 1 (release)
//   producer: sees done[s] (acquire), clears it, frees slot s.
// A consumer reads only the descriptor and table entries of the tile it
// holds, whose box is not done yet; the producer rewrites a slot only after
// its box is done and a table entry only once every box of the tile it held
// is done, so no consumer reads an entry while it changes.  Counters are 32
// bits: before *pub would pass tile_limit the producer stops appending, lets
// the ring drain and every consumer leave, and starts again from tile 0
// (rebase; the caller zeroes *head).
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

namespace chemgpu {

template <class Box>   // Box: a trivially copyable descriptor with an int64_t tile_pre
class ServeRing {
 public:
  // boxes[cap], done[cap], tile_slot[tile_cap] and *pub are shared with the
  // consumers; tile_cap is a power of two.
  void init(Box* boxes, unsigned* tile_slot, unsigned* pub, int* done, unsigned cap, unsigned tile_cap,
            unsigned tile_limit) {
    boxes_ = boxes;
    tile_slot_ = tile_slot;
    pub_ = pub;
    done_ = done;
    cap_ = cap;
    tile_cap_ = tile_cap;
    tile_limit_ = tile_limit;
    busy_.assign(cap, 0);
    live_.clear();
    free_.clear();
    for (unsigned s = cap; s-- > 0;) free_.push_back(s);
    for (unsigned s = 0; s < cap; ++s) __atomic_store_n(&done_[s], 0, __ATOMIC_RELAXED);
    tiles_ = 0;
    __atomic_store_n(pub_, 0u, __ATOMIC_RELEASE);
  }

  // Largest box (in tiles) that can ever be appended.
  unsigned max_box_tiles() const { return tile_cap_ / 4; }
  unsigned published() const { return tiles_; }
  unsigned live() const { return (unsigned)live_.size(); }
  bool idle() const { return live_.empty(); }
  // True when a box of `tiles` tiles would pass the 32-bit tile limit.
  bool needs_rebase(unsigned tiles) const { return (uint64_t)tiles_ + tiles > tile_limit_; }

  // True when a box of `tiles` tiles fits now: a free slot, table entries
  // no live box still uses, and room below the tile limit.
  bool can_append(unsigned tiles) const {
    if (tiles == 0 || tiles > max_box_tiles() || free_.empty() || needs_rebase(tiles)) return false;
    const uint64_t end = (uint64_t)tiles_ + tiles;
    return end <= (uint64_t)oldest_live_tile() + tile_cap_;
  }

  // Publish `b` (its tile_pre is set here).  Returns the slot, or -1 when
  // can_append(tiles) is false.
  int append(Box b, unsigned tiles) {
    if (!can_append(tiles)) return -1;
    const unsigned s = free_.back();
    free_.pop_back();
    b.tile_pre = (int64_t)tiles_;
    boxes_[s] = b;
    for (unsigned t = 0; t < tiles; ++t) tile_slot_[(tiles_ + t) & (tile_cap_ - 1)] = s;
    busy_[s] = 1;
    live_.push_back(s);
    tiles_ += tiles;
    __atomic_store_n(pub_, tiles_, __ATOMIC_RELEASE);
    return (int)s;
  }

  // Calls on_done(slot) for every live box whose done flag is set, then
  // frees its slot.  Returns the number of boxes collected.
  template <class F>
  int collect(F&& on_done) {
    int got = 0;
    for (size_t i = 0; i < live_.size();) {
      const unsigned s = live_[i];
      if (__atomic_load_n(&done_[s], __ATOMIC_ACQUIRE) != 0) {
        on_done(s);
        __atomic_store_n(&done_[s], 0, __ATOMIC_RELAXED);
        busy_[s] = 0;
        free_.push_back(s);
        live_[i] = live_.back();
        live_.pop_back();
        ++got;
      } else {
        ++i;
      }
    }
    return got;
  }

  // Back to tile 0.  Only while idle() and with no consumer running; the
  // caller zeroes the consumers' claim counter before they run again.
  void rebase() {
    tiles_ = 0;
    __atomic_store_n(pub_, 0u, __ATOMIC_RELEASE);
  }

  const Box& box(unsigned s) const { return boxes_[s]; }

 private:
  unsigned oldest_live_tile() const {
    unsigned lo = tiles_;
    for (unsigned s : live_) lo = std::min(lo, (unsigned)boxes_[s].tile_pre);
    return lo;
  }

  Box* boxes_ = nullptr;
  unsigned* tile_slot_ = nullptr;
  unsigned* pub_ = nullptr;
  int* done_ = nullptr;
  unsigned cap_ = 0, tile_cap_ = 0, tile_limit_ = 0;
  unsigned tiles_ = 0;
  std::vector<unsigned char> busy_;
  std::vector<unsigned> live_, free_;
};

// A request of n cells split into the fewest boxes of at most max_cells
// cells, sizes differing by at most one.
inline std::vector<int64_t> serve_split(int64_t n, int64_t max_cells) {
  const int64_t nb = n > 0 ? (n + max_cells - 1) / max_cells : 0;
  std::vector<int64_t> sizes((size_t)nb, nb ? n / nb : 0);
  for (int64_t i = 0; i < (nb ? n % nb : 0); ++i) sizes[(size_t)i]++;
  return sizes;
}

// Request layout (T[n], then Y[S n] SoA) to per-box layout (box after box,
// each T[nb] then Y[S nb]), and back.
inline void serve_pack(const double* in, int64_t n, int S, const std::vector<int64_t>& box_n, double* out) {
  int64_t a = 0;
  for (int64_t nb : box_n) {
    std::memcpy(out, in + a, sizeof(double) * (size_t)nb);
    for (int k = 0; k < S; ++k)
      std::memcpy(out + (size_t)(k + 1) * nb, in + (size_t)n + (size_t)k * n + a, sizeof(double) * (size_t)nb);
    out += (size_t)(S + 1) * nb;
    a += nb;
  }
}

inline void serve_unpack(const double* in, int64_t n, int S, const std::vector<int64_t>& box_n, double* out) {
  int64_t a = 0;
  for (int64_t nb : box_n) {
    std::memcpy(out + a, in, sizeof(double) * (size_t)nb);
    for (int k = 0; k < S; ++k)
      std::memcpy(out + (size_t)n + (size_t)k * n + a, in + (size_t)(k + 1) * nb, sizeof(double) * (size_t)nb);
    in += (size_t)(S + 1) * nb;
    a += nb;
  }
}

}  // namespace chemgpu
