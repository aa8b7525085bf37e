// chem_internal.h -- device tables and launch interface shared by the host
// library (chem_host.cpp) and the gfx950 kernels (chem_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace chemgpu {

constexpr int kMaxSide = 3;              // species per reaction side
constexpr int kSlots = 2 * kMaxSide;     // reactant slots 0..2, product slots 3..5
constexpr int kQMax = 5;                 // highest BDF order
constexpr int kRecRows = 9;              // per-cell record rows (see chem.h)
constexpr int kStatCount = 12;           // device stats counters

// Physical constants (CODATA 2018 gas constant, thermochemical calorie).
constexpr double kRu = 8.31446261815324;       // J/(mol K)
constexpr double kRuCgs = 8.31446261815324e7;  // erg/(mol K)
constexpr double kPatm = 101325.0;             // Pa, standard-state pressure of K_c
constexpr double kTref = 298.15;               // K, reference of the species thermo

// One reaction of Eq. 1 with its rate-constant parameters (Eq. 2's k vector):
// ln A, temperature exponent and activation temperature Ea/R, plus the
// low-pressure limit of a falloff reaction and Troe's broadening parameters.
// sp[] holds the species of the reactant slots 0..nr-1 and product slots
// 3..3+np-1 (-1 when unused).  eff_off/eff_n locate the reaction's collision
// efficiencies other than 1 in DevMech::eff_k/eff_v.
struct alignas(16) RxParams {
  double lnA, b, EaR;
  double lnA0, b0, EaR0;
  double troe[4];  // alpha, T3, T1, T2 (CHEMKIN's T***, T*, T**)
  int type;      // 0 elementary, 1 third body (+M), 2 falloff (Lindemann, times Troe's F when ntroe > 0)
  int rev;       // 1 reversible (reverse rate from K_c), 0 irreversible
  int nr, np;
  int sp[kSlots];
  int ntroe;     // 0, 3 or 4 Troe parameters
  int eff_off, eff_n;
  int pad;
};

// Device-resident mechanism tables (all pointers are device memory).
struct DevMech {
  int S, R, N;       // species, reactions, N = S + 1 unknowns per cell
  int nch;           // reaction chunks of NP reactions for the group layout
  int np_width;      // lanes per cell (16, 32 or 64)
  const double* W;   // [S] molecular weight g/mol
  const double* a0;  // [S] cp/R = a0 + a1 T
  const double* a1;
  const double* hf;  // [S] formation enthalpy at 298.15 K, J/mol
  const double* s0;  // [S] entropy at 298.15 K, J/(mol K)
  const RxParams* rx;      // [R]
  const int* csr_off;      // [S * (nch + 1)] start of species k's entries in chunk c
  const int* csr_ent;      // entries (j << 3) | (nu_kj + 4), sorted by j per species
  int nasa;                // 1: every species' thermo from nasa_c (NASA 7-coefficient polynomials)
  const double* nasa_c;    // [15][S]: T_mid, then c1..c7 for T <= T_mid, then c1..c7 above
  const int* eff_k;        // collision efficiencies other than 1: species index
  const double* eff_v;     //   and efficiency minus 1
  // The fields every rate evaluation reads, one array per field (reaction j
  // at j), so that the lanes of a wave, which hold consecutive reactions,
  // read them with coalesced loads:
  const double* rx_lnA;    // [R] ln A, temperature exponent, Ea/R
  const double* rx_b;
  const double* rx_EaR;
  const int4* rx_meta;     // [R] x: type | rev << 2 | nr << 3 | np << 5 | (ntroe > 0) << 7
                           //     y, z: species of slots 0..2 and 3..5, 8 bits each (255 = none)
                           //     w: eff_off | eff_n << 20
  const int2* rx_net;      // [R] the species with a nonzero net coefficient, up to 6, 10 bits each
                           //     (species << 3 | nu + 4; 1023 = none), three in x and three in y
};

__host__ __device__ inline void net_slot(const int2& nt, const int p, int& k, int& nu) {
  const int v = ((p < 3 ? nt.x : nt.y) >> (10 * (p % 3))) & 1023;
  k = v == 1023 ? -1 : (v >> 3);
  nu = (v & 7) - 4;
}

__host__ __device__ inline int meta_slot(const int4& mt, const int s) {
  const int v = ((s < kMaxSide ? mt.y : mt.z) >> (8 * (s % kMaxSide))) & 255;
  return v == 255 ? -1 : v;
}

// One box of the batched entry point, in queue order.
struct BoxDev {
  double* T;           // [n] device
  double* Y;           // [S * n] device, SoA within the box
  int64_t n;           // cells
  double dt;           // flow step of this box, s
  int64_t cell_off;    // first column of this box in the record array
  int64_t tile_pre;    // first queue item of this box
  int box_id;          // index in the caller's box array
  int pad;
};

struct BoxJob {
  int n_boxes;
  unsigned total_tiles;
  int64_t total_cells;
};

// One box of a resident serving kernel: a request's cells (or a part of
// them), with its own state and records in device memory.
struct ServeBox {
  double* T;           // [n]
  double* Y;           // [S * n], SoA within the box
  int32_t* rec;        // [kRecRows * n], rows n apart
  int64_t n;           // cells
  double dt;           // flow step of this box, s
  int64_t tile_pre;    // first tile of this box (set when it is published)
};

// Work queue of a resident serving kernel (continuous batching); the host
// half of the protocol, and the protocol itself, are in chem_serve_ring.h.
// The host appends boxes while the kernel runs: box descriptors in ring
// slots, the slot of every published tile in tile_slot, the published tile
// count in pub (all host-mapped, coherent).  Lane 0 of a wave claims a tile
// below *pub by compare-and-swap on head (device memory) and reads only its
// own box; the wave that finishes a box's last tile resets the slot's
// finished counter and sets done[slot] (host-mapped).  A wave leaves after
// idle_polls empty polls, at the stop flag, or between tiles once it has
// run for `quantum` ticks of the 100 MHz real-time counter (0: never), so
// every launch ends and the host relaunches while boxes are live.
struct ServeQueue {
  const ServeBox* boxes;       // host-mapped [ring slots]
  const unsigned* tile_slot;   // host-mapped [tile_mask + 1]
  const unsigned* pub;         // host-mapped: tiles published
  const int* stop;             // host-mapped
  unsigned* head;              // device: next tile to claim
  int* finished;               // device [ring slots]: tiles finished of the slot's box
  int* done;                   // host-mapped [ring slots]
  unsigned tile_mask;
  int idle_polls;
  int64_t quantum;
};

struct IntParams {
  double p, dt, rtol, atol;
  int max_steps, q_max, fixed_T, fixed_step_n;
  int lu_fp32, ir_max;
  int jac_mode;   // 0 analytic Jacobian, 1 difference quotients, 2 analytic with a difference-quotient T column
  int jac_reuse;  // 1: keep the factored Newton matrix while recent; 0: fresh every attempt
};

// Launchers (chem_kernels.hip).  All enqueue on `stream` and return the HIP
// status of the launch.
hipError_t launch_integrate(const DevMech& m, const IntParams& prm, double* T, double* Y, int64_t n,
                            int32_t* rec, hipStream_t stream);
hipError_t launch_rates(const DevMech& m, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                        double* wdot, double* f, double* jac, hipStream_t stream);
hipError_t launch_boxes(const DevMech& m, const IntParams& prm, const BoxDev* boxes, const BoxJob* job,
                        unsigned* head, int* remaining, int32_t* rec, int* host_done, int grid, hipStream_t stream);
hipError_t launch_reduce_records(const int32_t* rec, int64_t n, unsigned long long* out, hipStream_t stream);
hipError_t launch_reduce_records_job(const int32_t* rec, const BoxJob* job, unsigned long long* out,
                                     hipStream_t stream);
size_t integrate_lds_bytes(int np_width, int N, bool f32, bool f32_in_place = false);
hipError_t launch_boxes_init(const BoxDev* boxes, const BoxJob* job, unsigned* head, int* remaining,
                             hipStream_t stream);
// Resident serving kernel of the group family on `grid` waves, and the
// waves of it one CU can hold (occupancy).
hipError_t launch_serve(const DevMech& m, const IntParams& prm, const ServeQueue& q, int grid, hipStream_t stream);
int serve_waves_per_cu(const DevMech& m, bool f32, int ir_max);
// Zero `count` unsigned words of device memory with a kernel (no memset node).
hipError_t launch_zero_u32(unsigned* p, int count, hipStream_t stream);

// Lane-per-cell kernels, generated per mechanism and compiled with hipRTC
// (chem_jit.cpp).  Largest state size N = S + 1 they serve.
constexpr int kLpcMaxN = 12;
hipError_t launch_lpc_integrate(void* fn, const IntParams& prm, double* T, double* Y, int64_t n, int32_t* rec,
                                hipStream_t stream);
hipError_t launch_lpc_rates(void* fn, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                            double* wdot, double* f, double* jac, hipStream_t stream);
hipError_t launch_lpc_boxes(void* fn, const IntParams& prm, const BoxDev* boxes, const BoxJob* job, unsigned* head,
                            int* remaining, int32_t* rec, int* host_done, int grid, hipStream_t stream);
hipError_t launch_lpc_serve(void* fn, const IntParams& prm, const ServeQueue& q, int grid, hipStream_t stream);
int lpc_serve_waves_per_cu(void* fn);

}  // namespace chemgpu
