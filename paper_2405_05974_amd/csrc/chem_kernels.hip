// chem_kernels.hip -- gfx950 kernels for per-cell stiff chemistry.
//
// Layout: one cell per group of NP lanes (NP = 16, 32 or 64 >= S + 1), 64/NP
// cells per wave, one wave per workgroup.  Lane r of a group owns component r
// of the state y = (Y_1..Y_S, T).  Reactions are spread over the group's
// lanes (reaction j on lane j mod NP, in chunks of NP); species
// concentrations and Gibbs energies are exchanged through LDS, production
// rates are gathered per species lane in reaction order, and the sparse part
// of the Jacobian is scattered by the reaction lanes into per-cell LDS rows
// with f64 LDS atomics.
// The Newton matrix lives in those LDS rows between phases and is factored in
// registers (one row per lane) with partial pivoting; the factors are stored
// back in pivot order so that the triangular solves broadcast from fixed
// lanes.  Group reductions, the pivot search and broadcasts use DPP inside
// 16-lane rows and readlane across rows: every lane of a group computes the
// same expression on the same operands, so group decisions never split.
#include "chem_internal.h"

#include <cfloat>
#include <cmath>

namespace chemgpu {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The lane index with its value hidden from the optimiser: comparisons on it
// are then evaluated where they are used instead of being hoisted out of the
// integration loop as live masks (an empty register-only asm statement).
__device__ __forceinline__ int opaque_lane() {
  int v = (int)(threadIdx.x & (kWave - 1));
  asm volatile("" : "+v"(v));
  return v;
}

// ----------------------------------------------------------- cross-lane ops

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

constexpr int kRor8 = 0x128, kRor4 = 0x124, kRor2 = 0x122, kRor1 = 0x121;

// Sum over the group (all lanes receive the same bits).
template <int NP>
__device__ __forceinline__ double gsum(double v) {
  v += dpp_d<kRor8>(v);
  v += dpp_d<kRor4>(v);
  v += dpp_d<kRor2>(v);
  v += dpp_d<kRor1>(v);
  if constexpr (NP == 32) {
    const int lane = threadIdx.x & (kWave - 1);
    const double a = readlane_d(v, 0) + readlane_d(v, 16);
    const double b = readlane_d(v, 32) + readlane_d(v, 48);
    v = lane < 32 ? a : b;
  } else if constexpr (NP == 64) {
    v = (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
  }
  return v;
}

// Largest value over the group (NaN entries are ignored, as by fmax).
template <int NP>
__device__ __forceinline__ double gmax(double v) {
  v = fmax(v, dpp_d<kRor8>(v));
  v = fmax(v, dpp_d<kRor4>(v));
  v = fmax(v, dpp_d<kRor2>(v));
  v = fmax(v, dpp_d<kRor1>(v));
  if constexpr (NP == 32) {
    const int lane = threadIdx.x & (kWave - 1);
    const double a = fmax(readlane_d(v, 0), readlane_d(v, 16));
    const double b = fmax(readlane_d(v, 32), readlane_d(v, 48));
    v = lane < 32 ? a : b;
  } else if constexpr (NP == 64) {
    v = fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
  }
  return v;
}

template <int NP>
__device__ __forceinline__ int gor(int v) {
  v |= dpp_i<kRor8>(v);
  v |= dpp_i<kRor4>(v);
  v |= dpp_i<kRor2>(v);
  v |= dpp_i<kRor1>(v);
  if constexpr (NP == 32) {
    const int lane = threadIdx.x & (kWave - 1);
    const int a = __builtin_amdgcn_readlane(v, 0) | __builtin_amdgcn_readlane(v, 16);
    const int b = __builtin_amdgcn_readlane(v, 32) | __builtin_amdgcn_readlane(v, 48);
    v = lane < 32 ? a : b;
  } else if constexpr (NP == 64) {
    v = (__builtin_amdgcn_readlane(v, 0) | __builtin_amdgcn_readlane(v, 16)) |
        (__builtin_amdgcn_readlane(v, 32) | __builtin_amdgcn_readlane(v, 48));
  }
  return v;
}

// Pivot of a column: the group lane holding the largest candidate, ties to
// the lowest lane.  A max reduction gives the value; a ballot of the lanes
// that hold it gives the lowest such lane as a bit index, without carrying
// (value, index) pairs through the reduction.  Candidates must not be NaN.
template <int NP>
__device__ __forceinline__ int gpivot(const double cand) {
  const double mx = gmax<NP>(cand);
  const unsigned long long hit = __ballot(cand == mx);
  const int lane = threadIdx.x & (kWave - 1);
  const int base = lane - lane % NP;
  const unsigned long long mine = (NP == kWave) ? hit : ((hit >> base) & ((1ull << (NP & 63)) - 1ull));
  return __builtin_ctzll(mine);
}

// Value of group lane k (a compile-time constant after unrolling) to every
// lane of the group.
template <int NP>
__device__ __forceinline__ double gbcast(double v, const int k) {
  if constexpr (NP == 16) {
    switch (k) {
      case 0: return dpp_d<0x150>(v);
      case 1: return dpp_d<0x151>(v);
      case 2: return dpp_d<0x152>(v);
      case 3: return dpp_d<0x153>(v);
      case 4: return dpp_d<0x154>(v);
      case 5: return dpp_d<0x155>(v);
      case 6: return dpp_d<0x156>(v);
      case 7: return dpp_d<0x157>(v);
      case 8: return dpp_d<0x158>(v);
      case 9: return dpp_d<0x159>(v);
      case 10: return dpp_d<0x15A>(v);
      case 11: return dpp_d<0x15B>(v);
      case 12: return dpp_d<0x15C>(v);
      case 13: return dpp_d<0x15D>(v);
      case 14: return dpp_d<0x15E>(v);
      default: return dpp_d<0x15F>(v);
    }
  } else if constexpr (NP == 32) {
    const int lane = threadIdx.x & (kWave - 1);
    const double a = readlane_d(v, k), b = readlane_d(v, 32 + k);
    return lane < 32 ? a : b;
  } else {
    return readlane_d(v, k);
  }
}

// Per-lane species constants (lane r < S holds species r; other lanes hold
// neutral values), loaded once per kernel.
struct Spc {
  double W, a0, a1, hf, s0;
};

__device__ __forceinline__ Spc load_species(const DevMech& m, const int r) {
  Spc c{1.0, 0.0, 0.0, 0.0, 0.0};
  if (r < m.S) {
    c.W = m.W[r];
    c.a0 = m.a0[r];
    c.a1 = m.a1[r];
    c.hf = m.hf[r];
    c.s0 = m.s0[r];
  }
  return c;
}

template <int NP>
__device__ __forceinline__ float gbcastf(float v, const int k) {
  // broadcast a float through the 64-bit path (exact: float -> double -> float)
  return (float)gbcast<NP>((double)v, k);
}

// ------------------------------------------------------------------ LDS map

// LDS carve-up for one wave (64/NP groups).  Reaction scratch is indexed by
// wave lane, per-species vectors by group base + species index, and each
// group owns N matrix rows of NP+1 doubles (rows N..NP-1 of the padded
// matrix are identity and are not stored).
struct Shared {
  double* J;      // [groups][rows][ldj]: Jacobian rows, then the pivot-ordered LU factors
  double* C;      // [64] concentrations (mol/cm^3)
  double* G;      // [64] G_k/(R T)
  double* H;      // [64] H_k, J/mol
  double* iW;     // [64] 1/W_c for species columns, 0 for the T and padding columns (written once per kernel)
  double* rq;     // [3][64]: per species, sums of nu Q, nu dQ/dT and nu q0 over the reactions
  double* prow;   // [2][64] pivot row, double-buffered: rows 1-2 of rq, which a group never
                  // uses while it factors (the sums are read into registers before)
  int* perm;      // [64] lane whose row holds pivot k
  float* F;       // [groups][rows][ldj] FP32 LU factors (mixed-precision option only)
  float* prow32;  // [2][64] FP32 pivot row
  int ldj;
  int rows;       // stored matrix rows per group: N; rows N..NP-1 are identity and not stored
};

// With f32_in_place (FP32 LU without refinement sweeps, one group per wave)
// the FP32 factors overwrite the group's FP64 Jacobian rows, which nothing
// reads after the factorisation then, and the LDS per wave stays that of the
// FP64 path.
__device__ __forceinline__ Shared carve(double* smem, int NP, int N, bool f32 = false, bool f32_in_place = false) {
  Shared s;
  s.ldj = NP + 1;
  s.rows = N;
  s.C = smem;
  s.G = s.C + kWave;
  s.H = s.G + kWave;
  s.iW = s.H + kWave;
  s.rq = s.iW + kWave;
  s.prow = s.rq + kWave;
  s.perm = reinterpret_cast<int*>(s.rq + 3 * kWave);
  s.J = s.rq + 3 * kWave + kWave / 2;   // perm takes 64 ints = 32 doubles
  const size_t jd = (size_t)(kWave / NP) * N * (NP + 1);
  if (f32 && f32_in_place) {
    s.F = reinterpret_cast<float*>(s.J);
    s.prow32 = reinterpret_cast<float*>(s.prow);   // unused: the 64-lane pivot row goes by readlane
  } else {
    s.F = f32 ? reinterpret_cast<float*>(s.J + jd) : nullptr;
    s.prow32 = f32 ? s.F + jd : nullptr;
  }
  return s;
}

}  // namespace

size_t integrate_lds_bytes(int np_width, int N, bool f32, bool f32_in_place) {
  const int groups = kWave / np_width;
  const size_t jd = (size_t)groups * N * (np_width + 1);
  const size_t doubles = 4 * kWave + 3 * kWave + kWave / 2 + jd;
  return doubles * sizeof(double) + (f32 && !f32_in_place ? (jd + 2 * kWave) * sizeof(float) : 0);
}

namespace {

// Troe's broadening factor of a falloff reaction (CHEMKIN form, logarithms
// base 10): F_cent = (1-a) e^(-T/T3) + a e^(-T/T1) [+ e^(-T2/T)],
// c = -0.4 - 0.67 log F_cent, n = 0.75 - 1.27 log F_cent, d = 0.14,
// f1 = (log Pr + c)/(n - d (log Pr + c)), log F = log F_cent / (1 + f1^2);
// log Pr is taken at max(Pr, 1e-300).  With JAC also d ln F/dT at fixed [M]
// (dlnPr = d ln Pr/dT) and d log F / d log Pr (0 where Pr <= 1e-300).
template <bool JAC>
__device__ __forceinline__ void troe_broadening(const RxParams& x, const double T, const double Pr,
                                                const double dlnPr, double& F, double& dlnF, double& dlogF_dlp) {
  const double a = x.troe[0], T3 = x.troe[1], T1 = x.troe[2];
  const double e3 = exp(-T / T3), e1 = exp(-T / T1);
  double Fc = (1.0 - a) * e3 + a * e1;
  double dFc = -(1.0 - a) / T3 * e3 - a / T1 * e1;
  if (x.ntroe == 4) {
    const double e2 = exp(-x.troe[3] / T);
    Fc += e2;
    dFc += x.troe[3] / (T * T) * e2;
  }
  const double kLn10 = 2.302585092994045684;
  const double Lc = log10(Fc);
  const bool live = Pr > 1e-300;
  const double lp = log10(live ? Pr : 1e-300);
  const double cc = -0.4 - 0.67 * Lc, nn = 0.75 - 1.27 * Lc;
  const double u = lp + cc, v = nn - 0.14 * u;
  const double f1 = u / v;
  const double den = 1.0 + f1 * f1;
  F = exp(kLn10 * (Lc / den));
  if (JAC) {
    const double df1_dlp = nn / (v * v);
    const double df1_dLc = (-0.67 * v - u * (-1.27 + 0.67 * 0.14)) / (v * v);
    dlogF_dlp = live ? -Lc * 2.0 * f1 * df1_dlp / (den * den) : 0.0;
    const double dlogF_dLc = 1.0 / den - Lc * 2.0 * f1 * df1_dLc / (den * den);
    const double dLc_dT = dFc / (Fc * kLn10);
    const double dlp_dT = live ? dlnPr / kLn10 : 0.0;
    dlnF = kLn10 * (dlogF_dlp * dlp_dT + dlogF_dLc * dLc_dT);
  } else {
    dlnF = 0.0;
    dlogF_dlp = 0.0;
  }
}

// Right-hand side of the constant-pressure adiabatic reactor for the group's
// cell at state component yr; with JAC also J = df/dy, left in the group's
// LDS rows (row r = lane r's row; padding rows zero).
//   Eq. 2: Q_j = k_f prod C^nu' - k_r prod C^nu''   (times [M] for third body)
//   Eq. 3: wdot_k = sum_j nu_kj Q_j
//   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum H_k wdot_k / sum C_k Cp_k
// The Jacobian (Eq. 7 in the state (Y, T)) is assembled from the sparse
// concentration-space part A = dwdot/dC (slot products, scattered in LDS by
// each reaction lane into its participants' rows), the
// rank-1 part of [M] (its unit part; efficiencies other than 1 are scattered
// as sparse corrections), the closed-form T derivatives, and
// the chain rule through C_k(Y, T) and rho(Y, T).
template <int NP, bool JAC>
__device__ __forceinline__ void rhs_eval(const DevMech& m, const Spc& sc, const double p, const int fixedT,
                                         const double yr, double& fr, double& wd_out, const Shared& sh) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int g = lane / NP;
  const int base = g * NP;
  const int S = m.S;
  const bool isSp = r < S;
  double* Jg = sh.J + (size_t)g * sh.rows * sh.ldj;

  const double T = __shfl(yr, base + S);
  const double lnT = log(T);
  const double invT = 1.0 / T;

  const double W = sc.W, a0 = sc.a0, a1 = sc.a1, hf = sc.hf, s0 = sc.s0;
  const double Yr = isSp ? yr : 0.0;
  const double sumYW = gsum<NP>(Yr / W);
  const double Wbar = 1.0 / sumYW;
  const double rho = (p * 10.0) * Wbar / (kRuCgs * T);
  const double C = isSp ? rho * Yr / W : 0.0;
  const double Mconc = gsum<NP>(C);
  double H = 0.0, Cp = 0.0, Gd = 0.0, dCp = 0.0;
  if (isSp) {
    double Sm;
    if (m.nasa) {
      // NASA 7-coefficient polynomials of the range holding T (T <= T_mid: low)
      const double* c = m.nasa_c + (T <= m.nasa_c[r] ? 1 : 8) * S + r;
      const double c1 = c[0], c2 = c[S], c3 = c[2 * S], c4 = c[3 * S], c5 = c[4 * S], c6 = c[5 * S],
                   c7 = c[6 * S];
      Cp = kRu * (c1 + T * (c2 + T * (c3 + T * (c4 + T * c5))));
      H = kRu * (T * (c1 + T * (c2 * 0.5 + T * (c3 * (1.0 / 3.0) + T * (c4 * 0.25 + T * (c5 * 0.2))))) + c6);
      Sm = kRu * (c1 * lnT + T * (c2 + T * (c3 * 0.5 + T * (c4 * (1.0 / 3.0) + T * (c5 * 0.25)))) + c7);
      dCp = kRu * (c2 + T * (2.0 * c3 + T * (3.0 * c4 + T * (4.0 * c5))));
    } else {
      H = hf + kRu * (a0 * (T - kTref) + a1 * (T * T - kTref * kTref) * 0.5);
      Sm = s0 + kRu * (a0 * log(T / kTref) + a1 * (T - kTref));
      Cp = kRu * (a0 + a1 * T);
      dCp = kRu * a1;
    }
    Gd = (H - T * Sm) / (kRu * T);
  }
  sh.C[lane] = C;
  sh.G[lane] = Gd;
  sh.H[lane] = H;
  // per-species sums of nu Q, nu dQ/dT and nu q0, added by the reaction lanes
  sh.rq[0 * kWave + lane] = 0.0;
  sh.rq[1 * kWave + lane] = 0.0;
  sh.rq[2 * kWave + lane] = 0.0;
  if (JAC && r < sh.rows) {
#pragma unroll
    for (int c = 0; c < NP; ++c) Jg[r * sh.ldj + c] = 0.0;
  }
  wave_sync();

  const double lnc0 = log(kPatm / (kRu * T) * 1.0e-6);   // ln(p0/(R T)) in mol/cm^3
  const double invRT = 1.0 / (kRu * T);
  double wd = 0.0, bT = 0.0, ak = 0.0;
  double* rq = sh.rq;
  for (int ch = 0; ch < m.nch; ++ch) {
    const int j = ch * NP + r;
    double Q = 0.0, dQdT = 0.0, q0 = 0.0;
    double dq[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) dq[s] = 0.0;
    if (j < m.R) {
      const int4 mt = m.rx_meta[j];
      const int type = mt.x & 3, rev = (mt.x >> 2) & 1, nr = (mt.x >> 3) & 3, np = (mt.x >> 5) & 3;
      const int eff_off = mt.w & 0xFFFFF, eff_n = mt.w >> 20;
      const double xb = m.rx_b[j], xEaR = m.rx_EaR[j];
      // third-body concentration with this reaction's efficiencies
      double Mj = Mconc;
      for (int i = 0; i < eff_n; ++i) Mj += m.eff_v[eff_off + i] * sh.C[base + m.eff_k[eff_off + i]];
      const double kinf = exp(m.rx_lnA[j] + xb * lnT - xEaR * invT);
      double dlnkf = (xb + xEaR * invT) * invT;
      double kf = kinf, dkfdM = 0.0;
      if (type == 2) {   // falloff: the rarer fields from the full record
        const RxParams& x = m.rx[j];
        const double k0 = exp(x.lnA0 + x.b0 * lnT - x.EaR0 * invT);
        const double dlnk0 = (x.b0 + x.EaR0 * invT) * invT;
        const double Pr = k0 * Mj / kinf;
        const double dlnPr = dlnk0 - dlnkf;
        kf = kinf * Pr / (1.0 + Pr);
        dlnkf = dlnkf + dlnPr / (1.0 + Pr);
        dkfdM = k0 / ((1.0 + Pr) * (1.0 + Pr));
        if ((mt.x >> 7) & 1) {
          double F, dlnF, dlogF_dlp;
          troe_broadening<JAC>(x, T, Pr, dlnPr, F, dlnF, dlogF_dlp);
          if (JAC) {
            dkfdM = F * dkfdM + F * k0 / (1.0 + Pr) * dlogF_dlp;
            dlnkf += dlnF;
          }
          kf *= F;
        }
      }
      int sp[kSlots];
#pragma unroll
      for (int s = 0; s < kSlots; ++s) sp[s] = meta_slot(mt, s);
      double cs[kSlots];
#pragma unroll
      for (int s = 0; s < kSlots; ++s) cs[s] = (sp[s] >= 0) ? sh.C[base + sp[s]] : 1.0;
      double pf = 1.0, pr = 1.0;
#pragma unroll
      for (int s = 0; s < kMaxSide; ++s) {
        if (s < nr) pf *= cs[s];
        if (s < np) pr *= cs[kMaxSide + s];
      }
      double kr = 0.0, dkr = 0.0, dkrdM = 0.0;
      if (rev) {
        double sg = 0.0, shh = 0.0;
#pragma unroll
        for (int s = 0; s < kMaxSide; ++s) {
          if (s < np) {
            sg += sh.G[base + sp[kMaxSide + s]];
            if (JAC) shh += sh.H[base + sp[kMaxSide + s]];
          }
          if (s < nr) {
            sg -= sh.G[base + sp[s]];
            if (JAC) shh -= sh.H[base + sp[s]];
          }
        }
        const int dnu = np - nr;
        // k_r = k_f / K_c,  K_c = exp(-sum nu G/RT) (p0/RT)^dnu
        const double ratio = exp(sg - dnu * lnc0);
        kr = kf * ratio;
        if (JAC) {
          const double dlnKc = shh * invRT * invT - dnu * invT;
          dkr = kr * (dlnkf - dlnKc);
          dkrdM = dkfdM * ratio;
        }
      }
      const double mf = (type == 1) ? Mj : 1.0;
      const double net = kf * pf - kr * pr;
      Q = mf * net;
      if (JAC) {
        dQdT = mf * (kf * dlnkf * pf - dkr * pr);
        q0 = (type == 1) ? net : ((type == 2) ? dkfdM * pf - dkrdM * pr : 0.0);
#pragma unroll
        for (int s = 0; s < kMaxSide; ++s) {
          if (s < nr) {
            double t = 1.0;
#pragma unroll
            for (int s2 = 0; s2 < kMaxSide; ++s2)
              if (s2 != s && s2 < nr) t *= cs[s2];
            dq[s] = mf * kf * t;
          }
          if (s < np) {
            double t = 1.0;
#pragma unroll
            for (int s2 = 0; s2 < kMaxSide; ++s2)
              if (s2 != s && s2 < np) t *= cs[kMaxSide + s2];
            dq[kMaxSide + s] = -mf * kr * t;
          }
        }
      }
    }
    // production rates and, for JAC, the concentration-space Jacobian,
    // reaction by reaction: every species k with a nonzero net coefficient
    // nu_kj gets nu_kj Q_j (and nu_kj dQ_j/dT, nu_kj q0_j) in its sums and
    // nu_kj dQ_j/dC_c for each slot species c in its LDS row; with
    // efficiencies other than 1 also nu_kj q0 (eps_jc - 1) in column c (the 1
    // is the rank-one part of [M])
    if (j < m.R) {
      const int4 mt = m.rx_meta[j];
      const int2 nt = m.rx_net[j];
      const int eo = mt.w & 0xFFFFF, en = mt.w >> 20;
#pragma unroll
      for (int p = 0; p < kSlots; ++p) {
        int kp, nup;
        net_slot(nt, p, kp, nup);
        if (kp < 0) continue;
        const double nu = (double)nup;
        __hip_atomic_fetch_add(&rq[0 * kWave + base + kp], nu * Q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (JAC) {
          __hip_atomic_fetch_add(&rq[1 * kWave + base + kp], nu * dQdT, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
          __hip_atomic_fetch_add(&rq[2 * kWave + base + kp], nu * q0, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
#pragma unroll
          for (int s = 0; s < kSlots; ++s) {
            const int c = meta_slot(mt, s);
            if (c >= 0)
              __hip_atomic_fetch_add(&Jg[kp * sh.ldj + c], nu * dq[s], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
          for (int i = 0; i < en; ++i)
            __hip_atomic_fetch_add(&Jg[kp * sh.ldj + m.eff_k[eo + i]], nu * q0 * m.eff_v[eo + i],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
      }
    }
  }
  wave_sync();
  if (isSp) {
    wd = rq[0 * kWave + lane];
    if (JAC) {
      bT = rq[1 * kWave + lane];
      ak = rq[2 * kWave + lane];
    }
  }

  // ODE right-hand side
  const double num = gsum<NP>(isSp ? H * wd : 0.0);
  const double den = gsum<NP>(isSp ? C * Cp : 0.0);
  fr = 0.0;
  if (isSp) fr = W * wd / rho;
  if (r == S) fr = fixedT ? 0.0 : -num / den;
  wd_out = wd;

  if (JAC) {
    // species rows: A_k. = sparse LDS part + rank-1 [M] part
    double AC = 0.0;
    if (isSp)
      for (int c = 0; c < S; ++c) AC += (Jg[r * sh.ldj + c] + ak) * sh.C[base + c];
    const double dwdT = bT - AC * invT;
    const double HA = gsum<NP>(isSp ? H * ak : 0.0);
    const double HAC = gsum<NP>(isSp ? H * AC : 0.0);
    const double HdwdT = gsum<NP>(isSp ? H * dwdT : 0.0);
    const double Cpw = gsum<NP>(isSp ? Cp * wd : 0.0);
    const double Ca1 = gsum<NP>(isSp ? C * dCp : 0.0);
    // column sums sum_k H_k A_kj for column j = r (LDS column read)
    double colsum = HA;
    if (isSp)
      for (int k = 0; k < S; ++k) colsum += sh.H[base + k] * Jg[k * sh.ldj + r];
    wave_sync();   // all column reads done before rows are overwritten
    if (isSp) {
      const double fac = W / rho;
      const double fw = W * wd / rho;
      const double tT = fac * dwdT + fw * invT;
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        // species column c: (W_r/rho) dwdot_r/dY_c + (W_r wdot_r/rho) Wbar/W_c; T column: tT
        const double iWc = sh.iW[base + c];
        Jg[r * sh.ldj + c] = fac * ((Jg[r * sh.ldj + c] + ak) * rho * iWc - Wbar * iWc * AC) + fw * Wbar * iWc +
                             ((c == S) ? 1.0 : 0.0) * tT;
      }
    }
    // temperature row, one column per lane (lanes beyond S write 0)
    double tcol = 0.0;
    if (!fixedT) {
      if (isSp) {
        const double dN = (rho / W) * colsum - (Wbar / W) * HAC;
        const double dD = (rho * Cp - Wbar * den) / W;
        tcol = -dN / den + num * dD / (den * den);
      } else if (r == S) {
        const double dN = Cpw + HdwdT;
        const double dD = -den * invT + Ca1;
        tcol = -dN / den + num * dD / (den * den);
      }
    }
    Jg[S * sh.ldj + r] = tcol;
    wave_sync();
  }
}

// Newton matrix M = I - c J from the group's LDS rows, factored with partial
// pivoting (largest |m_rk| among unused rows, ties to the lowest row) one row
// per lane in registers; the pivot row of each column is published through
// LDS.  On return the LDS rows hold the factors in pivot order (row k = L row
// k below the diagonal, U row k on and above it), perm[k] names the lane whose
// original row became row k, and rdiag = 1/u_rr for lane r's position.
// NC (a multiple of 8, N <= NC <= NP) is the number of columns carried: the
// rows and columns NC..NP-1 hold only identity rows of padding lanes, and the
// elimination steps k >= N change no stored row, so stopping at NC is exact.
template <int NP, int NC = NP>
__device__ __forceinline__ void factor_newton_matrix(const Shared& sh, const double cfac, double& rdiag) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int base = lane - r;
  double* Jg = sh.J + (size_t)(lane / NP) * sh.rows * sh.ldj;
  double a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) a[c] = ((c == r) ? 1.0 : 0.0) - (r < sh.rows ? cfac * Jg[r * sh.ldj + c] : 0.0);
  bool used = false;
  int pos = -1;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double cand = used ? -1.0 : fabs(a[k]);
    if (!(cand == cand)) cand = -1.0;
    const int idx = gpivot<NP>(cand);
    if constexpr (NP == kWave) {
      // one cell per wave: the pivot lane is wave-uniform, and its row reaches
      // every lane by readlane, straight into scalar registers; rows already
      // used take the multiplier 0 and stay as they are (no branch, and no LDS
      // round trip per column pair, which register pressure had serialised)
      if (r == idx) {
        used = true;
        pos = k;
        sh.perm[base + k] = r;
      }
      const double pk = readlane_d(a[k], idx);
      const double l = used ? 0.0 : a[k] / pk;
      if (!used) a[k] = l;
#pragma unroll
      for (int c = k + 1; c < NC; ++c) a[c] -= l * readlane_d(a[c], idx);
    } else {
      double* prow = sh.prow + (k & 1) * kWave + base;
      if (r == idx) {
        used = true;
        pos = k;
        sh.perm[base + k] = r;
#pragma unroll
        for (int c = k; c < NC; ++c) prow[c] = a[c];
      }
      wave_sync();
      if (!used) {
        const double l = a[k] / prow[k];
        a[k] = l;
#pragma unroll
        for (int c = k + 1; c < NC; ++c) a[c] -= l * prow[c];
      }
    }
  }
  // store the rows in pivot order (every lane pivots exactly once).  The
  // identity rows of lanes r >= N pivot at their own position k = r (their
  // column k < N entries are zero and stay zero), so positions >= N are the
  // identity and are not stored.
  if (pos >= 0 && pos < sh.rows) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Jg[pos * sh.ldj + c] = a[c];
  }
  if (r >= NC) sh.perm[base + r] = r;   // padding lanes past NC keep their own position
  wave_sync();
  rdiag = r < sh.rows ? 1.0 / Jg[r * sh.ldj + r] : 1.0;
}

// Solve M x = b with the pivot-ordered factors; lane r holds b_r (component
// r) on entry and returns x_r.
template <int NP, int NC = NP>
__device__ __forceinline__ double lu_solve(const Shared& sh, const double rdiag, const double b) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int base = lane - r;
  const double* Jg = sh.J + (size_t)(lane / NP) * sh.rows * sh.ldj;
  double z = __shfl(b, base + sh.perm[base + r]);   // b in pivot order
#pragma unroll
  for (int k = 0; k < NC - 1; ++k) {
    const double zk = gbcast<NP>(z, k);
    if (r > k && r < sh.rows) z -= Jg[r * sh.ldj + k] * zk;
  }
  double x = 0.0;
#pragma unroll
  for (int k = NC - 1; k >= 0; --k) {
    const double xk = gbcast<NP>(z * rdiag, k);
    if (r < k && r < sh.rows) z -= Jg[r * sh.ldj + k] * xk;
    if (r == k) x = xk;
  }
  return x;
}

// WRMS norm sqrt(sum (v w)^2 / N).  Cold cells can have right-hand sides
// near 1e240 whose squares overflow: then the same norm is taken as
// M sqrt(sum (v w / M)^2 / N) with M = max |v w| (M itself if not finite).
template <int NP>
__device__ __forceinline__ double wrms(const double v, const double w, const int N) {
  const double t = v * w;
  const double s = gsum<NP>(t * t);
  if (__builtin_expect(isfinite(s), 1)) return sqrt(s / N);
  const double M = gmax<NP>(fabs(t));
  if (!isfinite(M)) return M;
  const double u = t / M;
  return M * sqrt(gsum<NP>(u * u) / N);
}

// Columns j0..N-1 of the group's Jacobian rows by one-sided difference
// quotients at y (component yr on lane r), given fy = f(y): the
// finite-difference Jacobian of Sec. 3.2 (the temperature column alone,
// j0 = N-1, in Sec. 3.2.2).  The increment of column j is
// max(sqrt(u) |y_j|, m / w_j) with m = 1000 |h| u N ||f(y)||_w (1 when the
// norm is 0) and u the FP64 unit roundoff, the dense difference-quotient rule
// of the SUNDIALS CVODE documentation.  With j0 = 0 the columns N..NP-1 of the
// stored rows are cleared as well.  Returns the right-hand sides evaluated.
template <int NP>
__device__ __forceinline__ int jac_difference_quotients(const DevMech& m, const Spc& sc, const double p,
                                                        const int fixedT, const double yr, const double fy,
                                                        const double w, const double h, const int N,
                                                        const int j0, const Shared& sh) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int base = lane - r;
  double* Jg = sh.J + (size_t)(lane / NP) * sh.rows * sh.ldj;
  const double u = DBL_EPSILON;
  const double fnorm = wrms<NP>(fy, w, N);
  const double minc = fnorm != 0.0 ? 1000.0 * fabs(h) * u * N * fnorm : 1.0;
  double mine = 0.0;
  if (r < N) {
    const double a = sqrt(u) * fabs(yr), b = minc / w;
    mine = a > b ? a : b;
  }
  if (j0 == 0 && r < sh.rows) {
#pragma unroll
    for (int c = 0; c < NP; ++c)
      if (c >= N) Jg[r * sh.ldj + c] = 0.0;
  }
  for (int j = j0; j < N; ++j) {
    const double inc = __shfl(mine, base + j);
    double f1, wdx;
    rhs_eval<NP, false>(m, sc, p, fixedT, yr + ((r == j) ? inc : 0.0), f1, wdx, sh);
    if (r < N) Jg[r * sh.ldj + j] = (f1 - fy) / inc;
  }
  wave_sync();
  return N - j0;
}

// Mixed-precision option: the same pivoted factorisation of M = I - c J in
// FP32 (M rounded from FP64), factors kept in FP32 LDS rows in pivot order;
// J stays in FP64 for the refinement residuals.
template <int NP, int NC = NP>
__device__ __forceinline__ void factor_newton_matrix_f32(const Shared& sh, const double cfac, float& rdiag) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int base = lane - r;
  const double* Jg = sh.J + (size_t)(lane / NP) * sh.rows * sh.ldj;
  float* Fg = sh.F + (size_t)(lane / NP) * sh.rows * sh.ldj;
  float a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
    a[c] = (float)(((c == r) ? 1.0 : 0.0) - (r < sh.rows ? cfac * Jg[r * sh.ldj + c] : 0.0));
  bool used = false;
  int pos = -1;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double cand = used ? -1.0 : (double)fabsf(a[k]);
    if (!(cand == cand)) cand = -1.0;
    const int idx = gpivot<NP>(cand);
    if constexpr (NP == kWave) {   // pivot row by readlane, as in the FP64 factorisation
      if (r == idx) {
        used = true;
        pos = k;
        sh.perm[base + k] = r;
      }
      const float pk = readlane_f(a[k], idx);
      const float l = used ? 0.0f : a[k] / pk;
      if (!used) a[k] = l;
#pragma unroll
      for (int c = k + 1; c < NC; ++c) a[c] -= l * readlane_f(a[c], idx);
    } else {
      float* prow = sh.prow32 + (k & 1) * kWave + base;
      if (r == idx) {
        used = true;
        pos = k;
        sh.perm[base + k] = r;
#pragma unroll
        for (int c = k; c < NC; ++c) prow[c] = a[c];
      }
      wave_sync();
      if (!used) {
        const float l = a[k] / prow[k];
        a[k] = l;
#pragma unroll
        for (int c = k + 1; c < NC; ++c) a[c] -= l * prow[c];
      }
    }
  }
  // every lane's FP64 row has been read before any FP32 row is stored (the
  // factors may overwrite the FP64 rows, see carve)
  wave_sync();
  if (pos >= 0 && pos < sh.rows) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Fg[pos * sh.ldj + c] = a[c];
  }
  if (r >= NC) sh.perm[base + r] = r;   // padding lanes past NC keep their own position
  wave_sync();
  rdiag = r < sh.rows ? 1.0f / Fg[r * sh.ldj + r] : 1.0f;
}

template <int NP, int NC = NP>
__device__ __forceinline__ double lu_solve_f32(const Shared& sh, const float rdiag, const double b) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const int base = lane - r;
  const float* Fg = sh.F + (size_t)(lane / NP) * sh.rows * sh.ldj;
  float z = (float)__shfl(b, base + sh.perm[base + r]);
#pragma unroll
  for (int k = 0; k < NC - 1; ++k) {
    const float zk = gbcastf<NP>(z, k);
    if (r > k && r < sh.rows) z -= Fg[r * sh.ldj + k] * zk;
  }
  float x = 0.0f;
#pragma unroll
  for (int k = NC - 1; k >= 0; --k) {
    const float xk = gbcastf<NP>(z * rdiag, k);
    if (r < k && r < sh.rows) z -= Fg[r * sh.ldj + k] * xk;
    if (r == k) x = xk;
  }
  return (double)x;
}

// x with M x = b to FP64 accuracy from FP32 factors: x = LU32^-1 b, then
// refinement sweeps x += LU32^-1 (b - M x) with the residual in FP64
// (M x = x - c J x from the FP64 Jacobian rows), until the WRMS correction is
// below 1e-8 or ir_max sweeps have run.
template <int NP, int NC = NP>
__device__ __forceinline__ double solve_refined(const Shared& sh, const float rdiag, const double cfac, const double b,
                                                const double w, const int N, const int ir_max, int& sweeps) {
  const int lane = opaque_lane();
  const int r = lane % NP;
  const double* Jg = sh.J + (size_t)(lane / NP) * sh.rows * sh.ldj;
  double x = lu_solve_f32<NP, NC>(sh, rdiag, b);
  for (int s = 0; s < ir_max; ++s) {
    double jx = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) jx += (r < sh.rows ? Jg[r * sh.ldj + c] : 0.0) * gbcast<NP>(x, c);
    const double res = b - (x - cfac * jx);
    const double dx = lu_solve_f32<NP, NC>(sh, rdiag, res);
    x += dx;
    sweeps++;
    if (wrms<NP>(dx, w, N) <= 1e-8) break;
  }
  return x;
}

// U = R(1) for the difference rescaling: U_ij = prod_{l=1..i} (l - 1 - j)/l.
__device__ constexpr double kU[kQMax + 1][kQMax + 1] = {
    {0, 0, 0, 0, 0, 0},
    {0, -1, -2, -3, -4, -5},
    {0, 0, 1, 3, 6, 10},
    {0, 0, 0, -1, -4, -10},
    {0, 0, 0, 0, 1, 5},
    {0, 0, 0, 0, 0, -1},
};

// BDF coefficients g_j = sum_{i<=j} 1/i.
__device__ __forceinline__ double gamma_k(const int k) {
  switch (k) {
    case 1: return 1.0;
    case 2: return 1.5;
    case 3: return 1.0 + 1.0 / 2 + 1.0 / 3;
    case 4: return 1.0 + 1.0 / 2 + 1.0 / 3 + 1.0 / 4;
    case 5: return 1.0 + 1.0 / 2 + 1.0 / 3 + 1.0 / 4 + 1.0 / 5;
    default: return 1.0 + 1.0 / 2 + 1.0 / 3 + 1.0 / 4 + 1.0 / 5 + 1.0 / 6;
  }
}

// Backward differences D_1..D_mdim mapped to the step ratio rr: D <- D (R U),
// R_ij = prod_{l=1..i} (l - 1 - j rr)/l (Shampine & Reichelt), evaluated as
// v = D R followed by v U to keep few values live.
__device__ __forceinline__ void rescale(double (&D)[kQMax + 2], const int mdim, const double rr) {
  double v[kQMax + 1];
#pragma unroll
  for (int l = 1; l <= kQMax; ++l) {
    double pr = 1.0, acc = 0.0;
#pragma unroll
    for (int i = 1; i <= kQMax; ++i) {
      pr *= (i - 1 - l * rr) / i;
      if (i <= mdim) acc += D[i] * pr;
    }
    v[l] = (l <= mdim) ? acc : 0.0;
  }
#pragma unroll
  for (int j = 1; j <= kQMax; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int l = 1; l <= j; ++l) acc += v[l] * kU[l][j];
    if (j <= mdim) D[j] = acc;
  }
}

__device__ __forceinline__ double pick(const double (&D)[kQMax + 2], const int j) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < kQMax + 2; ++i)
    if (i == j) v = D[i];
  return v;
}

template <int NP>
__device__ __forceinline__ void init_shared_constants(const DevMech& m, const Shared& sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  sh.iW[lane] = (r < m.S) ? 1.0 / m.W[r] : 0.0;
}

// Variable-order BDF over [0, dt] for the group's cell; the same decisions as
// the oracle's per-cell integrator (predictor/corrector in backward
// differences, Newton with a fresh Jacobian and LU per attempt, WRMS error
// test, quasi-constant step size with order selection after k+2 steps, and
// rejection of steps that leave a mass fraction below -atol, projection of
// the mass fractions onto Y >= 0 after every accepted step; T follows its
// own equation).
// One group integrates cell `cell` of the SoA arrays (Tg, Yg, n) over [0, dt];
// its record goes to column rec_cell of the rec array with rec_n columns.
template <int NP, bool F32, int NC = NP>
__device__ __forceinline__ void integrate_group(const DevMech& m, const IntParams& P, const double dt,
                                                const Shared& sh, const Spc& sc, double* __restrict__ Tg,
                                                double* __restrict__ Yg, const int64_t n, const int64_t cell,
                                                int32_t* __restrict__ rec, const int64_t rec_n,
                                                const int64_t rec_cell) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int S = m.S, N = m.N;

  double y0 = 0.0;
  if (r < S) y0 = Yg[(int64_t)r * n + cell];
  else if (r == S) y0 = Tg[cell];
  int bad = 0;
  if (r < N && !isfinite(y0)) bad = 1;
  if (r == S && !(y0 > 0.0)) bad = 1;
  bad = gor<NP>(bad);

  int status = 0, steps = 0, attempts = 0, nrhs = 0, njac = 0, nnewton = 0, netf = 0, nnnf = 0, nir = 0;
  if (bad) {
    status = 3;
  } else {
    const int fixedT = P.fixed_T;
    const bool fixed = P.fixed_step_n > 0;
    const int q_max = P.q_max < 1 ? 1 : (P.q_max > kQMax ? kQMax : P.q_max);
    double D[kQMax + 2];
#pragma unroll
    for (int j = 0; j < kQMax + 2; ++j) D[j] = 0.0;
    D[0] = (r < N) ? y0 : 0.0;
    double f, wdx;
    rhs_eval<NP, false>(m, sc, P.p, fixedT, D[0], f, wdx, sh);
    nrhs++;
    double w = (r < N) ? 1.0 / (P.rtol * fabs(D[0]) + P.atol) : 0.0;
    double h;
    if (fixed) {
      h = dt / P.fixed_step_n;
    } else {
      const double nf = wrms<NP>(f, w, N);
      h = dt;
      if (nf * dt > 1.0) h = 1.0 / nf;
    }
    D[1] = h * f;
    int k = 1, etf = 0, nk = 0;
    double t = 0.0;
    // the factored Newton matrix (LDS rows, perm, rdiag) is kept across
    // attempts while it is recent
    bool have_lu = false, stale_fail = false;
    int steps_lu = 0;
    double c_lu = 0.0;
    double rdiag = 0.0;
    float rdiag32 = 0.0f;
    while (t < dt) {
      const int rl = opaque_lane() % NP;   // lane-index tests stay inside the loop
      if (attempts >= P.max_steps) {
        status = 1;
        break;
      }
      attempts++;
      bool last = false;
      if (fixed) {
        last = (steps + 1 == P.fixed_step_n);
      } else if (t + 1.1 * h >= dt) {   // end exactly at dt (stretch up to 10% or shorten)
        const double hn = dt - t;
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, hn / h);
        h = hn;
        nk = 0;
        last = true;
      }
      if (!(h > 16.0 * DBL_EPSILON * t) || !(h >= 1e-290)) {
        status = 2;
        break;
      }
      w = (rl < N) ? 1.0 / (P.rtol * fabs(D[0]) + P.atol) : 0.0;
      double pred = D[0], ss = 0.0;
#pragma unroll
      for (int j = 1; j <= kQMax; ++j)
        if (j <= k) {
          pred += D[j];
          ss += gamma_k(j) * D[j];
        }
      const double gk = gamma_k(k);
      const double psi = ss / gk;
      const double c = h / gk;

      // keep the factors while c is within 30% of the c they were formed with,
      // fewer than 20 accepted steps have passed and Newton has not failed
      // with them; otherwise a fresh Jacobian at the predictor (all of this
      // is group-uniform)
      const bool fresh = !P.jac_reuse || !have_lu || fabs(c / c_lu - 1.0) > 0.3 || steps - steps_lu >= 20 ||
                         stale_fail;
      double fp = 0.0;
      if (fresh) {
        if (P.jac_mode == 1) {
          // f(pred) serves the quotients and the first Newton residual
          rhs_eval<NP, false>(m, sc, P.p, fixedT, pred, fp, wdx, sh);
          nrhs += jac_difference_quotients<NP>(m, sc, P.p, fixedT, pred, fp, w, h, N, 0, sh);
        } else {
          rhs_eval<NP, true>(m, sc, P.p, fixedT, pred, fp, wdx, sh);
          if (P.jac_mode == 2)
            nrhs += jac_difference_quotients<NP>(m, sc, P.p, fixedT, pred, fp, w, h, N, N - 1, sh);
        }
        njac++;
        if constexpr (F32) factor_newton_matrix_f32<NP, NC>(sh, c, rdiag32);
        else factor_newton_matrix<NP, NC>(sh, c, rdiag);
        have_lu = true;
        c_lu = c;
        steps_lu = steps;
        stale_fail = false;
      }

      double d = 0.0;
      bool conv = false;
      double prev = 0.0;
      const int maxit = fixed ? 50 : 4;
      const double ntol = fixed ? 1e-10 : 0.03;
      for (int it = 1; it <= maxit; ++it) {
        double fi;
        if (it == 1 && fresh) {
          fi = fp;   // f at pred + 0 was evaluated with the Jacobian
        } else {
          rhs_eval<NP, false>(m, sc, P.p, fixedT, pred + d, fi, wdx, sh);
        }
        nrhs++;
        nnewton++;
        const double b = (rl < N) ? -(d - c * fi + psi) : 0.0;
        double delta;
        if constexpr (F32) delta = solve_refined<NP, NC>(sh, rdiag32, c, b, w, N, P.ir_max, nir);
        else delta = lu_solve<NP, NC>(sh, rdiag, b);
        d += delta;
        const double nrm = wrms<NP>(delta, w, N);
        if (nrm <= ntol) {
          conv = true;
          break;
        }
        if (it > 1 && nrm > 2.0 * prev) break;
        prev = nrm;
      }
      if (!conv && !fixed && !fresh) {   // kept factors failed: same step, fresh matrix
        nnnf++;
        stale_fail = true;
        continue;
      }
      if (!conv && !fixed) {
        nnnf++;
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, 0.25);
        h *= 0.25;
        nk = 0;
        continue;
      }
      // inequality constraint: a corrector with a mass fraction below -atol is
      // rejected like a failed error test
      if (!fixed && gor<NP>((rl < S && pred + d < -P.atol) ? 1 : 0)) {
        netf++;
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, 0.25);
        h *= 0.25;
        nk = 0;
        continue;
      }
      const double err = wrms<NP>(d, w, N) / (k + 1);
      if (!fixed && !(err <= 1.0)) {
        netf++;
        etf++;
        double rr;
        if (etf >= 3) {
          k = 1;
          nk = 0;
          rr = 0.1;
        } else {
          rr = 0.9 * pow(err, -1.0 / (k + 1));
          if (rr < 0.2) rr = 0.2;
        }
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, rr);
        h *= rr;
        nk = 0;
        continue;
      }
      // accept: D_{k+2} = d - D_{k+1}, D_{k+1} = d, D_j += D_{j+1} for j = k..0
      {
        const double Dk1 = pick(D, k + 1);
#pragma unroll
        for (int j = 0; j < kQMax + 2; ++j) {
          if (j == k + 2 && k < q_max) D[j] = d - Dk1;
          if (j == k + 1) D[j] = d;
        }
#pragma unroll
        for (int j = kQMax; j >= 0; --j)
          if (j <= k) D[j] = D[j] + D[j + 1];
      }
      // positivity projection: a negative mass fraction is set to zero with
      // all of its differences, so that the next predictor holds it there
      if (rl < S && D[0] < 0.0) {
#pragma unroll
        for (int j = 0; j < kQMax + 2; ++j) D[j] = 0.0;
      }
      t = last ? dt : t + h;
      steps++;
      nk++;
      etf = 0;
      int kn = k;
      double rr = 1.0;
      if (fixed) {
        kn = steps + 1 < q_max ? steps + 1 : q_max;
      } else if (nk >= k + 2) {
        const double tk = 1.2 * pow(err, 1.0 / (k + 1));
        rr = tk > 0.1 ? 1.0 / tk : 10.0;
        if (k > 1) {
          const double ekm1 = wrms<NP>(pick(D, k), w, N) / k;
          const double tm = 1.3 * pow(ekm1, 1.0 / k);
          const double rm = tm > 0.1 ? 1.0 / tm : 10.0;
          if (rm > rr) {
            rr = rm;
            kn = k - 1;
          }
        }
        if (k < q_max) {
          const double ekp1 = wrms<NP>(pick(D, k + 2), w, N) / (k + 2);
          const double tp = 1.4 * pow(ekp1, 1.0 / (k + 2));
          const double rp = tp > 0.1 ? 1.0 / tp : 10.0;
          if (rp > rr) {
            rr = rp;
            kn = k + 1;
          }
        }
        if (rr > 10.0) rr = 10.0;
        if (rr <= 1.0) {
          rr = 1.0;
          kn = k;
        }
      }
      if (kn != k) {
        k = kn;
        nk = 0;
      }
      if (rr != 1.0) {
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, rr);
        nk = 0;
      }
      h *= rr;
    }
    if (r < S) Yg[(int64_t)r * n + cell] = D[0];
    else if (r == S) Tg[cell] = D[0];
  }
  if (rec != nullptr && r == 0) {
    int32_t* rc = rec + rec_cell;
    rc[0 * rec_n] = status;
    rc[1 * rec_n] = steps;
    rc[2 * rec_n] = attempts;
    rc[3 * rec_n] = nrhs;
    rc[4 * rec_n] = njac;
    rc[5 * rec_n] = nnewton;
    rc[6 * rec_n] = netf;
    rc[7 * rec_n] = nnnf;
    rc[8 * rec_n] = nir;
  }
}

template <int NP, bool F32, int NC = NP>
__global__ __launch_bounds__(kWave) void integrate_kernel(const DevMech m, const IntParams P, double* __restrict__ Tg,
                                                          double* __restrict__ Yg, const int64_t n,
                                                          int32_t* __restrict__ rec) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, NP, m.N, F32, F32 && NP == kWave && P.ir_max == 0);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int64_t cell = (int64_t)blockIdx.x * (kWave / NP) + lane / NP;
  if (cell >= n) return;   // whole groups leave together
  init_shared_constants<NP>(m, sh);
  const Spc sc = load_species(m, r);
  integrate_group<NP, F32, NC>(m, P, P.dt, sh, sc, Tg, Yg, n, cell, rec, n, cell);
}

// Persistent variant for many boxes of uneven size and step: each wave takes
// (box, tile of 64/NP cells) items from a device counter until the queue is
// empty.  Items follow the box order given by the host (largest boxes first);
// the wave that finishes a box's last tile raises that box's flag in
// host-mapped memory (for latency timing on the host).
template <int NP, bool F32, int NC = NP>
__global__ __launch_bounds__(kWave) void boxes_kernel(const DevMech m, const IntParams P,
                                                      const BoxDev* __restrict__ boxes, const BoxJob* __restrict__ job,
                                                      unsigned* __restrict__ head, int* __restrict__ remaining,
                                                      int32_t* __restrict__ rec, int* __restrict__ host_done) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, NP, m.N, F32, F32 && NP == kWave && P.ir_max == 0);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  init_shared_constants<NP>(m, sh);
  const Spc sc = load_species(m, r);
  const int nbox = job->n_boxes;
  const unsigned total = job->total_tiles;
  const int64_t rec_n = job->total_cells;
  // The lane tests below use opaque_lane(), evaluated afresh in every
  // iteration: with a lane test computed once before the loop, the compiler
  // treats it as loop-invariant and may thread lane 0's two atomic regions
  // into a loop of their own, leaving lanes 1..63 to re-enter the body
  // without a new item.  The item is then taken from lane 0 by readlane,
  // which does not depend on which lanes are active.
  for (;;) {
    unsigned item = 0;
    if (opaque_lane() == 0) item = atomicAdd(head, 1u);
    item = (unsigned)__builtin_amdgcn_readlane((int)item, 0);
    if (item >= total) break;
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {   // last box whose first tile is <= item
      const int mid = (lo + hi + 1) >> 1;
      if (boxes[mid].tile_pre <= (int64_t)item) lo = mid;
      else hi = mid - 1;
    }
    const BoxDev bx = boxes[lo];
    const int64_t c = ((int64_t)item - bx.tile_pre) * (kWave / NP) + g;
    if (c < bx.n) integrate_group<NP, F32, NC>(m, P, bx.dt, sh, sc, bx.T, bx.Y, bx.n, c, rec, rec_n, bx.cell_off + c);
    if (opaque_lane() == 0) {
      const int left = atomicSub(&remaining[lo], 1);
      if (left == 1 && host_done != nullptr) {
        __threadfence_system();
        host_done[bx.box_id] = 1;
      }
    }
  }
}

// Resident serving kernel: the box loop of boxes_kernel over a queue the
// host appends to while it runs (see ServeQueue).  Lane 0 claims a tile by
// compare-and-swap below the published count, polling with s_sleep while
// none is published, for at most q.idle_spins empty polls or until q.stop.
// Device half of the serving queue protocol (the queue layout is described
// with ServeQueue).  serve_claim runs on lane 0 only: it returns 1 with the
// claimed tile and its ring slot, or 0 when the wave should leave.  The
// published count is polled with relaxed loads and backoff; the acquire
// fence after a successful claim pairs with the host's release of *pub.
__device__ int serve_claim(const ServeQueue& q, unsigned* item, unsigned* slot) {
  unsigned backoff = 1;
  int polls = 0;
  for (int tries = 0; tries < (1 << 22); ++tries) {
    if (__hip_atomic_load(q.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) return 0;
    const unsigned pub = __hip_atomic_load(q.pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned h = __hip_atomic_load(q.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (h < pub) {
      if (__hip_atomic_compare_exchange_strong(q.head, &h, h + 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        *item = h;
        *slot = __hip_atomic_load(&q.tile_slot[h & q.tile_mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return 1;
      }
      continue;   // another wave took tile h: look again at once
    }
    if (++polls >= q.idle_polls) return 0;
    for (unsigned z = 0; z < backoff; ++z) __builtin_amdgcn_s_sleep(127);
    if (backoff < 16) backoff <<= 1;
  }
  return 0;
}

// Lane 0, after the wave's stores of the tile: count the tile, and on the
// box's last one reset the counter for the slot's next box and raise done.
__device__ void serve_finish(const ServeQueue& q, unsigned slot, int tiles) {
  const int fin = __hip_atomic_fetch_add(&q.finished[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
  if (fin == tiles) {
    __hip_atomic_store(&q.finished[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q.done[slot], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// A box descriptor read by lane 0 from host-mapped memory (atomic loads, so
// that no cached copy of an earlier box in the slot is used) and broadcast.
struct ServeBoxRegs {
  double* T;
  double* Y;
  int32_t* rec;
  int64_t n, tile_pre;
  double dt;
};

__device__ __forceinline__ uint64_t bcast_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t load_sys_u64(const void* p) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int NP, bool F32, int NC = NP>
__global__ __launch_bounds__(kWave) void serve_kernel(const DevMech m, const IntParams P, const ServeQueue q) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, NP, m.N, F32, F32 && NP == kWave && P.ir_max == 0);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  constexpr int kCpt = kWave / NP;
  init_shared_constants<NP>(m, sh);
  const Spc sc = load_species(m, r);
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    unsigned item = 0, slot = 0;
    int got = 0;
    uint64_t w[6] = {0, 0, 0, 0, 0, 0};
    if (lane == 0) {
      got = serve_claim(q, &item, &slot);
      if (got) {
        const uint64_t* d = reinterpret_cast<const uint64_t*>(&q.boxes[slot]);
        for (int i = 0; i < 6; ++i) w[i] = load_sys_u64(d + i);
      }
    }
    if (!__builtin_amdgcn_readfirstlane(got)) break;
    item = (unsigned)__builtin_amdgcn_readfirstlane((int)item);
    slot = (unsigned)__builtin_amdgcn_readfirstlane((int)slot);
    ServeBoxRegs bx;
    bx.T = reinterpret_cast<double*>(bcast_u64(w[0]));
    bx.Y = reinterpret_cast<double*>(bcast_u64(w[1]));
    bx.rec = reinterpret_cast<int32_t*>(bcast_u64(w[2]));
    bx.n = (int64_t)bcast_u64(w[3]);
    bx.dt = __builtin_bit_cast(double, bcast_u64(w[4]));
    bx.tile_pre = (int64_t)bcast_u64(w[5]);
    const int64_t c = ((int64_t)item - bx.tile_pre) * kCpt + g;
    if (c < bx.n) integrate_group<NP, F32, NC>(m, P, bx.dt, sh, sc, bx.T, bx.Y, bx.n, c, bx.rec, bx.n, c);
    __syncthreads();
    if (lane == 0) serve_finish(q, slot, (int)((bx.n + kCpt - 1) / kCpt));
    if (q.quantum > 0 && (int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > q.quantum) break;
  }
}

__global__ void zero_u32_kernel(unsigned* __restrict__ p, const int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}


// Queue counters for boxes_kernel: head = 0, remaining[i] = tiles of box i.
__global__ void boxes_init_kernel(const BoxDev* __restrict__ boxes, const BoxJob* __restrict__ job,
                                  unsigned* __restrict__ head, int* __restrict__ remaining) {
  const int nbox = job->n_boxes;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbox; i += gridDim.x * blockDim.x) {
    const int64_t next = (i + 1 < nbox) ? boxes[i + 1].tile_pre : (int64_t)job->total_tiles;
    remaining[i] = (int)(next - boxes[i].tile_pre);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *head = 0u;
}

template <int NP>
__global__ __launch_bounds__(kWave) void rates_kernel(const DevMech m, const double p, const int fixedT,
                                                      const double* __restrict__ Tg, const double* __restrict__ Yg,
                                                      const int64_t n, double* __restrict__ wdot,
                                                      double* __restrict__ fout, double* __restrict__ jac) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, NP, m.N);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  const int S = m.S, N = m.N;
  const int64_t cell = (int64_t)blockIdx.x * (kWave / NP) + g;
  if (cell >= n) return;
  init_shared_constants<NP>(m, sh);
  const Spc sc = load_species(m, r);
  double y = 0.0;
  if (r < S) y = Yg[(int64_t)r * n + cell];
  else if (r == S) y = Tg[cell];
  double f, wd;
  if (jac != nullptr) rhs_eval<NP, true>(m, sc, p, fixedT, y, f, wd, sh);
  else rhs_eval<NP, false>(m, sc, p, fixedT, y, f, wd, sh);
  if (r < S) wdot[(int64_t)r * n + cell] = wd * 1.0e6;   // mol/(cm^3 s) -> mol/(m^3 s)
  if (fout != nullptr && r < N) fout[(int64_t)r * n + cell] = f;
  if (jac != nullptr && r < N) {
    const double* Jg = sh.J + (size_t)g * sh.rows * sh.ldj;
    for (int c = 0; c < N; ++c) jac[((int64_t)r * N + c) * n + cell] = Jg[r * sh.ldj + c];
  }
}

__global__ void reduce_records_kernel(const int32_t* __restrict__ rec, int64_t n,
                                      unsigned long long* __restrict__ out, const BoxJob* __restrict__ job) {
  if (job != nullptr) n = job->total_cells;
  __shared__ unsigned long long part[kStatCount][256];
  unsigned long long acc[kStatCount];
#pragma unroll
  for (int i = 0; i < kStatCount; ++i) acc[i] = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int st = rec[c];
    const unsigned long long steps = (unsigned)rec[1 * n + c];
    acc[0] += steps;
    acc[1] = acc[1] > steps ? acc[1] : steps;
    acc[2] += (unsigned)rec[2 * n + c];
    acc[3] += (unsigned)rec[3 * n + c];
    acc[4] += (unsigned)rec[4 * n + c];
    acc[5] += (unsigned)rec[5 * n + c];
    acc[6] += (unsigned)rec[6 * n + c];
    acc[7] += (unsigned)rec[7 * n + c];
    acc[8] += (st != 0) ? 1u : 0u;
    acc[9] += (unsigned)rec[8 * n + c];
  }
#pragma unroll
  for (int i = 0; i < kStatCount; ++i) part[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int i = 0; i < kStatCount; ++i) {
        if (i == 1) {
          const unsigned long long a = part[i][threadIdx.x], b = part[i][threadIdx.x + s];
          part[i][threadIdx.x] = a > b ? a : b;
        } else {
          part[i][threadIdx.x] += part[i][threadIdx.x + s];
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < kStatCount; ++i) {
      if (i == 1) atomicMax(&out[i], part[i][0]);
      else atomicAdd(&out[i], part[i][0]);
    }
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int cnt) {
  const int i = threadIdx.x;
  if (i < cnt) p[i] = 0;
}

// Columns carried by the factorisations (FP64 and FP32) of the 64-lane
// kernels when the cell's N fits (S up to 55): eight padding columns fewer to
// eliminate, solve and refine.  Larger mechanisms take all 64.
constexpr int kNarrowCols = 56;

template <int NP>
hipError_t launch_integrate_np(const DevMech& m, const IntParams& prm, double* T, double* Y, int64_t n,
                               int32_t* rec, hipStream_t stream) {
  const int cpw = kWave / NP;
  const int64_t blocks = (n + cpw - 1) / cpw;
  const bool f32 = prm.lu_fp32 != 0;
  const size_t lds = integrate_lds_bytes(NP, m.N, f32, f32 && NP == kWave && prm.ir_max == 0);
  if constexpr (NP == kWave) {
    if (m.N <= kNarrowCols) {
      if (f32)
        hipLaunchKernelGGL((integrate_kernel<NP, true, kNarrowCols>), dim3((unsigned)blocks), dim3(kWave), lds,
                           stream, m, prm, T, Y, n, rec);
      else
        hipLaunchKernelGGL((integrate_kernel<NP, false, kNarrowCols>), dim3((unsigned)blocks), dim3(kWave), lds,
                           stream, m, prm, T, Y, n, rec);
      return hipGetLastError();
    }
  }
  if (f32)
    hipLaunchKernelGGL((integrate_kernel<NP, true>), dim3((unsigned)blocks), dim3(kWave), lds, stream, m, prm, T, Y,
                       n, rec);
  else
    hipLaunchKernelGGL((integrate_kernel<NP, false>), dim3((unsigned)blocks), dim3(kWave), lds, stream, m, prm, T,
                       Y, n, rec);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_rates_np(const DevMech& m, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                           double* wdot, double* f, double* jac, hipStream_t stream) {
  const int cpw = kWave / NP;
  const int64_t blocks = (n + cpw - 1) / cpw;
  const size_t lds = integrate_lds_bytes(NP, m.N, false);
  hipLaunchKernelGGL(rates_kernel<NP>, dim3((unsigned)blocks), dim3(kWave), lds, stream, m, p, fixed_T, T, Y, n,
                     wdot, f, jac);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_boxes_np(const DevMech& m, const IntParams& prm, const BoxDev* boxes, const BoxJob* job,
                           unsigned* head, int* remaining, int32_t* rec, int* host_done, int grid,
                           hipStream_t stream) {
  const bool f32 = prm.lu_fp32 != 0;
  const size_t lds = integrate_lds_bytes(NP, m.N, f32, f32 && NP == kWave && prm.ir_max == 0);
  hipLaunchKernelGGL(boxes_init_kernel, dim3(64), dim3(256), 0, stream, boxes, job, head, remaining);
  if constexpr (NP == kWave) {
    if (m.N <= kNarrowCols) {
      if (f32)
        hipLaunchKernelGGL((boxes_kernel<NP, true, kNarrowCols>), dim3(grid), dim3(kWave), lds, stream, m, prm,
                           boxes, job, head, remaining, rec, host_done);
      else
        hipLaunchKernelGGL((boxes_kernel<NP, false, kNarrowCols>), dim3(grid), dim3(kWave), lds, stream, m, prm,
                           boxes, job, head, remaining, rec, host_done);
      return hipGetLastError();
    }
  }
  if (f32)
    hipLaunchKernelGGL((boxes_kernel<NP, true>), dim3(grid), dim3(kWave), lds, stream, m, prm, boxes, job, head,
                       remaining, rec, host_done);
  else
    hipLaunchKernelGGL((boxes_kernel<NP, false>), dim3(grid), dim3(kWave), lds, stream, m, prm, boxes, job, head,
                       remaining, rec, host_done);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_serve_np(const DevMech& m, const IntParams& prm, const ServeQueue& q, int grid, hipStream_t stream) {
  const bool f32 = prm.lu_fp32 != 0;
  const size_t lds = integrate_lds_bytes(NP, m.N, f32, f32 && NP == kWave && prm.ir_max == 0);
  if constexpr (NP == kWave) {
    if (m.N <= kNarrowCols) {
      if (f32)
        hipLaunchKernelGGL((serve_kernel<NP, true, kNarrowCols>), dim3(grid), dim3(kWave), lds, stream, m, prm, q);
      else
        hipLaunchKernelGGL((serve_kernel<NP, false, kNarrowCols>), dim3(grid), dim3(kWave), lds, stream, m, prm, q);
      return hipGetLastError();
    }
  }
  if (f32)
    hipLaunchKernelGGL((serve_kernel<NP, true>), dim3(grid), dim3(kWave), lds, stream, m, prm, q);
  else
    hipLaunchKernelGGL((serve_kernel<NP, false>), dim3(grid), dim3(kWave), lds, stream, m, prm, q);
  return hipGetLastError();
}

template <int NP>
int serve_waves_np(const DevMech& m, bool f32, int ir_max) {
  int blocks = 0;
  const size_t lds = integrate_lds_bytes(NP, m.N, f32, f32 && NP == kWave && ir_max == 0);
  if constexpr (NP == kWave) {
    if (m.N <= kNarrowCols) {
      const hipError_t e =
          f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, serve_kernel<NP, true, kNarrowCols>, kWave, lds)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, serve_kernel<NP, false, kNarrowCols>, kWave, lds);
      return e == hipSuccess && blocks > 0 ? blocks : 1;
    }
  }
  const hipError_t e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, serve_kernel<NP, true>, kWave, lds)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, serve_kernel<NP, false>, kWave, lds);
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_serve(const DevMech& m, const IntParams& prm, const ServeQueue& q, int grid, hipStream_t stream) {
  switch (m.np_width) {
    case 16: return launch_serve_np<16>(m, prm, q, grid, stream);
    case 32: return launch_serve_np<32>(m, prm, q, grid, stream);
    case 64: return launch_serve_np<64>(m, prm, q, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

int serve_waves_per_cu(const DevMech& m, bool f32, int ir_max) {
  switch (m.np_width) {
    case 16: return serve_waves_np<16>(m, f32, ir_max);
    case 32: return serve_waves_np<32>(m, f32, ir_max);
    case 64: return serve_waves_np<64>(m, f32, ir_max);
    default: return 1;
  }
}

hipError_t launch_zero_u32(unsigned* p, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((count + 255) / 256 < 64 ? (count + 255) / 256 : 64), dim3(256), 0, stream,
                     p, count);
  return hipGetLastError();
}

hipError_t launch_boxes_init(const BoxDev* boxes, const BoxJob* job, unsigned* head, int* remaining,
                             hipStream_t stream) {
  hipLaunchKernelGGL(boxes_init_kernel, dim3(64), dim3(256), 0, stream, boxes, job, head, remaining);
  return hipGetLastError();
}

hipError_t launch_boxes(const DevMech& m, const IntParams& prm, const BoxDev* boxes, const BoxJob* job,
                        unsigned* head, int* remaining, int32_t* rec, int* host_done, int grid,
                        hipStream_t stream) {
  switch (m.np_width) {
    case 16: return launch_boxes_np<16>(m, prm, boxes, job, head, remaining, rec, host_done, grid, stream);
    case 32: return launch_boxes_np<32>(m, prm, boxes, job, head, remaining, rec, host_done, grid, stream);
    case 64: return launch_boxes_np<64>(m, prm, boxes, job, head, remaining, rec, host_done, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_integrate(const DevMech& m, const IntParams& prm, double* T, double* Y, int64_t n, int32_t* rec,
                            hipStream_t stream) {
  switch (m.np_width) {
    case 16: return launch_integrate_np<16>(m, prm, T, Y, n, rec, stream);
    case 32: return launch_integrate_np<32>(m, prm, T, Y, n, rec, stream);
    case 64: return launch_integrate_np<64>(m, prm, T, Y, n, rec, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rates(const DevMech& m, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                        double* wdot, double* f, double* jac, hipStream_t stream) {
  switch (m.np_width) {
    case 16: return launch_rates_np<16>(m, p, fixed_T, T, Y, n, wdot, f, jac, stream);
    case 32: return launch_rates_np<32>(m, p, fixed_T, T, Y, n, wdot, f, jac, stream);
    case 64: return launch_rates_np<64>(m, p, fixed_T, T, Y, n, wdot, f, jac, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_records(const int32_t* rec, int64_t n, unsigned long long* out, hipStream_t stream) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, out, kStatCount);
  if (n > 0) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(reduce_records_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, rec, n, out,
                       (const BoxJob*)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_records_job(const int32_t* rec, const BoxJob* job, unsigned long long* out,
                                     hipStream_t stream) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, out, kStatCount);
  hipLaunchKernelGGL(reduce_records_kernel, dim3(1024), dim3(256), 0, stream, rec, (int64_t)0, out, job);
  return hipGetLastError();
}

}  // namespace chemgpu
