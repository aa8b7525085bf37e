// chem_kernels.hip -- gfx950 kernels for per-cell stiff chemistry.
//
// Layout: one cell per group of NP lanes (NP = 16, 32 or 64 >= S + 1), 64/NP
// cells per wave, one wave per workgroup.  Lane r of a group owns component r
// of the state y = (Y_1..Y_S, T) and row r of the cell's Newton matrix, held
// in VGPRs.  Reactions are spread over the group's lanes (reaction j on lane
// j mod NP, in chunks of NP); species concentrations and Gibbs energies are
// exchanged through LDS, production rates are gathered per species lane in
// reaction order, and the sparse part of the Jacobian is scattered into
// LDS rows with f64 LDS atomics before each lane loads its row.  Group sums
// and the pivot search use xor-butterfly shuffles, whose commutative adds
// give every lane of the group the same bits, so group decisions never split.
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

template <int NP>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int o = NP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int NP>
__device__ __forceinline__ int gor(int v) {
#pragma unroll
  for (int o = NP / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}

// Largest value in the group, ties to the lowest lane index.
template <int NP>
__device__ __forceinline__ void gargmax(double& v, int& idx) {
#pragma unroll
  for (int o = NP / 2; o > 0; o >>= 1) {
    double ov = __shfl_xor(v, o);
    int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// LDS carve-up for one wave (64/NP groups).  Reaction scratch is indexed by
// wave lane, vectors by group base + species index.
struct Shared {
  double* J;      // [groups][N][ldj]
  double* C;      // [64] concentrations
  double* G;      // [64] G_k/(R T)
  double* H;      // [64] H_k, J/mol
  double* W;      // [64] molecular weights (written once per kernel)
  double* iW;     // [64] 1/W_c for species columns, 0 for the T and padding columns
  double* isT;    // [64] 1 for the temperature column, else 0
  double* rq;     // [9][64]: Q, dQ/dT, q0, dQ/dC slots 0..5
  double* prow;   // [2][64] pivot row, double-buffered
  int* perm;      // [64] lane holding the pivot of column k
  int ldj;
  int N;
};

__device__ __forceinline__ Shared carve(double* smem, int N, int NP) {
  Shared s;
  s.N = N;
  s.ldj = NP + 1;
  s.C = smem;
  s.G = s.C + kWave;
  s.H = s.G + kWave;
  s.W = s.H + kWave;
  s.iW = s.W + kWave;
  s.isT = s.iW + kWave;
  s.rq = s.isT + kWave;
  s.prow = s.rq + 9 * kWave;
  s.perm = reinterpret_cast<int*>(s.prow + 2 * kWave);
  s.J = s.prow + 2 * kWave + kWave / 2;   // perm takes 64 ints = 32 doubles
  return s;
}

}  // namespace

size_t integrate_lds_bytes(int np_width, int N) {
  const int groups = kWave / np_width;
  const size_t doubles = 6 * kWave + 9 * kWave + 2 * kWave + kWave / 2 + (size_t)groups * N * (np_width + 1);
  return doubles * sizeof(double);
}

namespace {

// Right-hand side of the constant-pressure adiabatic reactor (and, with JAC,
// lane r's row of J = df/dy) for the group's cell at state component yr.
//   Eq. 2: Q_j = k_f prod C^nu' - k_r prod C^nu''   (times [M] for third body)
//   Eq. 3: wdot_k = sum_j nu_kj Q_j
//   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum H_k wdot_k / sum C_k Cp_k
// The Jacobian (Eq. 7 in the state (Y, T)) is assembled from the sparse
// concentration-space part A = dwdot/dC (slot products, scattered in LDS), the
// rank-1 part of [M] (unit efficiencies), the closed-form T derivatives, and
// the chain rule through C_k(Y, T) and rho(Y, T).
template <int NP, bool JAC>
__device__ __forceinline__ void rhs_eval(const DevMech& m, const double p, const int fixedT, const double yr,
                                         double& fr, double& wd_out, double (&jrow)[NP], const Shared& sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  const int base = g * NP;
  const int S = m.S;
  const bool isSp = r < S;
  double* Jg = sh.J + (size_t)g * sh.N * sh.ldj;

  const double T = __shfl(yr, base + S);
  const double lnT = log(T);
  const double invT = 1.0 / T;

  double W = 1.0, a0 = 0.0, a1 = 0.0, hf = 0.0, s0 = 0.0;
  if (isSp) {
    W = m.W[r];
    a0 = m.a0[r];
    a1 = m.a1[r];
    hf = m.hf[r];
    s0 = m.s0[r];
  }
  const double Yr = isSp ? yr : 0.0;
  const double sumYW = gsum<NP>(Yr / W);
  const double Wbar = 1.0 / sumYW;
  const double rho = (p * 10.0) * Wbar / (kRuCgs * T);
  const double C = isSp ? rho * Yr / W : 0.0;
  const double Mconc = gsum<NP>(C);
  double H = 0.0, Cp = 0.0, Gd = 0.0;
  if (isSp) {
    H = hf + kRu * (a0 * (T - kTref) + a1 * (T * T - kTref * kTref) * 0.5);
    const double Sm = s0 + kRu * (a0 * log(T / kTref) + a1 * (T - kTref));
    Cp = kRu * (a0 + a1 * T);
    Gd = (H - T * Sm) / (kRu * T);
  }
  sh.C[lane] = C;
  sh.G[lane] = Gd;
  sh.H[lane] = H;
  if (JAC && isSp) {
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
      const RxParams x = m.rx[j];
      const double kinf = exp(x.lnA + x.b * lnT - x.EaR * invT);
      double dlnkf = (x.b + x.EaR * invT) * invT;
      double kf = kinf, dkfdM = 0.0;
      if (x.type == 2) {
        const double k0 = exp(x.lnA0 + x.b0 * lnT - x.EaR0 * invT);
        const double dlnk0 = (x.b0 + x.EaR0 * invT) * invT;
        const double Pr = k0 * Mconc / kinf;
        kf = kinf * Pr / (1.0 + Pr);
        dlnkf = dlnkf + (dlnk0 - dlnkf) / (1.0 + Pr);
        dkfdM = k0 / ((1.0 + Pr) * (1.0 + Pr));
      }
      double cs[kSlots];
#pragma unroll
      for (int s = 0; s < kSlots; ++s) cs[s] = (x.sp[s] >= 0) ? sh.C[base + x.sp[s]] : 1.0;
      double pf = 1.0, pr = 1.0;
#pragma unroll
      for (int s = 0; s < kMaxSide; ++s) {
        if (s < x.nr) pf *= cs[s];
        if (s < x.np) pr *= cs[kMaxSide + s];
      }
      double kr = 0.0, dkr = 0.0, dkrdM = 0.0;
      if (x.rev) {
        double sg = 0.0, shh = 0.0;
#pragma unroll
        for (int s = 0; s < kMaxSide; ++s) {
          if (s < x.np) {
            sg += sh.G[base + x.sp[kMaxSide + s]];
            shh += sh.H[base + x.sp[kMaxSide + s]];
          }
          if (s < x.nr) {
            sg -= sh.G[base + x.sp[s]];
            shh -= sh.H[base + x.sp[s]];
          }
        }
        const int dnu = x.np - x.nr;
        // k_r = k_f / K_c,  K_c = exp(-sum nu G/RT) (p0/RT)^dnu
        const double ratio = exp(sg - dnu * lnc0);
        kr = kf * ratio;
        if (JAC) {
          const double dlnKc = shh * invRT * invT - dnu * invT;
          dkr = kr * (dlnkf - dlnKc);
          dkrdM = dkfdM * ratio;
        }
      }
      const double mf = (x.type == 1) ? Mconc : 1.0;
      const double net = kf * pf - kr * pr;
      Q = mf * net;
      if (JAC) {
        dQdT = mf * (kf * dlnkf * pf - dkr * pr);
        q0 = (x.type == 1) ? net : ((x.type == 2) ? dkfdM * pf - dkrdM * pr : 0.0);
#pragma unroll
        for (int s = 0; s < kMaxSide; ++s) {
          if (s < x.nr) {
            double t = 1.0;
#pragma unroll
            for (int s2 = 0; s2 < kMaxSide; ++s2)
              if (s2 != s && s2 < x.nr) t *= cs[s2];
            dq[s] = mf * kf * t;
          }
          if (s < x.np) {
            double t = 1.0;
#pragma unroll
            for (int s2 = 0; s2 < kMaxSide; ++s2)
              if (s2 != s && s2 < x.np) t *= cs[kMaxSide + s2];
            dq[kMaxSide + s] = -mf * kr * t;
          }
        }
      }
    }
    rq[0 * kWave + lane] = Q;
    if (JAC) {
      rq[1 * kWave + lane] = dQdT;
      rq[2 * kWave + lane] = q0;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) rq[(3 + s) * kWave + lane] = dq[s];
    }
    wave_sync();
    if (isSp) {
      const int* off = m.csr_off + r * (m.nch + 1) + ch;
      const int e0 = off[0], e1 = off[1];
      for (int e = e0; e < e1; ++e) {
        const int ent = m.csr_ent[e];
        const int jj = ent >> 3;
        const double nu = (double)((ent & 7) - 4);
        const int src = base + (jj - ch * NP);
        wd += nu * rq[src];
        if (JAC) {
          bT += nu * rq[1 * kWave + src];
          ak += nu * rq[2 * kWave + src];
          const int* sp = m.rx[jj].sp;
#pragma unroll
          for (int s = 0; s < kSlots; ++s) {
            const int c = sp[s];
            if (c >= 0)
              __hip_atomic_fetch_add(&Jg[r * sh.ldj + c], nu * rq[(3 + s) * kWave + src], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
        }
      }
    }
    wave_sync();
  }

  // ODE right-hand side
  const double num = gsum<NP>(isSp ? H * wd : 0.0);
  const double den = gsum<NP>(isSp ? C * Cp : 0.0);
  fr = 0.0;
  if (isSp) fr = W * wd / rho;
  if (r == S) fr = fixedT ? 0.0 : -num / den;
  wd_out = wd;

  if (JAC) {
    // species rows: A_k. = sparse LDS part + rank-1 [M] part (read twice from LDS)
    double AC = 0.0;
    if (isSp)
      for (int c = 0; c < S; ++c) AC += (Jg[r * sh.ldj + c] + ak) * sh.C[base + c];
    const double dwdT = bT - AC * invT;
    const double HA = gsum<NP>(isSp ? H * ak : 0.0);
    const double HAC = gsum<NP>(isSp ? H * AC : 0.0);
    const double HdwdT = gsum<NP>(isSp ? H * dwdT : 0.0);
    const double Cpw = gsum<NP>(isSp ? Cp * wd : 0.0);
    const double Ca1 = gsum<NP>(isSp ? C * kRu * a1 : 0.0);
    // column sums sum_k H_k A_kj for column j = r (LDS column read)
    double colsum = HA;
    if (isSp)
      for (int k = 0; k < S; ++k) colsum += sh.H[base + k] * Jg[k * sh.ldj + r];
    const double fac = W / rho;
    const double fw = W * wd / rho;
    const double tT = fac * dwdT + fw * invT;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      // species column c: (W_r/rho) dwdot_r/dY_c + (W_r wdot_r/rho) Wbar/W_c; T column: tT
      const double iWc = sh.iW[base + c];
      const double v = fac * ((Jg[r * sh.ldj + c] + ak) * rho * iWc - Wbar * iWc * AC) + fw * Wbar * iWc +
                       sh.isT[base + c] * tT;
      jrow[c] = isSp ? v : 0.0;
    }
    wave_sync();   // all column and row reads done before row S is written
    // temperature row, one column per lane, through LDS row S
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
    Jg[S * sh.ldj + r] = tcol;   // lanes beyond S write 0
    wave_sync();
    if (r == S) {
#pragma unroll
      for (int c = 0; c < NP; ++c) jrow[c] = Jg[S * sh.ldj + c];
    }
    wave_sync();
  }
}

// In-place LU with partial pivoting of the group's matrix, one row per lane.
// Rows are never moved: the lane whose row wins the pivot search of column k
// (largest |a_rk| among unused rows, ties to the lowest row) records pos = k
// and publishes its row through LDS; the other unused rows store their
// multiplier in a[k] and update columns > k.  perm[k] names the pivot lane.
// Returns 1/u_kk of the lane's own pivot in rdiag.
template <int NP>
__device__ __forceinline__ void lu_factor(double (&a)[NP], int& pos, double& rdiag, const Shared& sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int base = lane - r;
  bool used = false;
  pos = -1;
  double dg = 1.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double cand = used ? -1.0 : fabs(a[k]);
    if (!(cand == cand)) cand = -1.0;
    int idx = r;
    gargmax<NP>(cand, idx);
    double* prow = sh.prow + (k & 1) * kWave + base;
    if (r == idx) {
      used = true;
      pos = k;
      dg = a[k];
      sh.perm[base + k] = r;
#pragma unroll
      for (int c = k; c < NP; ++c) prow[c] = a[c];
    }
    wave_sync();
    if (!used) {
      const double l = a[k] / prow[k];
      a[k] = l;
#pragma unroll
      for (int c = k + 1; c < NP; ++c) a[c] -= l * prow[c];
    }
  }
  rdiag = 1.0 / dg;
}

// Solve M x = b with the factors of lu_factor; lane r holds b_r on entry and
// returns x_r.
template <int NP>
__device__ __forceinline__ double lu_solve(const double (&a)[NP], const int pos, const double rdiag, double b,
                                           const Shared& sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int base = lane - r;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int pl = sh.perm[base + k];
    const double zk = __shfl(b, base + pl);
    if (pos > k) b -= a[k] * zk;
  }
  double x = 0.0;
#pragma unroll
  for (int k = NP - 1; k >= 0; --k) {
    const int pl = sh.perm[base + k];
    const double xk = __shfl(b * rdiag, base + pl);
    if (pos < k) b -= a[k] * xk;
    if (r == k) x = xk;
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

template <int NP>
__device__ __forceinline__ double wrms(const double v, const double w, const int N) {
  const double t = v * w;
  return sqrt(gsum<NP>(t * t) / N);
}

// Mixture enthalpy sum_k Y_k H_k(T)/W_k of the group's cell (J/g).
template <int NP>
__device__ __forceinline__ double mix_enthalpy(const DevMech& m, const double Yr, const double T, const int r) {
  double v = 0.0;
  if (r < m.S) {
    const double a0 = m.a0[r], a1 = m.a1[r];
    const double Hk = m.hf[r] + kRu * (a0 * (T - kTref) + a1 * (T * T - kTref * kTref) * 0.5);
    v = Yr * Hk / m.W[r];
  }
  return gsum<NP>(v);
}

// Temperature at which the mixture with composition Y has enthalpy h: the
// positive root of gamma T^2 + beta T + (alpha - h) = 0 in cancellation-free form.
template <int NP>
__device__ __forceinline__ double temperature_from_h(const DevMech& m, const double Yr, const double h, const int r) {
  double al = 0.0, be = 0.0, ga = 0.0;
  if (r < m.S) {
    const double w = Yr / m.W[r];
    const double a0 = m.a0[r], a1 = m.a1[r];
    al = w * (m.hf[r] - kRu * a0 * kTref - kRu * a1 * kTref * kTref / 2.0);
    be = w * kRu * a0;
    ga = w * kRu * a1 / 2.0;
  }
  al = gsum<NP>(al);
  be = gsum<NP>(be);
  ga = gsum<NP>(ga);
  const double c = h - al;
  return 2.0 * c / (be + sqrt(be * be + 4.0 * ga * c));
}

template <int NP>
__device__ __forceinline__ double pick(const double (&D)[kQMax + 2], const int j) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < kQMax + 2; ++i)
    if (i == j) v = D[i];
  return v;
}

// Variable-order BDF over [0, dt] for the group's cell; the same decisions as
// the oracle's per-cell integrator (predictor/corrector in backward
// differences, Newton with a fresh Jacobian and LU per attempt, WRMS error
// test, quasi-constant step size with order selection after k+2 steps, and
// enthalpy projection of T after every accepted step).
template <int NP>
__global__ __launch_bounds__(kWave) void integrate_kernel(const DevMech m, const IntParams P, double* __restrict__ Tg,
                                                          double* __restrict__ Yg, const int64_t n,
                                                          int32_t* __restrict__ rec) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, m.N, NP);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  const int S = m.S, N = m.N;
  const int64_t cell = (int64_t)blockIdx.x * (kWave / NP) + g;
  if (cell >= n) return;   // whole groups leave together
  sh.W[lane] = (r < S) ? m.W[r] : 1.0;
  sh.iW[lane] = (r < S) ? 1.0 / m.W[r] : 0.0;
  sh.isT[lane] = (r == S) ? 1.0 : 0.0;

  double y0 = 0.0;
  if (r < S) y0 = Yg[(int64_t)r * n + cell];
  else if (r == S) y0 = Tg[cell];
  int bad = 0;
  if (r < N && !isfinite(y0)) bad = 1;
  if (r == S && !(y0 > 0.0)) bad = 1;
  bad = gor<NP>(bad);

  int status = 0, steps = 0, attempts = 0, nrhs = 0, njac = 0, nnewton = 0, netf = 0, nnnf = 0;
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
    const double T0 = __shfl(y0, (lane - r) + S);
    const double h0 = mix_enthalpy<NP>(m, D[0], T0, r);
    double jrow[NP];
    double dummy[NP];
    double f, wdx;
    rhs_eval<NP, false>(m, P.p, fixedT, D[0], f, wdx, dummy, sh);
    nrhs++;
    double w = (r < N) ? 1.0 / (P.rtol * fabs(D[0]) + P.atol) : 0.0;
    double h;
    if (fixed) {
      h = P.dt / P.fixed_step_n;
    } else {
      const double nf = wrms<NP>(f, w, N);
      h = P.dt;
      if (nf * P.dt > 1.0) h = 1.0 / nf;
    }
    D[1] = h * f;
    int k = 1, etf = 0, nk = 0;
    double t = 0.0;
    while (t < P.dt) {
      if (attempts >= P.max_steps) {
        status = 1;
        break;
      }
      attempts++;
      bool last = false;
      if (fixed) {
        last = (steps + 1 == P.fixed_step_n);
      } else if (t + 1.1 * h >= P.dt) {   // end exactly at dt (stretch up to 10% or shorten)
        const double hn = P.dt - t;
        rescale(D, k + 1 <= q_max ? k + 1 : q_max, hn / h);
        h = hn;
        nk = 0;
        last = true;
      }
      if (!(h > 16.0 * DBL_EPSILON * t) || !(h >= 1e-290)) {
        status = 2;
        break;
      }
      w = (r < N) ? 1.0 / (P.rtol * fabs(D[0]) + P.atol) : 0.0;
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

      double fp;
      rhs_eval<NP, true>(m, P.p, fixedT, pred, fp, wdx, jrow, sh);
      njac++;
#pragma unroll
      for (int cc = 0; cc < NP; ++cc) jrow[cc] = ((cc == r) ? 1.0 : 0.0) - c * jrow[cc];
      int pos;
      double rdiag;
      lu_factor<NP>(jrow, pos, rdiag, sh);

      double d = 0.0;
      bool conv = false;
      double prev = 0.0;
      const int maxit = fixed ? 50 : 4;
      const double ntol = fixed ? 1e-10 : 0.03;
      for (int it = 1; it <= maxit; ++it) {
        double fi;
        if (it == 1) {
          fi = fp;   // f at pred + 0 was evaluated with the Jacobian
        } else {
          rhs_eval<NP, false>(m, P.p, fixedT, pred + d, fi, wdx, dummy, sh);
        }
        nrhs++;
        nnewton++;
        const double b = (r < N) ? -(d - c * fi + psi) : 0.0;
        const double delta = lu_solve<NP>(jrow, pos, rdiag, b, sh);
        d += delta;
        const double nrm = wrms<NP>(delta, w, N);
        if (nrm <= ntol) {
          conv = true;
          break;
        }
        if (it > 1 && nrm > 2.0 * prev) break;
        prev = nrm;
      }
      if (!conv && !fixed) {
        nnnf++;
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
        const double Dk1 = pick<NP>(D, k + 1);
        double Dn[kQMax + 2];
#pragma unroll
        for (int j = 0; j < kQMax + 2; ++j) Dn[j] = D[j];
#pragma unroll
        for (int j = 0; j < kQMax + 2; ++j) {
          if (j == k + 2 && k < q_max) Dn[j] = d - Dk1;
          if (j == k + 1) Dn[j] = d;
        }
#pragma unroll
        for (int j = kQMax; j >= 0; --j)
          if (j <= k) Dn[j] = Dn[j] + Dn[j + 1];
#pragma unroll
        for (int j = 0; j < kQMax + 2; ++j) D[j] = Dn[j];
      }
      if (!fixedT) {
        const double Tn = temperature_from_h<NP>(m, D[0], h0, r);
        if (r == S) D[0] = Tn;
      }
      t = last ? P.dt : t + h;
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
          const double ekm1 = wrms<NP>(pick<NP>(D, k), w, N) / k;
          const double tm = 1.3 * pow(ekm1, 1.0 / k);
          const double rm = tm > 0.1 ? 1.0 / tm : 10.0;
          if (rm > rr) {
            rr = rm;
            kn = k - 1;
          }
        }
        if (k < q_max) {
          const double ekp1 = wrms<NP>(pick<NP>(D, k + 2), w, N) / (k + 2);
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
    rec[0 * n + cell] = status;
    rec[1 * n + cell] = steps;
    rec[2 * n + cell] = attempts;
    rec[3 * n + cell] = nrhs;
    rec[4 * n + cell] = njac;
    rec[5 * n + cell] = nnewton;
    rec[6 * n + cell] = netf;
    rec[7 * n + cell] = nnnf;
  }
}

template <int NP>
__global__ __launch_bounds__(kWave) void rates_kernel(const DevMech m, const double p, const int fixedT,
                                                      const double* __restrict__ Tg, const double* __restrict__ Yg,
                                                      const int64_t n, double* __restrict__ wdot,
                                                      double* __restrict__ fout, double* __restrict__ jac) {
  extern __shared__ double smem[];
  const Shared sh = carve(smem, m.N, NP);
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane % NP;
  const int g = lane / NP;
  const int S = m.S, N = m.N;
  const int64_t cell = (int64_t)blockIdx.x * (kWave / NP) + g;
  if (cell >= n) return;
  sh.W[lane] = (r < S) ? m.W[r] : 1.0;
  sh.iW[lane] = (r < S) ? 1.0 / m.W[r] : 0.0;
  sh.isT[lane] = (r == S) ? 1.0 : 0.0;
  double y = 0.0;
  if (r < S) y = Yg[(int64_t)r * n + cell];
  else if (r == S) y = Tg[cell];
  double f, wd;
  double jrow[NP];
  if (jac != nullptr) rhs_eval<NP, true>(m, p, fixedT, y, f, wd, jrow, sh);
  else rhs_eval<NP, false>(m, p, fixedT, y, f, wd, jrow, sh);
  if (r < S) wdot[(int64_t)r * n + cell] = wd * 1.0e6;   // mol/(cm^3 s) -> mol/(m^3 s)
  if (fout != nullptr && r < N) fout[(int64_t)r * n + cell] = f;
  if (jac != nullptr && r < N) {
#pragma unroll
    for (int c = 0; c < NP; ++c)
      if (c < N) jac[((int64_t)r * N + c) * n + cell] = jrow[c];
  }
}

__global__ void reduce_records_kernel(const int32_t* __restrict__ rec, const int64_t n,
                                      unsigned long long* __restrict__ out) {
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

template <int NP>
hipError_t launch_integrate_np(const DevMech& m, const IntParams& prm, double* T, double* Y, int64_t n,
                               int32_t* rec, hipStream_t stream) {
  const int cpw = kWave / NP;
  const int64_t blocks = (n + cpw - 1) / cpw;
  const size_t lds = integrate_lds_bytes(NP, m.N);
  hipLaunchKernelGGL(integrate_kernel<NP>, dim3((unsigned)blocks), dim3(kWave), lds, stream, m, prm, T, Y, n, rec);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_rates_np(const DevMech& m, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                           double* wdot, double* f, double* jac, hipStream_t stream) {
  const int cpw = kWave / NP;
  const int64_t blocks = (n + cpw - 1) / cpw;
  const size_t lds = integrate_lds_bytes(NP, m.N);
  hipLaunchKernelGGL(rates_kernel<NP>, dim3((unsigned)blocks), dim3(kWave), lds, stream, m, p, fixed_T, T, Y, n,
                     wdot, f, jac);
  return hipGetLastError();
}

}  // namespace

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
    hipLaunchKernelGGL(reduce_records_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, rec, n, out);
  }
  return hipGetLastError();
}

}  // namespace chemgpu
