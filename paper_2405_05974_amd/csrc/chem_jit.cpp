// chem_jit.cpp -- mechanism-specific lane-per-cell kernels.
//
// The paper generates source code for each mechanism's production rates and
// analytic Jacobian (Sec. 3.2) so that every species index and coefficient is
// a constant the compiler can fold.  This file does the same at load time:
// it writes HIP source for ch_eval<JAC> (rates of Eq. 2, production rates of
// Eq. 3, the reactor right-hand side and its Jacobian, Eq. 7) with literal
// indices and parameters, appends the lane-per-cell BDF integrator
// (chem_lpc_body.inc), and compiles the result with hipRTC for the device's
// architecture.  With all indices static the Newton matrix and its LU stay in
// registers, one cell per lane, which suits mechanisms up to kLpcMaxN state
// components.  Modules are cached per (device, source).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cinttypes>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "chem_handle.h"
#include "chem_internal.h"

namespace chemgpu {

namespace {

const char* kLpcBody =
#include "chem_lpc_body.inc"
    ;

const char* kChExp =
#include "chem_exp.inc"
    ;

// exact double literal (hexadecimal floating point)
std::string lit(double v) {
  if (v == 0.0) return std::signbit(v) ? "(-0.0)" : "0.0";
  char buf[64];
  std::snprintf(buf, sizeof buf, "%a", v);
  return std::string("(") + buf + ")";
}

std::string C(int k) { return "C[" + std::to_string(k) + "]"; }

// product of the concentrations of `sp` except slot `skip` (-1: none)
std::string product(const std::vector<int>& sp, int skip) {
  std::string s;
  for (size_t i = 0; i < sp.size(); ++i) {
    if ((int)i == skip) continue;
    s += s.empty() ? C(sp[i]) : " * " + C(sp[i]);
  }
  return s.empty() ? "1.0" : s;
}

// Strongly connected components of the QSS dependency graph (App. B), in
// the order they can be solved.  QSS species q depends on n when the closure
// entry A_qn is structurally nonzero: n is the one QSS reactant of a kept
// direction that changes q.  Tarjan's algorithm (one depth-first search with
// discovery indices and low links) completes a component only after every
// component it depends on, so its output order is the solve order.  Species
// indices are the generator's internal ones (QSS species from ST on); nz
// receives the structure [nq][nq].
std::vector<std::vector<int>> qss_groups(const HostMech& m, int ST, std::vector<std::vector<char>>& nz) {
  const int S = (int)m.W.size(), nq = S - ST;
  nz.assign(nq, std::vector<char>(nq, 0));
  for (const HostReaction& x : m.rx) {
    std::vector<int> nu(S, 0);
    for (int k : x.reac) nu[k] -= 1;
    for (int k : x.prod) nu[k] += 1;
    for (int dir = 0; dir < 2; ++dir) {
      if (dir == 0 && x.drop_f) continue;
      if (dir == 1 && (!x.rev || x.drop_r)) continue;
      int n = -1;
      for (int k : dir == 0 ? x.reac : x.prod)
        if (k >= ST) n = k - ST;
      if (n < 0) continue;
      for (int q = 0; q < nq; ++q)
        if (nu[ST + q]) nz[q][n] = 1;
    }
  }
  std::vector<std::vector<int>> out;
  std::vector<int> index(nq, -1), low(nq, 0), stack;
  std::vector<char> on(nq, 0);
  int counter = 0;
  std::function<void(int)> visit = [&](int v) {
    index[v] = low[v] = counter++;
    stack.push_back(v);
    on[v] = 1;
    for (int w = 0; w < nq; ++w) {
      if (w == v || !nz[v][w]) continue;
      if (index[w] < 0) {
        visit(w);
        low[v] = std::min(low[v], low[w]);
      } else if (on[w]) {
        low[v] = std::min(low[v], index[w]);
      }
    }
    if (low[v] == index[v]) {
      std::vector<int> comp;
      int w;
      do {
        w = stack.back();
        stack.pop_back();
        on[w] = 0;
        comp.push_back(w);
      } while (w != v);
      std::sort(comp.begin(), comp.end());
      out.push_back(comp);
    }
  };
  for (int v = 0; v < nq; ++v)
    if (index[v] < 0) visit(v);
  return out;
}

void emit_nu_update(std::ostringstream& o, const char* arr, int k, int nu, const std::string& v) {
  if (nu == 1) o << "    " << arr << "[" << k << "] += " << v << ";\n";
  else if (nu == -1) o << "    " << arr << "[" << k << "] -= " << v << ";\n";
  else o << "    " << arr << "[" << k << "] += " << lit((double)nu) << " * " << v << ";\n";
}

}  // namespace

std::string lpc_source(const HostMech& m_in, bool reuse) {
  // With QSS species the generated code numbers the species internally with
  // the transported ones first (in their order, so that internal index =
  // state index) and the QSS ones after them; without, the numbering is the
  // mechanism's own.
  const int S = (int)m_in.W.size(), R = (int)m_in.rx.size();
  const int nq = (int)m_in.qss.size(), ST = S - nq, N = ST + 1;
  std::vector<int> order, inv(S, -1);
  {
    std::vector<char> isq(S, 0);
    for (int k : m_in.qss) isq[k] = 1;
    for (int k = 0; k < S; ++k)
      if (!isq[k]) order.push_back(k);
    for (int k : m_in.qss) order.push_back(k);
    for (int i = 0; i < S; ++i) inv[order[i]] = i;
  }
  HostMech m = m_in;
  for (int i = 0; i < S; ++i) {
    const int k = order[i];
    m.W[i] = m_in.W[k];
    m.a0[i] = m_in.a0[k];
    m.a1[i] = m_in.a1[k];
    m.hf[i] = m_in.hf[k];
    m.s0[i] = m_in.s0[k];
    m.nasa[i] = m_in.nasa[k];
  }
  for (HostReaction& x : m.rx) {
    for (int& k : x.reac) k = inv[k];
    for (int& k : x.prod) k = inv[k];
    for (int& k : x.eff_k) k = inv[k];
  }
  // Mechanism parameters are read from a __constant__ table (scalar loads,
  // several constants per instruction) rather than written as literals, each
  // of which costs two scalar moves wherever it is used.
  std::vector<double> pool;
  std::map<unsigned long long, int> pool_idx;
  auto kc = [&](double v) {
    unsigned long long bits;
    std::memcpy(&bits, &v, sizeof bits);
    auto it = pool_idx.find(bits);
    int idx;
    if (it != pool_idx.end()) {
      idx = it->second;
    } else {
      idx = (int)pool.size();
      pool.push_back(v);
      pool_idx[bits] = idx;
    }
    return "K[" + std::to_string(idx) + "]";
  };
  std::ostringstream o;
  // which species need a Gibbs energy
  std::vector<char> needG(S, 0);
  for (const HostReaction& x : m.rx)
    if (x.rev) {
      for (int k : x.reac) needG[k] = 1;
      for (int k : x.prod) needG[k] = 1;
    }
  const double kcal_to_K = 4184.0 / kRu;
  // WD: also hand back the net production rates (mol cm^-3 s^-1) for chem_rates
  o << "template <bool JAC, bool WD = false>\n__device__ __forceinline__ void ch_eval(const double (&y)[CH_N], "
       "const double p, const int fixedT, double (&f)[CH_N], double (&J)[CH_N][CH_N], double* wdo = nullptr) {\n";
  // K reads the table through the constant address space, so loads stay scalar.  At the top
  // and before every fourth reaction the pointer passes through an empty asm statement: the
  // compiler can no longer hoist every table load out of the step loop (about 130 doubles kept
  // live in scalar registers and spilled), and loads each group's constants from the scalar
  // cache where they are used.
  o << "  typedef const __attribute__((address_space(4))) double* ch_kptr;\n";
  o << "  ch_kptr __restrict__ K = (ch_kptr)ch_K;\n  asm volatile(\"\" : \"+s\"(K));\n";
  o << "  const double T = y[CH_S];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
  // Divisions by constants are multiplications by their exact reciprocals;
  // enthalpy and heat capacity are re-evaluated where they are used so that
  // only the Jacobian keeps them across the reactions.  For a species with
  // NASA 7-coefficient thermo each coefficient is selected by the range flag
  // lo<k> (T <= T_mid), and the divisions of the H and S polynomials are
  // folded into the constants.
  auto isN = [&](int k) { return !m.nasa[k].empty(); };
  auto nc = [&](int k, int i, double scale) {   // coefficient c_(i+1) of species k times scale
    return "(lo" + std::to_string(k) + " ? " + kc(m.nasa[k][1 + i] * scale) + " : " +
           kc(m.nasa[k][8 + i] * scale) + ")";
  };
  auto Hk = [&](int k) {
    if (isN(k))
      return "(CH_RU * (T * (" + nc(k, 0, 1.0) + " + T * (" + nc(k, 1, 0.5) + " + T * (" + nc(k, 2, 1.0 / 3.0) +
             " + T * (" + nc(k, 3, 0.25) + " + T * " + nc(k, 4, 0.2) + ")))) + " + nc(k, 5, 1.0) + "))";
    return "(" + kc(m.hf[k]) + " + CH_RU * (" + kc(m.a0[k]) + " * (T - CH_TREF) + " + kc(m.a1[k]) +
           " * (T * T - CH_TREF * CH_TREF) * 0.5))";
  };
  auto Cpk = [&](int k) {
    if (isN(k))
      return "(CH_RU * (" + nc(k, 0, 1.0) + " + T * (" + nc(k, 1, 1.0) + " + T * (" + nc(k, 2, 1.0) + " + T * (" +
             nc(k, 3, 1.0) + " + T * " + nc(k, 4, 1.0) + ")))))";
    return "(CH_RU * (" + kc(m.a0[k]) + " + " + kc(m.a1[k]) + " * T))";
  };
  auto dCpk = [&](int k) {
    if (isN(k))
      return "(CH_RU * (" + nc(k, 1, 1.0) + " + T * (" + nc(k, 2, 2.0) + " + T * (" + nc(k, 3, 3.0) + " + T * " +
             nc(k, 4, 4.0) + "))))";
    return "CH_RU * " + kc(m.a1[k]);
  };
  for (int k = 0; k < S; ++k)
    if (isN(k)) o << "  const bool lo" << k << " = T <= " << kc(m.nasa[k][0]) << ";\n";
  o << "  double sumYW = 0.0;\n";
  for (int k = 0; k < ST; ++k) o << "  sumYW += y[" << k << "] * " << kc(1.0 / m.W[k]) << ";\n";
  o << "  const double Wbar = 1.0 / sumYW;\n";
  o << "  const double rho = (p * 10.0) * Wbar / (CH_RU_CGS * T);\n";
  o << "  const double irho = 1.0 / rho;\n";
  o << "  double C[CH_SA];\n  double Mc = 0.0;\n";
  for (int k = 0; k < ST; ++k) o << "  C[" << k << "] = rho * y[" << k << "] * " << kc(1.0 / m.W[k]) << ";\n";
  for (int k = 0; k < ST; ++k) o << "  Mc += C[" << k << "];\n";
  o << "  const double lnTr = log(T * " << kc(1.0 / kTref) << ");\n";
  o << "  const double invRT = 1.0 / (CH_RU * T);\n";
  o << "  const double lnc0 = log(CH_PATM * invRT * 1.0e-6);\n";
  o << "  double H[CH_SA], G[CH_SA];\n";
  o << "  if (JAC) {\n";
  for (int k = 0; k < S; ++k) o << "    H[" << k << "] = " << Hk(k) << ";\n";
  o << "  }\n";
  for (int k = 0; k < S; ++k) {
    if (needG[k] && isN(k))
      o << "  G[" << k << "] = (" << Hk(k) << " - T * (CH_RU * (" << nc(k, 0, 1.0) << " * lnT + T * ("
        << nc(k, 1, 1.0) << " + T * (" << nc(k, 2, 0.5) << " + T * (" << nc(k, 3, 1.0 / 3.0) << " + T * "
        << nc(k, 4, 0.25) << "))) + " << nc(k, 6, 1.0) << "))) * invRT;\n";
    else if (needG[k])
      o << "  G[" << k << "] = (" << Hk(k) << " - T * (" << kc(m.s0[k]) << " + CH_RU * (" << kc(m.a0[k])
        << " * lnTr + " << kc(m.a1[k]) << " * (T - CH_TREF)))) * invRT;\n";
    else
      o << "  G[" << k << "] = 0.0;\n";
  }
  o << "  (void)lnc0; (void)invRT; (void)lnT; (void)Mc;\n";
  // Rate constants of reaction x (Eq. 2's k vector): k_f (with falloff and
  // Troe's factor) and, for reversible reactions, k_r from K_c; with JAC their
  // T and [M] derivatives.  Emitted in two parts around the reactant and
  // product concentration products.
  auto emit_kf = [&](const HostReaction& x) {
    o << "    const double kinf = ch_exp(" << kc(std::log(x.A)) << " + " << kc(x.b) << " * lnT - "
      << kc(x.Ea * kcal_to_K) << " * invT);\n";
    o << "    double kf = kinf;\n";
    o << "    double dlnkf = (" << kc(x.b) << " + " << kc(x.Ea * kcal_to_K) << " * invT) * invT;\n";
    o << "    double dkfdM = 0.0;\n    (void)dlnkf; (void)dkfdM;\n";
    // third-body concentration with this reaction's collision efficiencies
    if (x.type != 0) {
      o << "    const double Mj = Mc";
      for (size_t i = 0; i < x.eff_k.size(); ++i)
        if (x.eff_k[i] < ST) o << " + " << kc(x.eff_v[i] - 1.0) << " * " << C(x.eff_k[i]);
      o << ";\n";
    }
    if (x.type == 2) {
      o << "    const double k0 = ch_exp(" << kc(std::log(x.A0)) << " + " << kc(x.b0) << " * lnT - "
        << kc(x.Ea0 * kcal_to_K) << " * invT);\n";
      o << "    const double dlnk0 = (" << kc(x.b0) << " + " << kc(x.Ea0 * kcal_to_K) << " * invT) * invT;\n";
      o << "    const double Pr = k0 * Mj / kinf;\n";
      o << "    const double dlnPr = dlnk0 - dlnkf;\n";
      o << "    kf = kinf * Pr / (1.0 + Pr);\n";
      o << "    dlnkf = dlnkf + dlnPr / (1.0 + Pr);\n";
      o << "    dkfdM = k0 / ((1.0 + Pr) * (1.0 + Pr));\n";
      o << "    (void)dlnPr;\n";
      if (x.ntroe) {
        // Troe's broadening factor (CHEMKIN form, logarithms base 10; log Pr at max(Pr, 1e-300))
        const double a = x.troe[0];
        o << "    {\n      const double e3 = ch_exp(-T * " << kc(1.0 / x.troe[1]) << "), e1 = ch_exp(-T * "
          << kc(1.0 / x.troe[2]) << ");\n";
        o << "      double Fc = " << kc(1.0 - a) << " * e3 + " << kc(a) << " * e1;\n";
        o << "      double dFc = -" << kc((1.0 - a) / x.troe[1]) << " * e3 - " << kc(a / x.troe[2]) << " * e1;\n";
        if (x.ntroe == 4) {
          o << "      const double e2 = ch_exp(-" << kc(x.troe[3]) << " * invT);\n";
          o << "      Fc += e2;\n      dFc += " << kc(x.troe[3]) << " * invT * invT * e2;\n";
        }
        o << "      const double Lc = log(Fc) * CH_INV_LN10;\n";
        o << "      const bool live = Pr > 1e-300;\n";
        o << "      const double lp = log(live ? Pr : 1e-300) * CH_INV_LN10;\n";
        o << "      const double cc = -0.4 - 0.67 * Lc, nn = 0.75 - 1.27 * Lc;\n";
        o << "      const double u = lp + cc, v = nn - 0.14 * u;\n";
        o << "      const double f1 = u / v;\n      const double dn = 1.0 + f1 * f1;\n";
        o << "      const double F = ch_exp(CH_LN10 * (Lc / dn));\n";
        o << "      if (JAC) {\n";
        o << "        const double iv2 = 1.0 / (v * v);\n";
        o << "        const double dlogF_dlp = live ? -Lc * 2.0 * f1 * (nn * iv2) / (dn * dn) : 0.0;\n";
        o << "        const double df1_dLc = (-0.67 * v - u * (-1.27 + 0.67 * 0.14)) * iv2;\n";
        o << "        const double dlogF_dLc = 1.0 / dn - Lc * 2.0 * f1 * df1_dLc / (dn * dn);\n";
        o << "        const double dLc_dT = dFc / Fc * CH_INV_LN10;\n";
        o << "        const double dlp_dT = live ? dlnPr * CH_INV_LN10 : 0.0;\n";
        o << "        dkfdM = F * dkfdM + F * k0 / (1.0 + Pr) * dlogF_dlp;\n";
        o << "        dlnkf += CH_LN10 * (dlogF_dlp * dlp_dT + dlogF_dLc * dLc_dT);\n      }\n";
        o << "      kf *= F;\n    }\n";
      }
    }
  };
  auto emit_kr = [&](const HostReaction& x, const std::vector<int>& nu, int dnu) {
    o << "    double kr = 0.0, dkr = 0.0, dkrdM = 0.0;\n    (void)dkr; (void)dkrdM;\n";
    if (x.rev) {
      // sum_k nu_k G_k / RT and sum_k nu_k H_k over the net stoichiometry
      std::string sg, shh;
      for (int k = 0; k < S; ++k) {
        if (!nu[k]) continue;
        const std::string term = (nu[k] == 1 || nu[k] == -1) ? "" : lit((double)std::abs(nu[k])) + " * ";
        const char* sign = nu[k] > 0 ? (sg.empty() ? "" : " + ") : (sg.empty() ? "-" : " - ");
        sg += sign + term + "G[" + std::to_string(k) + "]";
        shh += sign + term + "H[" + std::to_string(k) + "]";
      }
      if (sg.empty()) {
        sg = "0.0";
        shh = "0.0";
      }
      o << "    const double ratio = ch_exp((" << sg << ") - " << lit((double)dnu) << " * lnc0);\n";
      o << "    kr = kf * ratio;\n";
      o << "    if (JAC) {\n";
      o << "      const double dlnKc = (" << shh << ") * invRT * invT - " << lit((double)dnu) << " * invT;\n";
      o << "      dkr = kr * (dlnkf - dlnKc);\n";
      o << "      dkrdM = dkfdM * ratio;\n    }\n";
    }
  };
  auto nu_of = [&](const HostReaction& x) {
    std::vector<int> nu(S, 0);
    for (int k : x.reac) nu[k] -= 1;
    for (int k : x.prod) nu[k] += 1;
    return nu;
  };
  // row k of the concentration-space Jacobian: transported rows accumulate in
  // J (state block) or, for a QSS column, in ATQ; QSS rows in AQT
  auto jac_row = [&](int k, int c) -> std::string {
    if (k < ST) return c < ST ? "    J[" + std::to_string(k) + "]" : "    ATQ[" + std::to_string(k) + "]";
    return "    AQT[" + std::to_string(k - ST) + "]";
  };
  auto jac_col = [&](int c) { return c < ST ? c : c - ST; };
  // QSS groups in solve order, and which closure entries are structurally nonzero
  std::vector<std::vector<char>> nzA;
  const std::vector<std::vector<int>> groups = qss_groups(m, ST, nzA);
  std::vector<int> group_of(nq, -1);
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int q : groups[gi]) group_of[q] = (int)gi;
  if (nq > 0) {
    // QSS closure (Eq. 4-6): with the quadratic couplings removed each kept
    // direction carries at most one QSS concentration as a factor, so the QSS
    // production rates are affine, qA C_Q - qb; the system is solved group by
    // group in the dependency order of its strongly connected components
    // (App. B), found with Tarjan's algorithm when the source is generated.
    o << "  double qA[CH_NQ][CH_NQ], qb[CH_NQ];\n";
    o << "#pragma unroll\n  for (int a = 0; a < CH_NQ; ++a) {\n    qb[a] = 0.0;\n"
         "#pragma unroll\n    for (int b = 0; b < CH_NQ; ++b) qA[a][b] = 0.0;\n  }\n";
    for (int j = 0; j < R; ++j) {
      const HostReaction& x = m.rx[j];
      const std::vector<int> nu = nu_of(x);
      bool touches = false;
      for (int k = ST; k < S; ++k) touches |= nu[k] != 0;
      if (!touches) continue;
      const int dnu = (int)x.prod.size() - (int)x.reac.size();
      o << "  asm volatile(\"\" : \"+s\"(K));\n  {  // closure terms of reaction " << j << "\n";
      emit_kf(x);
      emit_kr(x, nu, dnu);
      o << "    const double mf = " << (x.type == 1 ? "Mj" : "1.0") << ";\n";
      for (int dir = 0; dir < 2; ++dir) {
        if (dir == 0 && x.drop_f) continue;
        if (dir == 1 && (!x.rev || x.drop_r)) continue;
        const std::vector<int>& side = dir == 0 ? x.reac : x.prod;
        int n = -1;
        std::string c = dir == 0 ? "mf * kf" : "mf * kr";
        for (int k : side) {
          if (k >= ST) n = k - ST;
          else c += " * " + C(k);
        }
        o << "    {\n      const double cq = " << c << ";\n";
        for (int k = ST; k < S; ++k) {
          if (!nu[k]) continue;
          const int sgn = dir == 0 ? nu[k] : -nu[k];
          const std::string v = (sgn == 1 ? "" : (sgn == -1 ? "-" : lit((double)sgn) + " * ")) + std::string("cq");
          if (n >= 0) o << "      qA[" << k - ST << "][" << n << "] += " << v << ";\n";
          else o << "      qb[" << k - ST << "] -= " << v << ";\n";
        }
        o << "    }\n";
      }
      o << "  }\n";
    }
    o << "  asm volatile(\"\" : \"+s\"(K));\n";
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const std::vector<int>& g = groups[gi];
      const int n = (int)g.size();
      o << "  {  // QSS group";
      for (int q : g) o << " " << q;
      o << "\n    double a[" << n << "][" << n << "], r[" << n << "][1];\n";
      for (int i = 0; i < n; ++i) {
        for (int jj = 0; jj < n; ++jj) o << "    a[" << i << "][" << jj << "] = qA[" << g[i] << "][" << g[jj] << "];\n";
        o << "    r[" << i << "][0] = qb[" << g[i] << "]";
        for (int q = 0; q < nq; ++q)
          if (group_of[q] < (int)gi && nzA[g[i]][q]) o << " - qA[" << g[i] << "][" << q << "] * C[" << ST + q << "]";
        o << ";\n";
      }
      o << "    ch_gauss<" << n << ", 1>(a, r);\n";
      for (int i = 0; i < n; ++i) o << "    C[" << ST + g[i] << "] = r[" << i << "][0];\n";
      o << "  }\n";
    }
  }
  o << "  double wd[CH_S];\n";
  // For JAC the species block of J first accumulates A = d wdot / dC at fixed
  // T (without the [M] rank-one part, kept in ak) and is turned into the
  // (Y, T) Jacobian in place at the end.
  o << "  double bT[CH_S], ak[CH_S];\n";
  o << "#pragma unroll\n  for (int k = 0; k < CH_S; ++k) {\n    wd[k] = 0.0;\n    bT[k] = 0.0;\n    ak[k] = 0.0;\n"
       "    if (JAC) {\n#pragma unroll\n      for (int c = 0; c < CH_S; ++c) J[k][c] = 0.0;\n    }\n  }\n";
  if (nq > 0) {
    // blocks of the concentration-space Jacobian that involve QSS species
    o << "  double ATQ[CH_S][CH_NQ], AQT[CH_NQ][CH_S], bTQ[CH_NQ], akQ[CH_NQ];\n";
    o << "  if (JAC) {\n#pragma unroll\n    for (int a = 0; a < CH_NQ; ++a) {\n      bTQ[a] = 0.0;\n      akQ[a] = 0.0;\n"
         "#pragma unroll\n      for (int k = 0; k < CH_S; ++k) {\n        ATQ[k][a] = 0.0;\n        AQT[a][k] = 0.0;\n"
         "      }\n    }\n  }\n";
  }
  for (int j = 0; j < R; ++j) {
    const HostReaction& x = m.rx[j];
    const std::vector<int> nu = nu_of(x);
    const int dnu = (int)x.prod.size() - (int)x.reac.size();
    // the table pointer is made opaque every 4 reactions: their constants are
    // loaded together, and not all at the top of the function (which would
    // exhaust the scalar registers)
    if (j % 4 == 0) o << "  asm volatile(\"\" : \"+s\"(K));\n";
    o << "  {  // reaction " << j << "\n";
    emit_kf(x);
    // a direction removed by the linearisation has a zero concentration product
    o << "    const double pf = " << (x.drop_f ? std::string("0.0") : product(x.reac, -1)) << ";\n";
    o << "    const double pr = " << (x.drop_r ? std::string("0.0") : product(x.prod, -1)) << ";\n";
    emit_kr(x, nu, dnu);
    o << "    const double mf = " << (x.type == 1 ? "Mj" : "1.0") << ";\n";
    o << "    const double net = kf * pf - kr * pr;\n";
    o << "    const double Q = mf * net;\n";
    for (int k = 0; k < ST; ++k)
      if (nu[k]) emit_nu_update(o, "wd", k, nu[k], "Q");
    o << "    if (JAC) {\n";
    o << "      const double dQdT = mf * (kf * dlnkf * pf - dkr * pr);\n";
    for (int k = 0; k < S; ++k)
      if (nu[k]) emit_nu_update(o, k < ST ? "  bT" : "  bTQ", jac_col(k), nu[k], "dQdT");
    if (x.type == 1 || x.type == 2) {
      o << "      const double q0 = " << (x.type == 1 ? "net" : "dkfdM * pf - dkrdM * pr") << ";\n";
      for (int k = 0; k < S; ++k)
        if (nu[k]) emit_nu_update(o, k < ST ? "  ak" : "  akQ", jac_col(k), nu[k], "q0");
      // efficiencies other than 1: d[M]_j/dC_c = 1 + (eps_c - 1), the 1 being the rank-one part in ak
      for (size_t i = 0; i < x.eff_k.size(); ++i) {
        if (x.eff_k[i] >= ST) continue;     // QSS species do not collide
        o << "      {\n        const double dq = q0 * " << kc(x.eff_v[i] - 1.0) << ";\n";
        for (int k = 0; k < S; ++k)
          if (nu[k]) emit_nu_update(o, jac_row(k, x.eff_k[i]).c_str(), x.eff_k[i], nu[k], "dq");
        o << "      }\n";
      }
    }
    for (size_t sl = 0; sl < x.reac.size() && !x.drop_f; ++sl) {
      const int c = x.reac[sl];
      o << "      {\n        const double dq = mf * kf * " << product(x.reac, (int)sl) << ";\n";
      for (int k = 0; k < S; ++k)
        if (nu[k] && !(k >= ST && c >= ST)) emit_nu_update(o, jac_row(k, c).c_str(), jac_col(c), nu[k], "dq");
      o << "      }\n";
    }
    for (size_t sl = 0; sl < x.prod.size() && !x.drop_r; ++sl) {
      const int c = x.prod[sl];
      o << "      {\n        const double dq = -mf * kr * " << product(x.prod, (int)sl) << ";\n";
      for (int k = 0; k < S; ++k)
        if (nu[k] && !(k >= ST && c >= ST)) emit_nu_update(o, jac_row(k, c).c_str(), jac_col(c), nu[k], "dq");
      o << "      }\n";
    }
    o << "    }\n  }\n";
  }
  if (nq > 0) {
    // Jacobian through the closure (Sec. 3.2): the QSS concentrations follow
    // the transported ones and T, so with X = qA^-1 [A_QT | b_Q] the state
    // block becomes A_TT - A_TQ X and the T column b_T - A_TQ X_T
    o << "  if (JAC) {\n    double X[CH_NQ][CH_N];\n";
    o << "#pragma unroll\n    for (int a = 0; a < CH_NQ; ++a) {\n"
         "#pragma unroll\n      for (int c = 0; c < CH_S; ++c) X[a][c] = AQT[a][c] + akQ[a];\n"
         "      X[a][CH_S] = bTQ[a];\n    }\n";
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const std::vector<int>& g = groups[gi];
      const int n = (int)g.size();
      o << "    {  // QSS group";
      for (int q : g) o << " " << q;
      o << "\n      double a[" << n << "][" << n << "], r[" << n << "][CH_N];\n";
      for (int i = 0; i < n; ++i) {
        for (int jj = 0; jj < n; ++jj) o << "      a[" << i << "][" << jj << "] = qA[" << g[i] << "][" << g[jj] << "];\n";
        o << "#pragma unroll\n      for (int c = 0; c < CH_N; ++c) r[" << i << "][c] = X[" << g[i] << "][c]";
        for (int q = 0; q < nq; ++q)
          if (group_of[q] < (int)gi && nzA[g[i]][q]) o << " - qA[" << g[i] << "][" << q << "] * X[" << q << "][c]";
        o << ";\n";
      }
      o << "      ch_gauss<" << n << ", CH_N>(a, r);\n";
      for (int i = 0; i < n; ++i)
        o << "#pragma unroll\n      for (int c = 0; c < CH_N; ++c) X[" << g[i] << "][c] = r[" << i << "][c];\n";
      o << "    }\n";
    }
    o << "#pragma unroll\n    for (int k = 0; k < CH_S; ++k) {\n"
         "#pragma unroll\n      for (int a = 0; a < CH_NQ; ++a) {\n"
         "#pragma unroll\n        for (int c = 0; c < CH_S; ++c) J[k][c] -= ATQ[k][a] * X[a][c];\n"
         "        bT[k] -= ATQ[k][a] * X[a][CH_S];\n      }\n    }\n  }\n";
  }
  // right-hand side
  o << "  double num = 0.0, den = 0.0;\n";
  for (int k = 0; k < ST; ++k) {
    o << "  num += (JAC ? H[" << k << "] : " << Hk(k) << ") * wd[" << k << "];\n";
    o << "  den += C[" << k << "] * " << Cpk(k) << ";\n";
  }
  o << "  const double iden = 1.0 / den;\n";
  for (int k = 0; k < ST; ++k) o << "  f[" << k << "] = " << kc(m.W[k]) << " * wd[" << k << "] * irho;\n";
  o << "  f[CH_S] = fixedT ? 0.0 : -num * iden;\n";
  o << "  if (WD) {\n#pragma unroll\n    for (int k = 0; k < CH_S; ++k) wdo[k] = wd[k];\n  }\n";
  // Jacobian: row sums AC_k = sum_c A_kc C_c and the temperature row (which
  // needs the column sums sum_k H_k A_kc) from A, then the species rows in place
  o << "  if (JAC) {\n";
  o << "    double AC[CH_S], dwdT[CH_S];\n";
  o << "#pragma unroll\n    for (int k = 0; k < CH_S; ++k) {\n      double s = 0.0;\n"
       "#pragma unroll\n      for (int c = 0; c < CH_S; ++c) s += (J[k][c] + ak[k]) * C[c];\n"
       "      AC[k] = s;\n      dwdT[k] = bT[k] - s * invT;\n    }\n";
  o << "    double iW[CH_S], Wk[CH_S], Cp[CH_S];\n";
  for (int k = 0; k < ST; ++k) o << "    Cp[" << k << "] = " << Cpk(k) << ";\n";
  for (int k = 0; k < ST; ++k) o << "    iW[" << k << "] = " << kc(1.0 / m.W[k]) << ";\n";
  for (int k = 0; k < ST; ++k) o << "    Wk[" << k << "] = " << kc(m.W[k]) << ";\n";
  o << "    if (fixedT) {\n#pragma unroll\n      for (int c = 0; c < CH_N; ++c) J[CH_S][c] = 0.0;\n    } else {\n";
  o << "      double HAC = 0.0, HdwdT = 0.0, Cpw = 0.0, Ca1 = 0.0;\n";
  o << "#pragma unroll\n      for (int k = 0; k < CH_S; ++k) {\n        HAC += H[k] * AC[k];\n"
       "        HdwdT += H[k] * dwdT[k];\n        Cpw += Cp[k] * wd[k];\n      }\n";
  for (int k = 0; k < ST; ++k) o << "      Ca1 += C[" << k << "] * " << dCpk(k) << ";\n";
  o << "#pragma unroll\n      for (int c = 0; c < CH_S; ++c) {\n        double colsum = 0.0;\n"
       "#pragma unroll\n        for (int k = 0; k < CH_S; ++k) colsum += H[k] * (J[k][c] + ak[k]);\n"
       "        const double dN = (rho * iW[c]) * colsum - (Wbar * iW[c]) * HAC;\n"
       "        const double dD = (rho * Cp[c] - Wbar * den) * iW[c];\n"
       "        J[CH_S][c] = -dN * iden + num * dD * (iden * iden);\n      }\n";
  o << "      const double dN = Cpw + HdwdT;\n      const double dD = -den * invT + Ca1;\n"
       "      J[CH_S][CH_S] = -dN * iden + num * dD * (iden * iden);\n    }\n";
  o << "#pragma unroll\n    for (int k = 0; k < CH_S; ++k) {\n"
       "      const double fac = Wk[k] * irho;\n      const double fw = Wk[k] * wd[k] * irho;\n"
       "#pragma unroll\n      for (int c = 0; c < CH_S; ++c)\n"
       "        J[k][c] = fac * ((J[k][c] + ak[k]) * rho * iW[c] - Wbar * iW[c] * AC[k]) + fw * Wbar * iW[c];\n"
       "      J[k][CH_S] = fac * dwdT[k] + fw * invT;\n    }\n";
  o << "  }\n}\n";
  std::ostringstream head;
  head << "// generated: lane-per-cell kernels for a mechanism with " << S << " species and " << R
       << " reactions\n";
  head << "#define CH_S " << ST << "\n#define CH_N " << N << "\n#define CH_SA " << S << "\n";
  if (nq > 0) {
    head << "#define CH_NQ " << nq << "\n";
    // dense solve of one QSS group: Gaussian elimination with partial
    // pivoting (a row moves up only when strictly larger in magnitude), NR
    // right-hand sides, solution left in r
    head << "template <int K, int NR>\n__device__ __forceinline__ void ch_gauss(double (&a)[K][K], double (&r)[K][NR]) {\n"
            "#pragma unroll\n  for (int c = 0; c < K; ++c) {\n"
            "#pragma unroll\n    for (int i = c + 1; i < K; ++i) {\n"
            "      const bool sw = fabs(a[i][c]) > fabs(a[c][c]);\n"
            "#pragma unroll\n      for (int j = c; j < K; ++j) {\n        const double t = a[c][j];\n"
            "        a[c][j] = sw ? a[i][j] : t;\n        a[i][j] = sw ? t : a[i][j];\n      }\n"
            "#pragma unroll\n      for (int q = 0; q < NR; ++q) {\n        const double t = r[c][q];\n"
            "        r[c][q] = sw ? r[i][q] : t;\n        r[i][q] = sw ? t : r[i][q];\n      }\n    }\n"
            "#pragma unroll\n    for (int i = c + 1; i < K; ++i) {\n      const double l = a[i][c] / a[c][c];\n"
            "#pragma unroll\n      for (int j = c + 1; j < K; ++j) a[i][j] -= l * a[c][j];\n"
            "#pragma unroll\n      for (int q = 0; q < NR; ++q) r[i][q] -= l * r[c][q];\n    }\n  }\n"
            "#pragma unroll\n  for (int i = K - 1; i >= 0; --i) {\n"
            "#pragma unroll\n    for (int q = 0; q < NR; ++q) {\n      double sum = r[i][q];\n"
            "#pragma unroll\n      for (int j = i + 1; j < K; ++j) sum -= a[i][j] * r[j][q];\n"
            "      r[i][q] = sum / a[i][i];\n    }\n  }\n}\n";
  }
  // Newton-matrix reuse is compiled in only when asked for: keeping the
  // factors across attempts holds them in registers through the whole step
  head << "#define CH_REUSE " << (reuse ? 1 : 0) << "\n";
  head << "#define CH_RU " << lit(kRu) << "\n#define CH_RU_CGS " << lit(kRuCgs) << "\n#define CH_PATM "
       << lit(kPatm) << "\n#define CH_TREF " << lit(kTref) << "\n";
  head << "#define CH_LN10 " << lit(std::log(10.0)) << "\n#define CH_INV_LN10 " << lit(1.0 / std::log(10.0)) << "\n";
  head << "__constant__ double ch_K[" << std::max<size_t>(pool.size(), 1) << "] = {";
  for (size_t i = 0; i < pool.size(); ++i) head << (i ? ", " : "") << lit(pool[i]);
  if (pool.empty()) head << "0.0";
  head << "};\n";
  // exp for the rate constants (chem_exp.inc)
  head << kChExp;
  return head.str() + o.str() + kLpcBody;
}

namespace {

struct LpcModule {
  hipModule_t mod = nullptr;
  hipFunction_t integrate = nullptr;
  hipFunction_t boxes = nullptr;
  hipFunction_t rates = nullptr;
  hipFunction_t serve = nullptr;
};

std::mutex g_jit_mu;
std::map<std::pair<int, std::string>, LpcModule> g_jit_cache;   // (device, source)

}  // namespace

// Compile (or fetch) the lane-per-cell module of `src` for the current device.
int lpc_module(const std::string& src, int device, void** integrate_fn, void** boxes_fn, void** rates_fn,
               void** serve_fn, std::string& log) {
  std::lock_guard<std::mutex> lk(g_jit_mu);
  auto key = std::make_pair(device, src);
  auto it = g_jit_cache.find(key);
  if (it != g_jit_cache.end()) {
    *integrate_fn = it->second.integrate;
    *boxes_fn = it->second.boxes;
    *rates_fn = it->second.rates;
    *serve_fn = it->second.serve;
    return 0;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    log = "hipGetDeviceProperties failed";
    return -1;
  }
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "chem_lpc.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    log = "hiprtcCreateProgram failed";
    return -1;
  }
  const std::string off = "--offload-arch=" + arch;
  // Machine LICM off: with the whole integration in one loop nest it hoists
  // constants and addresses out of the step loop, and with every register
  // in use they are then spilled to scratch and reloaded at each use.
  const char* opts[] = {off.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-mllvm", "-disable-machine-licm"};
  const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t log_size = 0;
  hiprtcGetProgramLogSize(prog, &log_size);
  if (log_size > 1) {
    log.resize(log_size);
    hiprtcGetProgramLog(prog, &log[0]);
  }
  if (rc != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    log = "hipRTC compile of the lane-per-cell kernels failed: " + log;
    return -1;
  }
  size_t code_size = 0;
  hiprtcGetCodeSize(prog, &code_size);
  std::vector<char> code(code_size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  LpcModule mod;
  if (hipModuleLoadData(&mod.mod, code.data()) != hipSuccess ||
      hipModuleGetFunction(&mod.integrate, mod.mod, "chem_lpc_integrate") != hipSuccess ||
      hipModuleGetFunction(&mod.boxes, mod.mod, "chem_lpc_boxes") != hipSuccess ||
      hipModuleGetFunction(&mod.rates, mod.mod, "chem_lpc_rates") != hipSuccess ||
      hipModuleGetFunction(&mod.serve, mod.mod, "chem_lpc_serve") != hipSuccess) {
    log = "loading the lane-per-cell module failed";
    return -1;
  }
  g_jit_cache[key] = mod;
  *integrate_fn = mod.integrate;
  *boxes_fn = mod.boxes;
  *rates_fn = mod.rates;
  *serve_fn = mod.serve;
  return 0;
}

namespace {
struct LpcParams {   // layout of ChParams in the generated source
  double p, dt, rtol, atol;
  int max_steps, q_max, fixed_T, fixed_step_n;
  int jac_reuse, pad;
};
LpcParams lpc_params(const IntParams& prm) {
  LpcParams q;
  q.p = prm.p;
  q.dt = prm.dt;
  q.rtol = prm.rtol;
  q.atol = prm.atol;
  q.max_steps = prm.max_steps;
  q.q_max = prm.q_max;
  q.fixed_T = prm.fixed_T;
  q.fixed_step_n = prm.fixed_step_n;
  q.jac_reuse = prm.jac_reuse;
  q.pad = 0;
  return q;
}
}  // namespace

hipError_t launch_lpc_integrate(void* fn, const IntParams& prm, double* T, double* Y, int64_t n, int32_t* rec,
                                hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  LpcParams q = lpc_params(prm);
  long long nn = n;
  void* args[] = {&T, &Y, &nn, &rec, &q};
  const unsigned blocks = (unsigned)((n + 63) / 64);
  return hipModuleLaunchKernel((hipFunction_t)fn, blocks, 1, 1, 64, 1, 1, 0, stream, args, nullptr);
}

hipError_t launch_lpc_rates(void* fn, double p, int fixed_T, const double* T, const double* Y, int64_t n,
                            double* wdot, double* f, double* jac, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long nn = n;
  void* args[] = {&T, &Y, &nn, &p, &fixed_T, &wdot, &f, &jac};
  const unsigned blocks = (unsigned)((n + 63) / 64);
  return hipModuleLaunchKernel((hipFunction_t)fn, blocks, 1, 1, 64, 1, 1, 0, stream, args, nullptr);
}

hipError_t launch_lpc_boxes(void* fn, const IntParams& prm, const BoxDev* boxes, const BoxJob* job, unsigned* head,
                            int* remaining, int32_t* rec, int* host_done, int grid, hipStream_t stream) {
  LpcParams q = lpc_params(prm);
  void* args[] = {&q, &boxes, &job, &head, &remaining, &rec, &host_done};
  return hipModuleLaunchKernel((hipFunction_t)fn, (unsigned)grid, 1, 1, 64, 1, 1, 0, stream, args, nullptr);
}

namespace {
struct LpcServeQ {   // layout of ChServeQ in the generated source
  const ServeBox* boxes;
  const unsigned* tile_slot;
  const unsigned* pub;
  const int* stop;
  unsigned* head;
  int* finished;
  int* done;
  unsigned tile_mask;
  int idle_polls;
  long long quantum;
};
static_assert(sizeof(ServeBox) == 48, "ChServeBox mirrors ServeBox");
}  // namespace

int lpc_serve_waves_per_cu(void* fn) {
  int blocks = 0;
  const hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (hipFunction_t)fn, 64, 0);
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

hipError_t launch_lpc_serve(void* fn, const IntParams& prm, const ServeQueue& q, int grid, hipStream_t stream) {
  LpcParams pq = lpc_params(prm);
  LpcServeQ sq{q.boxes, q.tile_slot, q.pub, q.stop, q.head, q.finished, q.done, q.tile_mask, q.idle_polls,
               (long long)q.quantum};
  void* args[] = {&pq, &sq};
  return hipModuleLaunchKernel((hipFunction_t)fn, (unsigned)grid, 1, 1, 64, 1, 1, 0, stream, args, nullptr);
}

}  // namespace chemgpu
