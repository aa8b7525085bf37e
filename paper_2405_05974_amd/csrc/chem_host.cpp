// chem_host.cpp -- C ABI of libchem: mechanism parsing and upload, options,
// integration and rates launches, per-call statistics.  See include/chem.h.
#include "../../include/chem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "chem_handle.h"
#include "chem_internal.h"

using chemgpu::DevMech;
using chemgpu::IntParams;
using chemgpu::RxParams;
using chemgpu::HostMech;
using chemgpu::HostReaction;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(CHEM_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Whitespace tokenizer that drops '#' comments.
class Tokens {
 public:
  explicit Tokens(const std::string& text) {
    std::istringstream in(text);
    std::string line;
    while (std::getline(in, line)) {
      const size_t hash = line.find('#');
      if (hash != std::string::npos) line.resize(hash);
      std::istringstream ls(line);
      std::string t;
      while (ls >> t) toks_.push_back(t);
    }
  }
  bool word(const char* w) { return pos_ < toks_.size() && toks_[pos_++] == w; }
  bool integer(int& v) {
    if (pos_ >= toks_.size()) return false;
    const std::string& t = toks_[pos_++];
    char* end = nullptr;
    const long x = std::strtol(t.c_str(), &end, 10);
    if (end == t.c_str() || *end) return false;
    v = (int)x;
    return true;
  }
  bool real(double& v) {
    if (pos_ >= toks_.size()) return false;
    const std::string& t = toks_[pos_++];
    char* end = nullptr;
    v = std::strtod(t.c_str(), &end);
    return end != t.c_str() && !*end && std::isfinite(v);
  }
  bool skip() { return pos_++ < toks_.size(); }
  // consume the next token only when it equals w
  bool opt_word(const char* w) {
    if (pos_ < toks_.size() && toks_[pos_] == w) {
      ++pos_;
      return true;
    }
    return false;
  }

 private:
  std::vector<std::string> toks_;
  size_t pos_ = 0;
};

}  // namespace

std::vector<double> chemgpu::HostMech::nasa_of(int k) const {
  if (!nasa[k].empty()) return nasa[k];
  const double Tr = chemgpu::kTref, R = chemgpu::kRu;
  std::vector<double> c(15, 0.0);
  c[0] = 1000.0;
  for (int r = 0; r < 2; ++r) {
    double* a = &c[1 + 7 * r];
    a[0] = a0[k];
    a[1] = a1[k];
    a[5] = hf[k] / R - (a0[k] * Tr + a1[k] * Tr * Tr * 0.5);
    a[6] = s0[k] / R - (a0[k] * std::log(Tr) + a1[k] * Tr);
  }
  return c;
}

namespace {

int parse_mechanism(const std::string& text, HostMech& m) {
  Tokens tk(text);
  int ver = 0, E = 0, S = 0, R = 0;
  if (!tk.word("chem-mech") || !tk.integer(ver) || ver != 1) return fail(CHEM_ERR_PARSE, "missing 'chem-mech 1' header");
  if (!tk.word("ELEMENTS") || !tk.integer(E) || E < 1 || E > 16) return fail(CHEM_ERR_PARSE, "bad ELEMENTS block");
  m.emass.resize(E);
  for (int e = 0; e < E; ++e)
    if (!tk.skip() || !tk.real(m.emass[e]) || !(m.emass[e] > 0)) return fail(CHEM_ERR_PARSE, "bad element line");
  if (!tk.word("SPECIES") || !tk.integer(S) || S < 1) return fail(CHEM_ERR_PARSE, "bad SPECIES block");
  m.atoms.assign(S, std::vector<int>(E, 0));
  m.W.resize(S); m.a0.resize(S); m.a1.resize(S); m.hf.resize(S); m.s0.resize(S);
  m.nasa.assign(S, {});
  std::vector<int> inert_of(S, 0);
  for (int k = 0; k < S; ++k) {
    int inert = 0, total = 0;
    if (!tk.skip() || !tk.integer(inert)) return fail(CHEM_ERR_PARSE, "bad species line");
    inert_of[k] = inert;
    double w = 0.0;
    for (int e = 0; e < E; ++e) {
      if (!tk.integer(m.atoms[k][e]) || m.atoms[k][e] < 0) return fail(CHEM_ERR_PARSE, "bad atom count");
      w += m.atoms[k][e] * m.emass[e];
      total += m.atoms[k][e];
    }
    if (total == 0) return fail(CHEM_ERR_PARSE, "species without atoms");
    m.W[k] = w;
    if (tk.opt_word("NASA7")) {
      m.nasa[k].resize(15);
      for (int i = 0; i < 15; ++i)
        if (!tk.real(m.nasa[k][i])) return fail(CHEM_ERR_PARSE, "bad NASA7 thermo of species " + std::to_string(k));
      if (!(m.nasa[k][0] > 0)) return fail(CHEM_ERR_PARSE, "bad NASA7 midpoint temperature");
    } else if (!tk.real(m.a0[k]) || !tk.real(m.a1[k]) || !tk.real(m.hf[k]) || !tk.real(m.s0[k])) {
      return fail(CHEM_ERR_PARSE, "bad species thermo");
    }
  }
  if (!tk.word("REACTIONS") || !tk.integer(R) || R < 0) return fail(CHEM_ERR_PARSE, "bad REACTIONS block");
  m.rx.resize(R);
  for (int j = 0; j < R; ++j) {
    HostReaction& x = m.rx[j];
    int nr = 0, np = 0;
    if (!tk.integer(x.rev) || !tk.integer(x.type) || x.type < 0 || x.type > 2 || x.rev < 0 || x.rev > 1)
      return fail(CHEM_ERR_PARSE, "bad reaction kind in reaction " + std::to_string(j));
    if (!tk.integer(nr) || nr < 1 || nr > chemgpu::kMaxSide) return fail(CHEM_ERR_PARSE, "bad reactant count");
    x.reac.resize(nr);
    for (int i = 0; i < nr; ++i)
      if (!tk.integer(x.reac[i]) || x.reac[i] < 0 || x.reac[i] >= S) return fail(CHEM_ERR_PARSE, "bad reactant index");
    if (!tk.integer(np) || np < 1 || np > chemgpu::kMaxSide) return fail(CHEM_ERR_PARSE, "bad product count");
    x.prod.resize(np);
    for (int i = 0; i < np; ++i)
      if (!tk.integer(x.prod[i]) || x.prod[i] < 0 || x.prod[i] >= S) return fail(CHEM_ERR_PARSE, "bad product index");
    if (!tk.real(x.A) || !tk.real(x.b) || !tk.real(x.Ea) || !(x.A > 0))
      return fail(CHEM_ERR_PARSE, "bad Arrhenius parameters in reaction " + std::to_string(j));
    if (x.type == 2 && (!tk.real(x.A0) || !tk.real(x.b0) || !tk.real(x.Ea0) || !(x.A0 > 0)))
      return fail(CHEM_ERR_PARSE, "bad falloff parameters in reaction " + std::to_string(j));
    if (tk.opt_word("TROE")) {
      if (x.type != 2 || !tk.integer(x.ntroe) || (x.ntroe != 3 && x.ntroe != 4))
        return fail(CHEM_ERR_PARSE, "bad TROE record in reaction " + std::to_string(j));
      for (int i = 0; i < x.ntroe; ++i)
        if (!tk.real(x.troe[i])) return fail(CHEM_ERR_PARSE, "bad TROE parameter in reaction " + std::to_string(j));
      if (x.troe[1] == 0.0 || x.troe[2] == 0.0)
        return fail(CHEM_ERR_PARSE, "TROE temperatures T3 and T1 must be nonzero");
    }
    if (tk.opt_word("EFF")) {
      int ne = 0;
      if (x.type == 0 || !tk.integer(ne) || ne < 0 || ne > 64)
        return fail(CHEM_ERR_PARSE, "bad EFF record in reaction " + std::to_string(j));
      for (int i = 0; i < ne; ++i) {
        int k = -1;
        double v = 0.0;
        if (!tk.integer(k) || k < 0 || k >= S || !tk.real(v) || !(v >= 0))
          return fail(CHEM_ERR_PARSE, "bad efficiency in reaction " + std::to_string(j));
        for (int k2 : x.eff_k)
          if (k2 == k) return fail(CHEM_ERR_PARSE, "repeated efficiency in reaction " + std::to_string(j));
        x.eff_k.push_back(k);
        x.eff_v.push_back(v);
      }
    }
    for (int e = 0; e < E; ++e) {
      int bal = 0;
      for (int s : x.prod) bal += m.atoms[s][e];
      for (int s : x.reac) bal -= m.atoms[s][e];
      if (bal != 0) return fail(CHEM_ERR_PARSE, "reaction " + std::to_string(j) + " is not atom balanced");
    }
  }
  // optional QSS record: species the quasi-steady-state approximation turns
  // into algebraic unknowns (Sec. 2.1, Eq. 4)
  std::vector<char> isq(S, 0);
  if (tk.opt_word("QSS")) {
    int nq = 0;
    if (!tk.integer(nq) || nq < 0 || nq >= S) return fail(CHEM_ERR_PARSE, "bad QSS record");
    for (int q = 0; q < nq; ++q) {
      int k = -1;
      if (!tk.integer(k) || k < 0 || k >= S || isq[k] || inert_of[k])
        return fail(CHEM_ERR_PARSE, "bad QSS species in the QSS record");
      isq[k] = 1;
      m.qss.push_back(k);
    }
  }
  // one-sided linearisation (Sec. 2.2): a direction with two or more QSS
  // reactants is removed, the other direction stays
  for (HostReaction& x : m.rx) {
    int nqr = 0, nqp = 0;
    for (int k : x.reac) nqr += isq[k];
    for (int k : x.prod) nqp += isq[k];
    x.drop_f = nqr >= 2;
    x.drop_r = nqp >= 2;
  }
  for (int k : m.qss) {
    bool consumed = false;
    for (const HostReaction& x : m.rx) {
      int nu = 0, inr = 0, inp = 0;
      for (int s : x.prod) { nu += (s == k); inp |= (s == k); }
      for (int s : x.reac) { nu -= (s == k); inr |= (s == k); }
      if ((nu < 0 && inr && !x.drop_f) || (nu > 0 && inp && x.rev && !x.drop_r)) consumed = true;
    }
    if (!consumed) return fail(CHEM_ERR_PARSE, "QSS species " + std::to_string(k) + " is never consumed");
  }
  if (!tk.word("END")) return fail(CHEM_ERR_PARSE, "missing END");
  return CHEM_OK;
}

}  // namespace

namespace {

int upload(chem_mech* h) {
  const HostMech& m = h->host;
  const int S = (int)m.W.size(), R = (int)m.rx.size(), N = S + 1;
  if (N > 64) return fail(CHEM_ERR_UNSUPPORTED, "mechanisms with more than 63 species are not supported");
  const int np = N <= 16 ? 16 : (N <= 32 ? 32 : 64);
  const int widths[3] = {16, 32, 64};

  std::vector<RxParams> rx(std::max(R, 1));
  std::vector<int> effk;
  std::vector<double> effv;
  const double kcal_to_K = 4184.0 / chemgpu::kRu;   // Ea/R per kcal/mol
  for (int j = 0; j < R; ++j) {
    const HostReaction& x = m.rx[j];
    RxParams& d = rx[j];
    std::memset(&d, 0, sizeof d);
    d.lnA = std::log(x.A);
    d.b = x.b;
    d.EaR = x.Ea * kcal_to_K;
    if (x.type == 2) {
      d.lnA0 = std::log(x.A0);
      d.b0 = x.b0;
      d.EaR0 = x.Ea0 * kcal_to_K;
    }
    d.ntroe = x.ntroe;
    for (int i = 0; i < 4; ++i) d.troe[i] = x.troe[i];
    d.eff_off = (int)effk.size();
    d.eff_n = (int)x.eff_k.size();
    for (size_t i = 0; i < x.eff_k.size(); ++i) {
      effk.push_back(x.eff_k[i]);
      effv.push_back(x.eff_v[i] - 1.0);
    }
    d.type = x.type;
    d.rev = x.rev;
    d.nr = (int)x.reac.size();
    d.np = (int)x.prod.size();
    for (int s = 0; s < chemgpu::kSlots; ++s) d.sp[s] = -1;
    for (int i = 0; i < d.nr; ++i) d.sp[i] = x.reac[i];
    for (int i = 0; i < d.np; ++i) d.sp[chemgpu::kMaxSide + i] = x.prod[i];
  }
  // the hot fields again, one array per field
  std::vector<double> rlnA(std::max(R, 1), 0.0), rb(std::max(R, 1), 0.0), rEaR(std::max(R, 1), 0.0);
  std::vector<int4> rmeta(std::max(R, 1));
  for (int j = 0; j < std::max(R, 1); ++j) rmeta[j] = int4{0, 0xFFFFFF, 0xFFFFFF, 0};
  for (int j = 0; j < R; ++j) {
    const RxParams& d = rx[j];
    if (d.eff_off >= (1 << 20) || d.eff_n >= (1 << 11))
      return fail(CHEM_ERR_UNSUPPORTED, "too many collision efficiencies");
    rlnA[j] = d.lnA;
    rb[j] = d.b;
    rEaR[j] = d.EaR;
    int4 mt;
    mt.x = d.type | (d.rev << 2) | (d.nr << 3) | (d.np << 5) | ((d.ntroe > 0) << 7);
    mt.y = 0;
    mt.z = 0;
    for (int s2 = 0; s2 < chemgpu::kSlots; ++s2) {
      const int v = d.sp[s2] < 0 ? 255 : d.sp[s2];
      if (s2 < chemgpu::kMaxSide) mt.y |= v << (8 * s2);
      else mt.z |= v << (8 * (s2 - chemgpu::kMaxSide));
    }
    mt.w = d.eff_off | (d.eff_n << 20);
    rmeta[j] = mt;
  }
  // net stoichiometry of each reaction (species order), for the Jacobian scatter
  std::vector<int2> rnet(std::max(R, 1), int2{0x3FFFFFFF, 0x3FFFFFFF});
  for (int j = 0; j < R; ++j) {
    int2 nt{0, 0};
    int cnt = 0;
    for (int k = 0; k < S; ++k) {
      int nu = 0;
      for (int sp2 : m.rx[j].prod) nu += (sp2 == k);
      for (int sp2 : m.rx[j].reac) nu -= (sp2 == k);
      if (nu == 0) continue;
      const int v = (k << 3) | (nu + 4);
      if (cnt < 3) nt.x |= v << (10 * cnt);
      else nt.y |= v << (10 * (cnt - 3));
      ++cnt;
    }
    for (int c2 = cnt; c2 < 6; ++c2) {
      if (c2 < 3) nt.x |= 1023 << (10 * c2);
      else nt.y |= 1023 << (10 * (c2 - 3));
    }
    rnet[j] = nt;
  }
  // per-species lists of (reaction, net coefficient) in reaction order; for
  // each group width the list is split in chunks of that many reactions
  std::vector<int> ent, ent_start(S + 1, 0);
  std::vector<int> ent_j;
  for (int k = 0; k < S; ++k) {
    ent_start[k] = (int)ent.size();
    for (int j = 0; j < R; ++j) {
      int nu = 0;
      for (int s : m.rx[j].prod) nu += (s == k);
      for (int s : m.rx[j].reac) nu -= (s == k);
      if (nu == 0) continue;
      ent.push_back((j << 3) | (nu + 4));
      ent_j.push_back(j);
    }
  }
  ent_start[S] = (int)ent.size();
  std::vector<int> offs[3];
  int nchs[3] = {0, 0, 0};
  for (int wi = 0; wi < 3; ++wi) {
    const int w = widths[wi];
    const int nch = std::max(1, (R + w - 1) / w);
    nchs[wi] = nch;
    offs[wi].assign((size_t)S * (nch + 1), 0);
    for (int k = 0; k < S; ++k)
      for (int c = 0; c <= nch; ++c) {
        int e = ent_start[k];
        while (e < ent_start[k + 1] && ent_j[e] < c * w) ++e;
        offs[wi][(size_t)k * (nch + 1) + c] = e;
      }
  }
  if (ent.empty()) ent.push_back(0);
  std::vector<int> off;
  size_t off_at[3];
  for (int wi = 0; wi < 3; ++wi) {
    off_at[wi] = off.size();
    off.insert(off.end(), offs[wi].begin(), offs[wi].end());
  }

  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_sp = 0;
  const size_t sz_sp = align(5 * sizeof(double) * S);
  const size_t o_rx = o_sp + sz_sp;
  const size_t sz_rx = align(sizeof(RxParams) * rx.size());
  const size_t o_off = o_rx + sz_rx;
  const size_t sz_off = align(sizeof(int) * off.size());
  const size_t o_ent = o_off + sz_off;
  const size_t sz_ent = align(sizeof(int) * ent.size());
  const bool nasa = m.any_nasa();
  const size_t o_nasa = o_ent + sz_ent;
  const size_t sz_nasa = nasa ? align(sizeof(double) * 15 * S) : 0;
  if (effk.empty()) {
    effk.push_back(0);
    effv.push_back(0.0);
  }
  const size_t o_effk = o_nasa + sz_nasa;
  const size_t sz_effk = align(sizeof(int) * effk.size());
  const size_t o_effv = o_effk + sz_effk;
  const size_t sz_effv = align(sizeof(double) * effv.size());
  const size_t sz_rk = align(sizeof(double) * rlnA.size());
  const size_t o_rlnA = o_effv + sz_effv, o_rb = o_rlnA + sz_rk, o_rEaR = o_rb + sz_rk, o_rmeta = o_rEaR + sz_rk;
  const size_t sz_rmeta = align(sizeof(int4) * rmeta.size());
  const size_t o_rnet = o_rmeta + sz_rmeta;
  const size_t sz_rnet = align(sizeof(int2) * rnet.size());
  const size_t total = o_rnet + sz_rnet;
  std::vector<char> blob(total, 0);
  double* sp = reinterpret_cast<double*>(blob.data() + o_sp);
  for (int k = 0; k < S; ++k) {
    sp[0 * S + k] = m.W[k];
    sp[1 * S + k] = m.a0[k];
    sp[2 * S + k] = m.a1[k];
    sp[3 * S + k] = m.hf[k];
    sp[4 * S + k] = m.s0[k];
  }
  std::memcpy(blob.data() + o_rx, rx.data(), sizeof(RxParams) * rx.size());
  std::memcpy(blob.data() + o_off, off.data(), sizeof(int) * off.size());
  std::memcpy(blob.data() + o_ent, ent.data(), sizeof(int) * ent.size());
  if (nasa) {
    double* nc = reinterpret_cast<double*>(blob.data() + o_nasa);
    for (int k = 0; k < S; ++k) {
      const std::vector<double> c = m.nasa_of(k);
      for (int i = 0; i < 15; ++i) nc[(size_t)i * S + k] = c[i];
    }
  }
  std::memcpy(blob.data() + o_effk, effk.data(), sizeof(int) * effk.size());
  std::memcpy(blob.data() + o_effv, effv.data(), sizeof(double) * effv.size());
  std::memcpy(blob.data() + o_rlnA, rlnA.data(), sizeof(double) * rlnA.size());
  std::memcpy(blob.data() + o_rb, rb.data(), sizeof(double) * rb.size());
  std::memcpy(blob.data() + o_rEaR, rEaR.data(), sizeof(double) * rEaR.size());
  std::memcpy(blob.data() + o_rmeta, rmeta.data(), sizeof(int4) * rmeta.size());
  std::memcpy(blob.data() + o_rnet, rnet.data(), sizeof(int2) * rnet.size());

  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  void* d = nullptr;
  e = hipMalloc(&d, total);
  if (e != hipSuccess) return fail(CHEM_ERR_OOM, std::string("hipMalloc of mechanism tables: ") + hipGetErrorString(e));
  h->blob = d;
  e = hipMemcpy(d, blob.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy of mechanism tables");
  char* base = static_cast<char*>(d);
  DevMech& dm = h->dev;
  dm.S = S;
  dm.R = R;
  dm.N = N;
  dm.np_width = np;
  const double* dsp = reinterpret_cast<const double*>(base + o_sp);
  dm.W = dsp;
  dm.a0 = dsp + S;
  dm.a1 = dsp + 2 * S;
  dm.hf = dsp + 3 * S;
  dm.s0 = dsp + 4 * S;
  dm.rx = reinterpret_cast<const RxParams*>(base + o_rx);
  for (int wi = 0; wi < 3; ++wi) {
    h->csr_off_np[wi] = reinterpret_cast<const int*>(base + o_off) + off_at[wi];
    h->nch_np[wi] = nchs[wi];
  }
  dm.csr_off = h->csr_off_np[np == 16 ? 0 : (np == 32 ? 1 : 2)];
  dm.nch = h->nch_np[np == 16 ? 0 : (np == 32 ? 1 : 2)];
  dm.csr_ent = reinterpret_cast<const int*>(base + o_ent);
  if (!m.qss.empty()) {
    // the state holds the transported species; QSS mechanisms run only in the
    // generated kernels, which carry the closure themselves
    dm.S = m.n_state_species();
    dm.N = dm.S + 1;
  }
  dm.nasa = nasa ? 1 : 0;
  dm.nasa_c = nasa ? reinterpret_cast<const double*>(base + o_nasa) : nullptr;
  dm.eff_k = reinterpret_cast<const int*>(base + o_effk);
  dm.eff_v = reinterpret_cast<const double*>(base + o_effv);
  dm.rx_lnA = reinterpret_cast<const double*>(base + o_rlnA);
  dm.rx_b = reinterpret_cast<const double*>(base + o_rb);
  dm.rx_EaR = reinterpret_cast<const double*>(base + o_rEaR);
  dm.rx_meta = reinterpret_cast<const int4*>(base + o_rmeta);
  dm.rx_net = reinterpret_cast<const int2*>(base + o_rnet);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess && prop.multiProcessorCount > 0)
    h->n_cu = prop.multiProcessorCount;
  e = hipMalloc(&h->dstats, sizeof(unsigned long long) * chemgpu::kStatCount);
  if (e != hipSuccess) return fail(CHEM_ERR_OOM, "hipMalloc of stats");
  if ((e = hipEventCreate(&h->ev0)) != hipSuccess || (e = hipEventCreate(&h->ev1)) != hipSuccess)
    return hip_fail(e, "hipEventCreate");
  return CHEM_OK;
}

int load_text(const std::string& text, chem_mech** out) {
  if (!out) return fail(CHEM_ERR_ARG, "out is NULL");
  *out = nullptr;
  chem_mech* h = new (std::nothrow) chem_mech();
  if (!h) return fail(CHEM_ERR_OOM, "host allocation failed");
  int rc = parse_mechanism(text, h->host);
  if (rc == CHEM_OK) rc = upload(h);
  if (rc != CHEM_OK) {
    chem_mech_free(h);
    return rc;
  }
  *out = h;
  g_last_error.clear();
  return CHEM_OK;
}

void fill_stats(chem_stats* stats, int64_t n_cells, const unsigned long long* hs, float ms) {
  stats->n_cells = n_cells;
  stats->n_steps_total = (int64_t)hs[0];
  stats->n_steps_max = (int64_t)hs[1];
  stats->n_attempts = (int64_t)hs[2];
  stats->n_rhs = (int64_t)hs[3];
  stats->n_jac = (int64_t)hs[4];
  stats->n_lu = (int64_t)hs[4];
  stats->n_newton_iters = (int64_t)hs[5];
  stats->n_err_test_fails = (int64_t)hs[6];
  stats->n_newton_fails = (int64_t)hs[7];
  stats->n_cells_failed = (int64_t)hs[8];
  stats->n_ir_sweeps = (int64_t)hs[9];
  stats->wall_ms = ms;
}

int ensure_records(chem_mech* h, int64_t n) {
  if (n <= h->rec_cap) return CHEM_OK;
  if (h->rec) {
    (void)hipFree(h->rec);
    h->rec = nullptr;
    h->rec_cap = 0;
  }
  const int64_t cap = std::max<int64_t>(n, 1024);
  hipError_t e = hipMalloc(&h->rec, sizeof(int32_t) * chemgpu::kRecRows * cap);
  if (e != hipSuccess) return fail(CHEM_ERR_OOM, std::string("hipMalloc of cell records: ") + hipGetErrorString(e));
  h->rec_cap = cap;
  return CHEM_OK;
}

}  // namespace

// ------------------------------------------------ kernel family selection

namespace {

// The kernel family the handle's options ask for (without compiling anything).
int kernel_choice(const chem_mech* m, bool* lpc) {
  const int N = m->dev.N;
  bool want = false;
  if (!m->host.qss.empty()) {
    // the QSS closure is generated per mechanism: lane-per-cell kernels only
    if (m->kernel_mode == 1)
      return fail(CHEM_ERR_UNSUPPORTED, "mechanisms with QSS species run in the generated lane-per-cell kernels");
    if (N > chemgpu::kLpcMaxN)
      return fail(CHEM_ERR_UNSUPPORTED, "mechanisms with QSS species run in the generated kernels, which serve up to " +
                                            std::to_string(chemgpu::kLpcMaxN) + " state components");
    if (m->lu_fp32 || m->jac_mode)
      return fail(CHEM_ERR_UNSUPPORTED, "the FP32-LU and difference-quotient options do not run with QSS species");
    *lpc = true;
    return CHEM_OK;
  }
  if (m->kernel_mode == 2) {
    if (N > chemgpu::kLpcMaxN)
      return fail(CHEM_ERR_UNSUPPORTED,
                  "lane-per-cell kernels serve up to " + std::to_string(chemgpu::kLpcMaxN) + " state components");
    if (m->lu_fp32) return fail(CHEM_ERR_UNSUPPORTED, "the FP32-LU option runs in the group kernels only");
    if (m->jac_mode) return fail(CHEM_ERR_UNSUPPORTED, "finite-difference Jacobians run in the group kernels only");
    want = true;
  } else if (m->kernel_mode == 0) {
    want = N <= chemgpu::kLpcMaxN && !m->lu_fp32 && !m->jac_mode;
  }
  *lpc = want;
  return CHEM_OK;
}

// True when the lane-per-cell module for the handle's device and options is loaded.
bool lpc_ready(const chem_mech* m) {
  return m->lpc_integrate && m->lpc_device == m->device && m->lpc_reuse == (m->jac_reuse ? 1 : 0);
}

}  // namespace

int chem_select_kernel(chem_mech* m, bool* lpc) {
  const int crc = kernel_choice(m, lpc);
  if (crc != CHEM_OK || !*lpc) return crc;
  std::lock_guard<std::mutex> lk(m->lpc_mu);
  const int reuse = m->jac_reuse ? 1 : 0;
  if (lpc_ready(m)) return CHEM_OK;
  if (m->lpc_src.empty() || m->lpc_reuse != reuse) m->lpc_src = chemgpu::lpc_source(m->host, reuse != 0);
  std::string log;
  if (chemgpu::lpc_module(m->lpc_src, m->device, &m->lpc_integrate, &m->lpc_boxes, &m->lpc_rates, &m->lpc_serve,
                          log) != 0)
    return fail(CHEM_ERR_DEVICE, log);
  m->lpc_device = m->device;
  m->lpc_reuse = reuse;
  return CHEM_OK;
}

hipError_t chem_launch_box_queue(chem_mech* m, bool lpc, const chemgpu::IntParams& prm, const chemgpu::BoxDev* boxes,
                                 const chemgpu::BoxJob* job, unsigned* head, int* remaining, int32_t* rec,
                                 int* host_done, int grid, hipStream_t stream) {
  if (!lpc) return chemgpu::launch_boxes(m->dev, prm, boxes, job, head, remaining, rec, host_done, grid, stream);
  const hipError_t e = chemgpu::launch_boxes_init(boxes, job, head, remaining, stream);
  if (e != hipSuccess) return e;
  return chemgpu::launch_lpc_boxes(m->lpc_boxes, prm, boxes, job, head, remaining, rec, host_done, grid, stream);
}

extern "C" {

int chem_mech_load_str(const char* text, chem_mech** out) {
  if (!text) return fail(CHEM_ERR_ARG, "text is NULL");
  try {
    return load_text(text, out);
  } catch (...) {
    return fail(CHEM_ERR_OOM, "exception while loading mechanism");
  }
}

int chem_mech_load(const char* path, chem_mech** out) {
  if (!path) return fail(CHEM_ERR_ARG, "path is NULL");
  try {
    std::ifstream in(path);
    if (!in) return fail(CHEM_ERR_ARG, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << in.rdbuf();
    return load_text(ss.str(), out);
  } catch (...) {
    return fail(CHEM_ERR_OOM, "exception while loading mechanism");
  }
}

void chem_mech_free(chem_mech* m) {
  if (!m) return;
  if (m->blob) (void)hipFree(m->blob);
  if (m->rec) (void)hipFree(m->rec);
  if (m->retry_in) (void)hipFree(m->retry_in);
  if (m->dstats) (void)hipFree(m->dstats);
  if (m->ev0) (void)hipEventDestroy(m->ev0);
  if (m->ev1) (void)hipEventDestroy(m->ev1);
  if (m->dboxes) (void)hipFree(m->dboxes);
  if (m->dremaining) (void)hipFree(m->dremaining);
  if (m->djob) (void)hipFree(m->djob);
  if (m->dhead) (void)hipFree(m->dhead);
  if (m->host_done) (void)hipHostFree(m->host_done);
  if (m->graph) (void)hipGraphExecDestroy(m->graph);
  if (m->capture_stream) (void)hipStreamDestroy(m->capture_stream);
  delete m;
}

int chem_mech_info(const chem_mech* m, int* n_species, int* n_reactions, int* n_elements) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_species) *n_species = m->dev.S;
  if (n_reactions) *n_reactions = m->dev.R;
  if (n_elements) *n_elements = (int)m->host.emass.size();
  return CHEM_OK;
}

int chem_set_stream(chem_mech* m, void* hip_stream) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  m->stream = static_cast<hipStream_t>(hip_stream);
  return CHEM_OK;
}

int chem_set_option(chem_mech* m, int key, double value) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (!std::isfinite(value)) return fail(CHEM_ERR_ARG, "option value is not finite");
  const long v = std::lround(value);
  switch (key) {
    case CHEM_OPT_MAX_STEPS:
      if (v < 1 || v > 100000000) return fail(CHEM_ERR_ARG, "max_steps out of range");
      m->max_steps = (int)v;
      return CHEM_OK;
    case CHEM_OPT_Q_MAX:
      if (v < 1 || v > chemgpu::kQMax) return fail(CHEM_ERR_ARG, "q_max must be 1..5");
      m->q_max = (int)v;
      return CHEM_OK;
    case CHEM_OPT_FIXED_T:
      m->fixed_T = v != 0;
      return CHEM_OK;
    case CHEM_OPT_FIXED_STEP:
      if (v < 0 || v > 100000000) return fail(CHEM_ERR_ARG, "fixed_step out of range");
      m->fixed_step_n = (int)v;
      return CHEM_OK;
    case CHEM_OPT_LU_FP32:
      m->lu_fp32 = v != 0;
      return CHEM_OK;
    case CHEM_OPT_IR_MAX:
      if (v < 0 || v > 20) return fail(CHEM_ERR_ARG, "ir_max must be 0..20");
      m->ir_max = (int)v;
      return CHEM_OK;
    case CHEM_OPT_GRAPH:
      m->use_graph = v != 0;
      return CHEM_OK;
    case CHEM_OPT_WAVES_PER_CU:
      if (v < 1 || v > 32) return fail(CHEM_ERR_ARG, "waves_per_cu must be 1..32");
      m->waves_per_cu = (int)v;
      return CHEM_OK;
    case CHEM_OPT_JAC:
      if (v != 0 && v != 1 && v != 2)
        return fail(CHEM_ERR_ARG, "jac must be 0 (analytic), 1 (difference quotients) or 2 (difference-quotient T column)");
      m->jac_mode = (int)v;
      return CHEM_OK;
    case CHEM_OPT_RETRY:
      if (v < 0 || v > 12) return fail(CHEM_ERR_ARG, "retry must be 0..12 halvings");
      m->retry = (int)v;
      return CHEM_OK;
    case CHEM_OPT_JAC_REUSE:
      m->jac_reuse = v != 0;
      return CHEM_OK;
    case CHEM_OPT_KERNEL:
      if (v != 0 && v != 1 && v != 2) return fail(CHEM_ERR_ARG, "kernel must be 0 (auto), 1 (group) or 2 (lane per cell)");
      m->kernel_mode = (int)v;
      return CHEM_OK;
    case CHEM_OPT_GROUP_WIDTH: {
      const int wi = v == 16 ? 0 : (v == 32 ? 1 : (v == 64 ? 2 : -1));
      if (wi < 0 || v < m->dev.N) return fail(CHEM_ERR_ARG, "group width must be 16, 32 or 64 and at least S+1");
      m->dev.np_width = (int)v;
      m->dev.csr_off = m->csr_off_np[wi];
      m->dev.nch = m->nch_np[wi];
      return CHEM_OK;
    }
    case CHEM_OPT_PROGRESS:
      if (!(value >= 0) || !std::isfinite(value)) return fail(CHEM_ERR_ARG, "progress interval must be >= 0");
      m->progress_s = value;
      return CHEM_OK;
    default:
      return fail(CHEM_ERR_ARG, "unknown option key " + std::to_string(key));
  }
}

namespace {

hipError_t launch_either(chem_mech* m, bool lpc, const IntParams& prm, double* T, double* Y, int64_t n, int32_t* rec) {
  if (lpc) return chemgpu::launch_lpc_integrate(m->lpc_integrate, prm, T, Y, n, rec, m->stream);
  return chemgpu::launch_integrate(m->dev, prm, T, Y, n, rec, m->stream);
}

// The paper's remedy for a failed chemistry step, applied per cell: a cell
// that failed (attempt limit or step-size underflow) is integrated again from
// its input state with dt split into 2, 4, ... 2^retry equal substeps, until
// one level passes every substep.  Passed cells get that state and status 0;
// every cell's counters include the retry work.  The gather and scatter run
// on the host: they only happen when cells failed.
int retry_failed_cells(chem_mech* m, const IntParams& prm, bool lpc, int64_t n, double* T, double* Y, int32_t* rec,
                       unsigned long long* hs) {
  const int S = m->dev.S, N = S + 1, rows = chemgpu::kRecRows;
  std::vector<int32_t> hrec((size_t)rows * n);
  hipError_t e = hipMemcpy(hrec.data(), rec, sizeof(int32_t) * hrec.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "retry: records");
  std::vector<int64_t> idx;
  for (int64_t i = 0; i < n; ++i)
    if (hrec[i] == 1 || hrec[i] == 2) idx.push_back(i);
  if (idx.empty()) return CHEM_OK;
  const int64_t mc = (int64_t)idx.size();
  std::vector<double> hin((size_t)N * n);
  e = hipMemcpy(hin.data(), m->retry_in, sizeof(double) * hin.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "retry: saved inputs");
  std::vector<char> done(mc, 0);
  std::vector<double> result((size_t)N * mc, 0.0);
  std::vector<int32_t> acc((size_t)rows * mc, 0);
  double* dwork = nullptr;
  int32_t* drec = nullptr;
  e = hipMalloc(&dwork, sizeof(double) * N * mc);
  if (e == hipSuccess) e = hipMalloc(&drec, sizeof(int32_t) * rows * mc);
  if (e != hipSuccess) {
    (void)hipFree(dwork);
    return fail(CHEM_ERR_OOM, "retry: device buffers");
  }
  int rc = CHEM_OK;
  for (int level = 1; level <= m->retry && rc == CHEM_OK; ++level) {
    std::vector<int64_t> todo;
    for (int64_t j = 0; j < mc; ++j)
      if (!done[j]) todo.push_back(j);
    if (todo.empty()) break;
    const int64_t mt = (int64_t)todo.size();
    std::vector<double> w((size_t)N * mt);
    for (int64_t t = 0; t < mt; ++t) {
      const int64_t i = idx[todo[t]];
      w[t] = hin[i];
      for (int k = 0; k < S; ++k) w[mt + (size_t)k * mt + t] = hin[n + (size_t)k * n + i];
    }
    e = hipMemcpy(dwork, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { rc = hip_fail(e, "retry: upload"); break; }
    const int nsub = 1 << level;
    IntParams q = prm;
    q.dt = prm.dt / nsub;
    std::vector<char> ok(mt, 1);
    std::vector<int32_t> hr((size_t)rows * mt);
    for (int s = 0; s < nsub; ++s) {
      e = launch_either(m, lpc, q, dwork, dwork + mt, mt, drec);
      if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), drec, sizeof(int32_t) * hr.size(), hipMemcpyDeviceToHost, m->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
      if (e != hipSuccess) { rc = hip_fail(e, "retry: substep"); break; }
      for (int64_t t = 0; t < mt; ++t) {
        if (hr[t] != 0) ok[t] = 0;
        for (int r = 1; r < rows; ++r) acc[(size_t)r * mc + todo[t]] += hr[(size_t)r * mt + t];
      }
    }
    if (rc != CHEM_OK) break;
    e = hipMemcpy(w.data(), dwork, sizeof(double) * w.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) { rc = hip_fail(e, "retry: download"); break; }
    for (int64_t t = 0; t < mt; ++t) {
      if (!ok[t]) continue;
      const int64_t j = todo[t];
      done[j] = 1;
      result[j] = w[t];
      for (int k = 0; k < S; ++k) result[mc + (size_t)k * mc + j] = w[mt + (size_t)k * mt + t];
    }
  }
  (void)hipFree(dwork);
  (void)hipFree(drec);
  if (rc != CHEM_OK) return rc;
  std::vector<double> hT(n), hY((size_t)S * n);
  e = hipMemcpy(hT.data(), T, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hY.data(), Y, sizeof(double) * hY.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "retry: state");
  for (int64_t j = 0; j < mc; ++j) {
    const int64_t i = idx[j];
    if (done[j]) {
      hT[i] = result[j];
      for (int k = 0; k < S; ++k) hY[(size_t)k * n + i] = result[mc + (size_t)k * mc + j];
      hrec[i] = 0;
    }
    for (int r = 1; r < rows; ++r) hrec[(size_t)r * n + i] += acc[(size_t)r * mc + j];
  }
  e = hipMemcpy(T, hT.data(), sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(Y, hY.data(), sizeof(double) * hY.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(rec, hrec.data(), sizeof(int32_t) * hrec.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = chemgpu::launch_reduce_records(rec, n, m->dstats, m->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hs, m->dstats, sizeof(unsigned long long) * chemgpu::kStatCount, hipMemcpyDeviceToHost,
                       m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return hip_fail(e, "retry: write-back");
  return CHEM_OK;
}

}  // namespace

int chem_integrate_ex(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt, double rtol,
                      double atol, chem_stats* stats, int32_t* cell_records) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_cells < 0) return fail(CHEM_ERR_ARG, "n_cells < 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEM_ERR_ARG, "dt must be positive and finite");
  if (!(rtol > 0) || !std::isfinite(rtol)) return fail(CHEM_ERR_ARG, "rtol must be positive");
  if (!(atol >= 0) || !std::isfinite(atol)) return fail(CHEM_ERR_ARG, "atol must be >= 0");
  if (!(p > 0) || !std::isfinite(p)) return fail(CHEM_ERR_ARG, "p must be positive");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n_cells == 0) return CHEM_OK;
  if (!T || !Y) return fail(CHEM_ERR_ARG, "T or Y is NULL");
  if (n_cells > (int64_t)INT32_MAX * 16) return fail(CHEM_ERR_ARG, "n_cells too large");
  int32_t* rec = cell_records;
  if (!rec) {
    const int rc = ensure_records(m, n_cells);
    if (rc != CHEM_OK) return rc;
    rec = m->rec;
  }
  IntParams prm{};
  prm.p = p;
  prm.dt = dt;
  prm.rtol = rtol;
  prm.atol = atol;
  prm.max_steps = m->max_steps;
  prm.q_max = m->q_max;
  prm.fixed_T = m->fixed_T;
  prm.fixed_step_n = m->fixed_step_n;
  prm.lu_fp32 = m->lu_fp32;
  prm.ir_max = m->ir_max;
  prm.jac_mode = m->jac_mode;
  prm.jac_reuse = m->jac_reuse;
  bool lpc = false;
  const int krc = chem_select_kernel(m, &lpc);
  if (krc != CHEM_OK) return krc;
  hipError_t e = hipSuccess;
  const int N = m->dev.S + 1;
  if (m->retry > 0) {   // keep the input state for cells that may need a retry
    if (m->retry_cap < n_cells) {
      if (m->retry_in) (void)hipFree(m->retry_in);
      m->retry_in = nullptr;
      m->retry_cap = 0;
      e = hipMalloc(&m->retry_in, sizeof(double) * N * n_cells);
      if (e != hipSuccess) return fail(CHEM_ERR_OOM, "hipMalloc of the retry copy");
      m->retry_cap = n_cells;
    }
    e = hipMemcpyAsync(m->retry_in, T, sizeof(double) * n_cells, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(m->retry_in + n_cells, Y, sizeof(double) * (N - 1) * n_cells, hipMemcpyDeviceToDevice,
                         m->stream);
    if (e != hipSuccess) return hip_fail(e, "retry copy");
  }
  e = hipEventRecord(m->ev0, m->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  e = launch_either(m, lpc, prm, T, Y, n_cells, rec);
  if (e != hipSuccess) return hip_fail(e, "integrate kernel launch");
  e = hipEventRecord(m->ev1, m->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  e = chemgpu::launch_reduce_records(rec, n_cells, m->dstats, m->stream);
  if (e != hipSuccess) return hip_fail(e, "stats reduction launch");
  unsigned long long hs[chemgpu::kStatCount];
  e = hipMemcpyAsync(hs, m->dstats, sizeof hs, hipMemcpyDeviceToHost, m->stream);
  if (e != hipSuccess) return hip_fail(e, "stats copy");
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return hip_fail(e, "integrate");
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, m->ev0, m->ev1);
  if (hs[8] && m->retry > 0) {
    const int rrc = retry_failed_cells(m, prm, lpc, n_cells, T, Y, rec, hs);
    if (rrc != CHEM_OK) return rrc;
  }
  if (stats) fill_stats(stats, n_cells, hs, ms);
  g_last_error.clear();
  return hs[8] ? CHEM_WARN_CELLS_FAILED : CHEM_OK;
}

int chem_integrate(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt, double rtol,
                   double atol, chem_stats* stats) {
  return chem_integrate_ex(m, n_cells, T, Y, p, dt, rtol, atol, stats, nullptr);
}

}  // extern "C"

// ------------------------------------------ integration without allocation
//
// chem_integrate_noalloc keeps its per-cell records and statistics counters
// in `scratch`, one fixed array per device that lives until the process
// ends.  In host code the array's name is only a stand-in for the device
// symbol: its device address is looked up once per device and used wherever
// the host passes the array to a kernel or copy.
namespace {

constexpr size_t kScratchStatBytes = 256;   // kStatCount counters, padded to the array's alignment
constexpr size_t kScratchBytes =
    kScratchStatBytes + sizeof(int32_t) * chemgpu::kRecRows * (size_t)CHEM_NOALLOC_MAX_CELLS;
static_assert(sizeof(unsigned long long) * chemgpu::kStatCount <= kScratchStatBytes, "stats do not fit");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` per device

// Device address of `scratch` on `device`, looked up on the first call for
// that device with the device current.
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(CHEM_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    unsigned char* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
    if (!ptr) return fail(CHEM_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return CHEM_OK;
}

}  // namespace

extern "C" {

int chem_integrate_noalloc(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt, double rtol,
                           double atol, chem_stats* stats) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_cells < 0) return fail(CHEM_ERR_ARG, "n_cells < 0");
  if (n_cells > CHEM_NOALLOC_MAX_CELLS)
    return fail(CHEM_ERR_ARG, "n_cells " + std::to_string(n_cells) + " exceeds the allocation-free limit of " +
                                  std::to_string((long long)CHEM_NOALLOC_MAX_CELLS) + " cells");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEM_ERR_ARG, "dt must be positive and finite");
  if (!(rtol > 0) || !std::isfinite(rtol)) return fail(CHEM_ERR_ARG, "rtol must be positive");
  if (!(atol >= 0) || !std::isfinite(atol)) return fail(CHEM_ERR_ARG, "atol must be >= 0");
  if (!(p > 0) || !std::isfinite(p)) return fail(CHEM_ERR_ARG, "p must be positive");
  if (m->retry > 0)
    return fail(CHEM_ERR_ARG, "the retry option (CHEM_OPT_RETRY) keeps a copy of the inputs and so allocates; "
                              "set it to 0 for the allocation-free call");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n_cells == 0) return CHEM_OK;
  if (!T || !Y) return fail(CHEM_ERR_ARG, "T or Y is NULL");
  bool lpc = false;
  const int krc = kernel_choice(m, &lpc);
  if (krc != CHEM_OK) return krc;
  if (lpc) {
    std::lock_guard<std::mutex> lk(m->lpc_mu);
    if (!lpc_ready(m))
      return fail(CHEM_ERR_ARG, "the mechanism's generated kernels are not loaded on this device for these options; "
                                "call chem_integrate once with the handle first (loading a code object allocates)");
  }
  unsigned char* base = nullptr;
  const int src = scratch_address(m->device, &base);
  if (src != CHEM_OK) return src;
  unsigned long long* dstats = reinterpret_cast<unsigned long long*>(base);
  int32_t* rec = reinterpret_cast<int32_t*>(base + kScratchStatBytes);
  const IntParams prm = make_int_params(m, p, dt, rtol, atol);
  hipError_t e = hipEventRecord(m->ev0, m->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  e = launch_either(m, lpc, prm, T, Y, n_cells, rec);
  if (e != hipSuccess) return hip_fail(e, "integrate kernel launch");
  e = hipEventRecord(m->ev1, m->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  // the reduction clears the counters with a kernel of its own before summing
  e = chemgpu::launch_reduce_records(rec, n_cells, dstats, m->stream);
  if (e != hipSuccess) return hip_fail(e, "stats reduction launch");
  unsigned long long hs[chemgpu::kStatCount];
  e = hipMemcpyAsync(hs, dstats, sizeof hs, hipMemcpyDeviceToHost, m->stream);
  if (e != hipSuccess) return hip_fail(e, "stats copy");
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return hip_fail(e, "integrate");
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, m->ev0, m->ev1);
  if (stats) fill_stats(stats, n_cells, hs, ms);
  g_last_error.clear();
  return hs[8] ? CHEM_WARN_CELLS_FAILED : CHEM_OK;
}

namespace {

int ensure_boxes(chem_mech* m, int n_boxes) {
  if (!m->djob) {
    if (hipMalloc(&m->djob, sizeof(chemgpu::BoxJob)) != hipSuccess || hipMalloc(&m->dhead, sizeof(unsigned)) != hipSuccess)
      return fail(CHEM_ERR_OOM, "hipMalloc of queue state");
  }
  if (!m->capture_stream && hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(CHEM_ERR_DEVICE, "hipStreamCreate");
  if (n_boxes <= m->box_cap) return CHEM_OK;
  // a captured graph holds the old buffers' addresses
  if (m->graph) (void)hipGraphExecDestroy(m->graph);
  m->graph = nullptr;
  if (m->dboxes) (void)hipFree(m->dboxes);
  if (m->dremaining) (void)hipFree(m->dremaining);
  if (m->host_done) (void)hipHostFree(m->host_done);
  m->dboxes = nullptr;
  m->dremaining = nullptr;
  m->host_done = nullptr;
  m->box_cap = 0;
  const int cap = std::max(n_boxes, 256);
  if (hipMalloc(&m->dboxes, sizeof(chemgpu::BoxDev) * cap) != hipSuccess ||
      hipMalloc(&m->dremaining, sizeof(int) * cap) != hipSuccess)
    return fail(CHEM_ERR_OOM, "hipMalloc of box descriptors");
  if (hipHostMalloc(reinterpret_cast<void**>(&m->host_done), sizeof(int) * cap, hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&m->host_done_dev), m->host_done, 0) != hipSuccess)
    return fail(CHEM_ERR_OOM, "hipHostMalloc of completion flags");
  m->box_cap = cap;
  return CHEM_OK;
}

// Enqueue queue reset + persistent kernel (+ stats reduction) on `s`.
hipError_t enqueue_boxes(chem_mech* m, bool lpc, const IntParams& prm, int grid, hipStream_t s) {
  hipError_t e = chem_launch_box_queue(m, lpc, prm, m->dboxes, m->djob, m->dhead, m->dremaining, m->rec,
                                       m->host_done_dev, grid, s);
  if (e != hipSuccess) return e;
  return chemgpu::launch_reduce_records_job(m->rec, m->djob, m->dstats, s);
}

}  // namespace

int chem_integrate_boxes(chem_mech* m, int n_boxes, const chem_box* boxes, double p, double rtol, double atol,
                         chem_stats* stats, double* box_ms) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_boxes < 0 || (n_boxes > 0 && !boxes)) return fail(CHEM_ERR_ARG, "bad box array");
  if (!(rtol > 0) || !std::isfinite(rtol)) return fail(CHEM_ERR_ARG, "rtol must be positive");
  if (!(atol >= 0) || !std::isfinite(atol)) return fail(CHEM_ERR_ARG, "atol must be >= 0");
  if (!(p > 0) || !std::isfinite(p)) return fail(CHEM_ERR_ARG, "p must be positive");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n_boxes == 0) return CHEM_OK;
  for (int b = 0; b < n_boxes; ++b) {
    if (boxes[b].n_cells < 0 || (boxes[b].n_cells > 0 && (!boxes[b].T || !boxes[b].Y)))
      return fail(CHEM_ERR_ARG, "box " + std::to_string(b) + ": bad arrays");
    if (!(boxes[b].dt > 0) || !std::isfinite(boxes[b].dt))
      return fail(CHEM_ERR_ARG, "box " + std::to_string(b) + ": dt must be positive");
  }
  try {
    // queue order: largest boxes first (their tiles start earliest)
    std::vector<int> order(n_boxes);
    for (int b = 0; b < n_boxes; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return boxes[a].n_cells > boxes[b].n_cells; });
    bool lpc = false;
    const int krc = chem_select_kernel(m, &lpc);
    if (krc != CHEM_OK) return krc;
    const int cpw = chem_cells_per_tile(m, lpc);
    std::vector<chemgpu::BoxDev> q(n_boxes);
    int64_t tiles = 0, cells = 0;
    for (int i = 0; i < n_boxes; ++i) {
      const chem_box& bx = boxes[order[i]];
      q[i].T = bx.T;
      q[i].Y = bx.Y;
      q[i].n = bx.n_cells;
      q[i].dt = bx.dt;
      q[i].cell_off = cells;
      q[i].tile_pre = tiles;
      q[i].box_id = order[i];
      q[i].pad = 0;
      tiles += (bx.n_cells + cpw - 1) / cpw;
      cells += bx.n_cells;
    }
    if (tiles > (int64_t)0x7fffffff) return fail(CHEM_ERR_ARG, "too many cells in one call");
    if (cells == 0) return CHEM_OK;
    int rc = ensure_boxes(m, n_boxes);
    if (rc != CHEM_OK) return rc;
    const void* old_rec = m->rec;
    rc = ensure_records(m, cells);
    if (rc != CHEM_OK) return rc;
    chemgpu::BoxJob job{n_boxes, (unsigned)tiles, cells};
    hipError_t e = hipMemcpyAsync(m->dboxes, q.data(), sizeof(chemgpu::BoxDev) * n_boxes, hipMemcpyHostToDevice,
                                  m->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m->djob, &job, sizeof job, hipMemcpyHostToDevice, m->stream);
    if (e != hipSuccess) return hip_fail(e, "box descriptor upload");
    e = hipStreamSynchronize(m->stream);   // host copies above read stack memory
    if (e != hipSuccess) return hip_fail(e, "box descriptor upload");
    std::memset(m->host_done, 0, sizeof(int) * n_boxes);
    IntParams prm;
    std::memset(&prm, 0, sizeof prm);   // padding included: the struct is compared bytewise
    prm.p = p;
    prm.dt = 0.0;
    prm.rtol = rtol;
    prm.atol = atol;
    prm.max_steps = m->max_steps;
    prm.q_max = m->q_max;
    prm.fixed_T = m->fixed_T;
    prm.fixed_step_n = m->fixed_step_n;
    prm.lu_fp32 = m->lu_fp32;
    prm.ir_max = m->ir_max;
    prm.jac_mode = m->jac_mode;
    prm.jac_reuse = m->jac_reuse;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)m->waves_per_cu * m->n_cu);
    const auto t0 = std::chrono::steady_clock::now();
    e = hipEventRecord(m->ev0, m->stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (m->use_graph) {
      const void* key[6] = {m->rec, m->dboxes, m->host_done_dev, m->blob, m->dremaining, m->dhead};
      const bool stale = !m->graph || std::memcmp(key, m->graph_key, sizeof key) != 0 || m->graph_grid != grid ||
                         m->graph_np != (lpc ? 1 : m->dev.np_width) || m->graph_f32 != m->lu_fp32 ||
                         old_rec != m->rec ||
                         std::memcmp(&prm, &m->graph_prm, sizeof prm) != 0;
      if (stale) {
        if (m->graph) (void)hipGraphExecDestroy(m->graph);
        m->graph = nullptr;
        hipGraph_t gr = nullptr;
        e = hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          const hipError_t le = enqueue_boxes(m, lpc, prm, grid, m->capture_stream);
          e = hipStreamEndCapture(m->capture_stream, &gr);
          if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&m->graph, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(e, "hipGraph capture of the box launch");
        std::memcpy(m->graph_key, key, sizeof key);
        m->graph_grid = grid;
        m->graph_np = lpc ? 1 : m->dev.np_width;
        m->graph_f32 = m->lu_fp32;
        m->graph_prm = prm;
      }
      // the captured kernels take their per-call parameters from device memory,
      // except the integration options baked into the capture
      e = hipGraphLaunch(m->graph, m->stream);
    } else {
      e = enqueue_boxes(m, lpc, prm, grid, m->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "box launch");
    e = hipEventRecord(m->ev1, m->stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (box_ms) {
      std::vector<char> seen(n_boxes, 0);
      int left = n_boxes;
      int64_t cells_done = 0;
      double next_report = m->progress_s * 1e3;
      volatile int* flags = m->host_done;
      while (left > 0) {
        for (int b = 0; b < n_boxes; ++b) {
          if (!seen[b] && flags[b]) {
            seen[b] = 1;
            --left;
            cells_done += boxes[b].n_cells;
            box_ms[b] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          }
        }
        const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (m->progress_s > 0 && el >= next_report) {
          std::fprintf(stderr, "chem_integrate_boxes: %d of %d boxes, %lld of %lld cells done after %.1f s\n",
                       n_boxes - left, n_boxes, (long long)cells_done, (long long)cells, el * 1e-3);
          std::fflush(stderr);
          next_report += m->progress_s * 1e3;
        }
        if (left > 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        if (left > 0 && hipStreamQuery(m->stream) != hipErrorNotReady) {
          // the stream is done (or failed): every remaining box is complete
          const double now = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          for (int b = 0; b < n_boxes; ++b)
            if (!seen[b]) box_ms[b] = flags[b] ? now : -1.0;
          left = 0;
        }
      }
    }
    unsigned long long hs[chemgpu::kStatCount];
    e = hipMemcpyAsync(hs, m->dstats, sizeof hs, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "box integration");
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, m->ev0, m->ev1);
    if (stats) fill_stats(stats, cells, hs, ms);
    g_last_error.clear();
    return hs[8] ? CHEM_WARN_CELLS_FAILED : CHEM_OK;
  } catch (...) {
    return fail(CHEM_ERR_OOM, "exception in chem_integrate_boxes");
  }
}

namespace {
struct TuneKey {
  int device, S, R;
  bool operator<(const TuneKey& o) const {
    return device != o.device ? device < o.device : (S != o.S ? S < o.S : R < o.R);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;

int apply_tuning(chem_mech* m, int width, int waves) {
  int rc = chem_set_option(m, CHEM_OPT_GROUP_WIDTH, width);
  if (rc == CHEM_OK) rc = chem_set_option(m, CHEM_OPT_WAVES_PER_CU, waves);
  return rc;
}
}  // namespace

int chem_autotune(chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p, double dt, double rtol,
                  double atol, int* best_width, int* best_waves) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_cells <= 0 || !T || !Y) return fail(CHEM_ERR_ARG, "autotune needs a non-empty sample");
  const TuneKey key{m->device, m->dev.S, m->dev.R};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      if (best_width) *best_width = it->second.first;
      if (best_waves) *best_waves = it->second.second;
      return apply_tuning(m, it->second.first, it->second.second);
    }
  }
  const int S = m->dev.S;
  double* scratch = nullptr;
  const size_t bytes = sizeof(double) * (size_t)(S + 1) * n_cells;
  if (hipMalloc(&scratch, bytes) != hipSuccess) return fail(CHEM_ERR_OOM, "hipMalloc of autotune scratch");
  const int64_t box = 4096;
  std::vector<chem_box> boxes;
  for (int64_t c0 = 0; c0 < n_cells; c0 += box) {
    const int64_t nb = std::min(box, n_cells - c0);
    boxes.push_back(chem_box{nullptr, nullptr, nb, dt});
  }
  // scratch layout: per box T[nb] then Y[S*nb]
  {
    int64_t off = 0;
    for (auto& b : boxes) {
      b.T = scratch + off;
      b.Y = scratch + off + b.n_cells;
      off += (S + 1) * b.n_cells;
    }
  }
  const int old_width = m->dev.np_width, old_waves = m->waves_per_cu;
  int best_w = old_width, best_v = old_waves;
  double best_ms = 1e300;
  int rc = CHEM_OK;
  const int widths[3] = {16, 32, 64};
  const int waves[4] = {4, 8, 12, 16};
  for (int w : widths) {
    if (w < m->dev.N) continue;
    for (int v : waves) {
      rc = apply_tuning(m, w, v);
      if (rc != CHEM_OK) break;
      // refresh the scratch copy of the sample (SoA per box)
      int64_t c0 = 0;
      hipError_t e = hipSuccess;
      for (auto& b : boxes) {
        e = hipMemcpyAsync(b.T, T + c0, sizeof(double) * b.n_cells, hipMemcpyDeviceToDevice, m->stream);
        for (int k = 0; k < S && e == hipSuccess; ++k)
          e = hipMemcpyAsync(b.Y + (int64_t)k * b.n_cells, Y + (int64_t)k * n_cells + c0,
                             sizeof(double) * b.n_cells, hipMemcpyDeviceToDevice, m->stream);
        c0 += b.n_cells;
      }
      if (e != hipSuccess) {
        rc = hip_fail(e, "autotune copy");
        break;
      }
      chem_stats st;
      rc = chem_integrate_boxes(m, (int)boxes.size(), boxes.data(), p, rtol, atol, &st, nullptr);
      if (rc < 0) break;
      rc = CHEM_OK;
      if (st.wall_ms < best_ms) {
        best_ms = st.wall_ms;
        best_w = w;
        best_v = v;
      }
    }
    if (rc != CHEM_OK) break;
  }
  (void)hipFree(scratch);
  if (rc != CHEM_OK) {
    (void)apply_tuning(m, old_width, old_waves);
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best_w, best_v};
  }
  if (best_width) *best_width = best_w;
  if (best_waves) *best_waves = best_v;
  return apply_tuning(m, best_w, best_v);
}

int chem_rates(chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p, double* wdot, double* f,
               double* jac) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_cells < 0) return fail(CHEM_ERR_ARG, "n_cells < 0");
  if (!(p > 0) || !std::isfinite(p)) return fail(CHEM_ERR_ARG, "p must be positive");
  if (n_cells == 0) return CHEM_OK;
  if (!T || !Y || !wdot) return fail(CHEM_ERR_ARG, "T, Y or wdot is NULL");
  // the same kernel family chem_integrate would use for these options
  bool lpc = false;
  const int krc = chem_select_kernel(m, &lpc);
  if (krc != CHEM_OK) return krc;
  hipError_t e = lpc ? chemgpu::launch_lpc_rates(m->lpc_rates, p, m->fixed_T, T, Y, n_cells, wdot, f, jac, m->stream)
                     : chemgpu::launch_rates(m->dev, p, m->fixed_T, T, Y, n_cells, wdot, f, jac, m->stream);
  if (e != hipSuccess) return hip_fail(e, "rates kernel launch");
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return hip_fail(e, "rates");
  g_last_error.clear();
  return CHEM_OK;
}

const char* chem_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
