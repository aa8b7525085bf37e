// chem_host.cpp -- C ABI of libchem: mechanism parsing and upload, options,
// integration and rates launches, per-call statistics.  See include/chem.h.
#include "../../include/chem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "chem_internal.h"

using chemgpu::DevMech;
using chemgpu::IntParams;
using chemgpu::RxParams;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(CHEM_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

struct HostReaction {
  int rev = 1, type = 0;
  std::vector<int> reac, prod;
  double A = 0, b = 0, Ea = 0;      // Ea in kcal/mol
  double A0 = 0, b0 = 0, Ea0 = 0;
};

struct HostMech {
  std::vector<double> emass;
  std::vector<std::vector<int>> atoms;  // [S][E]
  std::vector<double> W, a0, a1, hf, s0;
  std::vector<HostReaction> rx;
};

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

 private:
  std::vector<std::string> toks_;
  size_t pos_ = 0;
};

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
  for (int k = 0; k < S; ++k) {
    int inert = 0, total = 0;
    if (!tk.skip() || !tk.integer(inert)) return fail(CHEM_ERR_PARSE, "bad species line");
    double w = 0.0;
    for (int e = 0; e < E; ++e) {
      if (!tk.integer(m.atoms[k][e]) || m.atoms[k][e] < 0) return fail(CHEM_ERR_PARSE, "bad atom count");
      w += m.atoms[k][e] * m.emass[e];
      total += m.atoms[k][e];
    }
    if (total == 0) return fail(CHEM_ERR_PARSE, "species without atoms");
    m.W[k] = w;
    if (!tk.real(m.a0[k]) || !tk.real(m.a1[k]) || !tk.real(m.hf[k]) || !tk.real(m.s0[k]))
      return fail(CHEM_ERR_PARSE, "bad species thermo");
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
    for (int e = 0; e < E; ++e) {
      int bal = 0;
      for (int s : x.prod) bal += m.atoms[s][e];
      for (int s : x.reac) bal -= m.atoms[s][e];
      if (bal != 0) return fail(CHEM_ERR_PARSE, "reaction " + std::to_string(j) + " is not atom balanced");
    }
  }
  if (!tk.word("END")) return fail(CHEM_ERR_PARSE, "missing END");
  return CHEM_OK;
}

}  // namespace

struct chem_mech {
  HostMech host;
  DevMech dev{};
  void* blob = nullptr;          // device tables
  hipStream_t stream = nullptr;
  int device = 0;
  // options
  int max_steps = 100000, q_max = 5, fixed_T = 0, fixed_step_n = 0, lu_fp32 = 0, ir_max = 3;
  // workspace
  int32_t* rec = nullptr;
  int64_t rec_cap = 0;
  unsigned long long* dstats = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

int upload(chem_mech* h) {
  const HostMech& m = h->host;
  const int S = (int)m.W.size(), R = (int)m.rx.size(), N = S + 1;
  if (N > 64) return fail(CHEM_ERR_UNSUPPORTED, "mechanisms with more than 63 species are not supported");
  const int np = N <= 16 ? 16 : (N <= 32 ? 32 : 64);
  const int nch = std::max(1, (R + np - 1) / np);

  std::vector<RxParams> rx(std::max(R, 1));
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
    d.type = x.type;
    d.rev = x.rev;
    d.nr = (int)x.reac.size();
    d.np = (int)x.prod.size();
    for (int s = 0; s < chemgpu::kSlots; ++s) d.sp[s] = -1;
    for (int i = 0; i < d.nr; ++i) d.sp[i] = x.reac[i];
    for (int i = 0; i < d.np; ++i) d.sp[chemgpu::kMaxSide + i] = x.prod[i];
  }
  // per-species lists of (reaction, net coefficient), reaction order, split in chunks
  std::vector<int> off((size_t)S * (nch + 1), 0), ent;
  for (int k = 0; k < S; ++k) {
    int ch_next = 0;
    for (int j = 0; j < R; ++j) {
      int nu = 0;
      for (int s : m.rx[j].prod) nu += (s == k);
      for (int s : m.rx[j].reac) nu -= (s == k);
      if (nu == 0) continue;
      while (ch_next <= j / np) off[(size_t)k * (nch + 1) + ch_next++] = (int)ent.size();
      ent.push_back((j << 3) | (nu + 4));
    }
    while (ch_next <= nch) off[(size_t)k * (nch + 1) + ch_next++] = (int)ent.size();
  }
  if (ent.empty()) ent.push_back(0);

  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_sp = 0;
  const size_t sz_sp = align(5 * sizeof(double) * S);
  const size_t o_rx = o_sp + sz_sp;
  const size_t sz_rx = align(sizeof(RxParams) * rx.size());
  const size_t o_off = o_rx + sz_rx;
  const size_t sz_off = align(sizeof(int) * off.size());
  const size_t o_ent = o_off + sz_off;
  const size_t sz_ent = align(sizeof(int) * ent.size());
  const size_t total = o_ent + sz_ent;
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
  dm.nch = nch;
  dm.np_width = np;
  const double* dsp = reinterpret_cast<const double*>(base + o_sp);
  dm.W = dsp;
  dm.a0 = dsp + S;
  dm.a1 = dsp + 2 * S;
  dm.hf = dsp + 3 * S;
  dm.s0 = dsp + 4 * S;
  dm.rx = reinterpret_cast<const RxParams*>(base + o_rx);
  dm.csr_off = reinterpret_cast<const int*>(base + o_off);
  dm.csr_ent = reinterpret_cast<const int*>(base + o_ent);
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
  if (m->dstats) (void)hipFree(m->dstats);
  if (m->ev0) (void)hipEventDestroy(m->ev0);
  if (m->ev1) (void)hipEventDestroy(m->ev1);
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
    default:
      return fail(CHEM_ERR_ARG, "unknown option key " + std::to_string(key));
  }
}

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
  hipError_t e = hipEventRecord(m->ev0, m->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  e = chemgpu::launch_integrate(m->dev, prm, T, Y, n_cells, rec, m->stream);
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
  if (stats) {
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
    stats->n_ir_sweeps = 0;
    stats->wall_ms = ms;
  }
  g_last_error.clear();
  return hs[8] ? CHEM_WARN_CELLS_FAILED : CHEM_OK;
}

int chem_integrate(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt, double rtol,
                   double atol, chem_stats* stats) {
  return chem_integrate_ex(m, n_cells, T, Y, p, dt, rtol, atol, stats, nullptr);
}

int chem_rates(chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p, double* wdot, double* f,
               double* jac) {
  if (!m) return fail(CHEM_ERR_ARG, "mechanism is NULL");
  if (n_cells < 0) return fail(CHEM_ERR_ARG, "n_cells < 0");
  if (!(p > 0) || !std::isfinite(p)) return fail(CHEM_ERR_ARG, "p must be positive");
  if (n_cells == 0) return CHEM_OK;
  if (!T || !Y || !wdot) return fail(CHEM_ERR_ARG, "T, Y or wdot is NULL");
  hipError_t e = chemgpu::launch_rates(m->dev, p, m->fixed_T, T, Y, n_cells, wdot, f, jac, m->stream);
  if (e != hipSuccess) return hip_fail(e, "rates kernel launch");
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return hip_fail(e, "rates");
  g_last_error.clear();
  return CHEM_OK;
}

const char* chem_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
