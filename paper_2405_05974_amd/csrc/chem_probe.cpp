// chem_probe.cpp -- measurement probes for the roofline report (a separate
// library, libchem_probe.so; not part of the chemistry ABI).
//
//   fma     independent FP64 fused multiply-add chains: the chip's measured
//           FP64 vector rate, quoted beside the published 78.6 TFLOP/s;
//   chexp   the branch-free exp of the generated kernels (chem_exp.inc) in a
//           loop, and
//   libexp  the device library's exp in the same loop, and
//   loop    the loop alone: FP64 instruction counters of chexp/libexp minus
//           loop give the operations one exp costs on this chip (the c_exp of
//           the flop model).
// Kernels are compiled with hipRTC for the current device from the same
// chem_exp.inc text the mechanism kernels use, launched on the null stream,
// and timed with HIP events.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

const char* kChExp =
#include "chem_exp.inc"
    ;

const char* kProbes = R"PROBE(
extern "C" __global__ __launch_bounds__(256) void probe_fma(double* __restrict__ out, const double b, const double c,
                                                           const int iters) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = 1.0 + 1e-9 * (double)(gid + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = __builtin_fma(a[i], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += a[i];
  out[gid] = s;
}

template <int MODE>
__device__ __forceinline__ double probe_f(const double x) {
  if (MODE == 1) return ch_exp(x);
  if (MODE == 2) return exp(x);
  return x;
}

template <int MODE>
__device__ __forceinline__ void probe_loop_body(double* __restrict__ out, const double x0, const double dx,
                                                const int iters) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double x = x0 + dx * (double)(gid & 1023);
  double acc = 0.0;
  for (int it = 0; it < iters; ++it) {
    acc += probe_f<MODE>(x);
    x += dx;
  }
  out[gid] = acc;
}

// Production rates wdot = Q nu^T for many cells, two ways, with the rates of
// progress generated in registers (Q(cell, j) = 1 + 1e-6 cell + 1e-3 j) so
// that only the contraction differs; each thread repeats the contraction
// `iters` times (rates shifted by 1e-9 it) and writes the sum, so that the
// result write does not dominate the timing:
//   probe_wdot_mfma    the dense [cells x RP] x [RP x SP] product on FP64
//                      matrix cores, v_mfma_f64_16x16x4 (16 cells, 4
//                      reactions, 16 species per instruction), nu^T dense in
//                      global memory (L2), out[cell][SP];
//   probe_wdot_sparse  one cell per lane, per-species lists of (reaction,
//                      coefficient) as in the kernels, out[k][cells].
typedef double ch_v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double probe_q(const int cell, const int j, const int it) {
  return 1.0 + 1e-6 * (double)cell + 1e-3 * (double)j + 1e-9 * (double)it;
}

extern "C" __global__ __launch_bounds__(256) void probe_wdot_mfma(const double* __restrict__ nuT, double* __restrict__ out,
                                                                 const int RP, const int SP, const int ncells, const int iters) {
  const int lane = threadIdx.x & 63;
  const int tile = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (tile * 16 >= ncells) return;
  const int row = lane & 15, kq = lane >> 4;
  const int cell = tile * 16 + row;
  for (int nb = 0; nb < SP; nb += 16) {
    ch_v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
      for (int k = 0; k < RP; k += 4) {
        const double a = probe_q(cell, k + kq, it);              // A[cell row][reaction k + kq]
        const double b = nuT[(size_t)(k + kq) * SP + nb + row];  // B[reaction k + kq][species nb + row]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    // D[lane / 16 + 4 i][lane % 16] in register i (measured lane layout)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tile * 16 + kq + 4 * i;
      if (c < ncells) out[(size_t)c * SP + nb + row] = acc[i];
    }
  }
}

extern "C" __global__ __launch_bounds__(256) void probe_wdot_sparse(const int* __restrict__ off, const int* __restrict__ ent,
                                                                   double* __restrict__ out, const int S, const int ncells,
                                                                   const int iters) {
  const int cell = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (cell >= ncells) return;
  for (int k = 0; k < S; ++k) {
    double s = 0.0;
    for (int it = 0; it < iters; ++it)
      for (int e = off[k]; e < off[k + 1]; ++e) {
        const int x = ent[e];
        s += (double)((x & 7) - 4) * probe_q(cell, x >> 3, it);
      }
    out[(size_t)k * ncells + cell] = s;
  }
}

extern "C" __global__ __launch_bounds__(256) void probe_loop(double* out, double x0, double dx, int iters) {
  probe_loop_body<0>(out, x0, dx, iters);
}
extern "C" __global__ __launch_bounds__(256) void probe_chexp(double* out, double x0, double dx, int iters) {
  probe_loop_body<1>(out, x0, dx, iters);
}
extern "C" __global__ __launch_bounds__(256) void probe_libexp(double* out, double x0, double dx, int iters) {
  probe_loop_body<2>(out, x0, dx, iters);
}
)PROBE";

hipModule_t g_mod = nullptr;

int compile_module() {
  if (g_mod) return 0;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1;
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  const std::string src = std::string(kChExp) + kProbes;
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "chem_probe.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) return -1;
  const std::string off = "--offload-arch=" + arch;
  const char* opts[] = {off.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  if (hiprtcCompileProgram(prog, 7, opts) != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    std::fprintf(stderr, "chem_probe: compile failed: %s\n", log.c_str());
    hiprtcDestroyProgram(&prog);
    return -1;
  }
  size_t code_size = 0;
  hiprtcGetCodeSize(prog, &code_size);
  std::vector<char> code(code_size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return hipModuleLoadData(&g_mod, code.data()) == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" {

// Run probe `which` ("fma", "chexp", "libexp" or "loop") over `blocks` blocks
// of 256 threads for `iters` loop trips; *ms receives the kernel time.
// Returns 0, or -1 on any HIP or compile error (message on stderr).
int chem_probe_run(const char* which, int blocks, int iters, double* ms) {
  if (!which || blocks <= 0 || iters <= 0 || !ms) return -1;
  if (compile_module() != 0) return -1;
  const std::string w = which;
  const char* name = w == "fma" ? "probe_fma" : w == "chexp" ? "probe_chexp" : w == "libexp" ? "probe_libexp"
                                                                               : w == "loop" ? "probe_loop" : nullptr;
  if (!name) return -1;
  hipFunction_t fn = nullptr;
  if (hipModuleGetFunction(&fn, g_mod, name) != hipSuccess) return -1;
  double* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * (size_t)blocks * 256) != hipSuccess) return -1;
  double a = 0.999999, b = 1e-7;        // fma: a <- a * 0.999999 + 1e-7 stays finite
  double x0 = -60.0, dx = 1.0e-4;       // exp arguments in the rate-constant range
  int it = iters;
  void* args_fma[] = {&out, &a, &b, &it};
  void* args_exp[] = {&out, &x0, &dx, &it};
  void** args = w == "fma" ? args_fma : args_exp;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventRecord(e0, nullptr) != hipSuccess) rc = -1;
  if (rc == 0 && hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, 256, 1, 1, 0, nullptr, args, nullptr) != hipSuccess)
    rc = -1;
  if (rc == 0 && hipEventRecord(e1, nullptr) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -1;
  float t = 0.0f;
  if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -1;
  *ms = t;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return rc;
}

// wdot = Q nu^T for ncells cells, `iters` times per cell (summed), with the
// dense (nu[R][S], host, integer coefficients) stoichiometry padded to
// RP x SP ("mfma") or as per-species lists ("sparse"); `reps` launches are
// timed and *ms receives the mean time of one.  out (host, optional)
// receives the last result as [cell][S].
// Returns 0, or -1 on any error.
int chem_probe_wdot(const char* which, const int* nu, int R, int S, int ncells, int iters, int reps, double* out,
                    double* ms) {
  if (!which || !nu || R <= 0 || S <= 0 || ncells <= 0 || iters <= 0 || reps <= 0 || !ms) return -1;
  if (compile_module() != 0) return -1;
  const std::string w = which;
  if (w != "mfma" && w != "sparse") return -1;
  const int RP = (R + 3) / 4 * 4, SP = (S + 15) / 16 * 16;
  hipFunction_t fn = nullptr;
  if (hipModuleGetFunction(&fn, g_mod, w == "mfma" ? "probe_wdot_mfma" : "probe_wdot_sparse") != hipSuccess) return -1;
  std::vector<double> nuT((size_t)RP * SP, 0.0);
  std::vector<int> off(S + 1, 0), ent;
  for (int k = 0; k < S; ++k) {
    off[k] = (int)ent.size();
    for (int j = 0; j < R; ++j) {
      const int v = nu[(size_t)j * S + k];
      if (v < -4 || v > 3) return -1;
      nuT[(size_t)j * SP + k] = v;
      if (v) ent.push_back((j << 3) | (v + 4));
    }
  }
  off[S] = (int)ent.size();
  if (ent.empty()) ent.push_back(0);
  const size_t out_n = w == "mfma" ? (size_t)((ncells + 15) / 16 * 16) * SP : (size_t)S * ncells;
  double *d_nuT = nullptr, *d_out = nullptr;
  int *d_off = nullptr, *d_ent = nullptr;
  int rc = 0;
  if (hipMalloc(&d_nuT, sizeof(double) * nuT.size()) != hipSuccess || hipMalloc(&d_out, sizeof(double) * out_n) != hipSuccess ||
      hipMalloc(&d_off, sizeof(int) * off.size()) != hipSuccess || hipMalloc(&d_ent, sizeof(int) * ent.size()) != hipSuccess)
    rc = -1;
  if (rc == 0 && (hipMemcpy(d_nuT, nuT.data(), sizeof(double) * nuT.size(), hipMemcpyHostToDevice) != hipSuccess ||
                  hipMemcpy(d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice) != hipSuccess ||
                  hipMemcpy(d_ent, ent.data(), sizeof(int) * ent.size(), hipMemcpyHostToDevice) != hipSuccess))
    rc = -1;
  int rp = RP, sp = SP, s = S, nc = ncells, itn = iters;
  void* args_m[] = {&d_nuT, &d_out, &rp, &sp, &nc, &itn};
  void* args_s[] = {&d_off, &d_ent, &d_out, &s, &nc, &itn};
  void** args = w == "mfma" ? args_m : args_s;
  // mfma: one wave (64 threads) per 16 cells; sparse: one thread per cell
  const long long threads = w == "mfma" ? (long long)(ncells + 15) / 16 * 64 : (long long)ncells;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == 0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = -1;
  if (rc == 0 && hipModuleLaunchKernel(fn, blocks, 1, 1, 256, 1, 1, 0, nullptr, args, nullptr) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventRecord(e0, nullptr) != hipSuccess) rc = -1;
  for (int r = 0; r < reps && rc == 0; ++r)
    if (hipModuleLaunchKernel(fn, blocks, 1, 1, 256, 1, 1, 0, nullptr, args, nullptr) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventRecord(e1, nullptr) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -1;
  float t = 0.0f;
  if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -1;
  *ms = t / reps;
  if (rc == 0 && out) {
    std::vector<double> h(out_n);
    if (hipMemcpy(h.data(), d_out, sizeof(double) * out_n, hipMemcpyDeviceToHost) != hipSuccess) rc = -1;
    for (int c = 0; c < ncells && rc == 0; ++c)
      for (int k = 0; k < S; ++k)
        out[(size_t)c * S + k] = w == "mfma" ? h[(size_t)c * SP + k] : h[(size_t)k * ncells + c];
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_nuT);
  (void)hipFree(d_out);
  (void)hipFree(d_off);
  (void)hipFree(d_ent);
  return rc;
}

}  // extern "C"
