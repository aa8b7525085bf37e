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

}  // extern "C"
