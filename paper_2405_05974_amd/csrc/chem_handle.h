// chem_handle.h -- the library's mechanism handle (shared by the C-ABI
// sources of libchem; not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "chem_internal.h"

namespace chemgpu {

struct HostReaction {
  int rev = 1, type = 0;
  std::vector<int> reac, prod;
  double A = 0, b = 0, Ea = 0;      // Ea in kcal/mol
  double A0 = 0, b0 = 0, Ea0 = 0;
  int ntroe = 0;                    // 0, or 3/4 Troe parameters alpha, T3, T1 [, T2]
  double troe[4] = {0, 0, 0, 0};
  std::vector<int> eff_k;           // collision efficiencies other than 1 in [M]
  std::vector<double> eff_v;
  int drop_f = 0, drop_r = 0;       // direction removed by the one-sided linearisation of QSS couplings
};

struct HostMech {
  std::vector<double> emass;
  std::vector<std::vector<int>> atoms;  // [S][E]
  std::vector<double> W, a0, a1, hf, s0;
  // NASA 7-coefficient thermo per species: T_mid, c1..c7 (T <= T_mid), c1..c7
  // above; empty when the species uses the linear cp form
  std::vector<std::vector<double>> nasa;
  std::vector<HostReaction> rx;
  // quasi-steady-state species (algebraic, not in the state), in the order
  // of the mechanism's QSS record
  std::vector<int> qss;
  int n_state_species() const { return (int)W.size() - (int)qss.size(); }
  bool any_nasa() const {
    for (const auto& v : nasa)
      if (!v.empty()) return true;
    return false;
  }
  // The species' NASA coefficients; a linear-cp species written in that form
  // (both ranges equal: c1 = a0, c2 = a1, c6 and c7 from h_f and s0 at 298.15 K).
  std::vector<double> nasa_of(int k) const;
};

}  // namespace chemgpu

struct chem_mech {
  chemgpu::HostMech host;
  chemgpu::DevMech dev{};
  void* blob = nullptr;          // device tables
  const int* csr_off_np[3] = {nullptr, nullptr, nullptr};   // chunk offsets for 16/32/64 lanes per cell
  int nch_np[3] = {0, 0, 0};
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  // options
  int max_steps = 100000, q_max = 5, fixed_T = 0, fixed_step_n = 0, lu_fp32 = 0, ir_max = 3, jac_mode = 0, jac_reuse = 0;
  int retry = 0;                 // halvings of dt tried for failed cells (0: none)
  double* retry_in = nullptr;    // the call's input state [T | Y], kept for retries
  int64_t retry_cap = 0;
  int use_graph = 1, waves_per_cu = 8;
  double progress_s = 0.0;       // seconds between progress lines of chem_integrate_boxes (0: none)
  int kernel_mode = 0;           // 0 auto, 1 group kernels, 2 lane-per-cell kernels
  // lane-per-cell module (generated source, compiled on first use per device)
  std::mutex lpc_mu;
  std::string lpc_src;
  void* lpc_integrate = nullptr;
  void* lpc_boxes = nullptr;
  void* lpc_rates = nullptr;
  void* lpc_serve = nullptr;
  int lpc_device = -1;
  int lpc_reuse = -1;   // CH_REUSE of the loaded module
  // workspace
  int32_t* rec = nullptr;
  int64_t rec_cap = 0;
  unsigned long long* dstats = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // batched boxes
  chemgpu::BoxDev* dboxes = nullptr;
  int* dremaining = nullptr;
  int box_cap = 0;
  chemgpu::BoxJob* djob = nullptr;
  unsigned* dhead = nullptr;
  int* host_done = nullptr;      // pinned, mapped
  int* host_done_dev = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  const void* graph_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int graph_grid = 0, graph_np = 0, graph_f32 = -1;
  chemgpu::IntParams graph_prm{};   // integration parameters baked into the captured launch
};

namespace chemgpu {
std::string lpc_source(const HostMech& m, bool reuse);
int lpc_module(const std::string& src, int device, void** integrate_fn, void** boxes_fn, void** rates_fn,
               void** serve_fn, std::string& log);
}  // namespace chemgpu

// Kernel family for the next integration with this handle's options: sets
// *lpc and, for the lane-per-cell family, compiles its module for the
// handle's device on first use.  Returns a CHEM_* code.
int chem_select_kernel(chem_mech* m, bool* lpc);
// Cells per queue tile of the chosen family (64 for lane-per-cell).
inline int chem_cells_per_tile(const chem_mech* m, bool lpc) { return lpc ? 64 : 64 / m->dev.np_width; }
// Queue reset + persistent box kernel of the chosen family on `stream`.
hipError_t chem_launch_box_queue(chem_mech* m, bool lpc, const chemgpu::IntParams& prm, const chemgpu::BoxDev* boxes,
                                 const chemgpu::BoxJob* job, unsigned* head, int* remaining, int32_t* rec,
                                 int* host_done, int grid, hipStream_t stream);

// Integration parameters from a handle's options (padding zeroed so that the
// struct can be compared bytewise).
inline chemgpu::IntParams make_int_params(const chem_mech* m, double p, double dt, double rtol, double atol) {
  chemgpu::IntParams prm;
  __builtin_memset(&prm, 0, sizeof prm);
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
  return prm;
}
