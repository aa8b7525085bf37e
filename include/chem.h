/*
 * chem.h -- C ABI of the MI355X per-cell stiff chemistry library (libchem).
 *
 * The library advances, in every cell of a batch, the chemical state
 * phi = (Y_1..Y_S, T) of a constant-pressure adiabatic homogeneous reactor
 * over one flow step dt with an implicit BDF integrator whose Newton
 * iteration uses the analytic chemical Jacobian (difference quotients as an
 * option, CHEM_OPT_JAC).  This is the per-cell
 * problem stated in the paper's Sec. 3.1 (at every time step and in every
 * cell, the production rates of the state are evaluated and the state is
 * advanced implicitly with Newton's method and the Jacobian of Eq. 7); the
 * kinetics are Eq. 1-3 (mechanism, rates of progress, net production rates).
 *
 * Conventions for every call:
 *   - Units are SI at this interface: K, Pa, s, mass fractions, and
 *     mol/(m^3 s) for production rates.  (Rate parameters in the mechanism
 *     text are in mol-cm-s units with Ea in kcal/mol.)
 *   - Cell arrays are FP64, device memory (hipMalloc'd or torch CUDA
 *     tensors), 8-byte aligned, structure-of-arrays:
 *         T[i],  Y[k * n_cells + i]  (species-major, contiguous along cells)
 *   - Array arguments are owned by the caller and are not retained after the
 *     call returns.  The mechanism handle is owned by the library from
 *     chem_mech_load* until chem_mech_free.
 *   - A handle may be used by one host thread at a time.  Work is enqueued on
 *     the handle's stream (chem_set_stream; default: the null stream) and
 *     every call below returns only after that work has completed.
 *   - Return codes: 0 = CHEM_OK, > 0 warnings, < 0 errors.  On an error the
 *     outputs are unspecified and chem_last_error() describes the cause.
 *     No C++ exception crosses this interface.
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHEM_OK 0
#define CHEM_WARN_CELLS_FAILED 1  /* some cells failed; see stats and cell_status */
#define CHEM_ERR_ARG (-1)         /* null pointer, n < 0, dt <= 0, rtol <= 0, atol < 0, p <= 0, bad option */
#define CHEM_ERR_PARSE (-2)       /* malformed or unbalanced mechanism text */
#define CHEM_ERR_DEVICE (-3)      /* HIP runtime error (message kept) */
#define CHEM_ERR_OOM (-4)         /* device allocation failed */
#define CHEM_ERR_UNSUPPORTED (-5) /* mechanism outside the supported sizes (S+1 > 64) */

/* Per-cell status codes (chem_integrate_ex cell_status). */
#define CHEM_CELL_OK 0
#define CHEM_CELL_MAX_STEPS 1     /* step attempts exhausted; state left at the last accepted time */
#define CHEM_CELL_H_UNDERFLOW 2   /* step size could not make progress; state at last accepted time */
#define CHEM_CELL_BAD_INPUT 3     /* non-finite or non-positive T, or non-finite Y; cell untouched */

typedef struct chem_mech chem_mech; /* opaque */

/* Totals over the cells of one chem_integrate call; filled by the library. */
typedef struct {
  int64_t n_cells;
  int64_t n_steps_total;     /* accepted steps, summed over cells */
  int64_t n_steps_max;       /* largest accepted-step count of any cell */
  int64_t n_attempts;        /* step attempts (accepted + rejected) */
  int64_t n_rhs;             /* right-hand-side evaluations */
  int64_t n_jac;             /* Jacobian evaluations (one per attempt) */
  int64_t n_lu;              /* Newton-matrix factorisations */
  int64_t n_newton_iters;
  int64_t n_err_test_fails;
  int64_t n_newton_fails;
  int64_t n_cells_failed;
  int64_t n_ir_sweeps;       /* refinement sweeps of the FP32-LU option */
  double wall_ms;            /* device time of the integration kernels */
} chem_stats;

/* Option keys for chem_set_option (values are passed as double). */
#define CHEM_OPT_MAX_STEPS 1    /* step attempts per cell, default 100000 */
#define CHEM_OPT_Q_MAX 2        /* highest BDF order 1..5, default 5 */
#define CHEM_OPT_FIXED_T 3      /* 1: hold T constant (dT/dt = 0); default 0 */
#define CHEM_OPT_FIXED_STEP 4   /* n > 0: n equal steps, no error test (convergence studies); default 0 */
#define CHEM_OPT_LU_FP32 5      /* 1: factorise the Newton matrix in FP32 with FP64 residual refinement */
#define CHEM_OPT_IR_MAX 6       /* refinement sweeps per solve for CHEM_OPT_LU_FP32, default 3 */
#define CHEM_OPT_GRAPH 7        /* 1: chem_integrate_boxes replays a captured hipGraph (default 1) */
#define CHEM_OPT_WAVES_PER_CU 8 /* resident waves per CU for chem_integrate_boxes' persistent grid (1..32) */
#define CHEM_OPT_GROUP_WIDTH 9  /* lanes per cell: 16, 32 or 64, at least S+1 (default: the smallest) */
#define CHEM_OPT_KERNEL 10      /* kernel family: 0 auto (default), 1 group kernels (16-64 lanes per cell),
                                   2 lane-per-cell kernels generated for the mechanism and compiled at run
                                   time (S+1 <= 12, FP64 LU and analytic Jacobian only; auto picks them
                                   where they apply) */
#define CHEM_OPT_JAC 11         /* Newton Jacobian (Sec. 3.2): 0 analytic, Eq. 7 (default); 1 one-sided
                                   difference quotients in every column (N extra right-hand sides per
                                   Jacobian); 2 analytic species columns with a difference-quotient
                                   temperature column, as in Sec. 3.2.2 (one extra right-hand side).
                                   Increment of column j: max(sqrt(u)|y_j|, 1000 h u N ||f||_w / w_j),
                                   u the FP64 unit roundoff, w the error weights.  Group kernels only */
#define CHEM_OPT_RETRY 13       /* k > 0: chem_integrate(_ex) integrates every cell that failed (attempt
                                   limit or step-size underflow) again from its input state with dt split
                                   into 2, 4, ... 2^k equal substeps, until one level passes every
                                   substep (the paper's smaller-timestep restart, per cell); such cells
                                   get that state and status 0, counters include the retry work, and the
                                   stats are recomputed.  Keeps a device copy of the input state
                                   (16(S+1) bytes per cell); wall_ms times the first pass.  Default 0 */
#define CHEM_OPT_PROGRESS 14    /* s > 0: while chem_integrate_boxes waits for per-box completion times
                                   (box_ms given), it writes a line to stderr every s seconds with the
                                   boxes and cells completed so far, read from the completion flags
                                   (for long batches); default 0 (silent) */
#define CHEM_OPT_JAC_REUSE 12   /* 1: keep the factored Newton matrix M = I - cJ across attempts while c
                                   is within 30% of the c it was formed with, fewer than 20 accepted
                                   steps have passed and Newton has not failed with it (a failure
                                   retries the step with a fresh Jacobian), as CVODE does; 0 (default):
                                   a fresh Jacobian and LU every attempt */

/* Parse a mechanism from a file path / from text (format "chem-mech 1":
 * elements with masses; species with atom counts, inert flag and either a
 * linear heat capacity cp/R = a0 + a1 T plus formation enthalpy and entropy
 * at 298.15 K, or NASA 7-coefficient polynomials in two temperature ranges
 * (the CHEMKIN thermo form of real mechanisms); reactions of Eq. 1 with
 * Arrhenius parameters, optional third body or falloff (Lindemann, or Troe
 * with 3 or 4 parameters), with collision efficiencies).  Validates exact atom
 * balance of every reaction and uploads the tables to the current device.
 * On success *out receives a new handle.  Errors: CHEM_ERR_ARG (null
 * pointers, unreadable file), CHEM_ERR_PARSE, CHEM_ERR_UNSUPPORTED,
 * CHEM_ERR_DEVICE, CHEM_ERR_OOM. */
int chem_mech_load(const char* path, chem_mech** out);
int chem_mech_load_str(const char* text, chem_mech** out);

/* Release the handle and its device tables (NULL is ignored). */
void chem_mech_free(chem_mech* m);

/* Sizes of a loaded mechanism: species S, reactions R, elements E. */
int chem_mech_info(const chem_mech* m, int* n_species, int* n_reactions, int* n_elements);

/* Stream for subsequent calls (a hipStream_t, e.g. torch's
 * current_stream().cuda_stream); NULL selects the null stream. */
int chem_set_stream(chem_mech* m, void* hip_stream);

/* Set one option (keys above).  Errors: CHEM_ERR_ARG for an unknown key or
 * a value out of range. */
int chem_set_option(chem_mech* m, int key, double value);

/* Integrate n_cells reactors in place over [0, dt] at pressure p.
 * T[n_cells] and Y[S * n_cells] (device, SoA) are read and overwritten with
 * the state at dt.  rtol > 0, atol >= 0 set the WRMS error weights
 * 1/(rtol |y| + atol) used for every component, T included.  Steps that
 * would leave a mass fraction below -atol are rejected, and one left
 * negative is set to zero (outputs are >= 0); T follows its own equation,
 * so the mixture enthalpy is conserved to the integration tolerance.  stats
 * (host pointer, may be NULL) receives the totals.  Returns CHEM_OK,
 * CHEM_WARN_CELLS_FAILED if any cell failed (see the CHEM_CELL_* codes), or
 * an error code.  n_cells == 0 is a no-op returning CHEM_OK. */
int chem_integrate(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt,
                   double rtol, double atol, chem_stats* stats);

/* As chem_integrate, and additionally writes, when the pointer is not NULL,
 * per-cell records (device memory, int32 SoA of 9 rows x n_cells):
 * row 0 status (CHEM_CELL_*), 1 accepted steps, 2 attempts, 3 rhs
 * evaluations, 4 Jacobian evaluations, 5 Newton iterations, 6 error-test
 * failures, 7 Newton failures, 8 refinement sweeps (CHEM_OPT_LU_FP32). */
int chem_integrate_ex(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt,
                      double rtol, double atol, chem_stats* stats, int32_t* cell_records);

/* Allocation-free variant of chem_integrate, for callers that cannot
 * allocate device memory during the call: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results,
 * statistics and return codes as chem_integrate (the same kernels run), but
 * the per-cell records and statistics counters live in a fixed scratch array
 * of the library on each device (36 MiB for the limit below, held until the
 * process ends) instead of handle-owned workspace, and the call makes no
 * hipMalloc/hipFree or other allocating call.  Limits and errors:
 *   - n_cells <= CHEM_NOALLOC_MAX_CELLS, else CHEM_ERR_ARG;
 *   - CHEM_OPT_RETRY must be 0 (the retry keeps a copy of the input), else
 *     CHEM_ERR_ARG;
 *   - where the handle's options select the lane-per-cell kernels generated
 *     for the mechanism, they must already be loaded on the device (the first
 *     chem_integrate or chem_rates call with the handle and these options
 *     compiles and loads them), else CHEM_ERR_ARG.
 * Every call on a device shares that device's scratch array, which keeps the
 * last call's contents (the counters are cleared by each call on its stream):
 * calls that overlap on one device, from any handle or thread, race and must
 * be serialised by the caller. */
#define CHEM_NOALLOC_MAX_CELLS 1048576
int chem_integrate_noalloc(chem_mech* m, int64_t n_cells, double* T, double* Y, double p, double dt, double rtol,
                           double atol, chem_stats* stats);

/* One box of cells for chem_integrate_boxes (device SoA arrays of that box). */
typedef struct {
  double* T;        /* [n_cells] */
  double* Y;        /* [S * n_cells], Y[k * n_cells + i] */
  int64_t n_cells;
  double dt;        /* flow step of this box, s (> 0) */
} chem_box;

/* Integrate many boxes of uneven size, each over its own dt, in one
 * persistent launch: the paper's AMR setting, where every box of every level
 * advances its chemistry over the flow step (Sec. 5).  Work items are tiles
 * of one wave's cells taken from a device queue, largest boxes first; all
 * options of chem_integrate apply.  boxes is a host array; the T/Y arrays are
 * device memory, updated in place.  box_ms (host, optional, n_boxes entries)
 * receives each box's completion time in ms from the launch, observed on the
 * host through host-mapped flags.  stats totals cover every cell of every box.
 * Returns as chem_integrate. */
int chem_integrate_boxes(chem_mech* m, int n_boxes, const chem_box* boxes, double p, double rtol, double atol,
                         chem_stats* stats, double* box_ms);

/* Pick the lanes-per-cell group width (16/32/64, at least S+1) and the
 * persistent grid's waves per CU (4, 8, 12, 16) for this mechanism by timing
 * chem_integrate_boxes on scratch copies of a caller-supplied sample (device
 * T[n], Y[S*n], left unchanged; split into boxes of up to 4096 cells), and
 * set them on the handle.  The choice only changes speed: results are the
 * same for every candidate.  Choices are cached per (device, S, R) for the
 * process; best_width/best_waves (may be NULL) receive the choice. */
int chem_autotune(chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p, double dt, double rtol,
                  double atol, int* best_width, int* best_waves);

/* ------------------------------------------------------------ serving ---
 * A continuous-batching request server (the serving extension of the
 * batched solve, Sec. 5.1's many-small-boxes setting at request level).
 * Clients submit box-solve requests (host arrays, any loaded mechanism, own
 * dt) at any time.  A dispatcher thread admits them in arrival order while
 * their state and per-cell records fit in the device arena (the HBM budget),
 * copies them in, and appends their cells, in tiles, to the work queue of a
 * resident kernel already running for the same mechanism, pressure and
 * tolerances (a channel): its waves take the new tiles as they finish the
 * ones they hold, so requests join work in flight instead of waiting for a
 * launch.  A wave leaves after about 20 ms without work, or between tiles
 * after 200 ms (so that channels share the GPU); the dispatcher relaunches a
 * channel while it has work.  The last tile of a box raises a host-mapped
 * flag; results then come back through pinned memory.  Latency is submit to
 * results on the host.  The handles passed to submit must stay alive, and
 * their options unchanged, until the server is drained. */
typedef struct chem_server chem_server;

typedef struct {
  int64_t submitted, completed, cells_completed;
  int64_t launches;          /* resident-kernel launches */
  int64_t bytes_in_use, bytes_peak, budget_bytes;
  int64_t queued;            /* waiting for admission */
  int64_t in_flight;         /* admitted, not yet completed */
} chem_server_stats;

/* Create a server with an HBM budget (bytes) for request state and records
 * (8 (S+1) + 36 bytes per cell) and a number of channels (1..8): resident
 * kernels, each serving one (mechanism, pressure, tolerances) at a time.
 * With fewer channels than such keys in the traffic, a channel drains and
 * changes key.  The budget is reserved as one device arena at creation,
 * with pinned staging of a quarter of it (at most 8 GiB).  Errors:
 * CHEM_ERR_ARG, CHEM_ERR_OOM, CHEM_ERR_DEVICE. */
int chem_server_create(int64_t budget_bytes, int streams, chem_server** out);

/* Queue one request: n_cells cells of mechanism m with host arrays T[n] and
 * Y[S*n] (SoA, copied at submit), pressure p, step dt and tolerances.  *id
 * receives the request id.  A request larger than the whole budget (or the
 * staging area) is rejected with CHEM_ERR_OOM; after a device error every
 * submit returns CHEM_ERR_DEVICE. */
int chem_server_submit(chem_server* s, chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p,
                       double dt, double rtol, double atol, int64_t* id);

/* Non-blocking completion check.  Returns 1 and fills T_out/Y_out (host, may
 * be NULL), latency_ms and status when the request is done (the request is
 * then forgotten), 0 while pending, or an error code for an unknown id.
 * status: CHEM_OK, CHEM_WARN_CELLS_FAILED, the code of a refused kernel
 * choice (e.g. CHEM_ERR_UNSUPPORTED), or CHEM_ERR_DEVICE; on an error the
 * output arrays are left alone. */
int chem_server_poll(chem_server* s, int64_t id, double* T_out, double* Y_out, double* latency_ms, int* status);

/* Block until every submitted request has completed (CHEM_ERR_DEVICE if
 * the server met a device error). */
int chem_server_drain(chem_server* s);

int chem_server_stats_get(chem_server* s, chem_server_stats* out);

/* Stop the dispatcher and the resident kernels (each wave leaves after the
 * tile it holds) and release everything; pending requests are dropped. */
void chem_server_destroy(chem_server* s);

/* Rates of one state per cell (Eq. 2-3, Eq. 7): wdot[S * n] (mol m^-3 s^-1,
 * required), f[(S+1) * n] (optional, the ODE right-hand side dY/dt, dT/dt)
 * and jac[(S+1)^2 * n] (optional, the analytic J[i][j] = d f_i / d y_j stored
 * at (i*(S+1)+j) * n + cell).  T, Y as in chem_integrate; p in Pa.  The
 * CHEM_OPT_FIXED_T option applies to f and jac.  The values come from the
 * kernel family chem_integrate would run with the handle's options
 * (CHEM_OPT_KERNEL), so each family's rate and Jacobian code can be checked
 * on its own. */
int chem_rates(chem_mech* m, int64_t n_cells, const double* T, const double* Y, double p, double* wdot,
               double* f, double* jac);

/* Message for the last error on the calling thread ("" if none). */
const char* chem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEM_H */
