#!/usr/bin/env python3
"""Benchmark: reactor cells integrated per second over one flow step on one
MI355X, for the planar-flame box of G(10,25,3, seed 1) (64 x 64 x 256 =
1,048,576 cells, dt = 2e-6 s, rtol 1e-8, atol 1e-12, 1 atm).

One step = one chem_integrate call over the whole box from the same initial
state (a device-to-device reset copy of 92 MB precedes each call).  Prints one
JSON line with the throughput, the roofline of the integration kernel (an
algorithmic FP64 flop count from the device's own counters divided by the
kernel's HIP-event time on the library's stream), and the CPU oracle timed on
a strided sample of the same box (which also gives the accuracy figure).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reactor cells integrated/sec over dt (1 GPU) at stated accuracy; p50/p99 box latency"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 flop/clk)
C_EXP_DEFAULT = 20.0             # FP64 operations per exp when no measured figure is on file


def probe_figures():
    """Measured probe figures committed under profiles/ (on-box FP64 FMA rate
    and the FP64 operations of one exp per kernel family), or {}."""
    path = os.path.join(ROOT, "profiles", "probe_fp64_exp.json")
    return json.load(open(path)) if os.path.exists(path) else {}


def flops_step_model(stats, S, R, c_exp, q):
    """Algorithmic FP64 flops of one launch by the per-step model

        F_step = n_N F_rhs + F_J + 2N^3/3 + n_N 2N^2 + 10 N q,
        F_rhs = R (2 c_exp + 14) + 12 S + 8 R,   F_J = 64 R + 2 S^2 + 6 N^2,

    summed with the launch's own counters: every right-hand side (n_rhs, the
    Newton iterations plus one per cell to start), every fresh Newton matrix
    (n_jac Jacobians and factorisations), every Newton solve and every step
    attempt (order q taken as q_max, an upper bound of a term worth ~2%)."""
    N = S + 1
    f_rhs = R * (2 * c_exp + 14) + 12 * S + 8 * R
    f_j = 64 * R + 2 * S * S + 6 * N * N
    f_lu = 2.0 * N ** 3 / 3.0
    return (stats["n_rhs"] * f_rhs + stats["n_jac"] * (f_j + f_lu) + stats["n_newton_iters"] * 2 * N * N
            + stats["n_attempts"] * 10 * N * q)


def flops_itemised_model(stats, S, R, n_tb, n_falloff, c_exp=20.0):
    """A finer itemisation of the same work (per rhs: mixture, thermo with one
    exp/log per species, rates with two exps per reaction, falloff, sparse
    products; per fresh matrix: Jacobian extras, M = I - cJ and its LU; per
    attempt: step control; per Newton iteration: residual, solve, norm).  It
    charges more per rhs than the model above and is reported beside it."""
    N = S + 1
    nnz = 4 * R
    f_rhs = 32 * S + S * c_exp + R * (26 + 2 * c_exp) + n_falloff * (8 + c_exp) + n_tb + 2 * nnz
    f_jac = 26 * R + 12 * nnz + 13 * S * S + 10 * N
    f_setup = f_jac + 2 * N * N + 2.0 * N ** 3 / 3.0
    return (stats["n_rhs"] * f_rhs + stats["n_jac"] * f_setup + stats["n_attempts"] * 40 * N
            + stats["n_newton_iters"] * (2 * N * N + 7 * N))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shape", type=str, default=None,
                    help="flame box nx,ny,nz (x = flame axis); default 256,64,64 for --config 2, 256,64,16 for 3")
    ap.add_argument("--config", type=int, choices=[2, 3], default=2,
                    help="flame workload: 2 = G(10,25,3,s1), dt 2e-6, rtol 1e-8 (the headline box); "
                         "3 = G(53,325,4,s2), dt 1e-6, rtol 1e-6 (the mixed-precision case, with --lu-fp32)")
    ap.add_argument("--cpu-sample", type=int, default=8192, help="cells in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--q-max", type=int, default=5)
    ap.add_argument("--mode", choices=["flame", "boxes", "serve", "copy", "jacstudy", "sweep", "peak", "mfma"],
                    default="flame",
                    help="flame: the headline box; boxes: uneven AMR boxes in one persistent launch; "
                         "serve: Poisson request trace through the continuous-batching server; "
                         "copy: a plain device copy of known size (HBM counter calibration); "
                         "jacstudy: analytic vs finite-difference Newton Jacobian at S = 10, 30, 53; "
                         "sweep: error against the tight-tolerance truth and cost over rtol x dt; "
                         "peak: the FP64 FMA rate and the cost of one exp on this device (probe kernels)")
    ap.add_argument("--lu-fp32", action="store_true", help="FP32 Newton-matrix LU with FP64 refinement")
    ap.add_argument("--ir-max", type=int, default=3,
                    help="with --lu-fp32: refinement sweeps per Newton solve at most (0 = the FP32 solve alone; "
                         "Newton's own FP64 residual then corrects it)")
    ap.add_argument("--jac-reuse", action="store_true",
                    help="keep the factored Newton matrix across attempts while it is recent (CVODE's policy); "
                         "default: a fresh Jacobian and LU every attempt")
    ap.add_argument("--kernel", choices=["auto", "group", "lane"], default="auto",
                    help="kernel family: lane = generated lane-per-cell kernels (S+1 <= 12), group = 16-64 lanes "
                         "per cell; auto picks lane where it applies")
    ap.add_argument("--n-boxes", type=int, default=200)
    ap.add_argument("--max-box-cells", type=int, default=None,
                    help="boxes/serve: cap on the cells of one box (default: none, edges up to 64)")
    ap.add_argument("--rate", type=float, default=2000.0,
                    help="serve: arrivals per second (the full trace's 2000/s is far beyond one GPU's capacity)")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: trace length, s")
    ap.add_argument("--wall", type=float, default=150.0, help="serve: stop after this many seconds")
    ap.add_argument("--queue-gb", type=float, default=8.0,
                    help="serve: request state the host keeps waiting for the server; more is refused")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget")
    ap.add_argument("--mix", type=float, default=0.5, help="serve: probability that a request is G(53,325,4)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (cells are independent, so "
              "each GPU would integrate its own share of the cells).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_05974_amd import chem, synth

    dev = torch.device("cuda:0")
    if args.mode == "copy":
        return copy_calibration(torch, dev)
    if args.mode == "peak":
        return probe_peak(torch)
    if args.mode == "mfma":
        return probe_mfma(synth)
    if args.mode == "boxes":
        return bench_boxes(args, torch, dev, chem, synth)
    if args.mode == "serve":
        return bench_serve(args, torch, dev, chem, synth)
    if args.mode == "jacstudy":
        return bench_jacstudy(args, torch, dev, chem, synth)
    if args.mode == "sweep":
        return bench_sweep(args, torch, dev, chem, synth)
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    w = synth.config_workload(args.config, os.path.join(ROOT, "tests", "golden"), shape=shape)
    shape = w.shape if w.shape else shape
    m = w.mech
    n = w.n_cells
    n_tb = sum(r.kind == 1 for r in m.reactions)
    n_fo = sum(r.kind == 2 for r in m.reactions)
    t_load = time.perf_counter()
    gm = chem.Mechanism(m.to_text())
    load_ms = (time.perf_counter() - t_load) * 1e3
    gm.set_options(q_max=args.q_max, lu_fp32=int(args.lu_fp32), kernel=KERNEL_CODES[args.kernel],
                   jac_reuse=int(args.jac_reuse), ir_max=args.ir_max)
    kname = kernel_name(args, m.n_species + 1)
    T0 = torch.tensor(w.T, dtype=torch.float64, device=dev)
    Y0 = torch.tensor(w.Y, dtype=torch.float64, device=dev)
    T = torch.empty_like(T0)
    Y = torch.empty_like(Y0)

    def step():
        T.copy_(T0)
        Y.copy_(Y0)
        return gm.integrate(T, Y, w.p, w.dt, w.rtol, w.atol)

    first_ms = None
    for i in range(args.warmup):
        tw = time.perf_counter()
        st = step()
        if first_ms is None:
            first_ms = (time.perf_counter() - tw) * 1e3
        print(f"warmup {i}: {st['wall_ms']:.1f} ms kernel, rc={st['rc']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    kernel_ms, step_ms, stats = [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st = step()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        kernel_ms.append(st["wall_ms"])
        stats.append(st)
        print(f"step {i}: {st['wall_ms']:.1f} ms kernel, rc={st['rc']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = stats[-1]
    if st["n_cells_failed"]:
        print(f"warning: {st['n_cells_failed']} cells failed", file=sys.stderr)
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    k_ms = float(np.median(kernel_ms))
    lane = kname.startswith("chem_lpc_integrate")
    probes = probe_figures()
    c_exp = probes.get("c_exp_chexp" if lane else "c_exp_libexp", C_EXP_DEFAULT)
    flops = flops_step_model(st, m.n_species, m.n_reactions, c_exp, args.q_max)
    flops_item = flops_itemised_model(st, m.n_species, m.n_reactions, n_tb, n_fo)
    achieved = flops / (k_ms * 1e-3) / 1e12
    prof = measured_profile("chem_lpc_integrate") if (lane and args.config == 2 and shape == (256, 64, 64)) else None
    hw_frac = None
    if prof and "fp64_flops_per_launch_hw" in prof:
        # executed FP64 flops counted on all 64 lanes, weighted by the measured lane activity
        hw = prof["fp64_flops_per_launch_hw"] * prof.get("lane_activity", 1.0)
        hw_frac = hw / (k_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32lu" if args.lu_fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"planar flame box {shape[0]}x{shape[1]}x{shape[2]} = {n} cells, mechanism "
                         f"G{synth.CONFIG_MECH[args.config][:3]} seed {synth.CONFIG_MECH[args.config][3]}, "
                         f"T 300->2200 K tanh profile, dt {w.dt:g} s, rtol {w.rtol:g}, "
                         f"atol {w.atol:g}, p 1 atm, constant-pressure adiabatic, BDF q<={args.q_max}, "
                         + ("Newton matrix kept while recent" if args.jac_reuse else "fresh Newton matrix every attempt")),
            "cells": n, "species": m.n_species, "reactions": m.n_reactions,
            "parallelism": "none (1 GPU)",
        },
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "one whole-box chem_integrate call"},
        "setup_ms": {"mechanism_load": load_ms, "first_call": first_ms,
                     "what": "parse + table upload; the first call includes compiling the generated kernels "
                             "(lane-per-cell family) and is not timed in value"},
        "integration": {"steps_per_cell": st["n_steps_total"] / n, "attempts_per_cell": st["n_attempts"] / n,
                        "newton_per_cell": st["n_newton_iters"] / n, "max_steps_cell": st["n_steps_max"],
                        "failed_cells": st["n_cells_failed"],
                        "refinement_sweeps_per_newton": (st["n_ir_sweeps"] / max(st["n_newton_iters"], 1)
                                                         if args.lu_fp32 else None),
                        "ir_max": args.ir_max if args.lu_fp32 else None},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": prof["hbm_bytes_per_launch"] if prof else None,
            "kernel": kname, "kernel_ms": k_ms, "flops_per_launch": flops,
            "flop_model": (f"per step n_N F_rhs + F_J + 2N^3/3 + n_N 2N^2 + 10Nq with F_rhs = R(2c_exp+14)+12S+8R, "
                           f"F_J = 64R+2S^2+6N^2, c_exp = {c_exp:g} (measured FP64 operations of one exp of this "
                           f"kernel family), q = {args.q_max}; summed over the launch's rhs, Jacobian, Newton and "
                           f"attempt counts"),
            "itemised_model": {"flops_per_launch": flops_item,
                               "frac": flops_item / (k_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                               "what": "finer per-event itemisation (bench.py flops_itemised_model, c_exp 20)"},
            "hw_counter_frac": hw_frac,
            "hw_counter_what": "SQ_INSTS_VALU_FLOPS_FP64 x 64 x lane activity (SQ_THREAD_CYCLES_VALU / "
                               "(64 SQ_ACTIVE_INST_VALU)) from the committed profile of this kernel's sources",
            "peak_measured": probes.get("fma_tflops"),
            "peak_measured_what": "FP64 FMA chains on every CU (bench.py --mode peak), beside the published peak",
            "mfma_utilisation": 0.0,
            "timing": "kernel_ms = median of the timed launches (HIP events on the launch stream)",
        },
    }
    worst = None
    if args.lu_fp32:
        out["accuracy_vs_fp64_gpu"] = fp64_comparison(gm, T0, Y0, T, Y, w, torch)
        worst = out["accuracy_vs_fp64_gpu"].pop("_worst")
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(w, T, Y, args, worst)
    print(json.dumps(out), flush=True)


def fp64_comparison(gm, T0, Y0, T, Y, w, torch):
    """Every cell of the FP32-LU result (T, Y) against the plain FP64 GPU path
    on the same inputs (T0, Y0) and settings: the difference isolates the LU
    precision.  Errors are absolute in Y and relative in T, max and p99 over
    the cells."""
    print("fp64 comparison: plain FP64 integration of the same box", file=sys.stderr, flush=True)
    gm.set_options(lu_fp32=0)
    T6, Y6 = T0.clone(), Y0.clone()
    st = gm.integrate(T6, Y6, w.p, w.dt, w.rtol, w.atol)
    gm.set_options(lu_fp32=1)
    print(f"fp64 comparison: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    dY = (Y - Y6).abs().amax(dim=0)
    dT = ((T - T6).abs() / T6)
    q = lambda t: float(torch.quantile(t.float().cpu(), 0.99))
    err = torch.maximum(dY, dT)
    over = int((err > 1e-6).sum())
    worst = torch.topk(err, min(8, err.numel())).indices
    wi = worst.cpu().numpy()
    return {"vs": "plain FP64 GPU path, same inputs and settings, every cell", "cells": int(T.numel()),
            "max_abs_dY": float(dY.max()), "p99_abs_dY": q(dY), "max_rel_dT": float(dT.max()), "p99_rel_dT": q(dT),
            "cells_over_1e-6": over, "fraction_over_1e-6": over / T.numel(),
            "worst_cells": [{"cell": int(i), "T0": float(T0[i]), "rel_dT": float(dT[i]), "abs_dY": float(dY[i])}
                            for i in wi],
            "fp64_kernel_ms": st["wall_ms"],
            "_worst": (wi, T6[worst].cpu().numpy(), Y6[:, worst].cpu().numpy())}


def measured_profile(kernel):
    """The HBM traffic and FP64 counter figures that profiles/traffic.json
    records for `kernel`, if the kernel's sources are unchanged since they
    were measured (None otherwise)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec if h.hexdigest()[:16] == rec["source_hash"] else None


KERNEL_CODES = {"auto": 0, "group": 1, "lane": 2}
LANE_MAX_N = 12          # largest S+1 the lane-per-cell kernels serve


def kernel_name(args, N):
    lane = args.kernel == "lane" or (args.kernel == "auto" and N <= LANE_MAX_N and not args.lu_fp32)
    if lane:
        return "chem_lpc_integrate (generated for the mechanism, hipRTC)"
    np_ = 16 if N <= 16 else (32 if N <= 32 else 64)
    cols = 56 if (np_ == 64 and N <= 56) else np_       # columns the 64-lane factorisations carry
    return f"integrate_kernel<{np_}, {'true' if args.lu_fp32 else 'false'}, {cols}>"


def cpu_baseline(w, Tg, Yg, args, worst=None):
    """The oracle, built for this host (-march=native), on a strided sample of
    the same box with all host threads: the median of three timed runs; the
    results also give the accuracy figures.  `worst` = (cells, FP64 GPU T, Y
    there) for the FP32-LU run: those cells also go through the oracle at the
    same settings and at the tight tolerance, so that the FP32-LU and FP64
    results there are both measured against the oracle and the truth."""
    import tempfile
    import oracle
    n = w.n_cells
    tmpdir = tempfile.mkdtemp(prefix="oracle_native_")
    try:
        lib_path = oracle.build_native(tmpdir)
        build = "gcc -O3 -march=native -fopenmp -ffp-contract=off (no fast-math)"
    except Exception as exc:             # keep the portable build if the host compiler refuses
        print(f"cpu baseline: native build failed ({exc}); using the portable build", file=sys.stderr, flush=True)
        lib_path, build = None, "gcc -O3 -fopenmp -ffp-contract=off (portable build)"
    om = oracle.Mech(w.mech.to_text(), lib_path=lib_path)
    threads = oracle.max_threads()
    # size the sample to about 15 s per run: a pilot of 2 cells per thread, strided over the box
    pilot = np.unique(np.linspace(0, n - 1, min(n, 2 * threads)).astype(np.int64))
    t0 = time.perf_counter()
    om.integrate(w.T[pilot], w.Y[:, pilot], w.p, w.dt, w.rtol, w.atol, q_max=args.q_max, nthreads=threads,
                 jac_reuse=args.jac_reuse, want_stats=False)
    per_cell = (time.perf_counter() - t0) / pilot.size
    k = int(max(threads, min(args.cpu_sample, n, 15.0 / max(per_cell, 1e-9))))
    print(f"cpu baseline: pilot {pilot.size} cells in {per_cell * pilot.size:.1f} s; sample {k} cells",
          file=sys.stderr, flush=True)
    idx = np.unique(np.linspace(0, n - 1, k).astype(np.int64))
    runs = []
    for r in range(3):
        print(f"cpu baseline: oracle run {r + 1}/3 on {idx.size} cells, {threads} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        To, Yo, so = om.integrate(w.T[idx], w.Y[:, idx], w.p, w.dt, w.rtol, w.atol, q_max=args.q_max,
                                  nthreads=threads, jac_reuse=args.jac_reuse, want_stats=(r == 0))
        runs.append(time.perf_counter() - t0)
        print(f"cpu baseline: {runs[-1]:.1f} s", file=sys.stderr, flush=True)
    el = float(np.median(runs))
    Tgs = Tg.cpu().numpy()[idx]
    Ygs = Yg.cpu().numpy()[:, idx]
    acc = {"vs": "CPU oracle, same inputs and settings", "cells": int(idx.size),
           "max_abs_dY": float(np.abs(Ygs - Yo).max()),
           "max_rel_dT": float((np.abs(Tgs - To) / To).max()),
           "p99_abs_dY": float(np.percentile(np.abs(Ygs - Yo).max(axis=0), 99)),
           "p99_rel_dT": float(np.percentile(np.abs(Tgs - To) / To, 99))}
    # against the tight-tolerance truth (the oracle at rtol 1e-12, atol 1e-20, fresh Newton matrices)
    # on a sub-sample of at most 128 cells sized to about 20 s of host time; a truth cell costs about
    # 8x a same-settings cell, 20x when the same-settings run kept its Newton matrices
    per_cell_truth = el * threads / idx.size * (20.0 if args.jac_reuse else 8.0)
    n_sub = int(min(128, idx.size, 20.0 * threads / per_cell_truth))
    if n_sub < 4:
        acc["vs_truth"] = {"cells": 0, "what": f"skipped: about {per_cell_truth:.0f} s per truth cell on one core"}
    else:
        sub = idx[:: max(1, idx.size // n_sub)]
        pos = np.searchsorted(idx, sub)
        print(f"cpu baseline: truth reference on {sub.size} cells", file=sys.stderr, flush=True)
        Tt, Yt, _ = om.integrate(w.T[sub], w.Y[:, sub], w.p, w.dt, 1e-12, 1e-20, q_max=args.q_max,
                                 nthreads=threads, want_stats=False)
        acc["vs_truth"] = {"cells": int(sub.size), "max_abs_dY_gpu": float(np.abs(Ygs[:, pos] - Yt).max()),
                           "max_rel_dT_gpu": float((np.abs(Tgs[pos] - Tt) / Tt).max()),
                           "max_abs_dY_oracle": float(np.abs(Yo[:, pos] - Yt).max()),
                           "max_rel_dT_oracle": float((np.abs(To[pos] - Tt) / Tt).max()),
                           "what": "truth = the oracle at rtol 1e-12, atol 1e-20"}
    if worst is not None:
        wi, T6w, Y6w = worst
        print(f"cpu baseline: oracle and truth on the {wi.size} cells where FP32 LU and FP64 differ most",
              file=sys.stderr, flush=True)
        Tow, Yow, _ = om.integrate(w.T[wi], w.Y[:, wi], w.p, w.dt, w.rtol, w.atol, q_max=args.q_max,
                                   nthreads=threads, want_stats=False)
        Ttw, Ytw, _ = om.integrate(w.T[wi], w.Y[:, wi], w.p, w.dt, 1e-12, 1e-20, q_max=args.q_max,
                                   nthreads=threads, want_stats=False)
        Tgw, Ygw = Tg.cpu().numpy()[wi], Yg.cpu().numpy()[:, wi]

        def e(Ta, Ya, Tb, Yb):
            return {"max_abs_dY": float(np.abs(Ya - Yb).max()), "max_rel_dT": float((np.abs(Ta - Tb) / Tb).max())}
        acc["worst_fp32_cells"] = {
            "cells": [int(i) for i in wi],
            "fp32lu_vs_oracle": e(Tgw, Ygw, Tow, Yow), "fp64_gpu_vs_oracle": e(T6w, Y6w, Tow, Yow),
            "fp32lu_vs_truth": e(Tgw, Ygw, Ttw, Ytw), "fp64_gpu_vs_truth": e(T6w, Y6w, Ttw, Ytw),
            "oracle_vs_truth": e(Tow, Yow, Ttw, Ytw),
            "what": "oracle = same settings (FP64 LU); truth = the oracle at rtol 1e-12, atol 1e-20"}
    # one core on a sub-sample of about 4 s
    n1 = int(max(1, min(idx.size, 4.0 * idx.size / (el * threads))))
    sub1 = idx[:: max(1, idx.size // n1)]
    print(f"cpu baseline: one core on {sub1.size} cells", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    om.integrate(w.T[sub1], w.Y[:, sub1], w.p, w.dt, w.rtol, w.atol, q_max=args.q_max, nthreads=1,
                 jac_reuse=args.jac_reuse, want_stats=False)
    el1 = time.perf_counter() - t1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    base = {"value": idx.size / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": (f"{idx.size} cells evenly strided over the {n}-cell box; median of 3 runs "
                       f"({', '.join(f'{r:.1f}' for r in runs)} s)"),
            "build": build,
            "one_core": {"value": sub1.size / el1, "cells": int(sub1.size), "seconds": el1},
            "cpu_model": model}
    return base, acc


def copy_calibration(torch, dev):
    """A plain device copy of 256 MiB, three times: the FETCH_SIZE and
    WRITE_SIZE counters of its dispatches against the known bytes give the
    scale factor applied to the integration kernel's counters."""
    n = (256 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_dispatch": n * 8, "bytes_written_per_dispatch": n * 8}))


def probe_peak(torch):
    """The probe kernels of libchem_probe.so: FP64 FMA throughput over the
    whole chip, and timed exp loops (their FP64 instruction counters, taken
    with rocprofv3 --pmc on this mode, give the operations of one exp)."""
    import ctypes as C
    torch.cuda.init()
    lib = C.CDLL(os.path.join(ROOT, "paper_2405_05974_amd", "libchem_probe.so"))
    lib.chem_probe_run.argtypes = [C.c_char_p, C.c_int, C.c_int, C.POINTER(C.c_double)]
    ms = C.c_double()
    out = {"mode": "peak"}
    blocks, iters = 8192, 2048
    for i in range(3):
        if lib.chem_probe_run(b"fma", blocks, iters, C.byref(ms)) != 0:
            raise RuntimeError("fma probe failed")
        flops = 2.0 * 16 * iters * blocks * 256
        out.setdefault("fma_tflops_runs", []).append(flops / (ms.value * 1e-3) / 1e12)
        print(f"peak: fma run {i}: {out['fma_tflops_runs'][-1]:.2f} TFLOP/s", file=sys.stderr, flush=True)
    out["fma_tflops"] = max(out["fma_tflops_runs"])
    eb, ei = 2048, 4096
    for which in ("loop", "chexp", "libexp"):
        if lib.chem_probe_run(which.encode(), eb, ei, C.byref(ms)) != 0:
            raise RuntimeError(f"{which} probe failed")
        out[f"{which}_ns_per_eval_per_lane"] = ms.value * 1e6 / (eb * 256 * ei) * 256 * 1024
        out[f"{which}_dispatch"] = {"blocks": eb, "threads": 256, "iters": ei, "ms": ms.value}
        print(f"peak: {which}: {ms.value:.2f} ms", file=sys.stderr, flush=True)
    out["what"] = ("fma: 16 independent FMA chains per thread, 8192 blocks of 256 threads, 2048 trips; "
                   "exp probes: 2048 blocks of 256 threads, 4096 exps per thread, arguments in [-60, -19]")
    print(json.dumps(out), flush=True)


def probe_mfma(synth):
    """The production-rate contraction wdot = Q nu^T of the 10- and
    53-species mechanisms, as the dense [cells x R] x [R x S] product on FP64
    matrix cores (v_mfma_f64_16x16x4) and as the sparse per-species gather of
    the kernels, rates of progress generated in registers in both
    (libchem_probe.so).  Each result is checked against numpy on 100 cells
    first; then both are timed on a full box of cells, 64 contractions per
    cell per launch (so that writing the result does not dominate)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2405_05974_amd", "libchem_probe.so"))
    lib.chem_probe_wdot.argtypes = [C.c_char_p, C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]
    iters = 64
    res = {"mode": "mfma", "what": probe_mfma.__doc__.split("\n\n")[0].replace("\n    ", " ")}
    for cfg, ncells in ((2, 1 << 20), (3, 1 << 18)):
        m = synth.config_mechanism(cfg)
        S, R = m.n_species, m.n_reactions
        nu = np.zeros((R, S), dtype=np.int32)
        for j, r in enumerate(m.reactions):
            for k in r.reactants:
                nu[j, k] -= 1
            for k in r.products:
                nu[j, k] += 1
        nup = np.ascontiguousarray(nu).ctypes.data_as(C.POINTER(C.c_int))
        nchk = 100
        Q = 1.0 + 1e-6 * np.arange(nchk)[:, None] + 1e-3 * np.arange(R)[None, :]
        ref = Q @ nu.astype(float)
        row = {"species": S, "reactions": R, "cells": ncells, "nnz": int(np.count_nonzero(nu)),
               "dense_padded": [(R + 3) // 4 * 4, (S + 15) // 16 * 16]}
        for which in ("mfma", "sparse"):
            out = np.zeros((nchk, S))
            ms = C.c_double()
            if lib.chem_probe_wdot(which.encode(), nup, R, S, nchk, 1, 1, out.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(ms)) != 0:
                raise RuntimeError(f"{which} probe failed")
            err = float(np.abs(out - ref).max() / np.abs(ref).max())
            if err > 1e-13:
                raise RuntimeError(f"{which} probe wrong: {err}")
            if lib.chem_probe_wdot(which.encode(), nup, R, S, ncells, iters, 5, None, C.byref(ms)) != 0:
                raise RuntimeError(f"{which} probe failed")
            row[which] = {"ms": ms.value, "ns_per_contraction": ms.value * 1e6 / (ncells * iters),
                          "check_rel_err": err}
            print(f"mfma probe: G{cfg} {which}: {ms.value:.3f} ms for {ncells} cells", file=sys.stderr, flush=True)
        RP, SP = row["dense_padded"]
        row["contractions_per_cell"] = iters
        row["flops_per_contraction"] = {"mfma_executed": 2 * RP * SP, "sparse_algorithmic": 2 * row["nnz"]}
        row["mfma_tflops_executed"] = 2 * RP * SP * ncells * iters / (row["mfma"]["ms"] * 1e-3) / 1e12
        row["mfma_over_sparse_time"] = row["mfma"]["ms"] / row["sparse"]["ms"]
        res[f"G{m.n_species}_{m.n_reactions}"] = row
    print(json.dumps(res), flush=True)


def bench_boxes(args, torch, dev, chem, synth):
    """Uneven AMR boxes of G(30,180,4, seed 3) with per-box dt, one persistent
    launch; edges log-uniform 8..64 cells, capped at --max-box-cells when
    given.  The library reports completed boxes every 20 s during a launch."""
    m = synth.config_mechanism(4)
    boxes = synth.amr_boxes(m, args.n_boxes, synth.config_seed(4), max_cells=args.max_box_cells)
    gm = chem.Mechanism(m.to_text())
    gm.set_options(q_max=args.q_max, lu_fp32=int(args.lu_fp32), kernel=KERNEL_CODES[args.kernel],
                   jac_reuse=int(args.jac_reuse), progress=20, ir_max=args.ir_max)
    src = [(torch.tensor(b.T, device=dev), torch.tensor(b.Y, device=dev), b.dt) for b in boxes]
    work = [(t.clone(), y.clone(), dt) for t, y, dt in src]
    sample_T = torch.cat([t[: min(256, t.numel())] for t, _, _ in src[:8]])
    sample_Y = torch.cat([y[:, : min(256, y.shape[1])] for _, y, _ in src[:8]], dim=1).contiguous()
    width, waves = gm.autotune(sample_T, sample_Y, synth.P_ATM, float(np.median([b.dt for b in boxes])), 1e-8, 1e-12)
    n = sum(b.T.size for b in boxes)

    def reset():
        for (t, y, _), (t0, y0, _) in zip(work, src):
            t.copy_(t0)
            y.copy_(y0)

    for _ in range(args.warmup):
        reset()
        gm.integrate_boxes(work, synth.P_ATM, 1e-8, 1e-12)
    times, lat, stats = [], [], None
    for i in range(args.steps):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, ms = gm.integrate_boxes(work, synth.P_ATM, 1e-8, 1e-12, box_ms=True)
        times.append(time.perf_counter() - t0)
        lat.extend(ms)
        print(f"boxes step {i}: {times[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    el = float(np.median(times))
    print(json.dumps({
        "mode": "boxes", "metric": METRIC, "value": n / el, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "ms_per_step": el * 1e3, "dtype": "f64+f32lu" if args.lu_fp32 else "f64",
        "box_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "what": "launch to box completion, host-observed"},
        "config": {"workload": f"{len(boxes)} boxes of G(30,180,4,seed 3), edges log-uniform 8..64"
                               + (f" capped at {args.max_box_cells} cells" if args.max_box_cells else "")
                               + ", per-box dt log-uniform 1e-7..1e-5 s, rtol 1e-8, "
                               + ("Newton matrix kept while recent" if args.jac_reuse else "fresh Newton matrix"),
                   "cells": n, "group_width": width, "waves_per_cu": waves},
        "integration": {"steps_per_cell": stats["n_steps_total"] / n, "failed_cells": stats["n_cells_failed"]},
    }), flush=True)


def bench_jacstudy(args, torch, dev, chem, synth):
    """The paper's analytic-vs-finite-difference Jacobian comparison (Sec. 3.2,
    the speedup column of its Table 4) on the GPU: the same cells integrated
    by the group kernels with the analytic Jacobian, with difference quotients
    in every column, with only the temperature column by differences
    (Sec. 3.2.2), and with the analytic Jacobian and kept Newton matrices.  Mechanisms G(10,25,3), G(30,180,4), G(53,325,4); flame-box
    states for S = 10 and 53, AMR-box states for S = 30.  One timed call per
    (mechanism, mode) after a warm-up call."""
    golden = os.path.join(ROOT, "tests", "golden")
    cases = []
    w2 = synth.config_workload(2, golden, shape=(256, 4, 4))
    cases.append(("G(10,25,3,seed 1)", w2.mech, w2.T, w2.Y, w2.dt, w2.rtol, w2.atol, "flame 256x4x4"))
    m4 = synth.config_mechanism(4)
    bx = synth.amr_boxes(m4, 64, synth.config_seed(4), max_cells=64)
    T4 = np.concatenate([b.T for b in bx])[:2048]
    Y4 = np.concatenate([b.Y for b in bx], axis=1)[:, :2048]
    cases.append(("G(30,180,4,seed 3)", m4, T4, Y4, 1e-6, 1e-8, 1e-12, f"AMR-box states, dt 1e-6 s"))
    w3 = synth.config_workload(3, golden, shape=(256, 2, 2))
    cases.append(("G(53,325,4,seed 2)", w3.mech, w3.T, w3.Y, w3.dt, w3.rtol, w3.atol, "flame 256x2x2"))
    rows = []
    for name, m, T0n, Y0n, dt, rtol, atol, what in cases:
        gm = chem.Mechanism(m.to_text())
        T0 = torch.tensor(np.asarray(T0n, dtype=np.float64), device=dev)
        Y0 = torch.tensor(np.ascontiguousarray(Y0n, dtype=np.float64), device=dev)
        row = {"mechanism": name, "species": m.n_species, "reactions": m.n_reactions, "cells": int(T0.numel()),
               "states": what, "dt": dt, "rtol": rtol}
        for mode, key, reuse in ((0, "analytic", 0), (1, "fd", 0), (2, "fd_T", 0), (0, "analytic_kept", 1)):
            gm.set_options(q_max=args.q_max, kernel=KERNEL_CODES["group"], jac=mode, jac_reuse=reuse)
            T, Y = T0.clone(), Y0.clone()
            gm.integrate(T, Y, synth.P_ATM, dt, rtol, atol)                       # warm-up
            T.copy_(T0)
            Y.copy_(Y0)
            st = gm.integrate(T, Y, synth.P_ATM, dt, rtol, atol)
            n = T0.numel()
            row[key] = {"kernel_ms": st["wall_ms"], "steps_per_cell": st["n_steps_total"] / n,
                        "jacobians_per_cell": st["n_jac"] / n,
                        "rhs_per_cell": st["n_rhs"] / n, "newton_per_cell": st["n_newton_iters"] / n,
                        "failed_cells": st["n_cells_failed"]}
            print(f"jacstudy {name} {key}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
        row["speedup_analytic_vs_fd"] = row["fd"]["kernel_ms"] / row["analytic"]["kernel_ms"]
        row["speedup_analytic_vs_fd_T"] = row["fd_T"]["kernel_ms"] / row["analytic"]["kernel_ms"]
        row["speedup_kept_matrix_vs_analytic"] = row["analytic"]["kernel_ms"] / row["analytic_kept"]["kernel_ms"]
        rows.append(row)
    print(json.dumps({"mode": "jacstudy", "dtype": "f64", "data": "synthetic", "kernel": "group kernels",
                      "rows": rows}), flush=True)


def bench_sweep(args, torch, dev, chem, synth):
    """Accuracy against cost over tolerance and substep (the paper's
    substep-by-tolerance study, Sec. 3.1): flame-box states of G(10,25,3) on the
    GPU for rtol in {1e-6, 1e-8, 1e-10} and dt in {1e-7, 1e-6, 1e-5} s; the
    error is measured on a strided sample against the oracle at rtol 1e-12,
    atol 1e-20."""
    import oracle
    golden = os.path.join(ROOT, "tests", "golden")
    w = synth.config_workload(2, golden, shape=(256, 4, 4))
    n = w.n_cells
    sub = np.arange(0, n, n // 48)
    gm = chem.Mechanism(w.mech.to_text())
    gm.set_options(q_max=args.q_max, kernel=KERNEL_CODES[args.kernel])
    om = oracle.Mech(w.mech.to_text())
    T0 = torch.tensor(w.T, device=dev)
    Y0 = torch.tensor(w.Y, device=dev)
    rows = []
    for dt in (1e-7, 1e-6, 1e-5):
        print(f"sweep: truth for dt {dt:g} on {sub.size} cells", file=sys.stderr, flush=True)
        Tt, Yt, _ = om.integrate(w.T[sub], w.Y[:, sub], w.p, dt, 1e-12, 1e-20, nthreads=oracle.max_threads())
        for rtol in (1e-6, 1e-8, 1e-10):
            T, Y = T0.clone(), Y0.clone()
            gm.integrate(T, Y, w.p, dt, rtol, 1e-12)                      # warm-up
            T.copy_(T0)
            Y.copy_(Y0)
            st = gm.integrate(T, Y, w.p, dt, rtol, 1e-12)
            Tg, Yg = T.cpu().numpy()[sub], Y.cpu().numpy()[:, sub]
            rows.append({"dt": dt, "rtol": rtol, "kernel_ms": st["wall_ms"], "cells_per_s": n / (st["wall_ms"] * 1e-3),
                         "steps_per_cell": st["n_steps_total"] / n, "failed_cells": st["n_cells_failed"],
                         "max_rel_dT_vs_truth": float((np.abs(Tg - Tt) / Tt).max()),
                         "max_abs_dY_vs_truth": float(np.abs(Yg - Yt).max())})
            print(f"sweep: dt {dt:g} rtol {rtol:g}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"mode": "sweep", "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"flame box 256x4x4 = {n} cells of G(10,25,3,seed 1), atol 1e-12; "
                                             f"error on {sub.size} strided cells"},
                      "rows": rows}), flush=True)


def bench_serve(args, torch, dev, chem, synth):
    """The serving workload: Poisson arrivals at --rate req/s over --duration s
    of box-solve requests, each drawing G(10,25,3,s1) or G(53,325,4,s2) with
    p = --mix (0.5) and a cubic box of edge log-uniform in 8..64 cells (capped at
    --max-box-cells when given), T, Y and dt as in the uneven-box workload,
    served under an HBM budget of --budget-gb.  A request's cells are drawn
    when it arrives.  The host keeps at most --queue-gb of request state
    waiting for the server; arrivals beyond that are refused at the door and
    counted.  The run stops at --wall seconds; requests still queued or on the
    GPU then are counted, not waited for.  Latency is trace arrival to results
    on the host."""
    mechs_ = [synth.config_mechanism(2), synth.config_mechanism(3)]
    handles = [chem.Mechanism(m.to_text()) for m in mechs_]
    for h in handles:
        # FP32 LU where a kernel family has it: the group kernels of G(53,325,4); G(10,25,3)
        # stays on the lane-per-cell kernels, which keep the whole 11x11 matrix in FP64 registers
        lane = h.N <= LANE_MAX_N
        h.set_options(q_max=args.q_max, lu_fp32=int(args.lu_fp32 and not lane), jac_reuse=int(args.jac_reuse),
                      kernel=KERNEL_CODES[args.kernel] if lane or args.kernel != "lane" else 0, ir_max=args.ir_max)
    arrivals = synth.poisson_trace(1005, args.rate, args.duration)
    pick = (np.random.default_rng(1005).random(arrivals.size) < args.mix).astype(int)
    srv = chem.Server(int(args.budget_gb * (1 << 30)), streams=4)
    queue_cap = args.queue_gb * (1 << 30)
    pending = {}                  # id -> (arrival s, cells, bytes)
    lat, lat_by = [], {0: [], 1: []}
    cells_by = {0: 0, 1: 0}
    cells_done = accepted = refused = 0
    held = 0.0
    t0 = time.perf_counter()
    next_report = 10.0
    i = 0
    while True:
        now = time.perf_counter() - t0
        if now >= args.wall or (i >= arrivals.size and not pending):
            break
        while i < arrivals.size and arrivals[i] <= now:
            k = int(pick[i])
            S = mechs_[k].n_species
            # the box's edge is the first draw of its generator (synth.amr_boxes), so a refused
            # request costs no cell generation
            L = int(round(math.exp(np.random.default_rng(10_000 + i).uniform(math.log(8), math.log(64)))))
            n_est = L ** 3 if args.max_box_cells is None else min(L ** 3, args.max_box_cells)
            nbytes = 8.0 * (S + 1) * n_est
            if held + nbytes > queue_cap:
                refused += 1
            else:
                bx = synth.amr_boxes(mechs_[k], 1, 10_000 + i, max_cells=args.max_box_cells)[0]
                rid = srv.submit(handles[k], bx.T, bx.Y, synth.P_ATM, bx.dt, 1e-8, 1e-12)
                pending[rid] = (arrivals[i], bx.T.size, nbytes, k)
                held += nbytes
                accepted += 1
            i += 1
        for rid in list(pending):
            r = srv.poll(rid)
            if r is not None:
                ta, nc, nbytes, k = pending.pop(rid)
                held -= nbytes
                lt = (time.perf_counter() - t0 - ta) * 1e3
                lat.append(lt)
                lat_by[k].append(lt)
                cells_done += nc
                cells_by[k] += nc
        if now >= next_report:
            print(f"serve: t={now:.0f}s offered {i} accepted {accepted} refused {refused} done {len(lat)} "
                  f"pending {len(pending)} cells done {cells_done}", file=sys.stderr, flush=True)
            next_report += 10.0
        time.sleep(0.0005)
    el = time.perf_counter() - t0
    st = srv.stats()
    unfinished = len(pending)
    print(f"serve: stopping after {el:.1f} s with {unfinished} requests unfinished", file=sys.stderr, flush=True)

    def q(v, p_):
        return float(np.percentile(v, p_)) if v else None
    print(json.dumps({
        "mode": "serve", "metric": METRIC, "value": cells_done / el, "unit": "cells/s", "n_gpus": 1,
        "dtype": "f64+f32lu" if args.lu_fp32 else "f64",
        "latency_ms": {"p50": q(lat, 50), "p99": q(lat, 99), "what": "trace arrival to results on the host, "
                       "completed requests only"},
        "latency_ms_by_mechanism": {"G(10,25,3)": {"n": len(lat_by[0]), "p50": q(lat_by[0], 50), "p99": q(lat_by[0], 99),
                                                   "cells": cells_by[0]},
                                    "G(53,325,4)": {"n": len(lat_by[1]), "p50": q(lat_by[1], 50), "p99": q(lat_by[1], 99),
                                                    "cells": cells_by[1]}},
        "requests": {"offered": int(i), "trace": int(arrivals.size), "accepted": accepted, "refused_at_door": refused,
                     "completed": len(lat), "unfinished_at_stop": unfinished},
        "config": {"workload": f"Poisson {args.rate:g} req/s over {args.duration:g} s, mechanisms G(10,25,3,s1) | "
                               f"G(53,325,4,s2) p={args.mix:g}, edges log-uniform 8..64"
                               + (", FP32 LU on G(53,325,4) (G(10,25,3) on the FP64 lane-per-cell kernels)"
                                  if args.lu_fp32 else "")
                               + (f" capped at {args.max_box_cells} cells" if args.max_box_cells else "")
                               + (", Newton matrix kept while recent" if args.jac_reuse else ""),
                   "budget_gb": args.budget_gb, "queue_gb": args.queue_gb, "wall_s": args.wall},
        "server": st, "wall_s": el,
    }), flush=True)
    srv.close()   # after the report: closing waits for the tiles the GPU holds


if __name__ == "__main__":
    main()
