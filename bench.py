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
C_EXP = 20.0                     # FP64 flops charged per exp/log (software sequence on gfx950)


def flop_model(S: int, R: int, n_tb: int, n_falloff: int):
    """Algorithmic FP64 flops per event of the method:
    per rhs evaluation, per Jacobian + Newton-matrix + LU (one per attempt),
    per Newton iteration (residual, solve, norm)."""
    N = S + 1
    nnz = 4 * R                                   # nonzeros of nu (<= 2 + 2 per reaction)
    f_rhs = 32 * S + S * C_EXP + R * (26 + 2 * C_EXP) + n_falloff * (8 + C_EXP) + n_tb + 2 * nnz
    f_jac = 26 * R + 12 * nnz + 13 * S * S + 10 * N
    f_lu = 2.0 * N ** 3 / 3.0
    f_attempt = f_jac + 2 * N * N + f_lu + 40 * N
    f_newton = 2 * N * N + 7 * N
    return f_rhs, f_attempt, f_newton


def algorithmic_flops(stats, S, R, n_tb, n_falloff):
    f_rhs, f_attempt, f_newton = flop_model(S, R, n_tb, n_falloff)
    return stats["n_rhs"] * f_rhs + stats["n_attempts"] * f_attempt + stats["n_newton_iters"] * f_newton


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shape", type=str, default="256,64,64", help="box nx,ny,nz (x = flame axis)")
    ap.add_argument("--cpu-sample", type=int, default=2048, help="cells in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--q-max", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(cells are independent; see DESIGN.md for how the work would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_05974_amd import chem, synth

    dev = torch.device("cuda:0")
    shape = tuple(int(v) for v in args.shape.split(","))
    w = synth.config_workload(2, os.path.join(ROOT, "tests", "golden"), shape=shape)
    m = w.mech
    n = w.n_cells
    n_tb = sum(r.kind == 1 for r in m.reactions)
    n_fo = sum(r.kind == 2 for r in m.reactions)
    gm = chem.Mechanism(m.to_text())
    gm.set_options(q_max=args.q_max)
    T0 = torch.tensor(w.T, dtype=torch.float64, device=dev)
    Y0 = torch.tensor(w.Y, dtype=torch.float64, device=dev)
    T = torch.empty_like(T0)
    Y = torch.empty_like(Y0)

    def step():
        T.copy_(T0)
        Y.copy_(Y0)
        return gm.integrate(T, Y, w.p, w.dt, w.rtol, w.atol)

    for i in range(args.warmup):
        st = step()
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
    flops = algorithmic_flops(st, m.n_species, m.n_reactions, n_tb, n_fo)
    k_ms = float(np.mean(kernel_ms))
    achieved = flops / (k_ms * 1e-3) / 1e12
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"planar flame box {shape[0]}x{shape[1]}x{shape[2]} = {n} cells, mechanism "
                         f"G(10,25,3,seed 1), T 300->2200 K tanh profile, dt {w.dt:g} s, rtol {w.rtol:g}, "
                         f"atol {w.atol:g}, p 1 atm, constant-pressure adiabatic, BDF q<={args.q_max}"),
            "cells": n, "species": m.n_species, "reactions": m.n_reactions,
            "parallelism": "none (1 GPU)",
        },
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "one whole-box chem_integrate call"},
        "integration": {"steps_per_cell": st["n_steps_total"] / n, "attempts_per_cell": st["n_attempts"] / n,
                        "newton_per_cell": st["n_newton_iters"] / n, "max_steps_cell": st["n_steps_max"],
                        "failed_cells": st["n_cells_failed"]},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
            "kernel": "integrate_kernel<16>", "kernel_ms": k_ms, "flops_per_launch": flops,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(w, T, Y, args)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, Tg, Yg, args):
    """The oracle on a strided sample of the same box, all host threads."""
    import oracle
    n = w.n_cells
    k = max(1, min(args.cpu_sample, n))
    idx = np.unique(np.linspace(0, n - 1, k).astype(np.int64))
    om = oracle.Mech(w.mech.to_text())
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    To, Yo, so = om.integrate(w.T[idx], w.Y[:, idx], w.p, w.dt, w.rtol, w.atol, q_max=args.q_max,
                              nthreads=threads)
    el = time.perf_counter() - t0
    Tgs = Tg.cpu().numpy()[idx]
    Ygs = Yg.cpu().numpy()[:, idx]
    acc = {"vs": "CPU oracle, same inputs and settings", "cells": int(idx.size),
           "max_abs_dY": float(np.abs(Ygs - Yo).max()),
           "max_rel_dT": float((np.abs(Tgs - To) / To).max()),
           "p99_abs_dY": float(np.percentile(np.abs(Ygs - Yo).max(axis=0), 99))}
    base = {"value": idx.size / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{idx.size} cells evenly strided over the {n}-cell box ({el:.1f} s)"}
    return base, acc


if __name__ == "__main__":
    main()
