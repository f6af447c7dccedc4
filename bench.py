#!/usr/bin/env python3
"""Throughput of the FV + IBM time step on one MI355X.

Default workload: the 3D turbulent channel at Re_tau = 180 on a
192 x 128 x 160 tanh-stretched grid, float32 stencils with float64
residual / refinement (the configuration the headline metric and the HBM
roofline target are quoted on).  One timed step = forward step
(predictor, boundary faces, PPE, CG / refinement, projection) and, once
available, its discrete adjoint with recomputation.

Prints ONE JSON line.  `value` = Mcell-updates/s of the whole job.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E peak

# algorithmic bytes per cell per launch (d = velocity components, s = bytes
# of the velocity type, v = bytes of the solve vectors)
def kernel_bytes(d: int, s: int, v: int, mixed: bool) -> dict:
    return {
        "predictor": 3 * d * s,                 # read u, f_b; write u*
        "ppe_rhs": d * s + 8,                   # read u*; write b (double)
        "residual": 8 + 8 + (4 + 4 if mixed else 8),  # read b, p; write r (+ clear inner iterate)
        "cg_dir": 3 * v,                        # read r, p_old; write p_new
        "cg_update": 5 * v,                     # read p, x, r; write x, r
        "ir_correct": 8 + 4 + 8,                # read p, d; write p
        "project": 2 * d * s + 8,               # read u*, p; write u
        "boundary": 0,
        "ib": 0,
        "adjoint": 0,
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8, help="max |div u| target of the PPE solve")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle sample timed on the host (0 = skip)")
    ap.add_argument("--no-fp64-compare", action="store_true")
    return ap.parse_args()


def make_workload(name):
    import fvib_workloads as W
    if name == "channel":
        return W.channel()
    return W.by_name(name, "full")


def run_gpu(w, precision, steps, warmup, tol):
    import torch
    import fvib_workloads as W
    import paper_2505_23940_amd as F
    g = F.Grid.from_workload(w, precision=precision, poisson_tol=tol, check_every=64)
    u0, fb = W.initial_fields(w)
    u = g.to_u(u0)
    fbt = g.to_u(fb)
    p = g.zeros_p()
    body = kc = None
    if w.body is not None:
        body = torch.tensor(W.body_state0(w), dtype=torch.float64, device=g.device)
        kc = torch.tensor(list(w.body.k) + list(w.body.c), dtype=torch.float64, device=g.device)
    for i in range(warmup):
        g.step(u, p, fbt, body, kc)
        print(f"[bench] warmup {precision} step {i}: {g.last_info()}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    g.timing_enable(True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(u, p, fbt, body, kc)
        infos.append(g.last_info())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] timed {steps} {precision} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)
    timing = g.timing_read()
    g.timing_enable(False)
    return t1 - t0, infos, timing, g


def cpu_baseline(w, budget_s):
    """The oracle as it stands, forward steps on the host cores."""
    import torch
    import fvib_workloads as W
    from oracle import Grid, init_state, make_params, step
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = max(1, min(cores, os.cpu_count() or 1))
    torch.set_num_threads(cores)
    og = Grid(w)
    u0, fb = W.initial_fields(w)
    st = init_state(og, u0, W.body_state0(w))
    pr = make_params(og, fb)
    with torch.no_grad():
        st, _ = step(og, st, pr)                 # warm-up (builds the eigenbases)
        n = 0
        t0 = time.perf_counter()
        while True:
            st, _ = step(og, st, pr)
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    return {"value": w.ncells * n / dt / 1e6, "unit": "Mcell-updates/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n} forward steps of the same workload (float64, exact Poisson solve), "
                      f"{dt:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {a.gpus}); "
              "multi-GPU sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    w = make_workload(a.workload)
    mixed = a.precision == "fp32"
    elapsed, infos, timing, g = run_gpu(w, a.precision, a.steps, a.warmup, a.tol)
    ncell = w.ncells
    mcells = ncell * a.steps / elapsed / 1e6
    s = 4 if mixed else 8
    kb = kernel_bytes(w.dim, s, 4 if mixed else 8, mixed)
    per_kernel = {}
    for name, (ms, n) in timing.items():
        if n == 0:
            continue
        bpl = kb.get(name, 0) * ncell
        avg_us = ms / n * 1e3
        per_kernel[name] = {"launches": n, "total_ms": round(ms, 3), "avg_us": round(avg_us, 2),
                            "GB_s": round(bpl / (avg_us * 1e-6) / 1e9, 1) if bpl else None}
    dom = max(per_kernel.items(), key=lambda kv: kv[1]["total_ms"])[0]
    dom_bytes = kb.get(dom, 0) * ncell
    dom_avg_s = per_kernel[dom]["avg_us"] * 1e-6
    achieved = dom_bytes / dom_avg_s / 1e9 if dom_bytes else 0.0
    cg = [i["cg_iters"] for i in infos]
    ir = [i["ir_iters"] for i in infos]
    out = {
        "metric": "Mcell-updates/s, fwd and fwd+adjoint step (FP32 vs FP64); % HBM roofline",
        "value": round(mcells, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "channel Re_tau=180, 192x128x160 tanh-stretched, laminar + 10% "
                               "seeded noise, uniform driving force" if a.workload == "channel"
                               else a.workload,
                   "cells": ncell, "precision": "fp32 stencils + fp64 residual/refinement"
                   if mixed else "fp64", "step": "forward", "poisson_tol": a.tol,
                   "cg_iters_per_step": float(np.mean(cg)), "ir_sweeps_per_step": float(np.mean(ir)),
                   "div_max": max(i["div_max"] for i in infos)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": dom_bytes, "traffic": None},
        "kernels": per_kernel,
    }
    if not a.no_fp64_compare and mixed:
        e64, inf64, _, _ = run_gpu(w, "fp64", max(2, a.steps // 2), 1, a.tol)
        v64 = ncell * max(2, a.steps // 2) / e64 / 1e6
        out["fp64_value"] = round(v64, 3)
        out["fp32_over_fp64"] = round(mcells / v64, 3)
        out["fp64_cg_iters_per_step"] = float(np.mean([i["cg_iters"] for i in inf64]))
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
