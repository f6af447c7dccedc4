#!/usr/bin/env python3
"""Throughput of the FV + IBM time step and its discrete adjoint on one MI355X.

Default workload: the 3D turbulent channel at Re_tau = 180 on a
192 x 128 x 160 tanh-stretched grid (x periodic, y walls, z periodic),
laminar profile plus 10% seeded noise, driven by a uniform body force;
float32 stencils with float64 residual / refinement.  One timed step is the
whole hot path: the forward step (predictor with forcing, boundary faces,
PPE right-hand side, refinement with the inner solve, projection) and its
discrete adjoint, run as a differentiable rollout (checkpoint every
--ckpt steps, recomputation inside segments) whose loss is the mean wall
shear stress after the last step; the gradient is taken with respect to
the body-force field.

Prints ONE JSON line; `value` = Mcell-updates/s of forward + adjoint.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E
# In the timed region one launch in TIMING_EVERY of the dominant class
# carries timestamp events (each idles the device for a few microseconds).
TIMING_EVERY = 4
MFMA_PEAK_TFS = {"fp32": 157.3, "fp64": 78.6}   # dense matrix-core peaks


def kernel_cost(d: int, s: int, mixed: bool, n: tuple, solver: str = "fdm"):
    """Algorithmic cost per launch per cell: ("bytes", B) or ("flops", F).

    d = velocity components, s = bytes per velocity value."""
    v = 4 if mixed else 8          # inner-solve vector type
    # 3D fast diagonalisation: the projection also stores the gauged pressure
    pg = 8 if (d == 3 and solver == "fdm") else 0
    return {
        "predictor": ("bytes", 3 * d * s),                 # read u, f_b; write u*
        "ppe_rhs": ("bytes", d * s + 8),                   # read u*; write b
        "rhs_res": ("bytes", d * s + 8 + 8 + v),           # read u*, p; write b, r
        "residual": ("bytes", 8 + 8 + v),                  # read b, p; write r
        "cg_dir": ("bytes", 3 * v),                        # read r, p_old; write p_new
        "cg_update": ("bytes", 5 * v),                     # read p, x, r; write x, r
        "ir_correct": ("bytes", 8 + v + 8),                # read p, d; write p
        "project": ("bytes", 2 * d * s + 8 + pg),          # read u*, p; write u (and p)
        "adj_momentum": ("bytes", 5 * d * s),              # read u, ustar_bar; write ubar; rw fbbar
        "adj_rhs": ("bytes", d * s + 8),                   # read ubar; write G^T ubar
        "adj_rhs_res": ("bytes", d * s + 8 + 8 + v),       # read ubar, mu; write y, r
        "adj_ustar": ("bytes", 2 * d * s + 8),             # read ubar, mu; write ustar_bar
        "fdm_x": ("flops", 2 * n[0]),                      # dense contraction along x
        "fdm_y": ("flops", 2 * n[1]),
        "fdm_z": ("flops", 2 * n[2]),
        # last axis forward + division + inverse in one launch
        "fdm_last": ("flops", 4 * n[2 if d == 3 else 1]),
        "fft": ("bytes", 2 * v),                           # read and write one vector
        "fft_acc": ("bytes", v + 16),                      # read d; read and write p
        # subgrid model (all passes of one step): nu_t (read u, write nu_t),
        # stress divergence (read u, nu_t, f_b; write g)
        "les": ("bytes", (d + 1) * s + (2 * d + 1 + d) * s),
        # its adjoint: nu_t again; sites (read u, gbar, nu_t; write 3 + 1 + 6);
        # cells (read nbar, 3 q, u; rw 3 w; write 3 s); edges (rw 3 p; read
        # 3 s); faces (read 3 w, 3 p, gbar; rw ubar, fbbar)
        "adj_les": ("bytes", (d + 1) * s + (2 * d + 1 + 10) * s + (1 + 3 + d + 6 + 3) * s
                    + 9 * s + (3 + 3 + 1 + 4) * s),
    }


def other_workloads(precision, tol, solver, steps=20):
    """Mcell-updates/s of the other workloads at their full sizes, same
    precision and solver: forward + adjoint (K = 1) and forward only, over
    `steps` steps after a warm-up of the same length.  Besides the five
    workloads: the channel with third-order Runge-Kutta steps, the channel
    with a roughness cube on its floor, and the 2-DOF VIV case strongly
    coupled (sub-iterations to a coupling error of 1e-5, at most 100)."""
    import fvib_workloads as W
    res = {}
    cases = [(n, W.by_name(n, "full"), None, None)
             for n in ("tgv2d", "tgv3d", "cylinder", "viv", "wmles")]
    cases.append(("channel_rk3", W.channel(), "rk3", None))
    cases.append(("channel_cube", W.channel_cube(), None, None))
    wv = W.viv(dof=2, coupling_iters=100, coupling_tol=1e-5)
    cases.append(("viv_2dof_strong", wv, None, (100, 1e-5)))
    for name, w, scheme, coupling in cases:
        g, ut, fbt, body, kc = setup(w, precision, tol, solver)
        fwd_adj_pass(g, w, ut, fbt, body, kc, steps, 1, scheme, coupling)
        el, _ = timed(lambda: fwd_adj_pass(g, w, ut, fbt, body, kc, steps, 1, scheme, coupling))
        elf, info = timed(lambda: fwd_pass(g, ut, fbt, body, kc, steps, scheme, coupling))
        g.check_infos(info, "forward step")
        res[name] = {"cells": w.ncells, "steps": steps,
                     "fwd_adj_value": round(w.ncells * steps / el / 1e6, 3),
                     "fwd_value": round(w.ncells * steps / elf / 1e6, 3)}
        if coupling is not None:
            from paper_2505_23940_amd import parse_info
            recs = parse_info(info)
            res[name]["coupling_iters_per_step"] = round(
                sum(r["coupling_iters"] for r in recs) / len(recs), 2)
        print(f"[bench] {name}: fwd+adj {res[name]['fwd_adj_value']} Mcell/s, "
              f"fwd {res[name]['fwd_value']} Mcell/s", file=sys.stderr, flush=True)
        del g
    return res


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--solver", default="fdm", choices=["fdm", "cg"])
    ap.add_argument("--ckpt", type=int, default=1, help="checkpoint interval of the rollout")
    ap.add_argument("--tol", type=float, default=1e-8, help="max |div u| target of the PPE solve")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle sample timed on the host (0 = skip)")
    ap.add_argument("--no-extra", action="store_true", help="skip the forward-only and fp64 runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def make_workload(name):
    import fvib_workloads as W
    if name == "channel":
        return W.channel()
    return W.by_name(name, "full")


def setup(w, precision, tol, solver):
    import torch
    import fvib_workloads as W
    import paper_2505_23940_amd as F
    g = F.Grid.from_workload(w, precision=precision, poisson_tol=tol, check_every=64,
                             solver=solver)
    u0, fb = W.initial_fields(w)
    ut = g.to_u(u0)
    fbt = g.to_u(fb)
    body = torch.tensor(W.body_state0(w), dtype=torch.float64, device=g.device)
    kcv = (list(w.body.k) + list(w.body.c)) if w.body is not None else [0.0] * 6
    kc = torch.tensor(kcv, dtype=torch.float64, device=g.device)
    return g, ut, fbt, body, kc


def fwd_adj_pass(g, w, ut, fbt, body, kc, steps, ckpt, scheme=None, coupling=None):
    """Differentiable rollout of `steps` steps, loss, backward."""
    from paper_2505_23940_amd.rollout import rms_lift, rollout, wall_shear
    fb = [x.detach().clone().requires_grad_(True) for x in fbt]
    kcr = kc.detach().clone().requires_grad_(True)
    uS, bS, Fh, _ = rollout(g, [x.clone() for x in ut], fb, kcr, body.clone(), steps,
                            ckpt_every=ckpt, scheme=scheme, coupling=coupling)
    if w.body is not None:
        J = rms_lift(g, Fh)
    elif w.bc[1] == ["noslip", "noslip"]:
        J = wall_shear(g, uS[0])
    else:
        # no loss of the paper's applies (periodic box): seed the adjoint
        # with a unit adjoint of the final streamwise velocity
        import torch
        torch.autograd.backward(uS[0], grad_tensors=torch.ones_like(uS[0]))
        return torch.zeros(())
    J.backward()
    return J


def fwd_pass(g, ut, fbt, body, kc, steps, scheme=None, coupling=None):
    """Forward steps in place, enqueued back to back (one step record per
    step, statuses checked after the last)."""
    import torch
    from paper_2505_23940_amd import INFO_DOUBLES
    u = [x.clone() for x in ut]
    p = g.zeros_p()
    b = body.clone()
    info = torch.zeros((steps, INFO_DOUBLES), dtype=torch.float64, device=g.device)
    g.defer_status(True)
    try:
        for n in range(steps):
            if coupling is not None:
                omega = torch.zeros(6, dtype=torch.float64, device=g.device)
                g.step(u, p, fbt, b, kc, info=info[n], coupling=coupling, omega=omega)
            else:
                g.step(u, p, fbt, b, kc, info=info[n], scheme=scheme)
    finally:
        g.defer_status(False)
    return info


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def host_cpu():
    """Model name and logical CPU count of the host (as lscpu / nproc show)."""
    model = "?"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def copy_bandwidth(device, nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: the best of `reps` device-to-device copies of
    nbytes (read + write counted), timed with events on the copy's stream."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        best = t if best is None else min(best, t)
    del src, dst
    return 2 * nbytes / best / 1e9


def cpu_baseline(w, budget_s):
    """The oracle as it stands, forward + adjoint like `value`: a rollout
    with autograd through every step (float64, exact Poisson solves), the
    same loss, backward to the body-force field; 2 warm-up steps, then 5
    timed steps, then 20 if the budget allows (the longer run is reported)."""
    import torch
    import fvib_workloads as W
    from oracle import Grid, init_state, make_params
    from oracle.step import rms_lift, rollout, wall_shear
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = max(1, min(cores, os.cpu_count() or 1))
    torch.set_num_threads(cores)
    og = Grid(w)
    u0, fb = W.initial_fields(w)

    def fwd_adj(n):
        st = init_state(og, u0, W.body_state0(w))
        pr = make_params(og, fb)
        pr["fb"] = [x.clone().requires_grad_(True) for x in pr["fb"]]
        st, Fh, _ = rollout(og, st, pr, n)
        J = wall_shear(og, st["u"]) if w.body is None else rms_lift(og, Fh)
        J.backward()

    fwd_adj(2)                                    # warm-up (builds the eigenbases)
    n = 5
    t0 = time.perf_counter()
    fwd_adj(n)
    dt = time.perf_counter() - t0
    if dt * 5.0 < budget_s:
        n = 20
        t0 = time.perf_counter()
        fwd_adj(n)
        dt = time.perf_counter() - t0
    model, nproc = host_cpu()
    return {"value": round(w.ncells * n / dt / 1e6, 3), "unit": "Mcell-updates/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n}-step rollout of the same workload, forward + autograd adjoint "
                      f"(float64, exact Poisson solve by per-axis eigen-decomposition, loss "
                      f"and backward to the body force as in `value`) in {dt:.1f} s after a "
                      f"2-step warm-up",
            "host": {"nproc": nproc, "cpu": model}}


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "hbm_traffic_channel_192x128x160_fp32.md")


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE, WRITE_SIZE, calibrated); None if absent or if a
    source file of the class changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        entry = json.loads(block).get(kernel_class)
    except (OSError, IndexError, ValueError):
        return None
    if not entry:
        return None
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2505_23940_amd", "csrc")
    for name, digest in entry["sources"].items():
        try:
            cur = hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest()[:16]
        except OSError:
            return None
        if cur != digest:
            return None
    return entry["traffic_bytes"]


def step_bytes(table, w, mixed, solver, nsteps):
    """Algorithmic HBM bytes of one step summed over the kernel classes of a
    timed pass of `nsteps` steps (launch counts of that pass; matrix-core
    contractions count their one read and one write of the vector)."""
    s = 4 if mixed else 8
    v = 4 if mixed else 8
    cost = kernel_cost(w.dim, s, mixed, w.n, solver)
    total, unmodeled = 0.0, []
    for name, row in table.items():
        if name not in cost:
            unmodeled.append(name)
            continue
        kind, per_cell = cost[name]
        per_cell = per_cell if kind == "bytes" else 2 * v
        total += per_cell * w.ncells * row["launches"]
    return total / nsteps, sorted(unmodeled)


def dominant(table, w, mixed, solver):
    """Kernel class with a cost model and the largest total time."""
    cost = kernel_cost(w.dim, 4 if mixed else 8, mixed, w.n, solver)
    return max((k for k in table if k in cost), key=lambda k: table[k]["total_ms"])


def roofline(timing, w, precision, mixed, solver, dom=None):
    ncell = w.ncells
    s = 4 if mixed else 8
    cost = kernel_cost(w.dim, s, mixed, w.n, solver)
    table = {}
    for name, (ms, nl) in timing.items():
        if nl == 0:
            continue
        avg_us = ms / nl * 1e3
        row = {"launches": nl, "total_ms": round(ms, 3), "avg_us": round(avg_us, 2)}
        if name in cost:
            kind, per_cell = cost[name]
            amount = per_cell * ncell
            if kind == "bytes":
                row["GB_s"] = round(amount / (avg_us * 1e-6) / 1e9, 1)
            else:
                row["TFLOP_s"] = round(amount / (avg_us * 1e-6) / 1e12, 2)
        table[name] = row
    if dom is None:
        dom = max((k for k in table if k in cost), key=lambda k: table[k]["total_ms"])
    kind, per_cell = cost[dom]
    amount = per_cell * ncell
    avg_s = table[dom]["avg_us"] * 1e-6
    if kind == "bytes":
        ach = amount / avg_s / 1e9
        rl = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
              "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
              "bytes_per_launch": amount, "traffic": None}
    else:
        ach = amount / avg_s / 1e12
        pk = MFMA_PEAK_TFS["fp32" if mixed else "fp64"]
        rl = {"bound": "mfma", "kernel": dom, "achieved": round(ach, 2), "peak": pk,
              "unit": "TFLOP/s", "frac": round(ach / pk, 4), "flops_per_launch": amount,
              "traffic": None}
    return rl, table


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); "
              "sharding the step across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    w = make_workload(a.workload)
    mixed = a.precision == "fp32"
    ncell = w.ncells
    g, ut, fbt, body, kc = setup(w, a.precision, a.tol, a.solver)
    # warm-up (not timed), then a pass of the same length with every kernel
    # class bracketed by HIP events -> per-class table and dominant kernel
    nw = max(1, a.warmup)
    fwd_adj_pass(g, w, ut, fbt, body, kc, nw, a.ckpt)
    # the table pass has the timed run's length, so its launch counts per
    # step (refinement sweeps included) are those of the timed run
    g.timing_enable(True)
    fwd_adj_pass(g, w, ut, fbt, body, kc, a.steps, a.ckpt)
    _, table = roofline(g.timing_read(), w, a.precision, mixed, a.solver)
    for name, (ms, nl) in g.timing_read(skipped=True).items():
        if nl and name in table:
            table[name]["skipped"] = nl
    g.timing_enable(False)
    dom = dominant(table, w, mixed, a.solver)
    print(f"[bench] warmup done ({nw} + {a.steps} steps); dominant kernel {dom}",
          file=sys.stderr, flush=True)
    # timed region: only a sample of the dominant class's launches carries
    # events, so the run stays close to an untimed one
    g.timing_enable(True, classes=[dom], every=TIMING_EVERY)
    el, J = timed(lambda: fwd_adj_pass(g, w, ut, fbt, body, kc, a.steps, a.ckpt))
    timing = g.timing_read()
    skipped = g.timing_read(skipped=True)
    g.timing_enable(False)
    print(f"[bench] fwd+adj {a.steps} steps in {el:.3f} s (J = {float(J.detach()):.6g})",
          file=sys.stderr, flush=True)
    rl, _ = roofline(timing, w, a.precision, mixed, a.solver, dom)
    # launches of speculative refinement sweeps that found the solve
    # converged return at once; they are left out of the average above
    rl["skipped_launches"] = skipped[dom][1]
    if a.workload == "channel" and mixed:
        rl["traffic"] = measured_traffic(dom)
    rl["timed_launches"] = timing[dom][1]
    rl["sampled_every"] = TIMING_EVERY
    value = ncell * a.steps / el / 1e6
    out = {
        "metric": "Mcell-updates/s, fwd and fwd+adjoint step (FP32 vs FP64); % HBM roofline",
        "value": round(value, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(el / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": ("channel Re_tau=180, 192x128x160 tanh-stretched, laminar + 10% "
                                "seeded noise, uniform driving force" if a.workload == "channel"
                                else a.workload),
                   "cells": ncell, "step": "forward + discrete adjoint (checkpointed rollout)",
                   "precision": ("fp32 stencils + fp64 residual/refinement" if mixed else "fp64"),
                   "poisson": a.solver, "poisson_tol": a.tol, "ckpt_every": a.ckpt},
        "roofline": rl,
        "kernels_table_pass": table,
    }
    sb, unmod = step_bytes(table, w, mixed, a.solver, a.steps)
    ach = sb / (el / a.steps) / 1e9
    out["roofline_step"] = {"bound": "hbm", "model_bytes_per_step": round(sb),
                            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4),
                            "launch_counts": f"kernel table pass ({a.steps} steps)",
                            "classes_without_model": unmod}
    if a.solver == "fdm" and "residual" in table:
        # refinement sweeps per Poisson solve (forward and adjoint, two per
        # step) from the table pass: residual launches that ran; the inner
        # solve is direct (no CG iterations)
        res = table["residual"]
        out["ir_sweeps_per_solve"] = round((res["launches"] - res.get("skipped", 0))
                                           / (2 * a.steps), 3)
        out["inner_iters_per_sweep"] = 0
    if not a.no_extra:
        if a.ckpt != 20 and a.steps >= 20:
            el20, _ = timed(lambda: fwd_adj_pass(g, w, ut, fbt, body, kc, a.steps, 20))
            out["ckpt20_value"] = round(ncell * a.steps / el20 / 1e6, 3)
            print(f"[bench] fwd+adj K=20 {a.steps} steps in {el20:.3f} s", file=sys.stderr,
                  flush=True)
        gi = g
        el_f, info = timed(lambda: fwd_pass(gi, ut, fbt, body, kc, a.steps))
        gi.check_infos(info, "forward step")
        from paper_2505_23940_amd import parse_info
        infos = parse_info(info)
        infos = infos if isinstance(infos, list) else [infos]
        out["fwd_value"] = round(ncell * a.steps / el_f / 1e6, 3)
        out["fwd_ir_sweeps_per_step"] = float(np.mean([i["ir_iters"] for i in infos]))
        out["fwd_div_max"] = max(i["div_max"] for i in infos)
        print(f"[bench] fwd {a.steps} steps in {el_f:.3f} s", file=sys.stderr, flush=True)
        if mixed:
            g64, u64, f64, b64, k64 = setup(w, "fp64", a.tol, a.solver)
            n64 = max(2, a.steps // 2)
            fwd_adj_pass(g64, w, u64, f64, b64, k64, 1, a.ckpt)
            el64, _ = timed(lambda: fwd_adj_pass(g64, w, u64, f64, b64, k64, n64, a.ckpt))
            out["fp64_value"] = round(ncell * n64 / el64 / 1e6, 3)
            out["fp32_over_fp64"] = round(value / out["fp64_value"], 3)
            print(f"[bench] fp64 fwd+adj {n64} steps in {el64:.3f} s", file=sys.stderr, flush=True)
    if not a.no_extra and a.workload == "channel":
        out["other_workloads"] = other_workloads(a.precision, a.tol, a.solver)
    # the fractions against a measured copy as well as against the peak
    cb = copy_bandwidth(g.device)
    for key in ("roofline", "roofline_step"):
        r = out.get(key)
        if r and r.get("unit") == "GB/s":
            r["copy_GB_s"] = round(cb, 1)
            r["frac_of_copy"] = round(r["achieved"] / cb, 4)
    if a.copy_probe:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device=g.device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
