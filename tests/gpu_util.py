"""Helpers shared by the GPU parity tests: run the same seeded workload
through libfvib and through the CPU oracle and compare."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import fvib_workloads as W


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs an MI355X")


def fvib():
    import paper_2505_23940_amd as F   # raises if libfvib.so is missing
    F.lib()
    return F


def make_grid(w, precision=None, **kw):
    F = fvib()
    args = {}
    if precision is not None:
        args["precision"] = precision
    args.update(kw)
    return F.Grid.from_workload(w, **args)


def rel_l2(a_list, b_list):
    num = sum(float(np.sum((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2))
              for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in b_list)
    return (num / max(den, 1e-300)) ** 0.5


def gpu_rollout(w, steps, precision="fp64", tol=1e-12, u0=None, body0=None, fb=None, kc=None,
                **kw):
    """Run `steps` steps on the GPU; returns dict of numpy results."""
    g = make_grid(w, precision=precision, poisson_tol=tol, **kw)
    if u0 is None or fb is None:
        uu, ff = W.initial_fields(w)
        u0 = uu if u0 is None else u0
        fb = ff if fb is None else fb
    u = g.to_u(u0)
    fbt = g.to_u(fb)
    p = g.zeros_p()
    body = None
    kct = None
    if w.body is not None:
        b0 = W.body_state0(w) if body0 is None else body0
        body = torch.tensor(b0, dtype=torch.float64, device=g.device)
        kvec = np.concatenate([np.asarray(w.body.k), np.asarray(w.body.c)]) if kc is None else kc
        kct = torch.tensor(kvec, dtype=torch.float64, device=g.device)
    forces, infos = [], []
    for _ in range(steps):
        g.step(u, p, fbt, body, kct)
        info = g.last_info()
        infos.append(info)
        forces.append(info["force"])
    torch.cuda.synchronize()
    out = {"u": [x.double().cpu().numpy() for x in u], "p": p.cpu().numpy(),
           "forces": np.asarray(forces), "infos": infos, "grid": g}
    out["body"] = body.cpu().numpy() if body is not None else None
    return out


def oracle_rollout(w, steps, u0=None, body0=None, fb=None, kc=None):
    from oracle import Grid, init_state, make_params, rollout
    og = Grid(w)
    if u0 is None or fb is None:
        uu, ff = W.initial_fields(w)
        u0 = uu if u0 is None else u0
        fb = ff if fb is None else fb
    b0 = W.body_state0(w) if body0 is None else body0
    st = init_state(og, u0, b0)
    k = c = None
    if kc is not None:
        k = torch.tensor(kc[:3], dtype=torch.float64)
        c = torch.tensor(kc[3:], dtype=torch.float64)
    pr = make_params(og, fb, k=k, c=c)
    with torch.no_grad():
        st, Fh, _ = rollout(og, st, pr, steps)
    return {"u": [x.numpy() for x in st["u"]], "p": st["p"].numpy(), "forces": Fh.numpy(),
            "body": st["body"].numpy(), "grid": og}


def gauge(p):
    return p - p.mean()
