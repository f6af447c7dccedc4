"""Workload-level gates on the GPU (through the C ABI):

* 3D Taylor-Green vortex 128^3, 500 steps: kinetic energy and enstrophy
  histories of the float32-mixed path against the float64 path;
* VIV at 256 x 128 (the reduced variant of the 1024 x 512 workload), 400
  steps, float64: dJ/dk and dJ/dc of the RMS lift from the adjoint rollout
  against central differences of the GPU forward (the point classes of the
  perturbed runs are checked to equal the base run's at every step, so the
  differences are those of the frozen-mask map) and against the oracle's
  autograd;
* cylinder 512 x 256, 5000 steps, float32-mixed: drag and lift histories
  (reported; the drag is checked to be finite and positive).  The force is
  the spreading sum of Eq. 20 weighted by the marker volumes (F = rho sum_k
  q_k dV_k); its absolute value depends on that reading and is not compared
  with the paper's figures.
"""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from gpu_util import make_grid, need_gpu

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _energy_enstrophy(g, u, h):
    """E = (1/2V) sum |u|^2 dv and Z = (1/2V) sum |omega|^2 dv on a uniform
    periodic grid, the vorticity on the cell edges (float64 reductions)."""
    a, b, c = (x.double() for x in u)     # (z, y, x) arrays, faces = cell index
    E = 0.5 * float((a * a + b * b + c * c).mean())
    # omega_x = dw/dy - dv/dz on x-edges, etc. (backward differences)
    wx = (c - torch.roll(c, 1, 1)) / h - (b - torch.roll(b, 1, 0)) / h
    wy = (a - torch.roll(a, 1, 0)) / h - (c - torch.roll(c, 1, 2)) / h
    wz = (b - torch.roll(b, 1, 2)) / h - (a - torch.roll(a, 1, 1)) / h
    Z = 0.5 * float((wx * wx + wy * wy + wz * wz).mean())
    return E, Z


def _tgv_history(w, precision):
    g = make_grid(w, precision=precision, poisson_tol=1e-12 if precision == "fp64" else 1e-8)
    u0, fb = W.initial_fields(w)
    u, p = g.to_u(u0), g.zeros_p()
    h = 2 * np.pi / w.n[0]
    hist = [_energy_enstrophy(g, u, h)]
    for _ in range(w.steps):
        g.step(u, p, None)
        hist.append(_energy_enstrophy(g, u, h))
    return np.asarray(hist)


def test_tgv3d_fp32_energy_enstrophy_history():
    need_gpu()
    w = W.tgv3d()                 # 128^3, 500 steps, dt 1e-3, Re 1600
    h64 = _tgv_history(w, "fp64")
    h32 = _tgv_history(w, "fp32")
    dE = float(np.abs(h32[:, 0] - h64[:, 0]).max() / np.abs(h64[:, 0]).max())
    dZ = float(np.abs(h32[:, 1] - h64[:, 1]).max() / np.abs(h64[:, 1]).max())
    print(f"TGV 128^3, 500 steps: E {h64[0, 0]:.6f} -> {h64[-1, 0]:.6f}, Z {h64[0, 1]:.6f} -> "
          f"{h64[-1, 1]:.6f}; float32 vs float64 max rel: E {dE:.2e}, Z {dZ:.2e}")
    assert dE <= 1e-5 and dZ <= 1e-5
    # viscous decay: the energy falls monotonically
    assert np.all(np.diff(h64[:, 0]) < 0)


def _viv_J(w, k, c, precision="fp64", classes=None):
    """Forward run; returns J (RMS lift) and, if asked, the point classes of
    every step."""
    g = make_grid(w, precision=precision, poisson_tol=1e-12)
    u0, fb = W.initial_fields(w)
    u, fbt, p = g.to_u(u0), g.to_u(fb), g.zeros_p()
    body = torch.tensor(W.body_state0(w), dtype=F64, device=g.device)
    kc = torch.tensor(np.concatenate([k, c]), dtype=F64, device=g.device)
    Fh = torch.zeros((w.steps, 8), dtype=F64, device=g.device)
    cls = [] if classes is not None else None
    for n in range(w.steps):
        if cls is not None:
            cc = g.test_ib_classify(body.clone())
            cls.append([x.cpu().numpy() for x in cc])
        g.step(u, p, fbt, body, kc, info=Fh[n])
    J = g.loss_rms_lift(Fh, 8, 5)
    torch.cuda.synchronize()
    return float(J[0]), cls


def test_viv_spring_gradients_fd_and_oracle():
    need_gpu()
    from paper_2505_23940_amd.rollout import rms_lift, rollout
    w = W.by_name("viv", "small")
    w.steps = 400
    k0 = np.asarray(w.body.k, dtype=np.float64)
    c0 = np.asarray(w.body.c, dtype=np.float64)
    # adjoint rollout on the GPU
    g = make_grid(w, precision="fp64", poisson_tol=1e-12)
    u0, fb = W.initial_fields(w)
    kct = torch.tensor(np.concatenate([k0, c0]), dtype=F64, device=g.device, requires_grad=True)
    b0 = torch.tensor(W.body_state0(w), dtype=F64, device=g.device)
    _, _, Fh, _ = rollout(g, g.to_u(u0), g.to_u(fb), kct, b0, w.steps, ckpt_every=20)
    J = rms_lift(g, Fh)
    J.backward()
    grad = kct.grad.cpu().numpy()
    J0, cls0 = _viv_J(w, k0, c0, classes=True)
    assert abs(J0 - float(J.detach())) <= 1e-13 * abs(J0)
    m, fn = float(w.body.m), float(w.meta["fn"])
    report = []
    for name, idx, delta in (("k", 1, 1e-4 * k0[1]), ("c", 4, 1e-4 * 2 * m * 2 * np.pi * fn)):
        vals = []
        for sgn in (+1, -1):
            kk, cc = k0.copy(), c0.copy()
            if name == "k":
                kk[1] += sgn * delta
            else:
                cc[1] += sgn * delta
            Jp, cls = _viv_J(w, kk, cc, classes=True)
            same = all(np.array_equal(a[q], b[q]) for a, b in zip(cls, cls0) for q in range(2))
            assert same, f"point classes changed along the {name} perturbation"
            vals.append(Jp)
        fd = (vals[0] - vals[1]) / (2 * delta)
        rel = abs(grad[idx] - fd) / abs(fd)
        report.append(f"dJ/d{name}: adjoint {grad[idx]:.10e}, central FD {fd:.10e}, rel {rel:.2e}")
        assert rel <= 1e-6, report[-1]
    # the oracle's autograd through the same 400 steps
    from oracle import Grid as OGrid
    from oracle import init_state, make_params
    from oracle.step import rms_lift as o_rms_lift
    from oracle.step import rollout as o_rollout
    og = OGrid(w)
    k = torch.tensor(k0, requires_grad=True)
    c = torch.tensor(c0, requires_grad=True)
    st = init_state(og, u0, W.body_state0(w))
    st, Fo, _ = o_rollout(og, st, make_params(og, fb, k=k, c=c), w.steps)
    Jo = o_rms_lift(og, Fo)
    Jo.backward()
    for name, idx, og_ in (("k", 1, float(k.grad[1])), ("c", 4, float(c.grad[1]))):
        rel = abs(grad[idx] - og_) / abs(og_)
        report.append(f"dJ/d{name}: oracle {og_:.10e}, rel {rel:.2e}")
        assert rel <= 1e-6, report[-1]
    assert abs(float(Jo.detach()) - J0) <= 1e-10 * J0
    print(f"VIV 256x128, 400 steps: J {J0:.12e} (oracle {float(Jo.detach()):.12e})\n" +
          "\n".join(report))


def test_cylinder_force_history():
    need_gpu()
    w = W.cylinder()              # 512 x 256, 5000 steps, dt 5e-3, Re 100
    g = make_grid(w, precision="fp32", poisson_tol=1e-8)
    u0, fb = W.initial_fields(w)
    u, fbt, p = g.to_u(u0), g.to_u(fb), g.zeros_p()
    body = torch.tensor(W.body_state0(w), dtype=F64, device=g.device)
    kc = torch.zeros(6, dtype=F64, device=g.device)
    infos = torch.zeros((w.steps, 8), dtype=F64, device=g.device)
    g.defer_status(True)
    try:
        for n in range(w.steps):
            g.step(u, p, fbt, body, kc, info=infos[n])
    finally:
        g.defer_status(False)
    g.check_infos(infos, "cylinder step")
    F = infos[:, 4:6].cpu().numpy()
    cd, cl = 2.0 * F[:, 0], 2.0 * F[:, 1]          # rho = U = D = 1
    last = slice(w.steps // 2, None)
    print(f"cylinder 512x256, {w.steps} steps (t = {w.steps * w.dt:g}): C_D mean over the second "
          f"half {cd[last].mean():.4f} (min {cd[last].min():.4f}, max {cd[last].max():.4f}); "
          f"C_L rms over the second half {np.sqrt((cl[last] ** 2).mean()):.3e}, "
          f"max |C_L| {np.abs(cl).max():.3e}; C_D at steps 100/1000/5000: {cd[99]:.4f} "
          f"{cd[999]:.4f} {cd[-1]:.4f}")
    assert np.all(np.isfinite(cd)) and np.all(np.isfinite(cl))
    assert cd[last].mean() > 0.0
    # symmetric start, no perturbation: the lift stays at round-off level
    assert np.abs(cl).max() < 1e-3 * cd[last].mean()
