"""P10: the oracle's adjoint (torch.autograd over the float64 step with the
masks frozen) against brute-force central finite differences, plus
conservation pins on bounded, stretched grids."""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from oracle import Grid, init_state, make_params, rollout
from oracle import fluid
from oracle.step import rms_lift, wall_shear

F64 = torch.float64


def _tiny_channel():
    return W.channel(nx=6, ny=8, nz=5, steps=3, dt=1e-4)


def _channel_J(g, u0, fb, nsteps):
    st = init_state(g, u0)
    pr = make_params(g, fb)
    st, _, _ = rollout(g, st, pr, nsteps)
    return wall_shear(g, st["u"])


def test_p10_channel_grad_fb_and_u0_vs_fd():
    w = _tiny_channel()
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    fbt = [torch.tensor(x, requires_grad=True) for x in fb]
    u0t = [torch.tensor(x, requires_grad=True) for x in u0]
    J = _channel_J(g, u0t, fbt, w.steps)
    J.backward()
    rng = np.random.default_rng(3)
    for comp in range(3):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in fb[comp].shape)
            for which, base, grad in (("fb", fb, fbt[comp].grad), ("u0", u0, u0t[comp].grad)):
                if which == "u0" and comp == 1 and idx[1] in (0, fb[1].shape[1] - 1):
                    continue   # wall-normal wall faces are boundary values
                delta = 1e-4
                vals = []
                for s in (+1, -1):
                    arrs = [x.copy() for x in base]
                    arrs[comp][idx] += s * delta
                    if which == "fb":
                        vals.append(float(_channel_J(g, u0, arrs, w.steps)))
                    else:
                        vals.append(float(_channel_J(g, arrs, fb, w.steps)))
                fd = (vals[0] - vals[1]) / (2 * delta)
                ad = float(grad[idx])
                assert abs(fd - ad) <= 1e-7 * max(abs(fd), 1e-6) + 1e-11, (which, comp, idx, fd, ad)


def _tiny_viv():
    return W.viv(nx=32, ny=16, lx=8.0, ly=4.0, center=(2.5, 2.0), markers=16, steps=6, dt=0.01,
                 d0=0.15)


def _viv_J(g, w, k, c, masks):
    u0, fb = W.initial_fields(w)
    st = init_state(g, u0, W.body_state0(w))
    pr = make_params(g, fb, k=k, c=c)
    st, Fh, used = rollout(g, st, pr, w.steps, masks_list=masks)
    return rms_lift(g, Fh), used


def test_p10_viv_grad_k_c_vs_frozen_mask_fd():
    w = _tiny_viv()
    g = Grid(w)
    k = torch.tensor(w.body.k, dtype=F64, requires_grad=True)
    c = torch.tensor([0.0, 0.3, 0.0], dtype=F64, requires_grad=True)
    J, masks = _viv_J(g, w, k, c, None)
    assert float(J.detach()) > 1e-6
    J.backward()
    for name, vec, grad in (("k", k, k.grad), ("c", c, c.grad)):
        base = vec.detach().clone()
        delta = 1e-4 * max(abs(float(base[1])), 0.1)
        vals = []
        for s in (+1, -1):
            v = base.clone()
            v[1] += s * delta
            kk, cc = (v, c.detach()) if name == "k" else (k.detach(), v)
            Jp, _ = _viv_J(g, w, kk, cc, masks)
            vals.append(float(Jp))
        fd = (vals[0] - vals[1]) / (2 * delta)
        ad = float(grad[1])
        assert abs(fd - ad) <= 1e-6 * abs(fd) + 1e-12, (name, fd, ad)


@pytest.mark.parametrize("wall", ["noslip", "freeslip"])
def test_conservation_bounded_stretched(wall):
    """On a stretched grid bounded by resting walls the volume-weighted sum
    of the convective term of the wall-parallel components telescopes to
    zero (no momentum flux through a wall)."""
    yf = W.tanh_faces(9, 1.4)
    xf = np.linspace(0, 2, 7)
    zf = np.linspace(0, 1, 6)
    w = W.generic(3, (6, 9, 5), [xf, yf, zf], [["periodic", "periodic"], [wall, wall],
                  ["periodic", "periodic"]], nu=0.01, dt=1e-3)
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, 9)]
    u[1][:, 0, :] = 0.0
    u[1][:, -1, :] = 0.0
    C = fluid.convection(g, u)
    for c in (0, 2):
        vol = g.bshape(c, g.dc[c][:-1])
        for b in range(3):
            if b != c:
                vol = vol * g.bshape(b, g.dx[b])
        s = float((C[c] * vol).sum())
        scale = float((C[c].abs() * vol).sum())
        assert abs(s) < 1e-13 * scale, (c, s, scale)


def test_energy_neutral_with_resting_walls():
    """Central convection with resting no-slip walls on a uniform grid is
    still energy neutral for a discretely divergence-free field."""
    n = 8
    f = np.linspace(0, 1, n + 1)
    w = W.generic(2, (n, n, 1), [f, f], [["periodic", "periodic"], ["noslip", "noslip"]],
                  nu=0.0, dt=1.0)
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, 21)]
    u[1][:, 0, :] = 0.0
    u[1][:, -1, :] = 0.0
    from oracle.poisson import solver
    b = fluid.flux_divergence(g, u)
    p = solver(g).solve(b - b.mean())
    up = [u[c] + fluid.pressure_gradient(g, p, c) for c in range(2)]
    assert float(fluid.divergence(g, up).abs().max()) < 1e-12
    C = fluid.convection(g, up)
    ev = [up[0], up[1][:, 1:-1, :]]          # faces advanced by the momentum eq.
    e = sum(float((ev[c] * C[c]).sum()) for c in range(2))
    scale = sum(float((ev[c].abs() * C[c].abs()).sum()) for c in range(2))
    assert abs(e) < 1e-13 * scale, (e, scale)
