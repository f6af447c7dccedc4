"""Pins of the oracle's strongly coupled step (Alg. 1 with N > 1) and of its
implicit gradient (Eq. 24).

* N = 1 is the weakly coupled step, value for value.
* The sub-iterations reach the fixed point w* = Phi(w*) of the coupling.
* Closed form: a freely moving body (no spring, no damper) in fluid at rest
  feels only the forcing of its own target velocity, F = -(rho / dt) S U
  with S = h^2 sum_f sum_k dV_k delta_h(x_f - X_k) over its forced faces;
  RK4 with a constant force gives v = v^n + dt F / m, so the coupled
  velocity is the fixed point U* = v^n / (1 + rho S / m) (an added-mass
  relation) and successive velocity corrections shrink by -rho S / m.
* The implicit gradient equals central differences of the converged map
  (masks frozen) and the gradient of the unrolled sub-iterations, for 1-DOF
  and 2-DOF bodies.
"""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from oracle import Grid, init_state, make_params, step
from oracle import ibm
from oracle.step import body_geometry, rms_lift
from oracle.strong import fluid_part, rollout_strong, step_strong, structure

F64 = torch.float64


def _tiny(dof=1, iters=100, tol=1e-5, steps=4):
    return W.viv(nx=32, ny=16, lx=8.0, ly=4.0, center=(2.5, 2.0), markers=16, steps=steps,
                 dt=0.01, d0=0.15, dof=dof, coupling_iters=iters, coupling_tol=tol)


def _state(g, w, seed=1):
    u0, fb = W.initial_fields(w)
    rng = np.random.default_rng(seed)
    u = [x + 0.2 * (2 * rng.random(x.shape) - 1) for x in u0]
    b0 = W.body_state0(w) + np.array([0.01, 0.0, 0.0, 0.05, -0.1, 0.0])
    return init_state(g, u, b0), make_params(g, fb)


@pytest.mark.parametrize("dof", [1, 2])
def test_single_iteration_is_the_weak_step(dof):
    w = _tiny(dof)
    g = Grid(w)
    st, pr = _state(g, w)
    with torch.no_grad():
        a, aux_a = step(g, st, pr)
        b, aux_b = step_strong(g, st, pr, tol=1e-5, nmax=1)
    for x, y in zip(a["u"], b["u"]):
        assert torch.equal(x, y)
    assert torch.equal(a["p"], b["p"])
    assert torch.equal(a["body"], b["body"])
    assert torch.equal(aux_a["F"], aux_b["F"])
    assert aux_b["iters"] == 1


@pytest.mark.parametrize("dof", [1, 2])
def test_sub_iterations_reach_the_fixed_point(dof):
    w = _tiny(dof)
    g = Grid(w)
    st, pr = _state(g, w, seed=2)
    with torch.no_grad():
        new, aux = step_strong(g, st, pr, tol=1e-26, nmax=200)
        xi = aux["xi"]
        assert xi[-1] < 1e-26 and aux["iters"] < 200
        assert all(b < a for a, b in zip(xi[1:-1], xi[2:]))     # contracts
        # Phi(w*) = w*: one more sub-iteration from the returned state
        _, _, F, _ = fluid_part(g, st["u"], pr, new["body"])
        again = structure(g, st["body"], F, pr)
        assert float((again - new["body"]).abs().max()) <= 1e-13 * float(new["body"].abs().max())
        # the weak step differs from the coupled one (the coupling matters)
        weak, _ = step(g, st, pr)
        assert float((weak["body"] - new["body"]).abs().max()) > 1e-8


def test_added_mass_fixed_point_closed_form():
    """Free body (k = c = 0) in fluid at rest, moving in x only."""
    w = _tiny(dof=1)
    w.body.free_dof = (1, 0, 0)
    w.body.k = (0.0, 0.0, 0.0)
    w.body.c = (0.0, 0.0, 0.0)
    w.bc_vel[:] = 0.0                 # no inflow: the fluid stays at rest
    g = Grid(w)
    u = [np.zeros(w.face_shape(c)) for c in range(2)]
    V0 = 0.3
    st = init_state(g, u, np.array([0.0, 0.0, 0.0, V0, 0.0, 0.0]))
    pr = make_params(g, None)
    with torch.no_grad():
        new, aux = step_strong(g, st, pr, tol=1e-28, nmax=200)
        om = aux["omega"]
        Xk, _, dV = body_geometry(g, om)
        masks = aux["masks"]
        # S from the face points of the forced u-faces and the markers
        h = float(g.dx[0][0])
        PX, PY = ibm.face_points_2d(g, 0)
        idx = masks[2][0][0].nonzero(as_tuple=False).numpy()
        S = 0.0
        for (j, i) in idx:
            for kk in range(Xk.shape[0]):
                rx = (PX[j, i] - float(Xk[kk, 0])) / h
                ry = (PY[j, i] - float(Xk[kk, 1])) / h
                S += h * h * float(dV[kk]) * _phi(rx) * _phi(ry) / (h * h)
        ratio = w.rho * S / w.body.m
        U = float(new["body"][3])
        assert abs(U * (1.0 + ratio) - V0) <= 1e-12 * V0, (U, ratio)
        assert 0.1 < ratio < 2.0


def _phi(r):
    """The 4-point kernel written from its printed piecewise form."""
    r = abs(r)
    if r <= 1.0:
        return (3.0 - 2.0 * r + np.sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0
    if r <= 2.0:
        return (5.0 - 2.0 * r - np.sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0
    return 0.0


def test_contraction_factor_is_the_added_mass_ratio():
    """Velocity corrections of successive sub-iterations shrink by -rho S / m
    (to first order: the markers also move by dt^2 dF / 2m between iterates,
    which changes S by a relative 1e-5 here)."""
    w = _tiny(dof=1)
    w.body.free_dof = (1, 0, 0)
    w.body.k = (0.0, 0.0, 0.0)
    w.body.c = (0.0, 0.0, 0.0)
    w.bc_vel[:] = 0.0
    g = Grid(w)
    u = [np.zeros(w.face_shape(c)) for c in range(2)]
    V0 = 0.3
    st = init_state(g, u, np.array([0.0, 0.0, 0.0, V0, 0.0, 0.0]))
    pr = make_params(g, None)
    with torch.no_grad():
        _, aux0 = step_strong(g, st, pr, tol=1e-28, nmax=1)
        masks = aux0["masks"]
        oms = [st["body"]]
        for _ in range(4):
            _, _, F, _ = fluid_part(g, st["u"], pr, oms[-1], masks)
            oms.append(structure(g, st["body"], F, pr))
        dU = [float(oms[i + 1][3] - oms[i][3]) for i in range(4)]
        r = [dU[i + 1] / dU[i] for i in range(3)]
        # S at the iterates' position (they differ by far less than their
        # displacement dt V0 from the time level)
        Xk, _, dV = body_geometry(g, oms[-1])
        h = float(g.dx[0][0])
        PX, PY = ibm.face_points_2d(g, 0)
        idx = masks[2][0][0].nonzero(as_tuple=False).numpy()
        S = sum(h * h * float(dV[kk]) * _phi((PX[j, i] - float(Xk[kk, 0])) / h)
                * _phi((PY[j, i] - float(Xk[kk, 1])) / h) / (h * h)
                for (j, i) in idx for kk in range(Xk.shape[0]))
        ratio = w.rho * S / w.body.m
        for x in r:
            assert abs(x + ratio) <= 1e-4 * ratio, (r, ratio)


def _J_strong(g, w, k, c, fb, tol, implicit=True, masks_list=None):
    u0, _ = W.initial_fields(w)
    st = init_state(g, u0, W.body_state0(w))
    pr = make_params(g, fb, k=k, c=c)
    st, Fh, _ = rollout_strong(g, st, pr, w.steps, tol=tol, nmax=200, implicit=implicit,
                               masks_list=masks_list)
    return rms_lift(g, Fh) + (st["body"][:2] ** 2).sum()


def _masks_of_run(g, w, k, c, fb, tol):
    u0, _ = W.initial_fields(w)
    st = init_state(g, u0, W.body_state0(w))
    pr = make_params(g, fb, k=k, c=c)
    masks = []
    with torch.no_grad():
        for _ in range(w.steps):
            st, aux = step_strong(g, st, pr, tol, 200)
            masks.append(aux["masks"])
    return masks


@pytest.mark.parametrize("dof", [1, 2])
def test_implicit_gradient_vs_fd_and_unrolled(dof):
    w = _tiny(dof, steps=4)
    g = Grid(w)
    tol = 1e-28
    _, fb = W.initial_fields(w)
    rng = np.random.default_rng(5)
    fbv = [0.05 * (2 * rng.random(x.shape) - 1) for x in fb]
    k0 = torch.tensor(w.body.k, dtype=F64)
    c0 = torch.tensor([0.2, 0.3, 0.0], dtype=F64) if dof == 2 else torch.tensor([0.0, 0.3, 0.0], dtype=F64)
    k = k0.clone().requires_grad_(True)
    c = c0.clone().requires_grad_(True)
    fbt = [torch.tensor(x, requires_grad=True) for x in fbv]
    J = _J_strong(g, w, k, c, fbt, tol)
    J.backward()
    # the unrolled sub-iterations differentiate the same converged map
    k2 = k0.clone().requires_grad_(True)
    c2 = c0.clone().requires_grad_(True)
    fbt2 = [torch.tensor(x, requires_grad=True) for x in fbv]
    J2 = _J_strong(g, w, k2, c2, fbt2, tol, implicit=False)
    J2.backward()
    assert abs(float(J2.detach()) - float(J.detach())) <= 1e-14 * abs(float(J.detach()))
    for a, b in ((k.grad, k2.grad), (c.grad, c2.grad)):
        assert float((a - b).abs().max()) <= 1e-8 * float(b.abs().max()) + 1e-14
    for a, b in zip(fbt, fbt2):
        assert float((a.grad - b.grad).abs().max()) <= 1e-8 * float(b.grad.abs().max())
    # central differences with the masks of the base run
    masks = _masks_of_run(g, w, k0, c0, fbv, tol)
    dofs = [1] if dof == 1 else [0, 1]
    for name, base, grad in (("k", k0, k.grad), ("c", c0, c.grad)):
        for a in dofs:
            delta = 1e-5 * max(abs(float(base[a])), 0.1)
            vals = []
            for s in (+1, -1):
                v = base.clone()
                v[a] += s * delta
                kk, cc = (v, c0) if name == "k" else (k0, v)
                with torch.no_grad():
                    vals.append(float(_J_strong(g, w, kk, cc, fbv, tol, masks_list=masks)))
            fd = (vals[0] - vals[1]) / (2 * delta)
            assert abs(fd - float(grad[a])) <= 1e-6 * abs(fd) + 1e-10, (name, a, fd, float(grad[a]))
    # one body-force entry near the body, per component
    for comp in range(2):
        idx = (0, 8, 10)
        delta = 1e-5
        vals = []
        for s in (+1, -1):
            arr = [x.copy() for x in fbv]
            arr[comp][idx] += s * delta
            with torch.no_grad():
                vals.append(float(_J_strong(g, w, k0, c0, arr, tol, masks_list=masks)))
        fd = (vals[0] - vals[1]) / (2 * delta)
        ad = float(fbt[comp].grad[idx])
        assert abs(fd - ad) <= 1e-6 * abs(fd) + 1e-10, (comp, fd, ad)
