"""Pins of the oracle's Runge-Kutta steps and CFL-adaptive time step
(Sec. 2.3.1, Sec. 2.5, Table 1):

* forward Euler in the Runge-Kutta form is the step itself, value for value;
* the shear mode u = sin(y) (no convection, projection inactive) is
  multiplied per step by the stability polynomial of the scheme at
  z = nu dt lam_h, lam_h = -(4/h^2) sin^2(h/2): 1 + z + z^2/2 (rk2) and
  1 + z + z^2/2 + z^3/6 (rk3), a closed form;
* on the nonlinear 2D Taylor-Green vortex at a fixed grid the error against
  a fine-step solution falls at order 1, 2 and 3 in dt;
* the adaptive step equals CFL h_min / max |u| (capped), and a rollout takes
  it at every step;
* the gradient through Runge-Kutta steps (autograd) equals central
  differences.
"""
import math

import numpy as np
import pytest
import torch

import fvib_workloads as W
from oracle import Grid, init_state, make_params, step
from oracle.rk import SCHEMES, cfl_dt, h_min, rollout_rk, step_rk

F64 = torch.float64


def _periodic(n, dim=2, nu=0.05, dt=2e-3):
    L = 2 * np.pi
    f = np.linspace(0, L, n + 1)
    bc = [["periodic", "periodic"]] * 3
    return W.generic(dim, (n, n, n if dim == 3 else 1), [f, f, f], bc, nu=nu, dt=dt)


def test_fe_form_is_the_step():
    w = W.tgv2d(n=16, steps=1, dt=1e-2)
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    st = init_state(g, u0)
    pr = make_params(g, fb)
    with torch.no_grad():
        a, _ = step(g, st, pr)
        b, _ = step_rk(g, st, pr, "fe")
    for x, y in zip(a["u"], b["u"]):
        assert torch.equal(x, y)
    assert torch.equal(a["p"], b["p"])


@pytest.mark.parametrize("scheme,poly", [("rk2", lambda z: 1 + z + z * z / 2),
                                         ("rk3", lambda z: 1 + z + z * z / 2 + z ** 3 / 6)])
@pytest.mark.parametrize("dim", [2, 3])
def test_shear_mode_stability_polynomial(scheme, poly, dim):
    n = 16 if dim == 2 else 12
    w = _periodic(n, dim, nu=0.05, dt=0.05)
    g = Grid(w)
    u0 = [np.zeros(g.face_shape(c)) for c in range(dim)]
    y = g.xc[1].numpy()
    u0[0][...] = np.sin(y)[None, :, None]
    st = init_state(g, u0)
    pr = make_params(g)
    nsteps = 20
    with torch.no_grad():
        st, dts = rollout_rk(g, st, pr, nsteps, scheme)
    h = 2 * np.pi / n
    z = w.nu * w.dt * (-(4.0 / h ** 2) * math.sin(h / 2) ** 2)
    amp = poly(z) ** nsteps
    ref = amp * np.sin(y)
    assert np.abs(st["u"][0].numpy() - ref[None, :, None]).max() < 1e-13
    for c in range(1, dim):
        assert st["u"][c].abs().max() < 1e-13
    # the schemes really differ: forward Euler's amplification is not rk's
    assert abs((1 + z) ** nsteps - amp) > 1e-6


def _tgv_final(scheme, dt, T=0.2, n=16):
    nsteps = int(round(T / dt))
    w = W.tgv2d(n=n, steps=nsteps, dt=dt, nu=0.05)
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    st = init_state(g, u0)
    with torch.no_grad():
        st, _ = rollout_rk(g, st, make_params(g, fb), nsteps, scheme)
    return st["u"]


@pytest.mark.parametrize("scheme,order", [("fe", 1), ("rk2", 2), ("rk3", 3)])
def test_temporal_order_tgv(scheme, order):
    ref = _tgv_final("rk3", 0.2 / 128)
    errs = []
    for dt in (0.2 / 8, 0.2 / 16, 0.2 / 32):
        u = _tgv_final(scheme, dt)
        errs.append(max(float((a - b).abs().max()) for a, b in zip(u, ref)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.25 for r in rates), (scheme, errs, rates)


def test_cfl_step_closed_form():
    w = _periodic(20, 2, dt=0.1)
    g = Grid(w)
    u = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(2)]
    u[0][0, 3, 4] = -2.5
    u[1][0, 7, 1] = 1.5
    h = 2 * np.pi / 20
    assert abs(h_min(g) - h) < 1e-15
    assert cfl_dt(g, u, 0.5, 0.1) == pytest.approx(0.5 * h / 2.5, rel=1e-15)
    assert cfl_dt(g, u, 0.5, 0.01) == 0.01                      # capped
    assert cfl_dt(g, [torch.zeros_like(x) for x in u], 0.5, 0.03) == 0.03
    # an adaptive rollout takes the rule at every step
    w2 = W.tgv2d(n=16, steps=5, dt=0.05, nu=0.05)
    g2 = Grid(w2)
    u0, fb = W.initial_fields(w2)
    st = init_state(g2, u0)
    pr = make_params(g2, fb)
    with torch.no_grad():
        s_ad, dts = rollout_rk(g2, st, pr, 5, "rk3", cfl=0.1, dt_max=0.05)
        s = st
        for n in range(5):
            g2.dt = cfl_dt(g2, s["u"], 0.1, 0.05)
            assert g2.dt == dts[n]
            s, _ = step_rk(g2, s, pr, "rk3")
        g2.dt = 0.05
    for a, b in zip(s["u"], s_ad["u"]):
        assert torch.equal(a, b)
    assert all(d < 0.05 for d in dts)


def test_rk3_gradient_vs_central_differences():
    w = _periodic(8, 2, nu=0.05, dt=0.05)
    g = Grid(w)
    rng = np.random.default_rng(3)
    u0 = W.random_fields(w, 5)
    from oracle import fluid
    # a divergence-free start: one forward-Euler step of the random field
    with torch.no_grad():
        st0, _ = step(g, init_state(g, u0), make_params(g))
    ub = [torch.tensor(rng.standard_normal(x.shape)) for x in st0["u"]]
    fbv = [0.1 * rng.standard_normal(x.shape) for x in st0["u"]]

    def J(fb):
        pr = make_params(g, fb)
        st, _ = rollout_rk(g, {"u": st0["u"], "p": st0["p"], "body": st0["body"]}, pr, 3, "rk3")
        return sum((a * b).sum() for a, b in zip(st["u"], ub))

    fbt = [torch.tensor(x, requires_grad=True) for x in fbv]
    J(fbt).backward()
    for comp, idx in ((0, (0, 2, 3)), (1, (0, 5, 1))):
        d = 1e-6
        vals = []
        for s in (+1, -1):
            arr = [x.copy() for x in fbv]
            arr[comp][idx] += s * d
            with torch.no_grad():
                vals.append(float(J(arr)))
        fd = (vals[0] - vals[1]) / (2 * d)
        ad = float(fbt[comp].grad[idx])
        assert abs(fd - ad) <= 1e-7 * max(1.0, abs(fd)), (comp, fd, ad)
    assert fluid is not None
