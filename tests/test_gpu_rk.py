"""Explicit Runge-Kutta steps (Sec. 2.3.1, Table 1) and the CFL-adaptive time
step (Sec. 2.5) through the C ABI against the oracle (oracle/rk.py):

* the "fe" scheme is the forward-Euler step bit for bit;
* rk2 / rk3 steps match the oracle's on periodic, walled and open grids;
* in-place and out-of-place steps agree;
* one-step vector-Jacobian products match the oracle's autograd;
* the CFL step equals the oracle's rule; an adaptive rk3 rollout takes the
  oracle's step sizes and its gradient matches the oracle's.
"""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from gpu_util import make_grid, need_gpu, rel_l2
from test_gpu_adjoint import _close

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _cases():
    bcv = np.zeros((3, 2, 3))
    bcv[0, 0, 0] = 1.0
    bcv[1, 1, 0] = 0.7
    return {
        "tgv2d": W.tgv2d(n=32, steps=6, dt=5e-3),
        "channel": W.channel(nx=24, ny=16, nz=20, steps=6, dt=1e-5),
        "box3d": W.generic(3, (12, 10, 9), [np.linspace(0, 2, 13), W.tanh_faces(10, 1.2),
                           np.linspace(0, 1.5, 10)], [["inflow", "outflow_conv"],
                           ["noslip", "freeslip"], ["periodic", "periodic"]], bc_vel=bcv,
                           nu=0.05, dt=2e-3, steps=6),
    }


def _gpu_run(w, precision, scheme, steps, inplace=True):
    g = make_grid(w, precision=precision, poisson_tol=1e-12 if precision == "fp64" else 1e-9)
    u0, fb = W.initial_fields(w)
    u, fbt, p = g.to_u(u0), g.to_u(fb), g.zeros_p()
    for _ in range(steps):
        if inplace:
            g.step(u, p, fbt, scheme=scheme)
        else:
            u2, p2 = g.zeros_u(), g.zeros_p()
            g.step(u, p, fbt, u_out=u2, p_out=p2, scheme=scheme)
            u, p = u2, p2
    torch.cuda.synchronize()
    return [x.double().cpu().numpy() for x in u], p.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fe_scheme_is_the_step(precision):
    need_gpu()
    w = _cases()["channel"]
    g = make_grid(w, precision=precision)
    u0, fb = W.initial_fields(w)
    a, fa, pa = g.to_u(u0), g.to_u(fb), g.zeros_p()
    b, pb = g.to_u(u0), g.zeros_p()
    for _ in range(3):
        g.step(a, pa, fa)
        g.step(b, pb, fa, scheme="fe")
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(pa, pb)


@pytest.mark.parametrize("case", list(_cases().keys()))
@pytest.mark.parametrize("scheme", ["rk2", "rk3"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rk_steps_match_oracle(case, scheme, precision):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import init_state, make_params
    from oracle.rk import rollout_rk
    w = _cases()[case]
    og = OGrid(w)
    u0, fb = W.initial_fields(w)
    with torch.no_grad():
        st, _ = rollout_rk(og, init_state(og, u0), make_params(og, fb), w.steps, scheme)
    gu, gp = _gpu_run(w, precision, scheme, w.steps)
    e = rel_l2(gu, [x.numpy() for x in st["u"]])
    tol = 1e-10 if precision == "fp64" else 1e-5
    print(f"{case} {scheme} {precision}: u rel L2 {e:.2e}")
    assert e <= tol, e
    if precision == "fp64":
        ep = rel_l2([gp - gp.mean()], [st["p"].numpy()])
        assert ep <= 1e-8, ep
    # in place and out of place agree
    gu2, _ = _gpu_run(w, precision, scheme, 2, inplace=False)
    gu3, _ = _gpu_run(w, precision, scheme, 2, inplace=True)
    assert rel_l2(gu2, gu3) <= (1e-13 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("case", list(_cases().keys()))
@pytest.mark.parametrize("scheme", ["rk2", "rk3"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rk_step_vjp(case, scheme, precision):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import init_state, make_params
    from oracle.rk import step_rk
    w = _cases()[case]
    og = OGrid(w)
    u = W.random_fields(w, 11)
    u0, _ = W.initial_fields(w)
    u = [a + 0.1 * b for a, b in zip(u0, u)]
    fb = W.random_fields(w, 12, 0.3)
    ubar = W.random_fields(w, 13)
    r32 = precision == "fp32"
    cast = (lambda a: torch.tensor(a).float().double()) if r32 else (lambda a: torch.tensor(a))
    if r32:
        ubar = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in ubar]
    ut = [cast(x).requires_grad_(True) for x in u]
    fbt = [cast(x).requires_grad_(True) for x in fb]
    st, _ = step_rk(og, init_state(og, ut), make_params(og, fbt), scheme)
    L = sum((st["u"][i] * torch.tensor(ubar[i])).sum() for i in range(w.dim))
    L.backward()
    g = make_grid(w, precision=precision, poisson_tol=1e-12 if not r32 else 1e-9)
    ugt, fgt = g.to_u(u), g.to_u(fb)
    ub1 = g.to_u(ubar)
    ub0, fbb = g.zeros_u(), g.zeros_u()
    z6 = torch.zeros(6, dtype=F64, device=g.device)
    g.step_adjoint(ugt, fgt, None, None, ub1, None, None, ub0, None, fbbar=fbb, scheme=scheme,
                   p=g.zeros_p())
    torch.cuda.synchronize()
    tol = 1e-9 if not r32 else 2e-4
    for i in range(w.dim):
        _close(ub0[i].double().cpu().numpy(), ut[i].grad.numpy(), tol, f"ubar[{i}]")
        _close(fbb[i].double().cpu().numpy(), fbt[i].grad.numpy(), tol, f"fbbar[{i}]")
    assert z6.abs().max() == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cfl_dt_matches_oracle(precision):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle.rk import cfl_dt
    w = _cases()["channel"]
    og = OGrid(w)
    g = make_grid(w, precision=precision)
    u = W.random_fields(w, 21)
    if precision == "fp32":
        u = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in u]
    ut = g.to_u(u)
    for cfl, dtmax in ((0.5, 1.0), (0.5, 1e-4), (0.05, 1.0)):
        dg = g.cfl_dt(ut, cfl, dtmax)
        do = cfl_dt(og, [torch.tensor(x) for x in u], cfl, dtmax)
        assert dg == pytest.approx(do, rel=1e-15, abs=0.0), (cfl, dtmax, dg, do)


def test_adaptive_rk3_rollout_gradient():
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import init_state, make_params
    from oracle.rk import rollout_rk
    from oracle.step import wall_shear
    from paper_2505_23940_amd.rollout import rollout, wall_shear as g_wall_shear
    w = W.channel(nx=16, ny=12, nz=10, steps=5, dt=4e-5)
    cfl = (0.01, 4e-5)
    og = OGrid(w)
    u0, fb = W.initial_fields(w)
    fbt = [torch.tensor(x, requires_grad=True) for x in fb]
    st, dts_o = rollout_rk(og, init_state(og, u0), make_params(og, fbt), w.steps, "rk3",
                           cfl=cfl[0], dt_max=cfl[1])
    Jo = wall_shear(og, st["u"])
    Jo.backward()
    g = make_grid(w, precision="fp64", poisson_tol=1e-12)
    fg = [x.requires_grad_(True) for x in g.to_u(fb)]
    kc = torch.zeros(6, dtype=F64, device=g.device)
    b0 = torch.zeros(6, dtype=F64, device=g.device)
    uS, _, _, _ = rollout(g, g.to_u(u0), fg, kc, b0, w.steps, ckpt_every=2, scheme="rk3",
                          cfl=cfl)
    J = g_wall_shear(g, uS[0])
    J.backward()
    torch.cuda.synchronize()
    assert g.dt == w.dt                       # restored
    assert all(d < cfl[1] for d in dts_o)     # the CFL limit is active
    assert abs(float(J.detach()) - float(Jo.detach())) <= 1e-10 * abs(float(Jo.detach()))
    e = rel_l2([x.grad.double().cpu().numpy() for x in fg], [x.grad.numpy() for x in fbt])
    print(f"adaptive rk3 channel: dts {dts_o}, J {float(J.detach()):.12e}, dJ/dfb rel L2 {e:.2e}")
    assert e <= 1e-8, e
