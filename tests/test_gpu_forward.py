"""GPU parity of the forward step against the CPU oracle (through the C ABI).

Tolerances: float64 path 1e-10 relative L2 (whole fields); float32-mixed
path 1e-5 relative L2; sub-kernels at 1e-12 (float64) / 1e-5 (float32)
relative to the field scale; point classes bit-exact.
"""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from gpu_util import gauge, gpu_rollout, make_grid, need_gpu, oracle_rollout, rel_l2

pytestmark = pytest.mark.gpu


def _cases():
    """Grids spanning several tiles with ragged tails and every BC kind."""
    bcv = np.zeros((3, 2, 3))
    bcv[0, 0, 0] = 1.0
    bcv[0, 0, 1] = 0.2          # inflow with a tangential component
    bcv[1, 1, 0] = 0.7          # moving wall
    return {
        "periodic2d": W.generic(2, (70, 37, 1), [np.linspace(0, 2, 71), np.linspace(0, 1, 38)],
                                [["periodic", "periodic"], ["periodic", "periodic"]], nu=0.03, dt=1e-3),
        "open2d": W.generic(2, (67, 13, 1), [np.linspace(0, 4, 68), np.linspace(0, 1, 14)],
                            [["inflow", "outflow_conv"], ["freeslip", "noslip"]], bc_vel=bcv,
                            nu=0.02, dt=1e-3),
        "neumann2d": W.generic(2, (33, 29, 1), [np.linspace(0, 1, 34), W.tanh_faces(29, 1.2)],
                               [["inflow", "outflow_neumann"], ["noslip", "noslip"]], bc_vel=bcv,
                               nu=0.02, dt=1e-3),
        "channel3d": W.channel(nx=67, ny=19, nz=9, dt=1e-5),
        "box3d": W.generic(3, (65, 6, 7), [np.linspace(0, 2, 66), W.tanh_faces(6, 1.1),
                           np.linspace(0, 1, 8)], [["inflow", "outflow_conv"],
                           ["noslip", "freeslip"], ["noslip", "noslip"]], bc_vel=bcv,
                           nu=0.05, dt=1e-3),
    }


@pytest.mark.parametrize("case", list(_cases().keys()))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("conv", ["central", "upwind"])
def test_momentum_rhs_parity(case, precision, conv):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import fluid
    w = _cases()[case]
    w.conv = conv
    g = make_grid(w, precision=precision)
    u = W.random_fields(w, 7)
    fb = W.random_fields(w, 8, 0.5)
    R = g.test_momentum(g.to_u(u), g.to_u(fb))
    og = OGrid(w)
    ut = [torch.tensor(x) for x in u]
    if precision == "fp32":        # the oracle sees exactly the rounded inputs
        ut = [x.float().double() for x in ut]
        fbt = [torch.tensor(x).float().double() for x in fb]
    else:
        fbt = [torch.tensor(x) for x in fb]
    Ro = fluid.momentum_rhs(og, ut, fbt)
    tol = 1e-12 if precision == "fp64" else 2e-5
    for c in range(w.dim):
        scale = float(Ro[c].abs().max())
        err = float((R[c].double().cpu() - Ro[c]).abs().max())
        assert err <= tol * scale, (case, c, err, scale)


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_ppe_rhs_and_operator_parity(case):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import fluid
    from oracle.poisson import apply_A
    w = _cases()[case]
    g = make_grid(w, precision="fp64")
    og = OGrid(w)
    us = W.random_fields(w, 3)
    b = g.test_ppe_rhs(g.to_u(us)).cpu()
    bo = -(w.rho / w.dt) * fluid.flux_divergence(og, [torch.tensor(x) for x in us])
    assert float((b - bo).abs().max()) <= 1e-12 * float(bo.abs().max())
    p = torch.tensor(W.random_cells(w, 4))
    Ap = g.test_apply_A(p.to(g.device)).cpu()
    Apo = apply_A(og, p)
    assert float((Ap - Apo).abs().max()) <= 1e-12 * float(Apo.abs().max())


@pytest.mark.parametrize("case", list(_cases().keys()))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("solver", ["cg", "fdm"])
def test_poisson_solution_parity(case, precision, solver):
    """CG (double, or float inside double refinement) and the fast
    diagonalisation inside double refinement reach the exact solution of the
    same discrete system."""
    need_gpu()
    from oracle import Grid as OGrid
    from oracle.poisson import solver as exact
    w = _cases()[case]
    g = make_grid(w, precision=precision, poisson_tol=1e-12, inner_rtol=1e-3, solver=solver)
    og = OGrid(w)
    b = torch.tensor(W.random_cells(w, 5))
    p, iters = g.test_poisson(b.to(g.device))
    pe = exact(og).solve(b - b.mean())
    err = float((gauge(p.cpu()) - pe).abs().max())
    if solver == "cg":
        assert iters > 0
    assert err <= 1e-9 * float(pe.abs().max()), (err, iters)


@pytest.mark.parametrize("dims", [(192, 128, 160), (64, 32, 96), (96, 256, 32),
                                  (48, 13, 10), (96, 5, 27)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_poisson_parity_channel_shapes(dims, precision):
    """Fast-diagonalisation solve at the channel's production shape (and
    shapes whose axes take the other operator-tile counts; the last two
    give the contiguous x FFT an odd line count that leaves its last block
    partly filled, 130 and 135 lines), against the oracle's exact solve."""
    need_gpu()
    from oracle import Grid as OGrid
    from oracle.poisson import solver as exact
    nx, ny, nz = dims
    w = W.channel(nx=nx, ny=ny, nz=nz)
    g = make_grid(w, precision=precision, poisson_tol=1e-12, inner_rtol=1e-3, solver="fdm")
    og = OGrid(w)
    b = torch.tensor(W.random_cells(w, 11))
    p, _ = g.test_poisson(b.to(g.device))
    pe = exact(og).solve(b - b.mean())
    err = float((gauge(p.cpu()) - pe).abs().max())
    assert err <= 1e-9 * float(pe.abs().max()), (dims, precision, err)


@pytest.mark.parametrize("name", ["cylinder", "viv"])
def test_ib_classification_bit_exact(name):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle import ibm
    w = W.by_name(name, "small")
    og = OGrid(w)
    g = make_grid(w, precision="fp64")
    for d in ([0.0, 0.0], [0.0, 0.1], [0.013, -0.271], [0.25, 0.3331]):
        body = torch.tensor([d[0], d[1], 0, 0, 0, 0], dtype=torch.float64, device=g.device)
        cls = g.test_ib_classify(body)
        X = w.body.X0 + np.asarray(d)[None, :]
        solid, ib, eps = ibm.classify(og, X)
        for c in range(2):
            exp = solid[c].numpy().astype(np.uint8) + 2 * ib[c].numpy().astype(np.uint8)
            assert np.array_equal(cls[c].cpu().numpy(), exp), (name, d, c)


# ------------------------------------------------------------ whole step
@pytest.mark.parametrize("solver", ["cg", "fdm"])
def test_tgv2d_fp64_100_steps(solver):
    """2D Taylor-Green vortex, 64 x 64, dt 1e-3, 100 steps, float64."""
    need_gpu()
    w = W.tgv2d()
    gr = gpu_rollout(w, w.steps, "fp64", tol=1e-13, solver=solver)
    orc = oracle_rollout(w, w.steps)
    eu = rel_l2(gr["u"], orc["u"])
    ep = rel_l2([gauge(gr["p"])], [orc["p"]])
    dm = max(i["div_max"] for i in gr["infos"])
    # error against the analytic decay at t = 0.1 (the discretisation error,
    # which the GPU shares with the oracle)
    t = w.steps * w.dt
    x, y = W.face_points(w, 0)[:2]
    ua = np.sin(x) * np.cos(y) * np.exp(-2 * w.nu * t)
    ea = float(np.abs(gr["u"][0] - ua).max())
    print(f"TGV 64^2 {solver}, 100 steps float64: u rel L2 vs oracle {eu:.2e}, p {ep:.2e}, "
          f"max div {dm:.2e}; max |u - analytic| {ea:.2e}")
    assert eu <= 1e-10
    assert ep <= 1e-10
    assert dm <= 1e-12
    assert ea <= 5e-3


@pytest.mark.parametrize("name", ["tgv3d", "channel", "cylinder", "viv"])
@pytest.mark.parametrize("solver", ["cg", "fdm"])
def test_small_workloads_fp64(name, solver):
    need_gpu()
    w = W.by_name(name, "small")
    gr = gpu_rollout(w, w.steps, "fp64", tol=1e-12, solver=solver)
    orc = oracle_rollout(w, w.steps)
    assert rel_l2(gr["u"], orc["u"]) <= 1e-10, name
    assert rel_l2([gauge(gr["p"])], [orc["p"]]) <= 1e-9, name
    if w.body is not None:
        assert np.abs(gr["forces"] - orc["forces"]).max() <= 1e-9 * max(1.0, np.abs(orc["forces"]).max())
        assert np.abs(gr["body"] - orc["body"]).max() <= 1e-12


@pytest.mark.parametrize("name", ["tgv3d", "channel", "cylinder", "viv"])
@pytest.mark.parametrize("solver", ["cg", "fdm"])
def test_small_workloads_fp32_mixed(name, solver):
    need_gpu()
    w = W.by_name(name, "small")
    gr = gpu_rollout(w, w.steps, "fp32", tol=1e-8, solver=solver)
    orc = oracle_rollout(w, w.steps)
    assert rel_l2(gr["u"], orc["u"]) <= 1e-5, name
    assert max(i["div_max"] for i in gr["infos"]) <= 1e-8
    assert all(i["status"] == 0 for i in gr["infos"])


def test_fp32_mixed_100_steps_channel():
    need_gpu()
    w = W.channel(nx=32, ny=24, nz=20, steps=100)
    gr = gpu_rollout(w, w.steps, "fp32", tol=1e-8)
    orc = oracle_rollout(w, w.steps)
    assert rel_l2(gr["u"], orc["u"]) <= 1e-5


def test_in_place_equals_out_of_place_and_deterministic():
    """Two in-place runs of the moving-body case agree bit for bit, and so
    does a run whose every step reads (u, p, body) from one set of tensors
    and writes a fresh set."""
    need_gpu()
    w = W.by_name("viv", "small")
    a = gpu_rollout(w, 3, "fp32", tol=1e-8)
    b = gpu_rollout(w, 3, "fp32", tol=1e-8)
    for x, y in zip(a["u"], b["u"]):
        assert np.array_equal(x, y)
    assert np.array_equal(a["p"], b["p"])
    g = make_grid(w, precision="fp32", poisson_tol=1e-8)
    u0, fb = W.initial_fields(w)
    u, fbt, p = g.to_u(u0), g.to_u(fb), g.zeros_p()
    body = torch.tensor(W.body_state0(w), dtype=torch.float64, device=g.device)
    kc = torch.tensor(np.concatenate([np.asarray(w.body.k), np.asarray(w.body.c)]),
                      dtype=torch.float64, device=g.device)
    for _ in range(3):
        u2 = [torch.full_like(x, float("nan")) for x in u]
        p2 = torch.full_like(p, float("nan"))
        b2 = torch.full_like(body, float("nan"))
        g.step(u, p, fbt, body, kc, u_out=u2, p_out=p2, body_out=b2)
        u, p, body = u2, p2, b2
    torch.cuda.synchronize()
    for x, y in zip(u, a["u"]):
        assert np.array_equal(x.double().cpu().numpy(), y)
    assert np.array_equal(p.cpu().numpy(), a["p"])
    assert np.array_equal(body.cpu().numpy(), a["body"])


@pytest.mark.parametrize("nx", [32, 16])      # 32: FFT pass adds the correction; 16: separate pass
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_out_of_place_pressure_guess(nx, precision):
    """A step that reads its pressure guess from one tensor and writes
    another equals the in-place step, also when the guess already meets the
    tolerance (the first refinement sweep is skipped on the device and must
    still carry the guess over)."""
    need_gpu()
    w = W.channel(nx=nx, ny=16, nz=24, steps=2, dt=1e-5)
    g = make_grid(w, precision=precision, poisson_tol=1e-8)
    u0, fb = W.initial_fields(w)
    fbt = g.to_u(fb)
    # in place from a zero guess
    u1 = g.to_u(u0)
    p1 = g.zeros_p()
    g.step(u1, p1, fbt)
    # out of place from the converged pressure: the first check passes at once
    for guess in (g.zeros_p(), p1.clone()):
        u2 = [torch.empty_like(x) for x in u1]
        p2 = torch.full_like(p1, float("nan"))
        ui = g.to_u(u0)
        g.step(ui, guess, fbt, u_out=u2, p_out=p2)
        torch.cuda.synchronize()
        assert torch.isfinite(p2).all()
        for a, b in zip(u2, u1):
            assert float((a.double() - b.double()).abs().max()) <= 1e-6 * float(b.abs().max())
        assert float((p2 - p1).abs().max()) <= 1e-6 * float(p1.abs().max())
        for a, b in zip(ui, g.to_u(u0)):        # the input state is untouched
            assert torch.equal(a, b)
