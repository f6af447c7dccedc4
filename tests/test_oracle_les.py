"""Pins of the oracle's LES terms (oracle/les.py): the Spalding-law solve
(Eq. 27) against the law evaluated forwards, its derivative against the
derivative of the law, the cell strain of a linear field against its exact
value, the stress divergence against the molecular Laplacian (constant
viscosity, divergence-free field) and against its own gradient (discrete
summation by parts: the subgrid term only dissipates), the wall model's
momentum balance against the stress the law prescribes (Eqs. 28-29), and
the LES step's gradient against central differences."""
import math

import numpy as np
import pytest
import torch

import fvib_workloads as W
from oracle import Grid, fluid, les
from oracle.poisson import solver
from oracle.step import init_state, make_params, step

F64 = torch.float64
KAPPA, B = 0.4, 5.0


def _yplus(up):
    """Eq. 27 evaluated forwards: y+ as a function of u+."""
    k = KAPPA * up
    return up + math.exp(-KAPPA * B) * (np.exp(k) - 1 - k - k * k / 2 - k ** 3 / 6)


def test_spalding_inverse_and_limits():
    up = np.array([0.05, 0.5, 3.0, 8.0, 11.0, 20.0, 30.0, 45.0])
    yp = _yplus(up)
    re = torch.tensor(up * yp)                   # U y / nu = u+ y+
    got = les.spalding_uplus(re, KAPPA, B).detach().numpy()
    assert np.abs(got / up - 1).max() < 1e-13
    # dimensional: u_tau from (U, y, nu)
    nu, ut = 1e-3, 0.37
    U = torch.tensor(up * ut)
    for i in range(up.size):
        y = yp[i] * nu / ut
        tau = les.wall_stress(U[i:i + 1], y, nu, KAPPA, B)
        assert abs(float(tau) / ut ** 2 - 1) < 1e-12
    # viscous sublayer: tau -> nu U / y; log layer: u+ -> ln(y+)/kappa + B
    U0 = torch.tensor([1e-6], dtype=F64)
    tau = les.wall_stress(U0, 0.01, 1e-3, KAPPA, B)
    assert abs(float(tau) / (1e-3 * 1e-6 / 0.01) - 1) < 1e-6
    y_big = 1e7
    up_big = float(les.spalding_uplus(torch.tensor([y_big * 40.0], dtype=F64), KAPPA, B))
    assert abs(up_big - (math.log(y_big * 40.0 / up_big) / KAPPA + B)) < 1e-3


def test_spalding_derivative():
    """du+/dRe = 1 / d(u+ y+)/du+, from differentiating the law forwards."""
    up = np.array([0.3, 4.0, 12.0, 25.0])
    k = KAPPA * up
    dyp = 1 + math.exp(-KAPPA * B) * KAPPA * (np.exp(k) - 1 - k - k * k / 2)
    yp = _yplus(up)
    expect = 1.0 / (yp + up * dyp)
    re = torch.tensor(up * yp, requires_grad=True)
    x = les.spalding_uplus(re, KAPPA, B)
    x.sum().backward()
    assert np.abs(re.grad.numpy() / expect - 1).max() < 1e-10


def _channel_grid(nx=8, ny=10, nz=6, les_cfg=None, seed=0):
    rng = np.random.default_rng(seed)
    fy = np.sort(np.concatenate([[-1.0, 1.0], rng.uniform(-0.95, 0.95, ny - 1)]))
    faces = [np.linspace(0, 2.0, nx + 1), fy, np.linspace(0, 1.3, nz + 1)]
    bc = [["periodic", "periodic"], ["noslip", "noslip"], ["periodic", "periodic"]]
    w = W.generic(3, (nx, ny, nz), faces, bc, nu=2e-3, dt=1e-3)
    w.les = les_cfg
    return w


def test_strain_of_linear_field():
    w = _channel_grid(nx=9, ny=11, nz=7)
    g = Grid(w)
    A = np.array([[0.3, -1.1, 0.7], [2.0, -0.5, 0.4], [-0.9, 1.6, 0.2]])
    u = []
    for c in range(3):
        x, y, z = W.face_points(w, c)
        u.append(torch.tensor(np.broadcast_to(A[c, 0] * x + A[c, 1] * y + A[c, 2] * z,
                                              w.face_shape(c)).copy()))
    S = les.strain(g, u)
    Sx = 0.5 * (A + A.T)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))     # away from the seam and walls
    for (i, j), v in S.items():
        assert np.abs(v[inner].numpy() - Sx[i, j]).max() < 1e-12, (i, j)
    cs = 0.17
    nut = les.nu_smagorinsky(g, u, cs)[inner].numpy()
    delta = les.filter_width(g)[inner].numpy()
    expect = (cs * delta) ** 2 * math.sqrt(2.0 * float((Sx * Sx).sum()))
    assert np.abs(nut - expect).max() < 1e-12 * expect.max()


def _periodic_grid(n=(8, 6, 10)):
    faces = [np.linspace(0, 2.0, n[0] + 1), np.linspace(0, 1.1, n[1] + 1),
             np.linspace(0, 2.7, n[2] + 1)]
    w = W.generic(3, n, faces, [["periodic", "periodic"]] * 3, nu=1e-2, dt=1e-3)
    return w, Grid(w)


def test_constant_viscosity_gives_laplacian():
    """For a discretely divergence-free field and constant nu the transpose
    term d_j d_c u_j = d_c div u vanishes: the stress divergence is nu lap u."""
    w, g = _periodic_grid()
    us = [torch.tensor(x) for x in W.random_fields(w, 3)]
    eps = [torch.zeros(g.face_shape(c), dtype=torch.bool) for c in range(3)]
    b = fluid.ppe_rhs(g, us, eps, us)
    u = fluid.project(g, us, solver(g).solve(b))
    assert float(fluid.divergence(g, u).abs().max()) < 1e-12
    nu0 = 0.37
    D = les.stress_divergence(g, u, torch.full(g.cell_shape(), nu0, dtype=F64))
    L = fluid.diffusion(g, u)
    for c in range(3):
        assert float((D[c] - nu0 * L[c]).abs().max()) < 1e-11 * float(L[c].abs().max())


def test_stress_divergence_is_dissipative():
    """Summation by parts on a periodic grid: sum over faces of dv u . div(T)
    = -(sum over cells of vol 2 nu (d_c u_c)^2 + sum over edges of vol_e nu_e G_e^2)."""
    w, g = _periodic_grid()
    u = [torch.tensor(x) for x in W.random_fields(w, 5)]
    rng = np.random.default_rng(6)
    nu_c = torch.tensor(rng.uniform(0.1, 1.0, g.cell_shape()))
    D = les.stress_divergence(g, u, nu_c)
    lhs = 0.0
    for c in range(3):
        dv = g.bshape(c, g.dc[c][:-1]) * g.face_area(c)
        lhs += float((dv * u[c] * D[c]).sum())
    vol = g.cell_volume()
    rhs = 0.0
    for c in range(3):
        rhs += float((vol * 2.0 * nu_c * les._diag_grad(g, u, c) ** 2).sum())
    for c, a in ((0, 1), (0, 2), (1, 2)):
        G = les.edge_grad(g, u, c, a)
        nu_e = les._edge_nu(g, nu_c, c, a, None)
        bb = 3 - a - c
        ve = g.bshape(c, g.dc[c]) * g.bshape(a, g.dc[a]) * g.bshape(bb, g.dx[bb])
        term = ve * nu_e * G * G
        # the lattice repeats the periodic first position at the end: count it once
        term = term.narrow(2 - c, 0, g.n[c]).narrow(2 - a, 0, g.n[a])
        rhs += float(term.sum())
    assert abs(lhs + rhs) <= 1e-12 * abs(rhs)


def test_wall_model_momentum_balance():
    """Every interior flux telescopes: the x- and z-momentum the diffusive
    terms (molecular + subgrid) add equals the wall stress of the Spalding
    law at the prescribed first-row speed, split by Eq. 29 and scaled by the
    Eq. 28 regulariser, on both walls."""
    cfg = {"cs": 0.13, "wall_model": True, "kappa": KAPPA, "B": B, "eps": 1e-6}
    w = _channel_grid(nx=8, ny=10, nz=6, les_cfg=cfg)
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, 9)]
    u[1][:, 0, :] = 0.0
    u[1][:, -1, :] = 0.0
    expect = {0: 0.0, 2: 0.0}
    area = 2.0 * 1.3
    for side, row, up, th in ((0, 0, 14.0, 0.3), (1, -1, 9.0, -0.7)):
        yw = 0.5 * float(g.dx[1][0] if side == 0 else g.dx[1][-1])
        ut = _yplus(up) * g.nu / yw                     # u_tau giving this u+ at yw
        U = up * ut
        u1, w1 = U * math.cos(th), U * math.sin(th)
        u[0][:, row, :] = u1
        u[2][:, row, :] = w1
        for comp, v in ((0, u1), (2, w1)):
            tau_i = ut * ut * v / U
            r = (v / yw) / (v / yw + cfg["eps"])
            expect[comp] -= area * tau_i * r
    S = les.sgs_force(g, u)
    L = fluid.diffusion(g, u)
    for comp in (0, 2):
        dv = g.bshape(comp, g.dc[comp][:-1]) * g.face_area(comp)
        tot = float((dv * (g.nu * L[comp] + S[comp])).sum())
        assert abs(tot - expect[comp]) <= 1e-11 * abs(expect[comp]), (comp, tot, expect[comp])


def test_galilean_invariance_of_nut():
    w, g = _periodic_grid()
    u = [torch.tensor(x) for x in W.random_fields(w, 2)]
    n0 = les.nu_smagorinsky(g, u, 0.1)
    n1 = les.nu_smagorinsky(g, [x + v for x, v in zip(u, (3.0, -1.0, 0.5))], 0.1)
    assert float((n0 - n1).abs().max()) < 1e-12 * float(n0.max())


def test_les_step_gradient_matches_central_differences():
    cfg = {"cs": 0.15, "wall_model": True, "kappa": KAPPA, "B": B, "eps": 1e-6}
    w = _channel_grid(nx=6, ny=8, nz=4, les_cfg=cfg, seed=1)
    w.nu = 1e-3
    g = Grid(w)
    rng = np.random.default_rng(4)
    u0 = W.random_fields(w, 11)
    u0[0] = u0[0] + 3.0
    for c in (1,):
        u0[c][:, 0, :] = 0.0
        u0[c][:, -1, :] = 0.0
    fb = W.random_fields(w, 12, 0.1)
    wgt = W.random_fields(w, 13)
    dirs = [rng.standard_normal(s) for s in (w.face_shape(c) for c in range(3))]
    dirs[1][:, 0, :] = 0.0
    dirs[1][:, -1, :] = 0.0

    def J(ulist, grad=False):
        ut = [torch.tensor(x, requires_grad=grad) for x in ulist]
        st, _ = step(g, init_state(g, ut), make_params(g, fb))
        val = sum((st["u"][c] * torch.tensor(wgt[c])).sum() for c in range(3))
        return val, ut

    val, ut = J(u0, True)
    val.backward()
    ad = sum(float((ut[c].grad * torch.tensor(dirs[c])).sum()) for c in range(3))
    h = 1e-6
    jp = float(J([x + h * d for x, d in zip(u0, dirs)])[0])
    jm = float(J([x - h * d for x, d in zip(u0, dirs)])[0])
    fd = (jp - jm) / (2 * h)
    assert abs(ad - fd) <= 1e-6 * abs(fd), (ad, fd)


def test_les_rejects_unsupported_grids():
    faces = [np.linspace(0, 1, 5)] * 3
    w = W.generic(3, (4, 4, 4), faces, [["inflow", "outflow_conv"], ["noslip", "noslip"],
                                        ["periodic", "periodic"]])
    w.les = {"cs": 0.1, "wall_model": False}
    with pytest.raises(ValueError):
        les.sgs_force(Grid(w), [torch.zeros(w.face_shape(c), dtype=F64) for c in range(3)])
