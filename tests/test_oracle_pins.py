"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what it pins and what plausible mistake it would catch.
All run on the CPU (no GPU marker).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg
import torch

import fvib_workloads as W
from oracle import Grid, init_state, make_params, rollout, step
from oracle import body as bodymod
from oracle import fluid, ibm
from oracle.poisson import solver

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F64 = torch.float64


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- P1 kernel
def test_p1_kernel_golden_values():
    """Eq. 22 at half-integer shifts (hand-evaluated closed forms)."""
    for s, v in _read_table("peskin4.txt"):
        got = float(ibm.phi4(torch.tensor([float(s)], dtype=F64))[0])
        assert abs(got - float(v)) < 2e-16, (s, got, v)


def test_p1_kernel_moment_identities():
    """Known identities of the 4-point kernel (Peskin 2002): partition of
    unity, zero first moment, even/odd sums 1/2, sum of squares 3/8, for
    every shift.  A wrong constant or sign in either branch breaks them."""
    shifts = torch.linspace(0.0, 1.0, 1001, dtype=F64)
    j = torch.arange(-4, 6, dtype=F64)
    r = shifts[:, None] - j[None, :]
    ph = ibm.phi4(r)
    assert torch.allclose(ph.sum(1), torch.ones_like(shifts), atol=1e-15)
    assert (r * ph).sum(1).abs().max() < 1e-15
    even = (j % 2 == 0)
    assert torch.allclose(ph[:, even].sum(1), 0.5 * torch.ones_like(shifts), atol=1e-15)
    assert torch.allclose(ph[:, ~even].sum(1), 0.5 * torch.ones_like(shifts), atol=1e-15)
    assert torch.allclose((ph * ph).sum(1), 0.375 * torch.ones_like(shifts), atol=1e-15)


def test_p1_kernel_scaling():
    """d_h(r) = phi(r/h)/h, so its integral over a uniform grid is 1."""
    h = 0.37
    x = torch.arange(-10, 11, dtype=F64) * h + 0.123
    assert abs(float(ibm.d_h(x, h).sum() * h) - 1.0) < 1e-14


# ------------------------------------------------------- P2 periodic fluid
def _shear_decay(n, dim):
    """u = sin(y) on a periodic grid: convection is identically zero and the
    projection inactive, so each step multiplies the mode by exactly
    1 + nu dt lam_h with lam_h = -(4/h^2) sin^2(h/2)."""
    L = 2 * np.pi
    f = np.linspace(0, L, n + 1)
    faces = [f, f, f]
    bc = [["periodic", "periodic"]] * 3
    w = W.generic(dim, (n, n, n if dim == 3 else 1), faces, bc, nu=0.05, dt=2e-3)
    g = Grid(w)
    u0 = [np.zeros(g.face_shape(c)) for c in range(dim)]
    y = g.xc[1].numpy()
    u0[0][...] = np.sin(y)[None, :, None]
    st = init_state(g, u0)
    pr = make_params(g)
    nsteps = 25
    st, _, _ = rollout(g, st, pr, nsteps)
    h = L / n
    lam = -(4.0 / h ** 2) * math.sin(h / 2) ** 2
    amp = (1.0 + w.nu * w.dt * lam) ** nsteps
    return st["u"], amp * np.sin(y)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_stokes_mode_closed_form(dim):
    u, ref = _shear_decay(12 if dim == 3 else 16, dim)
    assert np.abs(u[0].numpy() - ref[None, :, None]).max() < 1e-13
    for c in range(1, dim):
        assert u[c].abs().max() < 1e-13


def _tgv_error(n):
    w = W.tgv2d(n=n, steps=20, dt=1e-3)
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    st, _, _ = rollout(g, init_state(g, u0), make_params(g, fb), w.steps)
    t = w.steps * w.dt
    x, y, _ = g.face_coords(0)
    ua = (torch.sin(x)[None, None, :] * torch.cos(y)[None, :, None]) * math.exp(-2 * w.nu * t)
    return float((st["u"][0] - ua).abs().max())


def test_p2_tgv_second_order():
    """Analytic TGV decay: the error falls at second order in h (temporal
    error O(dt) is far smaller here)."""
    e = [_tgv_error(n) for n in (16, 32, 64)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, e


def test_p2_tgv_initial_divergence_free():
    w = W.tgv2d(n=32)
    g = Grid(w)
    u0, _ = W.initial_fields(w)
    d = fluid.divergence(g, [torch.tensor(x) for x in u0])
    assert float(d.abs().max()) < 1e-13


# ------------------------------------------------------- P3 walls, stretching
@pytest.mark.parametrize("stretched", [False, True])
def test_p3_couette_exact_steady_state(stretched):
    """A linear profile between a fixed and a moving wall is an exact
    discrete steady state (mirror ghosts, moving-wall value, stretched
    metrics).  A wrong ghost rule or centre spacing breaks it."""
    ny = 12
    yf = W.tanh_faces(ny, 1.3) if stretched else np.linspace(-1, 1, ny + 1)
    xf = np.linspace(0, 1, 5)
    bcv = np.zeros((3, 2, 3))
    bcv[1, 1, 0] = 2.5                      # top wall moves in +x
    w = W.generic(2, (4, ny, 1), [xf, yf], [["periodic", "periodic"], ["noslip", "noslip"]],
                  bc_vel=bcv, nu=0.3, dt=1e-3)
    g = Grid(w)
    yc = g.xc[1].numpy()
    u0 = [np.zeros(g.face_shape(0)), np.zeros(g.face_shape(1))]
    u0[0][...] = (2.5 * (yc + 1.0) / 2.0)[None, :, None]
    st, _, _ = rollout(g, init_state(g, u0), make_params(g), 10)
    assert np.abs(st["u"][0].numpy() - u0[0]).max() < 1e-13
    assert float(st["u"][1].abs().max()) < 1e-13


def _poiseuille_fixed_point(ny):
    """The step is affine in a streamwise-invariant profile u(y); its fixed
    point solves (I - M) u = s, with M and s read off the oracle step."""
    G, nu = 1.0, 1.0
    yf = np.linspace(-1, 1, ny + 1)
    w = W.generic(2, (2, ny, 1), [np.linspace(0, 1, 3), yf],
                  [["periodic", "periodic"], ["noslip", "noslip"]], nu=nu, dt=1e-3)
    g = Grid(w)
    fb = [np.full(g.face_shape(0), G), np.zeros(g.face_shape(1))]
    pr = make_params(g, fb)

    def apply(prof):
        u0 = [np.zeros(g.face_shape(0)), np.zeros(g.face_shape(1))]
        u0[0][...] = prof[None, :, None]
        st, _ = step(g, init_state(g, u0), pr)
        return st["u"][0][0, :, 0].numpy()

    s = apply(np.zeros(ny))
    M = np.stack([apply(np.eye(ny)[j]) - s for j in range(ny)], axis=1)
    u = np.linalg.solve(np.eye(ny) - M, s)
    yc = g.xc[1].numpy()
    exact = G / (2 * nu) * (1 - yc ** 2)
    return np.abs(u - exact).max()


def test_p3_poiseuille_second_order():
    """Steady channel flow converges to the parabola (G/2nu)(1 - y^2) at
    second order."""
    e = [_poiseuille_fixed_point(n) for n in (8, 16, 32)]
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


# --------------------------------------------------- P4 conservation / energy
def _random_periodic(dim, n, seed, conv="central"):
    L = 2 * np.pi
    f = np.linspace(0, L, n + 1)
    w = W.generic(dim, (n, n + 1, n + 2 if dim == 3 else 1), [f, np.linspace(0, L, n + 2),
                  np.linspace(0, L, n + 3)], [["periodic", "periodic"]] * 3, nu=0.02, dt=1e-3,
                  conv=conv)
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, seed)]
    return w, g, u


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("conv", ["central", "upwind"])
def test_p4_momentum_conservation(dim, conv):
    """Divergence-form fluxes telescope on a periodic grid: sum of C over
    all faces is zero, for central and upwind, with or without continuity.
    An index slip in a flux difference breaks the telescoping."""
    w, g, u = _random_periodic(dim, 6, 11, conv)
    C = fluid.convection(g, u)
    Lp = fluid.diffusion(g, u)
    for c in range(dim):
        assert abs(float(C[c].sum())) < 1e-12
        assert abs(float(Lp[c].sum())) < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_p4_central_energy_conservation(dim):
    """Divergence-form central convection on a uniform staggered grid is
    energy neutral for a discretely divergence-free field (Morinishi et al.
    1998): sum u . C(u) = 0.  Catches wrong averaging partners or a transposed
    edge flux."""
    n = 8
    L = 2 * np.pi
    f = np.linspace(0, L, n + 1)
    w = W.generic(dim, (n, n, n if dim == 3 else 1), [f, f, f], [["periodic", "periodic"]] * 3,
                  nu=0.0, dt=1e-3)
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, 5)]
    b = fluid.flux_divergence(g, u)
    p = solver(g).solve(b - b.mean())
    # remove the divergence with the exact projection (rho = dt = 1 scaling)
    up = [u[c] + fluid.pressure_gradient(g, p, c) for c in range(dim)]
    # sign convention: A p = -V D G p = b  =>  D(u + G p) = 0
    assert float(fluid.divergence(g, up).abs().max()) < 1e-12
    C = fluid.convection(g, up)
    e = sum(float((up[c] * C[c]).sum()) for c in range(dim))
    scale = sum(float((up[c].abs() * C[c].abs()).sum()) for c in range(dim))
    assert abs(e) < 1e-13 * scale


def test_p4_upwind_first_order_dissipative():
    """Upwinding adds dissipation: the kinetic energy of a divergence-free
    field decreases under pure convection (nu = 0), unlike central."""
    n = 8
    f = np.linspace(0, 2 * np.pi, n + 1)
    for conv, sign in (("upwind", -1), ("central", 0)):
        w = W.generic(2, (n, n, 1), [f, f], [["periodic", "periodic"]] * 2, nu=0.0, dt=1e-3,
                      conv=conv)
        g = Grid(w)
        u = [torch.tensor(x) for x in W.random_fields(w, 3)]
        b = fluid.flux_divergence(g, u)
        p = solver(g).solve(b - b.mean())
        up = [u[c] + fluid.pressure_gradient(g, p, c) for c in range(2)]
        C = fluid.convection(g, up)
        e = sum(float((up[c] * C[c]).sum()) for c in range(2))
        if sign < 0:
            assert e > 1e-3          # dE/dt = -sum u.C < 0
        else:
            assert abs(e) < 1e-12


# --------------------------------------------------------- P5 divergence
@pytest.mark.parametrize("name", ["cylinder", "viv", "channel", "tgv3d"])
def test_p5_post_projection_divergence(name):
    """D u^{n+1} = D[eps (u* - u_c)] (Eq. 8), which is zero for rigid
    bodies whose forced faces carry u* = u_c, and zero off-body."""
    w = W.by_name(name, "small")
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    st = init_state(g, u0, W.body_state0(w))
    pr = make_params(g, fb)
    for _ in range(2):
        st, aux = step(g, st, pr)
        d = fluid.divergence(g, st["u"])
        scale = max(float(x.abs().max()) for x in st["u"]) / min(float(g.dx[a].min()) for a in range(w.dim))
        assert float(d.abs().max()) < 1e-12 * scale


# ----------------------------------------------------------- P7 Poisson
def _assemble_sparse(g):
    """A assembled face by face from its definition (independent of the
    tensor-product solver)."""
    nx, ny, nz = g.n
    idx = lambda i, j, k: (k * ny + j) * nx + i
    rows, cols, vals = [], [], []
    N = [nx, ny, nz]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                cidx = [i, j, k]
                for a in range(g.dim):
                    for side in (0, 1):
                        nb = list(cidx)
                        nb[a] += -1 if side == 0 else 1
                        face = cidx[a] + side
                        if not g.periodic[a] and (nb[a] < 0 or nb[a] >= N[a]):
                            continue
                        nb[a] %= N[a]
                        area = 1.0
                        for b in range(g.dim):
                            if b != a:
                                area *= float(g.dx[b][cidx[b]])
                        coef = area / float(g.dc[a][face])
                        rows += [idx(*cidx), idx(*cidx)]
                        cols += [idx(*cidx), idx(*nb)]
                        vals += [coef, -coef]
    n = nx * ny * nz
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("case", ["periodic2d", "mixed2d", "channel3d", "box3d"])
def test_p7_exact_poisson_vs_sparse_direct(case):
    if case == "periodic2d":
        w = W.tgv2d(n=12)
    elif case == "mixed2d":
        w = W.cylinder(nx=14, ny=9, markers=8)
    elif case == "channel3d":
        w = W.channel(nx=6, ny=7, nz=5)
    else:
        w = W.generic(3, (5, 6, 4), [np.linspace(0, 1, 6), W.tanh_faces(6, 1.2),
                      np.linspace(0, 2, 5) ** 1.3], [["inflow", "outflow_conv"],
                      ["noslip", "freeslip"], ["noslip", "noslip"]])
    g = Grid(w)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(g.cell_shape())
    b -= b.mean()
    A = _assemble_sparse(g).tolil()
    rhs = b.reshape(-1).copy()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    rhs[0] = 0.0
    ref = scipy.sparse.linalg.spsolve(A.tocsr(), rhs)
    ref = ref - ref.mean()
    got = solver(g).solve(torch.tensor(b)).reshape(-1).numpy()
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


# ------------------------------------------------------------------ P8 IBM
def test_p8_polygon_classification_vs_half_planes():
    """Crossing-number test against the convex half-plane test for a
    regular polygon, on points away from the edges."""
    X0, _ = W.circle_markers(0.3, -0.2, 2.0, 37)
    rng = np.random.default_rng(0)
    P = rng.uniform(-1.5, 1.5, size=(20000, 2)) + np.array([0.3, -0.2])
    inside = ibm.inside_polygon(P[:, 0], P[:, 1], X0)
    M = X0.shape[0]
    margin = np.full(P.shape[0], np.inf)
    ref = np.ones(P.shape[0], dtype=bool)
    for k in range(M):
        a, b = X0[k], X0[(k + 1) % M]
        e = b - a
        nrm = np.array([e[1], -e[0]]) / np.hypot(*e)     # outward (CCW polygon)
        s = (P - a) @ nrm
        ref &= s < 0
        margin = np.minimum(margin, np.abs(s))
    ok = margin > 1e-9
    assert (inside[ok] == ref[ok]).all()


def test_p8_shepard_target_reproduces_rigid_velocity():
    w = W.by_name("viv", "small")
    g = Grid(w)
    bs = torch.tensor([0.0, 0.1, 0.0, 0.3, -0.7, 0.0], dtype=F64)
    from oracle.step import body_geometry
    Xk, U, dV = body_geometry(g, bs)
    masks = ibm.classify(g, Xk.numpy())
    us, uc = ibm.targets(g, masks, Xk, U, dV)
    for c in range(2):
        e = masks[2][c]
        assert e.sum() > 0
        assert torch.allclose(us[c][e], U[c].expand(int(e.sum())), atol=1e-15)
        assert float(us[c][~e].abs().max()) == 0.0
        assert masks[1][c].sum() > 0 and (masks[0][c] & masks[1][c]).sum() == 0


def test_p8_loads_partition_of_unity():
    """Constant forcing f on every face gives q_k = -f exactly (Eq. 20 with
    the partition of unity of the kernel), so F = -rho f sum_k dV_k."""
    w = W.by_name("viv", "small")
    g = Grid(w)
    Xk = torch.tensor(w.body.X0, dtype=F64)
    h = float(g.dx[0][0])
    dV = torch.tensor(w.body.ds, dtype=F64) * h
    allm = [torch.ones(g.face_shape(c), dtype=torch.bool) for c in range(2)]
    f = [torch.full(g.face_shape(0), 0.7, dtype=F64), torch.full(g.face_shape(1), -1.3, dtype=F64)]
    F = ibm.loads(g, (allm, allm, allm), f, Xk, dV)
    assert abs(float(F[0]) + 0.7 * float(dV.sum())) < 1e-13
    assert abs(float(F[1]) - 1.3 * float(dV.sum())) < 1e-13


def test_p8_comoving_body_is_a_fixed_point():
    """Uniform flow U in a periodic box with a body moving at U: the
    forcing vanishes and the flow stays uniform while the masks move."""
    n = 32
    f = np.linspace(0, 4, n + 1)
    X0, ds = W.circle_markers(2.0, 2.0, 1.0, 48)
    U = (0.4, -0.25)
    body = W.Body("spring", X0, ds, free_dof=(1, 1, 0), m=1.0, k=(0.0, 0.0, 0.0),
                  c=(0.0, 0.0, 0.0), v0=(U[0], U[1], 0.0))
    w = W.generic(2, (n, n, 1), [f, f], [["periodic", "periodic"]] * 2, nu=0.01, dt=0.01,
                  body=body)
    g = Grid(w)
    u0 = [np.full(g.face_shape(0), U[0]), np.full(g.face_shape(1), U[1])]
    st = init_state(g, u0, W.body_state0(w))
    pr = make_params(g)
    first = None
    for _ in range(6):
        st, aux = step(g, st, pr)
        if first is None:
            first = [e.clone() for e in aux["eps"]]
        for c in range(2):
            assert float(aux["f"][c].abs().max()) < 1e-12
            assert float((st["u"][c] - U[c]).abs().max()) < 1e-12
        assert float(aux["F"].abs().max()) < 1e-12
    assert any((first[c] != aux["eps"][c]).any() for c in range(2))
    assert abs(float(st["body"][0]) - 6 * 0.01 * U[0]) < 1e-14


# ----------------------------------------------------------------- P9 body
def test_p9_rk4_is_taylor_of_matrix_exponential():
    """For the linear oscillator the RK4 map equals sum_{j<=4} (dt A)^j / j!
    (a matrix identity), including the forcing term."""
    m, k, c, F, dt = 1.3, 2.1, 0.4, 0.9, 0.07
    A = np.array([[0.0, 1.0], [-k / m, -c / m]])
    T = sum(np.linalg.matrix_power(dt * A, j) / math.factorial(j) for j in range(5))
    # forcing: y' = A y + g  =>  y1 = T y0 + (sum_{j=1..4} dt^j A^{j-1}/j!) g
    S = sum(dt ** j * np.linalg.matrix_power(A, j - 1) / math.factorial(j) for j in range(1, 5))
    y0 = np.array([0.3, -0.2])
    g_ = np.array([0.0, F / m])
    ref = T @ y0 + S @ g_
    d1, v1 = bodymod.rk4(torch.tensor(0.3, dtype=F64), torch.tensor(-0.2, dtype=F64),
                         torch.tensor(F, dtype=F64), m, torch.tensor(k, dtype=F64),
                         torch.tensor(c, dtype=F64), dt)
    assert abs(float(d1) - ref[0]) < 1e-15 and abs(float(v1) - ref[1]) < 1e-15


def test_p9_free_oscillation_fourth_order():
    m, k = 1.5707963267948966, 2.4805021344239854
    om = math.sqrt(k / m)
    errs = []
    for dt in (0.04, 0.02):
        d = torch.tensor(0.1, dtype=F64)
        v = torch.tensor(0.0, dtype=F64)
        nsteps = int(round(3.6 / dt))   # not a multiple of the period (5)
        for _ in range(nsteps):
            d, v = bodymod.rk4(d, v, torch.tensor(0.0, dtype=F64), m, torch.tensor(k, dtype=F64),
                               torch.tensor(0.0, dtype=F64), dt)
        errs.append(abs(float(d) - 0.1 * math.cos(om * 3.6)))
    assert 14.0 < errs[0] / errs[1] < 18.0, errs


def test_p9_static_deflection():
    m, k, c, F = 1.0, 3.0, 2.0, 0.6
    d = torch.tensor(0.0, dtype=F64)
    v = torch.tensor(0.0, dtype=F64)
    for _ in range(4000):
        d, v = bodymod.rk4(d, v, torch.tensor(F, dtype=F64), m, torch.tensor(k, dtype=F64),
                           torch.tensor(c, dtype=F64), 0.01)
    assert abs(float(d) - F / k) < 1e-12 and abs(float(v)) < 1e-12


def test_p9_viv_constants_golden():
    vals = {k: float(v) for k, v in _read_table("viv_constants.txt")}
    w = W.viv()
    assert abs(w.body.m - vals["m"]) < 1e-15
    assert abs(w.meta["fn"] - vals["fn"]) < 1e-15
    assert abs(w.body.k[1] - vals["k"]) < 1e-14
    assert w.body.c[1] == vals["c"]


# ------------------------------------------------------ open boundaries
def _open_box(n=16, m=8):
    bcv = np.zeros((3, 2, 3))
    bcv[0, 0, 0] = 1.0
    return W.generic(2, (n, m, 1), [np.linspace(0, 4, n + 1), np.linspace(0, 2, m + 1)],
                     [["inflow", "outflow_conv"], ["freeslip", "freeslip"]], bc_vel=bcv,
                     nu=0.01, dt=0.01)


def test_open_boundaries_uniform_flow_fixed_point():
    """Uniform inflow through a free-slip channel with a convective outlet
    is a fixed point of the step (zero RHS, zero outflow correction)."""
    w = _open_box()
    g = Grid(w)
    u0 = [np.ones(g.face_shape(0)), np.zeros(g.face_shape(1))]
    st, _, _ = rollout(g, init_state(g, u0), make_params(g), 5)
    assert float((st["u"][0] - 1.0).abs().max()) < 1e-14
    assert float(st["u"][1].abs().max()) < 1e-14


def test_outflow_correction_balances_boundary_flux():
    """After the outflow correction the net flux through the boundary of
    the predicted field is zero, whatever the interior state."""
    w = _open_box()
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, 4)]
    eps = [torch.zeros(g.face_shape(c), dtype=torch.bool) for c in range(2)]
    zero = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(2)]
    ustar, _, _ = fluid.predictor(g, u, zero, eps, zero)
    net = float(fluid.flux_divergence(g, ustar).sum())
    assert abs(net) < 1e-13
    assert float((ustar[0][:, :, 0] - 1.0).abs().max()) == 0.0       # inflow held
    assert float(ustar[1][:, 0, :].abs().max()) == 0.0               # free-slip walls


def test_unused_ghost_layer_is_never_read(monkeypatch):
    """The ghost layer beyond a bounded axis' own boundary faces is filled
    with NaN: no NaN may reach R, so the stencils never read it."""
    real_zeros_like = torch.zeros_like

    def nan_ext(g, q, c):
        for a in range(g.dim):
            td = 2 - a
            n = q.shape[td]
            first, last = q.narrow(td, 0, 1), q.narrow(td, n - 1, 1)
            if g.periodic[a]:
                lo, hi = last, first
            elif a == c:
                lo = torch.full_like(first, float("nan"))
                hi = torch.full_like(last, float("nan"))
            else:
                lo = fluid._ghost(first, g.bc[a][0], g.bc_vel[a][0][c])
                hi = fluid._ghost(last, g.bc[a][1], g.bc_vel[a][1][c])
            q = torch.cat([lo, q, hi], dim=td)
        return q

    monkeypatch.setattr(fluid, "ext", nan_ext)
    for w in (_open_box(), W.by_name("channel", "small")):
        for conv in ("central", "upwind"):
            w.conv = conv
            g = Grid(w)
            u = [torch.tensor(x) for x in W.random_fields(w, 2)]
            fb = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(w.dim)]
            R = fluid.momentum_rhs(g, u, fb)
            assert all(torch.isfinite(r).all() for r in R)
    del real_zeros_like
