"""Pins of the oracle's stretched-grid stencils, boundary rules, losses and
pressure operator against exact discrete identities.

Every expected value here is computed from the raw face coordinates and
from closed forms (linear profiles, telescoping sums, a translating linear
outlet profile, a sinusoid, a face-by-face sparse assembly, a hand-drawn
mask), never from the oracle's own metric tables, so a wrong weight,
divisor, sign or neighbour rule in the oracle fails one of them.  CPU only.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import torch

import fvib_workloads as W
from oracle import Grid, init_state, make_params, step
from oracle import fluid, ibm
from oracle.poisson import apply_A
from oracle.step import rms_lift, wall_shear
from test_oracle_pins import _assemble_sparse

F64 = torch.float64
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _centres(f):
    return 0.5 * (f[:-1] + f[1:])


def _channel3d(nx=6, ny=11, nz=5, gamma=1.4, wall="noslip", nu=0.01, dt=1e-3):
    xf = np.linspace(0.0, 2.0, nx + 1)
    yf = W.tanh_faces(ny, gamma)
    zf = np.linspace(0.0, 1.0, nz + 1)
    w = W.generic(3, (nx, ny, nz), [xf, yf, zf],
                  [["periodic", "periodic"], [wall, wall], ["periodic", "periodic"]],
                  nu=nu, dt=dt)
    return w, xf, yf, zf


# ------------------------------------------------ linear interpolation (Eq. 4)
def test_stretched_cross_flux_exact_for_linear_profiles():
    """Carrying a cell quantity to a face of a stretched axis is linear
    interpolation between the two cell centres: for u and w linear in y and
    a uniform v, d(u v)/dy = b_u V and d(w v)/dy = b_w V exactly at every
    row whose two faces are interior, and the v-equation sees no flux
    difference.  Replacing the interpolation weight by 1/2, or swapping its
    two partners, breaks the identity on a stretched axis."""
    w, xf, yf, zf = _channel3d()
    g = Grid(w)
    yc = _centres(yf)
    au, bu, aw, bw, V = 0.3, 1.7, -0.4, 0.9, 0.65
    u = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(3)]
    u[0][...] = torch.tensor(au + bu * yc)[None, :, None]
    u[1][...] = V
    u[2][...] = torch.tensor(aw + bw * yc)[None, :, None]
    C = fluid.convection(g, u)
    ny = w.n[1]
    rows = slice(1, ny - 1)
    assert float((C[0][:, rows, :] - bu * V).abs().max()) < 1e-12 * bu * V
    assert float((C[2][:, rows, :] - bw * V).abs().max()) < 1e-12 * bw * V
    # v-equation: interior v faces 2 .. ny-2 (index 0 of C[1] is face 1)
    assert float(C[1][:, 1:ny - 2, :].abs().max()) < 1e-12


# ---------------------------------------------------- diffusion on stretching
def _diffusion_case(seed):
    w, xf, yf, zf = _channel3d()
    g = Grid(w)
    u = [torch.tensor(x) for x in W.random_fields(w, seed)]
    # wall rows of u and w at zero (their mirror ghosts are then zero too),
    # v zero on the wall faces
    u[0][:, 0, :] = 0.0
    u[0][:, -1, :] = 0.0
    u[2][:, 0, :] = 0.0
    u[2][:, -1, :] = 0.0
    u[1][:, 0, :] = 0.0
    u[1][:, -1, :] = 0.0
    return w, g, u, yf


def test_stretched_diffusion_telescopes_with_geometric_volumes():
    """Finite-volume diffusion is a difference of face fluxes divided by
    the control-volume width: weighted by the geometric widths (cells for u
    and w across y, the face control volume between two centres for v along
    y) the sum over y telescopes to the boundary fluxes, which vanish here.
    A wrong divisor in either the own-axis or the cross-axis term breaks
    it."""
    w, g, u, yf = _diffusion_case(31)
    yc = _centres(yf)
    dy = np.diff(yf)                          # cell widths
    dvc = yc[1:] - yc[:-1]                    # v control volumes, faces 1..ny-1
    L = fluid.diffusion(g, u)
    # x and z are uniform and periodic: their parts telescope in the total
    for c in (0, 2):
        s = float((L[c] * torch.tensor(dy)[None, :, None]).sum())
        scale = float((L[c].abs() * torch.tensor(dy)[None, :, None]).sum())
        assert abs(s) < 1e-13 * scale, c
    # v: evolved faces 1..ny-1; their y-flux telescopes to
    # (v_N - v_{N-1})/dy_{N-1} - (v_1 - v_0)/dy_0 = -v_{N-1}/dy_{N-1} - v_1/dy_0
    v = u[1]
    s = (L[1] * torch.tensor(dvc)[None, :, None]).sum(dim=1)
    # the x and z parts telescope over the periodic directions separately, so
    # compare the sum over all three directions
    tot = float(s.sum())
    exp = float((-v[:, -2, :] / dy[-1] - v[:, 1, :] / dy[0]).sum())
    assert abs(tot - exp) < 1e-12 * float((L[1].abs() * torch.tensor(dvc)[None, :, None]).sum())


def test_stretched_diffusion_green_identity():
    """Discrete Green identity of the y part of the Laplacian on a
    stretched axis: sum_j vol_j q_j (L q)_j = -sum_faces (q_j - q_{j-1})^2 / dist
    with the distances between the two points each face separates.  Pins the
    numerator spacings as well as the divisor."""
    w, xf, yf, zf = _channel3d(nx=3, nz=3)
    g = Grid(w)
    yc = _centres(yf)
    dy = np.diff(yf)
    rng = np.random.default_rng(5)
    ny = w.n[1]
    # x- and z-invariant fields: only the y part of the Laplacian acts
    qu = rng.uniform(-1, 1, ny)
    qu[0] = qu[-1] = 0.0
    qv = rng.uniform(-1, 1, ny + 1)
    qv[0] = qv[-1] = 0.0
    u = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(3)]
    u[0][...] = torch.tensor(qu)[None, :, None]
    u[1][...] = torch.tensor(qv)[None, :, None]
    L = fluid.diffusion(g, u)
    lu = L[0][0, :, 0].numpy()
    lhs = float(np.sum(dy * qu * lu))
    rhs = -float(np.sum((qu[1:] - qu[:-1]) ** 2 / (yc[1:] - yc[:-1])))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    lv = L[1][0, :, 0].numpy()                 # faces 1 .. ny-1
    dvc = yc[1:] - yc[:-1]
    lhs = float(np.sum(dvc * qv[1:-1] * lv))
    rhs = -float(np.sum((qv[1:] - qv[:-1]) ** 2 / dy))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


# --------------------------------------------- P3 stretched Poiseuille
def _tridiagonal_poiseuille(yf, G, nu):
    """-nu (F_{j+1} - F_j) / dy_j = G with F_j = (u_j - u_{j-1}) / (yc_j - yc_{j-1})
    on interior faces and no-slip mirror ghosts on the walls (F_0 = u_0 /
    (yc_0 - yf_0), F_N = -u_{N-1} / (yf_N - yc_{N-1})), solved as a banded
    system."""
    yc = _centres(yf)
    n = yc.size
    dy = np.diff(yf)
    kf = np.zeros(n + 1)
    kf[1:n] = 1.0 / (yc[1:] - yc[:-1])
    k0 = 1.0 / (yc[0] - yf[0])
    kN = 1.0 / (yf[-1] - yc[-1])
    diag = np.zeros(n)
    up = np.zeros(n)
    lo = np.zeros(n)
    for j in range(n):
        # nu/dy_j * [ (u_j - u_{j-1}) kf_j - (u_{j+1} - u_j) kf_{j+1} ] = G
        a_lo = kf[j] if j > 0 else 0.0
        a_hi = kf[j + 1] if j < n - 1 else 0.0
        wall = (k0 if j == 0 else 0.0) + (kN if j == n - 1 else 0.0)
        diag[j] = nu * (a_lo + a_hi + wall) / dy[j]
        if j > 0:
            lo[j] = -nu * a_lo / dy[j]
        if j < n - 1:
            up[j] = -nu * a_hi / dy[j]
    ab = np.zeros((3, n))
    ab[0, 1:] = up[:-1]
    ab[1] = diag
    ab[2, :-1] = lo[1:]
    return scipy.linalg.solve_banded((1, 1), ab, np.full(n, G))


@pytest.mark.parametrize("ny,gamma", [(12, 1.45), (17, 2.0)])
def test_p3_poiseuille_stretched_fixed_point_vs_tridiagonal(ny, gamma):
    """The step maps a streamwise-invariant profile affinely; its fixed
    point on a tanh-stretched wall-normal axis equals the independent
    banded solve of the 1D finite-volume balance to round-off."""
    G, nu = 1.3, 0.7
    yf = W.tanh_faces(ny, gamma)
    w = W.generic(2, (3, ny, 1), [np.linspace(0, 1, 4), yf],
                  [["periodic", "periodic"], ["noslip", "noslip"]], nu=nu, dt=1.0)
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
    ref = _tridiagonal_poiseuille(yf, G, nu)
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


# ------------------------------------------------- convective outflow (Table 1)
@pytest.mark.parametrize("side", ["high", "low"])
def test_convective_outflow_translates_a_linear_profile(side):
    """du/dt + U_c du/dn = 0 moves a profile linear in the normal coordinate
    rigidly at speed U_c; forward Euler with the one-sided difference does
    this exactly, so the predicted outlet face equals a + b (x_b -+ U_c dt)."""
    nx, ny = 12, 5
    xf = np.linspace(0.0, 4.0, nx + 1)
    bcv = np.zeros((3, 2, 3))
    if side == "high":
        bc = [["inflow", "outflow_conv"], ["freeslip", "freeslip"]]
        bcv[0, 0, 0] = 1.0
    else:
        bc = [["outflow_conv", "inflow"], ["freeslip", "freeslip"]]
        bcv[0, 1, 0] = -1.0
    w = W.generic(2, (nx, ny, 1), [xf, np.linspace(0, 1, ny + 1)], bc, bc_vel=bcv,
                  nu=0.01, dt=0.013, u_conv=0.7)
    g = Grid(w)
    a, b = 0.4, -0.35
    u = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(2)]
    u[0][...] = torch.tensor(a + b * xf)[None, None, :]
    out = fluid.boundary_normal(g, u, [x.clone() for x in u])
    if side == "high":
        exp = a + b * (xf[-1] - w.u_conv * w.dt)
        got = out[0][..., -1]
    else:
        exp = a + b * (xf[0] + w.u_conv * w.dt)
        got = out[0][..., 0]
    assert float((got - exp).abs().max()) < 1e-14


# ----------------------------------------------------- IB point classes
def _read_mask_fixture():
    poly, rows = None, {"u": [], "v": []}
    with open(os.path.join(GOLD, "ib_mask_square.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(None, 1)
            if key == "polygon":
                poly = np.array([float(x) for x in val.split()]).reshape(-1, 2)
            else:
                rows[key].append(val)
    return poly, rows


def test_ib_point_classes_match_hand_drawn_fixture():
    poly, rows = _read_mask_fixture()
    f = np.linspace(0.0, 12.0, 13)
    w = W.generic(2, (12, 12, 1), [f, f], [["periodic", "periodic"]] * 2)
    g = Grid(w)
    solid, ib, eps = ibm.classify(g, poly)
    code = {".": 0, "S": 1, "I": 2}
    for c, key in enumerate(("u", "v")):
        exp = np.array([[code[ch] for ch in r] for r in rows[key]])
        got = solid[c][0].numpy().astype(int) + 2 * ib[c][0].numpy().astype(int)
        assert np.array_equal(got, exp), (key, got)
        assert np.array_equal(eps[c][0].numpy(), exp > 0)


# ------------------------------------------------------------ losses
def test_wall_shear_of_linear_wall_profiles():
    """u = s (1 - |y|) near both walls: the one-sided wall gradient is s at
    each wall, so J = nu s."""
    w, xf, yf, zf = _channel3d(nx=4, ny=9, nz=3, nu=0.037)
    g = Grid(w)
    s = 2.3
    u = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(3)]
    u[0][...] = torch.tensor(s * (1.0 - np.abs(_centres(yf))))[None, :, None]
    J = float(wall_shear(g, u))
    assert abs(J - w.nu * s) < 1e-15 * max(1.0, w.nu * s)


def test_p6_channel_momentum_budget_ties_to_wall_shear():
    """Streamwise momentum of a channel with x, z periodic and resting
    walls changes per step by the body force minus the viscous wall drag:
    (M^{n+1} - M^n)/dt = sum f_b dV - 2 Lx Lz J(u^n).  Convection and the
    pressure gradient telescope; only the wall fluxes remain."""
    w, xf, yf, zf = _channel3d(nx=6, ny=8, nz=5, nu=0.05, dt=2e-3)
    g = Grid(w)
    u0 = W.random_fields(w, 41)
    u0[1][:, 0, :] = 0.0
    u0[1][:, -1, :] = 0.0
    fb = W.random_fields(w, 42, 0.8)
    st = init_state(g, u0)
    st1, _ = step(g, st, make_params(g, fb))
    dV = (np.diff(xf)[None, None, :] * np.diff(yf)[None, :, None] * np.diff(zf)[:, None, None])
    M0 = float(np.sum(u0[0] * dV))
    M1 = float(np.sum(st1["u"][0].numpy() * dV))
    Lx, Lz = xf[-1] - xf[0], zf[-1] - zf[0]
    J = float(wall_shear(g, [torch.tensor(x) for x in u0]))
    rhs = float(np.sum(fb[0] * dV)) - 2.0 * Lx * Lz * J
    assert abs((M1 - M0) / w.dt - rhs) < 1e-11 * (abs(rhs) + 2 * Lx * Lz * abs(J))


@pytest.mark.parametrize("u_ref,diameter", [(1.0, 1.0), (2.0, 0.5)])
def test_rms_lift_of_a_sinusoid(u_ref, diameter):
    """C_L = A sin(2 pi n / P) sampled over whole periods has RMS A / sqrt 2
    (the mean of sin^2 over P >= 3 equally spaced phases is 1/2)."""
    w = W.tgv2d(n=8)
    g = Grid(w)
    P, A = 8, 0.37
    n = np.arange(3 * P)
    Fh = np.zeros((n.size, 3))
    Fh[:, 1] = 0.5 * u_ref * u_ref * diameter * A * np.sin(2 * np.pi * n / P)
    Fh[:, 0] = 5.0                      # drag does not enter
    J = float(rms_lift(g, torch.tensor(Fh), u_ref=u_ref, diameter=diameter))
    assert abs(J - A / math.sqrt(2.0)) < 1e-15


# ------------------------------------------------------ pressure operator
@pytest.mark.parametrize("case", ["periodic2d", "mixed2d", "channel3d", "box3d"])
def test_apply_A_equals_face_by_face_assembly(case):
    """The matrix-free operator equals the matrix assembled face by face
    from the definition (A p)_c = sum_f (A_f / dc_f)(p_c - p_nb)."""
    if case == "periodic2d":
        w = W.tgv2d(n=9)
    elif case == "mixed2d":
        w = W.cylinder(nx=11, ny=7, markers=8)
    elif case == "channel3d":
        w = W.channel(nx=5, ny=7, nz=4)
    else:
        w = W.generic(3, (5, 6, 4), [np.linspace(0, 1, 6), W.tanh_faces(6, 1.2),
                      np.linspace(0, 2, 5) ** 1.3], [["inflow", "outflow_conv"],
                      ["noslip", "freeslip"], ["noslip", "noslip"]])
    g = Grid(w)
    A = _assemble_sparse(g)
    p = np.random.default_rng(8).standard_normal(g.cell_shape())
    ref = (A @ p.reshape(-1)).reshape(p.shape)
    got = apply_A(g, torch.tensor(p)).numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
