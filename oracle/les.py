"""Large-eddy simulation terms: the constant-coefficient Smagorinsky
subgrid model and the equilibrium wall-stress model (paper Sec. 2.5,
Table 1, and Sec. 3.4.5, Eqs. 27-29).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the models and the wall law but not their discretisation.
Readings taken here:

* the subgrid stress is tau_ij = -2 nu_t S_ij with the resolved strain
  S_ij = (d_j u_i + d_i u_j) / 2; its divergence is added to the momentum
  right-hand side R next to the molecular term nu lap(u), which keeps its
  Laplacian form, so nu_t = 0 gives the plain step back;
* nu_t = (C_s Delta)^2 |S| with |S| = sqrt(2 S_ij S_ij) and
  Delta = (dx dy dz)^(1/3), at cell centres (no anisotropy correction,
  no near-wall damping: "constant coefficient");
* S at a cell centre: the diagonal from the cell's two faces, an
  off-diagonal entry as the mean of the symmetric gradient
  (d_a u_c + d_c u_a) / 2 on the four cell edges around the centre in that
  plane; an edge gradient is the difference of the two values beside the
  edge over their centre spacing, ghost values behind a wall taken as for
  the molecular term (mirrored about the wall);
* the stress sits where its divergence needs it on the staggered grid:
  normal stresses at cell centres (nu_t of the cell), shear stresses on
  the cell edges with the mean nu_t of the four cells around the edge;
  on an edge lying on a wall the subgrid viscosity is zero unless the wall
  model sets it;
* wall model (walls normal to y, x and z periodic): at every streamwise
  face of the first cell row next to a wall, and at every spanwise face of
  that row, the tangential speed U = sqrt(u^2 + w^2) relative to the wall
  takes the other component as the mean of its four nearest faces in the
  row; the matching distance y is the half height of the wall cell; the
  Spalding law (Eq. 27) gives u_tau by a bracketed Newton-Raphson solve,
  tau_w = u_tau^2 (kinematic: the stress divided by rho), split by Eq. 29;
  Eq. 28 sets the subgrid viscosity of the wall edge, with du/dy the
  velocity gradient along the wall normal pointing into the fluid,
  (u - u_wall) / y, so that the wall edge carries the modelled stress;
* all grid axes are periodic or no-slip walls.
"""
from __future__ import annotations

import math

import torch

from . import fluid
from .grid import Grid, F64


def _cfg(g: Grid) -> dict:
    return getattr(g.w, "les", None)


# --------------------------------------------------------------- strain rate
def _diag_grad(g: Grid, u, c: int) -> torch.Tensor:
    """d_c u_c at the cell centres (cell shape)."""
    E = fluid.ext(g, u[c], c)
    spec = {a: (1, g.n[a] + 1) for a in range(3) if a != c}
    spec[c] = (1, g.n[c] + 2)                     # faces 0..N
    X = fluid._sl(E, spec)
    td = 2 - c
    d = X.narrow(td, 1, g.n[c]) - X.narrow(td, 0, g.n[c])
    return d / g.bshape(c, g.dx[c])


def edge_grad(g: Grid, u, c: int, a: int) -> torch.Tensor:
    """(d_a u_c + d_c u_a) on the (c, a) edge lattice: c-faces 0..N_c along
    c, a-faces 0..N_a along a, cells along the third axis."""
    b = 3 - a - c
    Ec = fluid.ext(g, u[c], c)
    Ea = fluid.ext(g, u[a], a)
    # d_a u_c: u_c on c-faces, cells j-1 and j along a (ext index j, j+1)
    s = {b: (1, g.n[b] + 1), c: (1, g.n[c] + 2), a: (0, g.n[a] + 2)}
    X = fluid._sl(Ec, s)
    ta = 2 - a
    dac = (X.narrow(ta, 1, g.n[a] + 1) - X.narrow(ta, 0, g.n[a] + 1)) / g.bshape(a, g.dc[a])
    # d_c u_a: u_a on a-faces, cells i-1 and i along c
    s = {b: (1, g.n[b] + 1), a: (1, g.n[a] + 2), c: (0, g.n[c] + 2)}
    Y = fluid._sl(Ea, s)
    tc = 2 - c
    dca = (Y.narrow(tc, 1, g.n[c] + 1) - Y.narrow(tc, 0, g.n[c] + 1)) / g.bshape(c, g.dc[c])
    return dac + dca


def _edge_to_cell(g: Grid, G: torch.Tensor, c: int, a: int) -> torch.Tensor:
    """Mean of the four edge values around each cell centre in the (c, a) plane."""
    tc, ta = 2 - c, 2 - a
    nc, na = g.n[c], g.n[a]
    s = (G.narrow(tc, 0, nc) + G.narrow(tc, 1, nc))
    return 0.25 * (s.narrow(ta, 0, na) + s.narrow(ta, 1, na))


def strain(g: Grid, u):
    """Cell-centred S: dict {(i, j): tensor} for i <= j."""
    S = {}
    for c in range(3):
        S[(c, c)] = _diag_grad(g, u, c)
    for c, a in ((0, 1), (0, 2), (1, 2)):
        S[(c, a)] = 0.5 * _edge_to_cell(g, edge_grad(g, u, c, a), c, a)
    return S


def filter_width(g: Grid) -> torch.Tensor:
    """Delta = (dx dy dz)^(1/3) per cell."""
    return g.cell_volume() ** (1.0 / 3.0)


def nu_smagorinsky(g: Grid, u, cs: float) -> torch.Tensor:
    """nu_t = (C_s Delta)^2 sqrt(2 S_ij S_ij) at the cell centres."""
    S = strain(g, u)
    ss = S[(0, 0)] ** 2 + S[(1, 1)] ** 2 + S[(2, 2)] ** 2 + \
        2.0 * (S[(0, 1)] ** 2 + S[(0, 2)] ** 2 + S[(1, 2)] ** 2)
    mag = torch.sqrt(2.0 * ss)
    return (cs * filter_width(g)) ** 2 * mag


# ------------------------------------------------------------- Spalding law
def spalding_yplus(up: torch.Tensor, kappa: float, B: float):
    """Eq. 27 read forwards: y+ as a function of u+, and dy+/du+."""
    k = kappa * up
    e = math.exp(-kappa * B)
    ek = torch.exp(k)
    yp = up + e * (ek - 1.0 - k - 0.5 * k * k - k * k * k / 6.0)
    dyp = 1.0 + e * kappa * (ek - 1.0 - k - 0.5 * k * k)
    return yp, dyp


def _spalding_h(t: torch.Tensor, lre: torch.Tensor, kappa: float, B: float):
    """h(t) = ln(u+ y+(u+)) - ln Re at u+ = e^t, and dh/dt.  Re = U y / nu
    equals u+ y+, so the root of h is the u+ of Eq. 27."""
    up = torch.exp(t)
    yp, dyp = spalding_yplus(up, kappa, B)
    return t + torch.log(yp) - lre, 1.0 + up * dyp / yp


def spalding_uplus(re: torch.Tensor, kappa: float = 0.4, B: float = 5.0) -> torch.Tensor:
    """u+ solving Eq. 27 for Re = U y / nu > 0 (u+ below 200).

    Newton-Raphson on h(t) above, t = ln u+: u+ y+ increases with u+, and
    in t the law is close to linear in the viscous sublayer (h ~ 2t) and
    in the log layer (h ~ kappa e^t), so the iteration needs few steps.  It
    starts from the upper end of the bracket t in [t_hi - 80, t_hi],
    t_hi = min(ln sqrt(Re), ln 200) (u+ <= sqrt(Re) because y+ >= u+); a
    step leaving the current bracket is replaced by bisection, and the
    iteration stops once a step is below 1e-13.  The root is found without
    gradients; one more Newton step from it, with gradients, brings it to
    rounding level (quadratic convergence) and carries the implicit-function
    derivative dt/dRe = -h_Re / h_t."""
    with torch.no_grad():
        lre = torch.log(re.detach())
        hi = torch.clamp(0.5 * lre, max=math.log(200.0))
        lo = hi - 80.0
        t = hi.clone()
        for _ in range(200):
            h, dh = _spalding_h(t, lre, kappa, B)
            lo = torch.where(h < 0, t, lo)
            hi = torch.where(h > 0, t, hi)
            tn = t - h / dh
            bad = (tn <= lo) | (tn >= hi)
            tn = torch.where(bad, 0.5 * (lo + hi), tn)
            done = bool(((tn - t).abs() <= 1e-13).all())
            t = tn
            if done:
                break
    h, dh = _spalding_h(t, torch.log(re), kappa, B)
    return torch.exp(t - h / dh)


def wall_stress(U: torch.Tensor, y: float, nu: float, kappa: float, B: float) -> torch.Tensor:
    """tau_w / rho = u_tau^2 with u_tau = U / u+ (Eq. 27), zero where U = 0."""
    pos = U > 0
    Us = torch.where(pos, U, torch.ones_like(U))
    up = spalding_uplus(Us * (y / nu), kappa, B)
    tau = (Us / up) ** 2
    return torch.where(pos, tau, torch.zeros_like(U))


# --------------------------------------------------------------- wall model
def _wall_row(q: torch.Tensor, side: int) -> torch.Tensor:
    """The first cell row next to wall `side` of the y axis, (z, x) slab."""
    return q[:, 0, :] if side == 0 else q[:, -1, :]


def wall_viscosity(g: Grid, u, cfg: dict):
    """Eq. 28 on the wall edges: {(comp, side): (nz, nx) tensor} for the
    streamwise (comp 0) and spanwise (comp 2) components and both walls."""
    kappa, B, eps = cfg["kappa"], cfg["B"], cfg["eps"]
    out = {}
    for side in (0, 1):
        h = float(g.dx[1][0] if side == 0 else g.dx[1][-1])
        y = 0.5 * h
        uw = g.bc_vel[1][side]
        ur = _wall_row(u[0], side) - uw[0]          # (nz, nx) on x-faces i
        wr = _wall_row(u[2], side) - uw[2]          # (nz, nx) on z-faces k
        # w at the x-faces: cells i-1, i along x; faces k, k+1 along z
        wx = wr + torch.roll(wr, 1, dims=1)                 # w(i-1) + w(i) on z-face k
        wx = 0.25 * (wx + torch.roll(wx, -1, dims=0))       # faces k and k+1
        # u at the z-faces: faces i, i+1 along x; cells k-1, k along z
        uz = ur + torch.roll(ur, -1, dims=1)
        uz = 0.25 * (uz + torch.roll(uz, 1, dims=0))
        for comp, own, other in ((0, ur, wx), (2, wr, uz)):
            U = torch.sqrt(own * own + other * other)
            tau = wall_stress(U, y, g.nu, kappa, B)
            Us = torch.where(U > 0, U, torch.ones_like(U))
            tau_i = torch.where(U > 0, tau * own / Us, torch.zeros_like(U))   # Eq. 29
            dudn = own / y
            out[(comp, side)] = tau_i / (dudn + eps) - g.nu                     # Eq. 28
    return out


# ------------------------------------------------------- stress divergence
def _edge_nu(g: Grid, nu_c: torch.Tensor, c: int, a: int, nu_w) -> torch.Tensor:
    """nu on the (c, a) edge lattice: four-cell mean inside, zero on a
    wall, the wall-model value on the wall edges it defines."""
    tc, ta = 2 - c, 2 - a
    # cell ext along c and a: periodic wrap (zeros behind walls, unused)
    E = nu_c
    for ax in (c, a):
        t = 2 - ax
        n = E.shape[t]
        if g.periodic[ax]:
            lo, hi = E.narrow(t, n - 1, 1), E.narrow(t, 0, 1)
        else:
            lo = hi = torch.zeros_like(E.narrow(t, 0, 1))
        E = torch.cat([lo, E, hi], dim=t)
    s = E.narrow(tc, 0, g.n[c] + 1) + E.narrow(tc, 1, g.n[c] + 1)
    nu_e = 0.25 * (s.narrow(ta, 0, g.n[a] + 1) + s.narrow(ta, 1, g.n[a] + 1))
    # edges on walls
    keep = torch.ones_like(nu_e, dtype=torch.bool)
    for ax, t in ((c, tc), (a, ta)):
        if not g.periodic[ax]:
            idx = [slice(None)] * 3
            idx[t] = 0
            keep[tuple(idx)] = False
            idx[t] = -1
            keep[tuple(idx)] = False
    nu_e = torch.where(keep, nu_e, torch.zeros_like(nu_e))
    if nu_w is not None and (c, a) in ((0, 1), (1, 2)):
        comp = 0 if (c, a) == (0, 1) else 2         # tangential component
        slabs = []
        for side in (0, 1):
            wv = nu_w[(comp, side)]                 # (nz, nx) on comp's faces
            # the lattice repeats the first periodic face position at the end
            wv = torch.cat([wv, wv[:, :1]], dim=1) if comp == 0 else \
                torch.cat([wv, wv[:1, :]], dim=0)
            slabs.append(wv.unsqueeze(1))
        nu_e = torch.cat([slabs[0], nu_e[:, 1:-1, :], slabs[1]], dim=1)
    return nu_e


def stress_divergence(g: Grid, u, nu_c: torch.Tensor, nu_w=None) -> list:
    """d_j [nu_e (d_j u_c + d_c u_j)] on the evolved faces of each component
    (zero elsewhere), given the cell-centred nu_c and the wall-edge values."""
    out = []
    G = {}
    NU = {}
    for c, a in ((0, 1), (0, 2), (1, 2)):
        G[(c, a)] = edge_grad(g, u, c, a)
        NU[(c, a)] = _edge_nu(g, nu_c, c, a, nu_w)
    for c in range(3):
        e0, e1 = fluid._evolved_range(g, c)
        td = 2 - c
        # normal stress 2 nu_t d_c u_c at cells; faces i use cells i-1, i
        T = 2.0 * nu_c * _diag_grad(g, u, c)
        n = g.n[c]
        if g.periodic[c]:
            Te = torch.cat([T.narrow(td, n - 1, 1), T], dim=td)      # cells -1..N-1
        else:
            Te = torch.cat([torch.zeros_like(T.narrow(td, 0, 1)), T], dim=td)
        m = e1 - e0
        D = (Te.narrow(td, e0 + 1, m) - Te.narrow(td, e0, m)) / g.bshape(c, g.dc[c][e0:e1])
        for a in range(3):
            if a == c:
                continue
            key = (min(c, a), max(c, a))
            S = NU[key] * G[key]                     # on (key0, key1) lattice
            ta = 2 - a
            Sf = S.narrow(td, e0, m)                 # c-faces e0..e1-1
            dS = Sf.narrow(ta, 1, g.n[a]) - Sf.narrow(ta, 0, g.n[a])
            D = D + dS / g.bshape(a, g.dx[a])
        out.append(fluid._place(torch.zeros(g.face_shape(c), dtype=F64), D, c, e0, e1))
    return out


def sgs_force(g: Grid, u) -> list:
    """The subgrid term added to R: divergence of 2 nu_t S with the
    Smagorinsky nu_t and, if enabled, the wall-model edges."""
    cfg = _cfg(g)
    check(g, cfg)
    nu_c = nu_smagorinsky(g, u, float(cfg["cs"]))
    nu_w = wall_viscosity(g, u, cfg) if cfg.get("wall_model") else None
    return stress_divergence(g, u, nu_c, nu_w)


def check(g: Grid, cfg: dict) -> None:
    if g.dim != 3:
        raise ValueError("the subgrid model is defined on 3D grids")
    for a in range(3):
        if not g.periodic[a] and tuple(g.bc[a]) != ("noslip", "noslip"):
            raise ValueError("LES grids need periodic axes or no-slip walls")
    if cfg.get("wall_model"):
        if not (g.periodic[0] and g.periodic[2]) or g.periodic[1]:
            raise ValueError("the wall model needs walls normal to y, x and z periodic")
