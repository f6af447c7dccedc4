"""Fluid sub-steps of the oracle (paper Sec. 2.3.1, Eqs. 4-10).

Readings of the paper taken here (it only says "staggered FVM, second-order
central or first-order upwind convection, central diffusion"):

* convection is in divergence form -div(u (x) u); a velocity carried to a
  cell centre along its own axis is the mean of its two faces, a velocity
  carried across a cell boundary of another axis is linearly interpolated
  between the two cell centres (the mean on a uniform axis);
* upwinding takes the transported velocity from the upstream side of the
  transporting velocity's sign, and a zero transport velocity gives a zero
  flux;
* ghost values behind a boundary: Dirichlet (no-slip wall, inflow)
  ``2 g - u_0`` mirrored about the boundary face, Neumann (free slip,
  outflow) ``u_0``, periodic wrap;
* an external body force f_b (e.g. the channel's driving pressure
  gradient) is part of the right-hand side R, so the direct forcing of
  Eq. 5 -- written as f = eps [ -R + (u_s - u)/dt ] -- still makes the
  predicted velocity equal the target on forced faces;
* faces normal to a bounded axis are not advanced by Eq. 4: walls and
  inflows keep their prescribed normal velocity, a convective outflow is
  advected with speed U_conv (a zero-gradient outflow copies the predicted
  neighbour), and the outflow faces then receive one uniform correction so
  that the net boundary flux is zero;
* the PPE (Eq. 9) is solved in its volume-integrated symmetric form with
  homogeneous Neumann conditions on bounded axes; its right-hand side has
  its mean removed and p is gauged to zero mean.
"""
from __future__ import annotations

import torch

from .grid import Grid, F64

DIRICHLET = ("noslip", "inflow")


def _sl(q: torch.Tensor, spec: dict) -> torch.Tensor:
    """Slice q with spec = {axis: (start, stop)} (physical axes)."""
    idx = [slice(None)] * 3
    for a, (s0, s1) in spec.items():
        idx[2 - a] = slice(s0, s1)
    return q[tuple(idx)]


def ext(g: Grid, q: torch.Tensor, c: int) -> torch.Tensor:
    """Component c extended by one ghost layer along every active axis.

    Along the component's own bounded axis the extra layer is never read;
    it is filled with zeros.
    """
    for a in range(g.dim):
        td = 2 - a
        n = q.shape[td]
        first = q.narrow(td, 0, 1)
        last = q.narrow(td, n - 1, 1)
        if g.periodic[a]:
            lo, hi = last, first
        elif a == c:
            lo, hi = torch.zeros_like(first), torch.zeros_like(last)
        else:
            lo = _ghost(first, g.bc[a][0], g.bc_vel[a][0][c])
            hi = _ghost(last, g.bc[a][1], g.bc_vel[a][1][c])
        q = torch.cat([lo, q, hi], dim=td)
    return q


def _ghost(v: torch.Tensor, kind: str, gval: float) -> torch.Tensor:
    if kind in DIRICHLET:
        return 2.0 * gval - v
    return v


def _interior(g: Grid, skip=()) -> dict:
    """Ext-array slice spec selecting the real cells along every active axis."""
    return {a: (1, g.n[a] + 1) for a in range(g.dim) if a not in skip}


def _evolved_range(g: Grid, c: int):
    """Index range (in face indices) of faces advanced along axis c."""
    return (0, g.n[c]) if g.periodic[c] else (1, g.n[c])


def convection(g: Grid, u) -> list:
    """C(u) = div(u (x) u) on the evolved faces of each component (Eq. 4)."""
    E = [ext(g, u[c], c) for c in range(g.dim)]
    out = []
    for c in range(g.dim):
        e0, e1 = _evolved_range(g, c)
        # --- own direction: cell-centre fluxes between consecutive c-faces
        spec = _interior(g, skip=(c,))
        spec_c = dict(spec)
        spec_c[c] = (0, g.nfaces(c) + 2)
        Ec = _sl(E[c], spec_c)
        td = 2 - c
        qL = Ec.narrow(td, 0, Ec.shape[td] - 1)
        qR = Ec.narrow(td, 1, Ec.shape[td] - 1)
        Qc = 0.5 * (qL + qR)            # position e <-> cell e - 1
        if g.conv == "upwind":
            flux = Qc * torch.where(Qc > 0, qL, torch.where(Qc < 0, qR, torch.zeros_like(qL)))
        else:
            flux = Qc * Qc
        # face i uses cells i-1 (pos i) and i (pos i+1)
        fR = _sl(flux, {c: (e0 + 1, e1 + 1)})
        fL = _sl(flux, {c: (e0, e1)})
        Cc = (fR - fL) / g.bshape(c, g.dc[c][e0:e1])
        out.append(Cc)
    # --- cross directions: edge fluxes shared by the c- and a-equations
    for c in range(g.dim):
        for a in range(g.dim):
            if a == c:
                continue
            # edge lattice: c-faces 0..N_c, a-faces 0..N_a, other axes cells
            other = [b for b in range(g.dim) if b not in (a, c)]
            spec_o = {b: (1, g.n[b] + 1) for b in other}
            # component c carried along a to a-faces (between ext j, j+1)
            s = dict(spec_o)
            s[c] = (1, g.n[c] + 2)
            s[a] = (0, g.n[a] + 2)
            Xc = _sl(E[c], s)
            ta = 2 - a
            cL = Xc.narrow(ta, 0, g.n[a] + 1)
            cR = Xc.narrow(ta, 1, g.n[a] + 1)
            wa = g.bshape(a, g.wi[a])
            Ua = (1.0 - wa) * cL + wa * cR
            # component a carried along c to c-faces
            s = dict(spec_o)
            s[a] = (1, g.n[a] + 2)
            s[c] = (0, g.n[c] + 2)
            Xa = _sl(E[a], s)
            tc = 2 - c
            aL = Xa.narrow(tc, 0, g.n[c] + 1)
            aR = Xa.narrow(tc, 1, g.n[c] + 1)
            wc = g.bshape(c, g.wi[c])
            Vc = (1.0 - wc) * aL + wc * aR
            if g.conv == "upwind":
                zero = torch.zeros_like(cL)
                flux_c = Vc * torch.where(Vc > 0, cL, torch.where(Vc < 0, cR, zero))
            else:
                flux_c = Ua * Vc
            # c-equation, evolved c-faces, cell j along a: X[j+1] - X[j]
            e0, e1 = _evolved_range(g, c)
            F = _sl(flux_c, {c: (e0, e1)})
            dF = F.narrow(ta, 1, g.n[a]) - F.narrow(ta, 0, g.n[a])
            out[c] = out[c] + dF / g.bshape(a, g.dx[a])
    return out


def diffusion(g: Grid, u) -> list:
    """Central second-order Laplacian of each component on its evolved faces."""
    out = []
    for c in range(g.dim):
        E = ext(g, u[c], c)
        e0, e1 = _evolved_range(g, c)
        L = 0.0
        for a in range(g.dim):
            spec = _interior(g, skip=(a, c))
            if a == c:
                spec[c] = (e0, e1 + 2)
                X = _sl(E, spec)
                td = 2 - c
                m = e1 - e0
                qm, q0, qp = X.narrow(td, 0, m), X.narrow(td, 1, m), X.narrow(td, 2, m)
                hp = g.bshape(c, g.dxe[c][e0 + 1:e1 + 1])   # cell i (between i, i+1)
                hm = g.bshape(c, g.dxe[c][e0:e1])           # cell i-1
                H = g.bshape(c, g.dc[c][e0:e1])
                L = L + ((qp - q0) / hp - (q0 - qm) / hm) / H
            else:
                spec[c] = (e0 + 1, e1 + 1)
                spec[a] = (0, g.n[a] + 2)
                X = _sl(E, spec)
                td = 2 - a
                m = g.n[a]
                qm, q0, qp = X.narrow(td, 0, m), X.narrow(td, 1, m), X.narrow(td, 2, m)
                hp = g.bshape(a, g.dc[a][1:m + 1])
                hm = g.bshape(a, g.dc[a][0:m])
                H = g.bshape(a, g.dx[a])
                L = L + ((qp - q0) / hp - (q0 - qm) / hm) / H
        out.append(L)
    return out


def momentum_rhs(g: Grid, u, fb) -> list:
    """R = -div(u (x) u) + nu lap(u) + f_b on the evolved faces (zero elsewhere),
    plus the divergence of the subgrid stress when the workload enables LES
    (``les.py``)."""
    C = convection(g, u)
    L = diffusion(g, u)
    out = []
    for c in range(g.dim):
        e0, e1 = _evolved_range(g, c)
        Rin = -C[c] + g.nu * L[c] + _sl(fb[c], {c: (e0, e1)})
        R = _place(torch.zeros(g.face_shape(c), dtype=F64), Rin, c, e0, e1)
        out.append(R)
    if getattr(g.w, "les", None) is not None:
        from . import les          # subgrid stress divergence (zero off the evolved faces)
        out = [R + S for R, S in zip(out, les.sgs_force(g, u))]
    return out


def _place(full: torch.Tensor, part: torch.Tensor, c: int, e0: int, e1: int):
    """Out-of-place write of part into full[.., e0:e1 along axis c, ..]."""
    td = 2 - c
    n = full.shape[td]
    pieces = []
    if e0 > 0:
        pieces.append(full.narrow(td, 0, e0))
    pieces.append(part)
    if e1 < n:
        pieces.append(full.narrow(td, e1, n - e1))
    return torch.cat(pieces, dim=td)


def predictor(g: Grid, u, fb, eps, us):
    """Eqs. 4-5: u* = u + dt [ R + f ], f = eps [ -R + (u_s - u)/dt ].

    Returns (u*, f, R).  Boundary-normal faces follow the boundary rules in
    the module docstring, then the outflow mass correction is applied.
    """
    R = momentum_rhs(g, u, fb)
    dt = g.dt
    ustar, force = [], []
    for c in range(g.dim):
        ev = g.evolved(c)
        f = torch.where(eps[c], -R[c] + (us[c] - u[c]) / dt, torch.zeros_like(u[c]))
        us_c = torch.where(ev, u[c] + dt * (R[c] + f), u[c])
        ustar.append(us_c)
        force.append(f)
    ustar = boundary_normal(g, u, ustar)
    ustar = outflow_correction(g, ustar)
    return ustar, force, R


def boundary_normal(g: Grid, u, ustar):
    out = list(ustar)
    for c in range(g.dim):
        if g.periodic[c]:
            continue
        td = 2 - c
        n = g.nfaces(c)
        for side in (0, 1):
            kind = g.bc[c][side]
            b = 0 if side == 0 else n - 1
            inner = 1 if side == 0 else n - 2
            ub = u[c].narrow(td, b, 1)
            if kind in ("noslip", "freeslip", "inflow"):
                val = torch.full_like(ub, float(g.bc_vel[c][side][c]))
            elif kind == "outflow_conv":
                h = float(g.dx[c][0] if side == 0 else g.dx[c][-1])
                val = ub - g.dt * g.u_conv * (ub - u[c].narrow(td, inner, 1)) / h
            elif kind == "outflow_neumann":
                val = out[c].narrow(td, inner, 1)
            else:
                raise ValueError(kind)
            out[c] = _place(out[c], val, c, b, b + 1)
    return out


def outflow_correction(g: Grid, ustar):
    """Uniform correction of outflow faces so the net boundary flux is zero."""
    outs = [(c, s) for c in range(g.dim) if not g.periodic[c] for s in (0, 1)
            if g.bc[c][s].startswith("outflow")]
    if not outs:
        return ustar
    net = 0.0
    area_out = 0.0
    for c in range(g.dim):
        if g.periodic[c]:
            continue
        td = 2 - c
        n = g.nfaces(c)
        A = g.face_area(c)
        for s in (0, 1):
            b = 0 if s == 0 else n - 1
            sign = -1.0 if s == 0 else 1.0
            flux = (ustar[c].narrow(td, b, 1) * A).sum()
            net = net + sign * flux
            if g.bc[c][s].startswith("outflow"):
                area_out = area_out + float((A.expand_as(ustar[c].narrow(td, b, 1))).sum())
    out = list(ustar)
    for c, s in outs:
        td = 2 - c
        n = g.nfaces(c)
        b = 0 if s == 0 else n - 1
        sign = -1.0 if s == 0 else 1.0
        val = out[c].narrow(td, b, 1) - sign * net / area_out
        out[c] = _place(out[c], val, c, b, b + 1)
    return out


def flux_divergence(g: Grid, q) -> torch.Tensor:
    """Sum over the faces of each cell of (outward sign) area x face value,
    i.e. the volume integral of div(q)."""
    s = torch.zeros(g.cell_shape(), dtype=F64)
    for c in range(g.dim):
        A = g.face_area(c)
        F = q[c] * A
        td = 2 - c
        if g.periodic[c]:
            s = s + (torch.roll(F, -1, dims=td) - F)
        else:
            n = g.n[c]
            s = s + (F.narrow(td, 1, n) - F.narrow(td, 0, n))
    return s


def divergence(g: Grid, q) -> torch.Tensor:
    """Cell-centred divergence (D q)_c."""
    return flux_divergence(g, q) / g.cell_volume()


def ppe_rhs(g: Grid, ustar, eps, uc) -> torch.Tensor:
    """Eq. 9 integrated over each cell: b = -(rho/dt) sum_f +-A_f u~_f with
    u~ = (1 - eps) u* + eps u_c; the mean of b is removed (compatibility)."""
    ut = [torch.where(eps[c], uc[c], ustar[c]) for c in range(g.dim)]
    b = -(g.rho / g.dt) * flux_divergence(g, ut)
    return b - b.mean()


def pressure_gradient(g: Grid, p: torch.Tensor, c: int) -> torch.Tensor:
    """(p_i - p_{i-1}) / dc_i on faces normal to axis c; zero on bounded-axis
    boundary faces (homogeneous Neumann)."""
    td = 2 - c
    if g.periodic[c]:
        return (p - torch.roll(p, 1, dims=td)) / g.bshape(c, g.dc[c][:-1])
    n = g.n[c]
    inner = (p.narrow(td, 1, n - 1) - p.narrow(td, 0, n - 1)) / g.bshape(c, g.dc[c][1:n])
    zero = torch.zeros_like(p.narrow(td, 0, 1))
    return torch.cat([zero, inner, zero], dim=td)


def project(g: Grid, ustar, p):
    """Eq. 10: u^{n+1} = u* - (dt/rho) grad p on every face that is not a
    boundary-normal face of a bounded axis."""
    return [ustar[c] - (g.dt / g.rho) * pressure_gradient(g, p, c) for c in range(g.dim)]
