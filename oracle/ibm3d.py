"""Static immersed bodies on 3D grids: axis-aligned boxes (the cubic
roughness elements on the channel wall of Sec. 3.4.2) forced by the
direct-forcing IBM (Sec. 2.3.1, Eq. 5; point classes of Sec. 2.2, Fig. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken here:

* point classes per velocity component on its own face points, as in 2D: a
  face point is solid if it lies in the half-open box x0 <= x < x1,
  y0 <= y < y1, z0 <= z < z1 (the rule the 2D crossing-number test gives a
  rectangle); it is an immersed-boundary point if it is not solid and one of
  its six axis neighbours on the same component grid is solid (neighbours
  outside the array are not solid); forced = (solid or IB) and advanced by
  the momentum equation: a boundary-normal face of a bounded axis keeps its
  boundary condition (Eq. 4 is not solved there, so Eq. 5 cannot force it),
  which matters for a body standing on a wall (the cubes of Sec. 3.4.2);
* the body is at rest: target and solid velocities are zero on every
  forced face;
* there are no Lagrangian markers on a 3D body, so the force on it is the
  momentum the forcing removes from the fluid, F = -rho sum_f f_f dv_f over
  the forced faces (dv_f the face control volume: centre spacing along the
  component's axis times the transverse cell widths).
"""
from __future__ import annotations

import numpy as np
import torch

from .grid import Grid, F64


def classify_box(g: Grid, lo, hi):
    """(solid, ib, eps) boolean arrays per component (face array shapes)."""
    solid, ib, eps = [], [], []
    for c in range(3):
        fx, fy, fz = (t.numpy() for t in g.face_coords(c))
        inx = (fx >= lo[0]) & (fx < hi[0])
        iny = (fy >= lo[1]) & (fy < hi[1])
        inz = (fz >= lo[2]) & (fz < hi[2])
        s = inz[:, None, None] & iny[None, :, None] & inx[None, None, :]
        nb = np.zeros_like(s)
        nb[:, :, 1:] |= s[:, :, :-1]
        nb[:, :, :-1] |= s[:, :, 1:]
        nb[:, 1:, :] |= s[:, :-1, :]
        nb[:, :-1, :] |= s[:, 1:, :]
        nb[1:, :, :] |= s[:-1, :, :]
        nb[:-1, :, :] |= s[1:, :, :]
        b = (~s) & nb
        solid.append(torch.tensor(s))
        ib.append(torch.tensor(b))
        eps.append(torch.tensor(s | b) & g.evolved(c))
    return solid, ib, eps


def face_volume(g: Grid, c: int) -> torch.Tensor:
    """Control volume of the faces of component c (broadcast shape)."""
    dcv = g.dc[c] if not g.periodic[c] else g.dc[c][:-1]
    return g.bshape(c, dcv) * g.face_area(c)


def box_force(g: Grid, eps, f) -> torch.Tensor:
    """F = -rho sum over forced faces of f dv (3 components)."""
    F = []
    for c in range(3):
        dv = face_volume(g, c).expand(g.face_shape(c))
        F.append(-g.rho * (f[c] * dv * eps[c].to(F64)).sum())
    return torch.stack(F)
