"""Staggered (MAC) grid metrics for the oracle -- Sec. 2.3.1 of the paper.

Pressure lives at cell centres and velocity component ``c`` on the faces
normal to axis ``c`` (the west/south/bottom face of cell ``i`` carries
index ``i``).  Arrays are (z, y, x) with x fastest.  Axis ``a`` of the
physical problem maps to tensor dimension ``2 - a``.

Per axis (``N`` cells, faces ``xf[0..N]``):

* ``dx[i]  = xf[i+1] - xf[i]``                       cell width
* ``xc[i]  = (xf[i] + xf[i+1]) / 2``                 cell centre
* ``xce``  centres extended by one ghost on each side: mirrored about the
  boundary face on a bounded axis, shifted by the period on a periodic one
* ``dc[f]  = xce[f+1] - xce[f]`` for faces f = 0..N  centre spacing, which is
  also the width of the control volume of a face-normal velocity
* ``wi[f]  = (xf[f] - xce[f]) / dc[f]``              linear-interpolation
  weight of the upper cell when a cell quantity is carried to face f.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


class Grid:
    """Grid, boundary description and physical constants of one workload."""

    def __init__(self, w):
        self.w = w
        self.dim = int(w.dim)
        self.n = tuple(int(v) for v in w.n)
        self.bc = [list(b) for b in w.bc]
        self.bc_vel = np.asarray(w.bc_vel, dtype=np.float64)
        self.nu = float(w.nu)
        self.rho = float(w.rho)
        self.dt = float(w.dt)
        self.u_conv = float(w.u_conv)
        self.conv = w.conv
        self.periodic = [self.bc[a][0] == "periodic" for a in range(3)]
        for a in range(3):
            if (self.bc[a][0] == "periodic") != (self.bc[a][1] == "periodic"):
                raise ValueError("periodic boundaries must be paired")
        self.xf, self.dx, self.xc, self.xce, self.dxe, self.dc, self.wi = ([] for _ in range(7))
        for a in range(3):
            f = np.asarray(w.faces[a], dtype=np.float64)
            N = self.n[a]
            assert f.size == N + 1
            dx = f[1:] - f[:-1]
            xc = 0.5 * (f[:-1] + f[1:])
            L = f[-1] - f[0]
            if self.periodic[a]:
                xce = np.concatenate([[xc[-1] - L], xc, [xc[0] + L]])
                dxe = np.concatenate([[dx[-1]], dx, [dx[0]]])
            else:
                xce = np.concatenate([[2.0 * f[0] - xc[0]], xc, [2.0 * f[-1] - xc[-1]]])
                dxe = np.concatenate([[dx[0]], dx, [dx[-1]]])
            dc = xce[1:] - xce[:-1]
            wi = (f - xce[:-1]) / dc
            for lst, v in ((self.xf, f), (self.dx, dx), (self.xc, xc), (self.xce, xce),
                           (self.dxe, dxe), (self.dc, dc), (self.wi, wi)):
                lst.append(torch.tensor(v, dtype=F64))

    # ------------------------------------------------------------------ shapes
    def nfaces(self, c: int) -> int:
        """Number of faces of component c along its own axis."""
        return self.n[c] if self.periodic[c] else self.n[c] + 1

    def face_shape(self, c: int) -> tuple:
        ext = list(self.n)
        ext[c] = self.nfaces(c)
        return (ext[2], ext[1], ext[0])

    def cell_shape(self) -> tuple:
        return (self.n[2], self.n[1], self.n[0])

    @staticmethod
    def bshape(a: int, v: torch.Tensor) -> torch.Tensor:
        """Reshape a 1D per-axis vector so it broadcasts along axis a."""
        s = [1, 1, 1]
        s[2 - a] = v.numel()
        return v.reshape(s)

    def evolved(self, c: int) -> torch.Tensor:
        """Boolean mask of faces of component c advanced by the momentum
        equation: every face on a periodic axis, interior faces otherwise."""
        m = torch.ones(self.face_shape(c), dtype=torch.bool)
        if not self.periodic[c]:
            idx = [slice(None)] * 3
            idx[2 - c] = 0
            m[tuple(idx)] = False
            idx[2 - c] = -1
            m[tuple(idx)] = False
        return m

    def face_coords(self, c: int):
        """Physical coordinates of the faces of component c (1D per axis)."""
        out = []
        for a in range(3):
            if a == c:
                f = self.xf[a]
                out.append(f if not self.periodic[a] else f[:-1])
            else:
                out.append(self.xc[a])
        return out

    def cell_volume(self) -> torch.Tensor:
        v = self.bshape(0, self.dx[0]) * self.bshape(1, self.dx[1])
        if self.dim == 3:
            v = v * self.bshape(2, self.dx[2])
        return v.expand(self.cell_shape())

    def face_area(self, c: int) -> torch.Tensor:
        """Area of faces of component c (product of the transverse widths)."""
        a_ = torch.ones((1, 1, 1), dtype=F64)
        for b in range(self.dim):
            if b != c:
                a_ = a_ * self.bshape(b, self.dx[b])
        return a_
