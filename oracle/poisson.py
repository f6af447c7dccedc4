"""Exact solution of the discrete pressure Poisson equation (paper Eq. 9).

The volume-integrated operator is

    (A p)_c = sum over interior faces f of cell c of (A_f / dc_f) (p_c - p_nb),

homogeneous Neumann on bounded axes (boundary faces carry no term) and
periodic wrap otherwise.  It separates into a Kronecker sum
A = sum_a (W_other (x) T_a) with T_a the 1D symmetric tridiagonal operator
of axis a and W_b = diag(dx_b).  Each 1D pencil T_a phi = lam W_a phi is
solved once with a dense symmetric generalized eigensolver, so that

    p = Phi diag(1 / (lam_x + lam_y + lam_z)) Phi^T b,   Phi^T W Phi = I,

with the single zero eigenvalue (constants) mapped to zero.  This is the
exact solution of the linear system (up to rounding), which the GPU path
reaches iteratively; p is then gauged to zero mean.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import torch

from .grid import Grid, F64


def axis_operator(g: Grid, a: int):
    """(T_a, W_a) for axis a as dense float64 numpy arrays."""
    N = g.n[a]
    dc = g.dc[a].numpy()
    T = np.zeros((N, N))
    faces = range(N) if g.periodic[a] else range(1, N)
    for f in faces:
        i, j = f % N, (f - 1) % N         # cells on both sides of face f
        coef = 1.0 / dc[f]
        T[i, i] += coef
        T[j, j] += coef
        T[i, j] -= coef
        T[j, i] -= coef
    W = np.diag(g.dx[a].numpy())
    return T, W


class ExactPoisson:
    def __init__(self, g: Grid):
        self.g = g
        self.phi, self.lam = [], []
        for a in range(g.dim):
            T, W = axis_operator(g, a)
            lam, phi = scipy.linalg.eigh(T, W)
            self.phi.append(torch.tensor(phi, dtype=F64))
            self.lam.append(torch.tensor(lam, dtype=F64))
        lsum = torch.zeros(g.cell_shape(), dtype=F64)
        for a in range(g.dim):
            lsum = lsum + g.bshape(a, self.lam[a])
        # the zero mode: the single smallest |eigenvalue| (constants)
        flat = lsum.reshape(-1)
        k0 = int(torch.argmin(flat.abs()))
        inv = torch.where(flat.abs() > 0, 1.0 / flat, torch.zeros_like(flat))
        inv[k0] = 0.0
        self.inv = inv.reshape(lsum.shape)

    def _apply(self, q: torch.Tensor, transpose: bool) -> torch.Tensor:
        for a in range(self.g.dim):
            M = self.phi[a].t() if transpose else self.phi[a]
            td = 2 - a
            q = torch.movedim(torch.tensordot(q, M, dims=([td], [1])), -1, td)
        return q

    def solve(self, b: torch.Tensor) -> torch.Tensor:
        bh = self._apply(b, transpose=True)       # Phi^T b
        p = self._apply(bh * self.inv, transpose=False)
        return p - p.mean()


def apply_A(g: Grid, p: torch.Tensor) -> torch.Tensor:
    """Matrix-free A p from its face-flux definition (used by the pins)."""
    out = torch.zeros_like(p)
    for a in range(g.dim):
        A = g.face_area(a)
        td = 2 - a
        n = g.n[a]
        if g.periodic[a]:
            flux = A * (p - torch.roll(p, 1, dims=td)) / g.bshape(a, g.dc[a][:-1])
            out = out + flux - torch.roll(flux, -1, dims=td)
        else:
            fl = A * (p.narrow(td, 1, n - 1) - p.narrow(td, 0, n - 1)) / g.bshape(a, g.dc[a][1:n])
            zero = torch.zeros_like(p.narrow(td, 0, 1))
            flux = torch.cat([zero, fl, zero], dim=td)       # faces 0..n
            out = out + flux.narrow(td, 0, n) - flux.narrow(td, 1, n)
    return out


def solver(g: Grid) -> ExactPoisson:
    """The exact solver of a grid, built once and kept on the grid."""
    s = getattr(g, "_exact_poisson", None)
    if s is None:
        s = ExactPoisson(g)
        g._exact_poisson = s
    return s
