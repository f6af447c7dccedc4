"""Immersed-boundary pieces of the oracle (paper Sec. 2.2 and Sec. 2.3.3).

Readings taken here:

* point classes (Sec. 2.2, Fig. 2) are evaluated per velocity component on
  that component's own face points.  A face point is *solid* if it lies
  inside the closed marker polygon (crossing-number test, half-open rule
  ``y_a <= y < y_b``, float64, evaluated as ``x < x_a + ((y - y_a)(x_b - x_a))
  / (y_b - y_a)`` in exactly that order).  It is an *IB point* if it is not
  solid and one of its axis neighbours on the same component grid is solid.
  The forcing mask of Eq. 5 is eps = solid OR IB (binary);
* the target velocity of Eq. 5 is the body velocity on solid points and, on
  IB points, the interpolation of Eqs. 18-19 in its normalised (Shepard)
  form  u_s(x) = sum_k U_k w_k / sum_k w_k  with  w_k = delta_h(x - X_k) dV_k.
  As printed, Eqs. 18-19 divide by a sum of kernel values without volume
  weights, which is not dimensionally consistent; the normalised form keeps
  the property the half-distribution normalisation is meant to give (a
  uniform body velocity is reproduced exactly).  The solid velocity u_c of
  Eqs. 8-9 is the rigid body velocity on every forced point;
* the marker volume is a shell one grid spacing thick, dV_k = ds_k h;
* the fluid-to-solid transfer follows Eq. 20, q_k = -sum_x f(x)
  delta_h(x - X_k) dv(x) with dv = h^2 the face control volume, and the
  total force on the body is F = rho sum_k q_k dV_k (Eq. 12 sums q over the
  markers; the volume weight makes the sum a force).
"""
from __future__ import annotations

import numpy as np
import torch

from .grid import Grid, F64


def phi4(s: torch.Tensor) -> torch.Tensor:
    """Dimensionless 4-point kernel of Eq. 22 (support |s| <= 2)."""
    s = s.abs()
    s1 = torch.clamp(s, 0.0, 1.0)
    s2 = torch.clamp(s, 1.0, 2.0)
    inner = (3.0 - 2.0 * s1 + torch.sqrt(1.0 + 4.0 * s1 - 4.0 * s1 * s1)) / 8.0
    outer = (5.0 - 2.0 * s2 - torch.sqrt(-7.0 + 12.0 * s2 - 4.0 * s2 * s2)) / 8.0
    zero = torch.zeros_like(s)
    return torch.where(s <= 1.0, inner, torch.where(s <= 2.0, outer, zero))


def d_h(r: torch.Tensor, h: float) -> torch.Tensor:
    """One-dimensional smoothing kernel d_h(r) of Eq. 22."""
    return phi4(r / h) / h


def delta_h(dx: torch.Tensor, dy: torch.Tensor, h: float) -> torch.Tensor:
    """Tensor-product regularised delta of Eq. 21."""
    return d_h(dx, h) * d_h(dy, h)


def inside_polygon(px: np.ndarray, py: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Crossing-number test of points against the closed polygon X (M, 2)."""
    inside = np.zeros(px.shape, dtype=bool)
    M = X.shape[0]
    for k in range(M):
        ax, ay = X[k]
        bx, by = X[(k + 1) % M]
        cond = ((ay <= py) & (py < by)) | ((by <= py) & (py < ay))
        if not cond.any():
            continue
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (py - ay) * (bx - ax)
            t = t / (by - ay)
            xint = ax + t
        inside ^= cond & (px < xint)
    return inside


def face_points_2d(g: Grid, c: int):
    """Broadcast grids (x, y) of the face points of component c, shape (ny, nx)."""
    fx, fy, _ = g.face_coords(c)
    X = np.broadcast_to(fx.numpy()[None, :], (fy.numel(), fx.numel()))
    Y = np.broadcast_to(fy.numpy()[:, None], (fy.numel(), fx.numel()))
    return X, Y


def classify(g: Grid, X: np.ndarray):
    """(solid, ib, eps) boolean arrays per component, shape of the face arrays.

    Points outside the bounding box of the polygon are outside it (a
    horizontal ray from such a point crosses the polygon an even number of
    times), so only the box is tested.
    """
    xmin, ymin = X.min(axis=0)
    xmax, ymax = X.max(axis=0)
    solid, ib, eps = [], [], []
    for c in range(2):
        PX, PY = face_points_2d(g, c)
        s = np.zeros(PX.shape, dtype=bool)
        box = (PX >= xmin) & (PX <= xmax) & (PY >= ymin) & (PY <= ymax)
        if box.any():
            s[box] = inside_polygon(PX[box], PY[box], X)
        nb = np.zeros_like(s)
        nb[:, 1:] |= s[:, :-1]
        nb[:, :-1] |= s[:, 1:]
        nb[1:, :] |= s[:-1, :]
        nb[:-1, :] |= s[1:, :]
        ibm = (~s) & nb
        solid.append(torch.tensor(s[None]))
        ib.append(torch.tensor(ibm[None]))
        eps.append(torch.tensor((s | ibm)[None]))
    return solid, ib, eps


def grid_spacing(g: Grid) -> float:
    h = float(g.dx[0][0])
    return h


def targets(g: Grid, masks, Xk: torch.Tensor, Ubody: torch.Tensor, dV: torch.Tensor):
    """Target velocity u_s and solid velocity u_c on the face arrays.

    Xk (M, 2) marker positions, Ubody (2,) rigid velocity (every marker
    moves with it), dV (M,) marker volumes.
    """
    solid, ib, eps = masks
    h = grid_spacing(g)
    us, uc = [], []
    for c in range(2):
        shape = g.face_shape(c)
        PX, PY = face_points_2d(g, c)
        Uc = Ubody[c]
        base = torch.zeros(shape, dtype=F64) + Uc * eps[c].to(F64)
        ibi = ib[c][0].nonzero(as_tuple=False)            # (n_ib, 2) -> (j, i)
        if ibi.shape[0] > 0:
            px = torch.tensor(PX[ibi[:, 0].numpy(), ibi[:, 1].numpy()], dtype=F64)
            py = torch.tensor(PY[ibi[:, 0].numpy(), ibi[:, 1].numpy()], dtype=F64)
            w = delta_h(px[:, None] - Xk[None, :, 0], py[:, None] - Xk[None, :, 1], h) * dV[None, :]
            num = (w * Uc).sum(dim=1)                    # every U_k = U (rigid)
            den = w.sum(dim=1)
            val = torch.where(den > 0, num / torch.where(den > 0, den, torch.ones_like(den)),
                              Uc.expand_as(den))
            flat = base.reshape(-1)
            lin = ibi[:, 0] * shape[2] + ibi[:, 1]
            flat = flat.index_put((lin,), val)
            base = flat.reshape(shape)
        us.append(base)
        uc.append(torch.zeros(shape, dtype=F64) + Uc * eps[c].to(F64))
    return us, uc


def loads(g: Grid, masks, f, Xk: torch.Tensor, dV: torch.Tensor) -> torch.Tensor:
    """Eq. 20 on each component's forced faces, then F = rho sum_k q_k dV_k."""
    _, _, eps = masks
    h = grid_spacing(g)
    dv = h * h
    F = []
    for c in range(2):
        PX, PY = face_points_2d(g, c)
        idx = eps[c][0].nonzero(as_tuple=False)
        if idx.shape[0] == 0:
            F.append(torch.zeros((), dtype=F64))
            continue
        px = torch.tensor(PX[idx[:, 0].numpy(), idx[:, 1].numpy()], dtype=F64)
        py = torch.tensor(PY[idx[:, 0].numpy(), idx[:, 1].numpy()], dtype=F64)
        fv = f[c][0][idx[:, 0], idx[:, 1]]
        dl = delta_h(px[:, None] - Xk[None, :, 0], py[:, None] - Xk[None, :, 1], h)
        q = -(fv[:, None] * dl * dv).sum(dim=0)          # q_k, (M,)
        F.append(g.rho * (q * dV).sum())
    return torch.stack(F + [torch.zeros((), dtype=F64)])
