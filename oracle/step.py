"""One weakly coupled FSI time step and rollouts (paper Alg. 1 with N = 1).

Order inside a step (Alg. 1, loop body):

1. markers X_k = X0_k + d^n, point classes and forcing mask (Sec. 2.2);
2. target / solid velocities from the body velocity (Eqs. 18-19, 23);
3. predictor with direct forcing (Eqs. 4-5) and boundary faces;
4. modified PPE (Eq. 9), exact solve, correction (Eq. 10);
5. loads on the body from the forcing (Eq. 20, Eq. 12 sums);
6. rigid-body update with RK4 (Eq. 12).

The state is (u, p, body) with body = [d_x, d_y, d_z, v_x, v_y, v_z]; the
differentiable parameters are the body-force field f_b and the spring
stiffness / damping vectors k, c.

Losses:

* ``wall_shear``: the two-wall mean of nu du/dy at the wall-adjacent
  streamwise faces, du/dy taken one-sided between the wall (velocity 0)
  and the first cell centre;
* ``rms_lift``: sqrt of the time mean of C_L^2 with C_L = 2 F_y / (rho U^2 D).
"""
from __future__ import annotations

import numpy as np
import torch

from . import body as bodymod
from . import fluid, ibm, ibm3d
from .grid import Grid, F64
from .poisson import solver


def _as64(x):
    return x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x), dtype=F64)


def make_params(g: Grid, fb=None, k=None, c=None):
    w = g.w
    if fb is None:
        fb = [torch.zeros(g.face_shape(cc), dtype=F64) for cc in range(g.dim)]
    else:
        fb = [_as64(x) for x in fb]
    bd = w.body
    kk = torch.tensor(bd.k if bd is not None else (0.0, 0.0, 0.0), dtype=F64) if k is None else k
    cc_ = torch.tensor(bd.c if bd is not None else (0.0, 0.0, 0.0), dtype=F64) if c is None else c
    return {"fb": fb, "k": kk, "c": cc_}


def init_state(g: Grid, u0, body0=None):
    u = [_as64(x) for x in u0]
    p = torch.zeros(g.cell_shape(), dtype=F64)
    if body0 is None:
        body0 = np.zeros(6)
    return {"u": u, "p": p, "body": _as64(body0)}


def body_geometry(g: Grid, bstate: torch.Tensor):
    """Marker positions, body velocity and marker volumes."""
    bd = g.w.body
    X0 = torch.tensor(bd.X0, dtype=F64)
    Xk = X0 + bstate[:2][None, :]
    h = ibm.grid_spacing(g)
    dV = torch.tensor(bd.ds, dtype=F64) * h
    U = bstate[3:5]
    return Xk, U, dV


def step(g: Grid, state: dict, params: dict, masks=None):
    """Advance (u, p, body) by one step; returns (new_state, aux)."""
    u, bs = state["u"], state["body"]
    bd = g.w.body
    bx = getattr(g.w, "box", None)
    if bd is None and bx is not None:
        # static box on a 3D grid (ibm3d): targets and solid velocity zero
        if masks is None:
            masks = ibm3d.classify_box(g, bx[0], bx[1])
        eps = masks[2]
        us = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(g.dim)]
        uc = us
    elif bd is not None:
        Xk, U, dV = body_geometry(g, bs)
        if masks is None:
            masks = ibm.classify(g, Xk.detach().numpy())
        us, uc = ibm.targets(g, masks, Xk, U, dV)
        eps = masks[2]
    else:
        eps = [torch.zeros(g.face_shape(c), dtype=torch.bool) for c in range(g.dim)]
        us = [torch.zeros(g.face_shape(c), dtype=F64) for c in range(g.dim)]
        uc = us
    ustar, f, R = fluid.predictor(g, u, params["fb"], eps, us)
    b = fluid.ppe_rhs(g, ustar, eps, uc)
    p = solver(g).solve(b)
    un = fluid.project(g, ustar, p)
    if bd is not None:
        F = ibm.loads(g, masks, f, Xk, dV)
        if bd.kind == "spring":
            bs_new = bodymod.advance(bs, F, bd.free_dof, float(bd.m), params["k"],
                                     params["c"], g.dt)
        else:
            bs_new = bs
    elif bx is not None:
        F = ibm3d.box_force(g, eps, f)
        bs_new = bs
    else:
        F = torch.zeros(3, dtype=F64)
        bs_new = bs
    aux = {"F": F, "f": f, "ustar": ustar, "b": b, "R": R, "eps": eps, "masks": masks}
    return {"u": un, "p": p, "body": bs_new}, aux


def rollout(g: Grid, state: dict, params: dict, nsteps: int, masks_list=None,
            keep_states: bool = False):
    """Alg. 2 semantics: repeat the step; returns (final_state, F history,
    masks used per step[, states])."""
    Fh, used, states = [], [], []
    for n in range(nsteps):
        mk = None if masks_list is None else masks_list[n]
        if keep_states:
            states.append(state)
        state, aux = step(g, state, params, masks=mk)
        Fh.append(aux["F"])
        used.append(aux["masks"])
    Fh = torch.stack(Fh) if Fh else torch.zeros((0, 3), dtype=F64)
    if keep_states:
        return state, Fh, used, states
    return state, Fh, used


def wall_shear(g: Grid, u) -> torch.Tensor:
    """Two-wall mean streamwise wall shear stress (rho = 1)."""
    yf, yc = g.xf[1], g.xc[1]
    lo = u[0][:, 0, :].mean() / (yc[0] - yf[0])
    hi = u[0][:, -1, :].mean() / (yf[-1] - yc[-1])
    return 0.5 * g.nu * (lo + hi)


def rms_lift(g: Grid, Fh: torch.Tensor, u_ref: float = 1.0, diameter: float = 1.0):
    cl = 2.0 * Fh[:, 1] / (g.rho * u_ref * u_ref * diameter)
    return torch.sqrt((cl * cl).mean())
