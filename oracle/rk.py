"""Explicit Runge-Kutta integration of the fluid and the CFL-adaptive time
step (paper Sec. 2.3.1 and Sec. 2.5, Table 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper offers explicit Runge-Kutta schemes next to forward Euler, and a
time step fixed or adapted to the CFL condition of the instantaneous maximum
velocity, without naming a scheme.  Readings taken here:

* a scheme is written in Shu-Osher form over the forward-Euler step
  S(v) = P(v + dt R(v)) of ``step.step`` (predictor, modified PPE, correction):
  v_0 = u^n, v_s = a_s u^n + b_s S(v_{s-1}) for s = 1..S, u^{n+1} = v_S.
  Every S(v) is divergence free and so is u^n, hence every stage is, and the
  scheme is the Runge-Kutta method of du/dt = P R(u):
    "fe"  (a, b) = (0, 1)                              forward Euler
    "rk2" (0, 1), (1/2, 1/2)                           Heun, second order
    "rk3" (0, 1), (3/4, 1/4), (1/3, 2/3)               third order (SSP)
* each stage's solve starts from the pressure of the previous stage (only an
  iterative solver sees it); the step returns the pressure of the last stage;
* grids without an immersed body only: a combination of stages would not keep
  the forced faces at the body velocity;
* adaptive step: dt = min(dt_max, CFL * h_min / max |u|), the maximum over
  every face value of every velocity component, h_min the smallest cell width
  of the grid; the step size is not differentiated.
"""
from __future__ import annotations

import torch

from .grid import Grid, F64
from .step import step

SCHEMES = {
    "fe": ((0.0, 1.0),),
    "rk2": ((0.0, 1.0), (0.5, 0.5)),
    "rk3": ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)),
}


def step_rk(g: Grid, state: dict, params: dict, scheme: str = "rk3"):
    """One Runge-Kutta step; returns (new_state, aux of the last stage)."""
    if g.w.body is not None or getattr(g.w, "box", None) is not None:
        raise ValueError("Runge-Kutta steps are defined for grids without an immersed body")
    u0 = state["u"]
    v, p = u0, state["p"]
    aux = None
    for a, b in SCHEMES[scheme]:
        st, aux = step(g, {"u": v, "p": p, "body": state["body"]}, params)
        v = [b * x if a == 0.0 else a * x0 + b * x for x0, x in zip(u0, st["u"])]
        p = st["p"]
    return {"u": v, "p": p, "body": state["body"]}, aux


def h_min(g: Grid) -> float:
    return min(float(g.dx[a].min()) for a in range(g.dim))


def cfl_dt(g: Grid, u, cfl: float, dt_max: float) -> float:
    """CFL-limited step from the instantaneous maximum velocity."""
    umax = max(float(x.detach().abs().max()) for x in u)
    if umax <= 0.0:
        return dt_max
    return min(dt_max, cfl * h_min(g) / umax)


def rollout_rk(g: Grid, state: dict, params: dict, nsteps: int, scheme: str = "rk3",
               cfl: float = None, dt_max: float = None):
    """nsteps Runge-Kutta steps; with cfl given, each step's dt follows
    cfl_dt (g.dt is restored afterwards).  Returns (state, dts)."""
    dt0 = g.dt
    dts = []
    try:
        for _ in range(nsteps):
            if cfl is not None:
                g.dt = cfl_dt(g, state["u"], cfl, dt_max if dt_max is not None else dt0)
            dts.append(g.dt)
            state, _ = step_rk(g, state, params, scheme)
    finally:
        g.dt = dt0
    return state, dts
