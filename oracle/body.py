"""Rigid-body oscillator of the oracle (paper Eq. 12).

m w'' + c w' + k w = F per translational degree of freedom, integrated with
the classic fourth-order Runge-Kutta scheme.  The fluid force F is the one
computed by the fluid step (Alg. 1 evaluates the load once per coupling
iteration), so it is held constant over the four stages.

Reading: the paper prints k = 2 m (2 pi f_n)^2, which contradicts f_n being
the natural frequency of m w'' + k w = 0; k = m (2 pi f_n)^2 is used by the
workloads.  The damping c = 2 m (2 pi f_n) zeta_s is as printed.
"""
from __future__ import annotations

import torch


def rk4(d: torch.Tensor, v: torch.Tensor, F: torch.Tensor, m: float,
        k: torch.Tensor, c: torch.Tensor, dt: float):
    """One RK4 step of (d, v) with d' = v, v' = (F - c v - k d) / m."""
    def rhs(dd, vv):
        return vv, (F - c * vv - k * dd) / m

    k1d, k1v = rhs(d, v)
    k2d, k2v = rhs(d + 0.5 * dt * k1d, v + 0.5 * dt * k1v)
    k3d, k3v = rhs(d + 0.5 * dt * k2d, v + 0.5 * dt * k2v)
    k4d, k4v = rhs(d + dt * k3d, v + dt * k3v)
    d1 = d + (dt / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d)
    v1 = v + (dt / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v)
    return d1, v1


def advance(state: torch.Tensor, F: torch.Tensor, free, m: float,
            k: torch.Tensor, c: torch.Tensor, dt: float) -> torch.Tensor:
    """Body state [d_x, d_y, d_z, v_x, v_y, v_z] after one step; fixed
    degrees of freedom keep their values."""
    d, v = state[:3], state[3:]
    d1, v1 = rk4(d, v, F, m, k, c, dt)
    fr = torch.tensor([bool(x) for x in free])
    return torch.cat([torch.where(fr, d1, d), torch.where(fr, v1, v)])
