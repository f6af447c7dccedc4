"""Strongly coupled FSI step (paper Alg. 1 with N > 1, Sec. 2.3.3) and its
gradient by implicit differentiation of the coupling fixed point (Sec. 2.4.1,
Eq. 24).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step from (u^n, p^n, w^n):

* the structural iterate starts at the previous time level, w_0 = w^n;
* sub-iteration k: the fluid advances from the previous time level u^n with
  the immersed body placed and moving as the current iterate w_{k-1}
  (point classes, target velocities, Eqs. 4-5, 9-10), the loads follow from
  its forcing (Eq. 20), and the structure advances from w^n under that load
  (Eq. 12, RK4) to give w_k;
* the coupling error xi_k = ||w_k - w_{k-1}||^2 / max(||w_{k-1}||^2, 1e-30)
  decides whether another sub-iteration follows (xi_k >= tol and k < N);
* the step returns the fluid state and the force of the last sub-iteration
  and w_K.

Readings (the algorithm overloads w^{t-1} as both the previous time level
and the previous iterate):
* the structure always integrates from the time level w^n, while the fluid
  sees the latest iterate;
* w is the whole rigid-body state (displacement and velocity, the response
  the RK4 of Eq. 12 returns); the printed error divides by w^{t-1}, which
  vanishes at rest, so the squared norm of the difference is taken relative
  to the squared norm of the previous iterate, floored at 1e-30;
* N = 1 is the weakly coupled step of ``step.step``.

Implicit differentiation: at the converged iterate w* = Phi(w*) with
Phi(w) = RK4(w^n, F(u^n, w)), the adjoint lambda solves
(I - dPhi/dw)^T lambda = dJ/dw (Eq. 24 with the residual w - Phi(w)), and the
input gradients are the partial derivatives of J + lambda . Phi at fixed w*.
The Jacobian dPhi/dw (6 x 6) is formed exactly by automatic differentiation
and the system is solved directly.  Point classes are frozen at those of w*.
"""
from __future__ import annotations

import torch

from . import body as bodymod
from . import fluid, ibm
from .grid import Grid, F64
from .poisson import solver
from .step import body_geometry


def fluid_part(g: Grid, u, params: dict, omega: torch.Tensor, masks=None):
    """Fluid update of one coupling iteration with the body at `omega`
    (positions X0 + d, rigid velocity v): predictor with direct forcing,
    modified PPE, correction and the loads.  Returns (u_new, p, F, masks)."""
    Xk, U, dV = body_geometry(g, omega)
    if masks is None:
        masks = ibm.classify(g, Xk.detach().numpy())
    us, uc = ibm.targets(g, masks, Xk, U, dV)
    eps = masks[2]
    ustar, f, _ = fluid.predictor(g, u, params["fb"], eps, us)
    b = fluid.ppe_rhs(g, ustar, eps, uc)
    p = solver(g).solve(b)
    un = fluid.project(g, ustar, p)
    F = ibm.loads(g, masks, f, Xk, dV)
    return un, p, F, masks


def structure(g: Grid, w_n: torch.Tensor, F: torch.Tensor, params: dict) -> torch.Tensor:
    """Rigid-body state after the step from the time level w_n under F."""
    bd = g.w.body
    return bodymod.advance(w_n, F, bd.free_dof, float(bd.m), params["k"], params["c"], g.dt)


def coupling_error(w_new: torch.Tensor, w_old: torch.Tensor) -> float:
    num = float(((w_new - w_old) ** 2).sum())
    den = max(float((w_old ** 2).sum()), 1e-30)
    return num / den


def step_strong(g: Grid, state: dict, params: dict, tol: float = 1e-5, nmax: int = 100,
                masks=None):
    """One strongly coupled step; returns (new_state, aux) with aux holding
    the force F of the last sub-iteration, the iterate it used ("omega"),
    the sub-iteration count and the error history."""
    u, w_n = state["u"], state["body"]
    omega = w_n
    xis = []
    for k in range(1, nmax + 1):
        un, p, F, mk = fluid_part(g, u, params, omega, masks)
        w_new = structure(g, w_n, F, params)
        xi = coupling_error(w_new.detach(), omega.detach())
        xis.append(xi)
        used = omega
        omega = w_new
        if xi < tol:
            break
    aux = {"F": F, "omega": used, "iters": k, "xi": xis, "masks": mk}
    return {"u": un, "p": p, "body": omega}, aux


class _StrongStep(torch.autograd.Function):
    """Forward: step_strong.  Backward: Eq. 24 at the converged iterate."""

    @staticmethod
    def forward(ctx, g, tol, nmax, masks, nd, *args):
        u = list(args[:nd])
        fb = list(args[nd:2 * nd])
        w_n, k, c = args[2 * nd:2 * nd + 3]
        params = {"fb": [x.detach() for x in fb], "k": k.detach(), "c": c.detach()}
        st = {"u": [x.detach() for x in u], "body": w_n.detach()}
        with torch.no_grad():
            new, aux = step_strong(g, st, params, tol, nmax, masks)
        ctx.g, ctx.nd = g, nd
        ctx.masks = aux["masks"]
        ctx.iters = aux["iters"]
        ctx.save_for_backward(aux["omega"].detach(), *args)
        return (*new["u"], new["p"], new["body"], aux["F"])

    @staticmethod
    def backward(ctx, *grads):
        g, nd = ctx.g, ctx.nd
        omega_s = ctx.saved_tensors[0]
        args = ctx.saved_tensors[1:]
        ubar = list(grads[:nd])
        wbar = grads[nd + 1]
        Fbar = grads[nd + 2]
        with torch.enable_grad():
            u = [x.detach().requires_grad_(True) for x in args[:nd]]
            fb = [x.detach().requires_grad_(True) for x in args[nd:2 * nd]]
            w_n, k, c = [x.detach().requires_grad_(True) for x in args[2 * nd:2 * nd + 3]]
            om = omega_s.clone().requires_grad_(True)
            params = {"fb": fb, "k": k, "c": c}
            un, _, F, _ = fluid_part(g, u, params, om, ctx.masks)
            Phi = structure(g, w_n, F, params)
            Jloc = torch.zeros((), dtype=F64)
            for i in range(nd):
                if ubar[i] is not None:
                    Jloc = Jloc + (un[i] * ubar[i]).sum()
            if Fbar is not None:
                Jloc = Jloc + (F * Fbar).sum()
            # dPhi/dw, row by row
            jac = torch.zeros((6, 6), dtype=F64)
            for r in range(6):
                gr, = torch.autograd.grad(Phi[r], om, retain_graph=True, allow_unused=True)
                if gr is not None:
                    jac[r] = gr
            a = torch.zeros(6, dtype=F64) if wbar is None else wbar.detach().clone()
            if Jloc.requires_grad:
                ga, = torch.autograd.grad(Jloc, om, retain_graph=True, allow_unused=True)
                if ga is not None:
                    a = a + ga
            lam = torch.linalg.solve((torch.eye(6, dtype=F64) - jac).t(), a)
            total = Jloc + (lam.detach() * Phi).sum()
            leaves = u + fb + [w_n, k, c]
            gs = torch.autograd.grad(total, leaves, allow_unused=True)
        return (None, None, None, None, None, *gs)


def step_strong_implicit(g: Grid, state: dict, params: dict, tol: float = 1e-5,
                         nmax: int = 100, masks=None):
    """Differentiable strongly coupled step whose gradient is the implicit
    one of Eq. 24.  Returns (new_state, F)."""
    nd = g.dim
    out = _StrongStep.apply(g, tol, nmax, masks, nd, *state["u"], *params["fb"], state["body"],
                            params["k"], params["c"])
    return {"u": list(out[:nd]), "p": out[nd], "body": out[nd + 1]}, out[nd + 2]


def rollout_strong(g: Grid, state: dict, params: dict, nsteps: int, tol: float = 1e-5,
                   nmax: int = 100, implicit: bool = True, masks_list=None):
    """Alg. 2 over strongly coupled steps; returns (final_state, F history,
    sub-iteration counts).  implicit=False differentiates through the
    unrolled sub-iterations instead (autograd of step_strong)."""
    Fh, its = [], []
    for n in range(nsteps):
        mk = None if masks_list is None else masks_list[n]
        if implicit:
            state, F = step_strong_implicit(g, state, params, tol, nmax, mk)
            its.append(None)
        else:
            state, aux = step_strong(g, state, params, tol, nmax, mk)
            F = aux["F"]
            its.append(aux["iters"])
        Fh.append(F)
    Fh = torch.stack(Fh) if Fh else torch.zeros((0, 3), dtype=F64)
    return state, Fh, its
