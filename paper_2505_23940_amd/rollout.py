"""Differentiable rollouts over libfvib (reverse mode through the discrete
adjoint of each step).

The forward pass repeats ``fvib_step`` (the paper's main loop, Alg. 2, with
one weakly coupled step per iteration, or one strongly coupled step of
``fvib_step_strong`` when a coupling is given) and keeps a checkpoint every
``ckpt_every`` steps.  The backward pass walks the segments in reverse:
it restores the segment's checkpoint, recomputes the states inside the
segment with the same (deterministic) forward step, then applies
``fvib_step_adjoint`` step by step.  Memory is O(S / K + K) states; K = 1
keeps every state and recomputes nothing.  Gradients flow to the initial
velocity, the body-force field, the spring constants (k, c) and the
initial body state; the loss may read the final velocity, the final body
state and the per-step force history.
"""
from __future__ import annotations

from typing import List, Optional

import torch

from . import Grid, INFO_DOUBLES


def _slots_like(x, n):
    """n fresh contiguous tensors shaped like x, carved from one allocation;
    each starts on a 256-byte boundary, as a separate allocation would (the
    library's vector loads need 16- and 32-byte alignment)."""
    es = x.element_size()
    per = -(-x.numel() * es // 256) * 256 // es
    flat = torch.empty((n, per), dtype=x.dtype, device=x.device)
    return [flat[s, :x.numel()].view(x.shape) for s in range(n)]


def _forward_steps(grid, nsteps, ckpt_every, u, p, body, fbd, kcd, info, ckpts, coupling=None,
                   omegas=None, scheme=None, cfl=None, dts=None):
    # The state entering a segment is kept as is; the segment's first step
    # writes its result into a fresh slot and the segment continues there in
    # place.  The slots of all segments but the last come from one
    # allocation per field (a device allocation per step stalls the
    # stream); the last segment, whose state is returned, has its own.
    nseg = (nsteps + ckpt_every - 1) // ckpt_every
    if nseg > 1:
        Us = [_slots_like(x, nseg - 1) for x in u]
        Ps, Bs = _slots_like(p, nseg - 1), _slots_like(body, nseg - 1)
    for n in range(nsteps):
        if cfl is not None:
            # CFL-adaptive step from the state entering step n
            dts[n] = grid.cfl_dt(u, cfl[0], cfl[1])
            grid.set_dt(dts[n])
        if n % ckpt_every == 0:
            ckpts[n] = (u, p, body)
            s = n // ckpt_every
            if s < nseg - 1:
                u2, p2, b2 = [X[s] for X in Us], Ps[s], Bs[s]
            else:
                u2 = [torch.empty_like(x) for x in u]
                p2, b2 = torch.empty_like(p), torch.empty_like(body)
            grid.step(u, p, fbd, body, kcd, u_out=u2, p_out=p2, body_out=b2, info=info[n],
                      coupling=coupling, omega=None if omegas is None else omegas[n],
                      scheme=scheme)
            u, p, body = u2, p2, b2
        else:
            grid.step(u, p, fbd, body, kcd, info=info[n], coupling=coupling,
                      omega=None if omegas is None else omegas[n], scheme=scheme)
    ckpts["final"] = (u, p, body)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid: Grid, nsteps: int, ckpt_every: int, coupling, scheme, cfl, nd: int,
                *tensors):
        u0 = list(tensors[:nd])
        fb = list(tensors[nd:2 * nd])
        kc, body0 = tensors[2 * nd], tensors[2 * nd + 1]
        dev = grid.device
        u = [x.detach().clone() for x in u0]
        p = grid.zeros_p()
        body = body0.detach().clone()
        fbd = [x.detach() for x in fb]
        kcd = kc.detach()
        info = torch.zeros((nsteps, INFO_DOUBLES), dtype=torch.float64, device=dev)
        ckpts = {}
        # strongly coupled steps keep the iterate each step's fluid saw last
        # (the linearisation point of their adjoint)
        omegas = None
        if coupling is not None:
            omegas = torch.zeros((nsteps, 6), dtype=torch.float64, device=dev)
        # CFL-adaptive steps keep the step size of every step (not differentiated)
        dt0 = grid.dt
        dts = [dt0] * nsteps
        # steps are enqueued back to back; their statuses are checked once
        grid.defer_status(True)
        try:
            _forward_steps(grid, nsteps, ckpt_every, u, p, body, fbd, kcd, info, ckpts, coupling,
                           omegas, scheme, cfl, dts)
        finally:
            grid.defer_status(False)
            if cfl is not None:
                grid.set_dt(dt0)
        u, p, body = ckpts.pop("final")
        grid.check_infos(info, "forward step")
        ctx.grid = grid
        ctx.nsteps = nsteps
        ctx.k = ckpt_every
        ctx.nd = nd
        ctx.ckpts = ckpts
        ctx.coupling = coupling
        ctx.omegas = omegas
        ctx.scheme = scheme
        ctx.dts = dts if cfl is not None else None
        ctx.dt0 = dt0
        ctx.save_for_backward(*fbd, kcd)
        Fh = info[:, 4:7].clone()
        ctx.mark_non_differentiable(p)
        return (*u, body, Fh, p)

    @staticmethod
    def backward(ctx, *grads):
        grid: Grid = ctx.grid
        nd, S, K = ctx.nd, ctx.nsteps, ctx.k
        saved = ctx.saved_tensors
        fb = list(saved[:nd])
        kc = saved[nd]
        gu = grads[:nd]
        gbody, gF = grads[nd], grads[nd + 1]
        ubar = [(g.contiguous().clone() if g is not None else torch.zeros(grid.layouts[c][0], dtype=grid.dtype, device=grid.device))
                for c, g in enumerate(gu)]
        ubar_tmp = grid.zeros_u()
        bbar = gbody.contiguous().clone() if gbody is not None else torch.zeros(6, dtype=torch.float64, device=grid.device)
        bbar_tmp = torch.zeros(6, dtype=torch.float64, device=grid.device)
        gF = gF.contiguous() if gF is not None else torch.zeros((S, 3), dtype=torch.float64, device=grid.device)
        fbbar = grid.zeros_u()
        kcbar = torch.zeros(6, dtype=torch.float64, device=grid.device)
        # adjoint pressure, carried from step to step as the next solve's guess
        mu = grid.zeros_p()
        starts = list(range(0, S, K))
        # states recomputed inside a segment, one allocation per field
        if K > 1:
            RU = [_slots_like(x, K - 1) for x in ubar]
            RB = _slots_like(bbar, K - 1)
            RP = grid.zeros_p()
        # recomputed and adjoint steps are enqueued back to back; their
        # statuses are checked once at the end
        infos = torch.zeros((2, S, INFO_DOUBLES), dtype=torch.float64, device=grid.device)
        infos_f, infos_a = infos[0], infos[1]
        dts = ctx.dts

        def use_dt(n):
            if dts is not None:
                grid.set_dt(dts[n])

        grid.defer_status(True)
        try:
            for s0 in reversed(starts):
                s1 = min(s0 + K, S)
                cu, cp, cb = ctx.ckpts[s0]
                # states n = s0 .. s1-1 of the segment: the checkpoint, then the
                # recomputed ones, each step writing into fresh velocity tensors
                states = [(cu, cb)]
                if s1 - s0 > 1:
                    p = RP
                    p.copy_(cp)
                    u, body = cu, cb
                    for n in range(s0, s1 - 1):
                        q = n - s0
                        u2 = [X[q] for X in RU]
                        b2 = RB[q]
                        use_dt(n)
                        grid.step(u, p, fb, body, kc, u_out=u2, p_out=p, body_out=b2,
                                  info=infos_f[n], coupling=ctx.coupling, scheme=ctx.scheme)
                        u, body = u2, b2
                        states.append((u, body))
                for n in reversed(range(s0, s1)):
                    un, bn = states[n - s0]
                    dF = gF[n].contiguous()
                    use_dt(n)
                    grid.step_adjoint(un, fb, bn, kc, ubar, bbar, dF, ubar_tmp, bbar_tmp,
                                      fbbar=fbbar, kcbar=kcbar, info=infos_a[n], mu=mu,
                                      omega=None if ctx.omegas is None else ctx.omegas[n],
                                      scheme=ctx.scheme,
                                      p=(cp if n == s0 else RP) if ctx.scheme else None)
                    ubar, ubar_tmp = ubar_tmp, ubar
                    bbar, bbar_tmp = bbar_tmp, bbar
        finally:
            grid.defer_status(False)
            if dts is not None:
                grid.set_dt(ctx.dt0)
        host = infos.cpu()             # one read of both sets of records
        grid.check_infos(host[0], "recomputed step")
        grid.check_infos(host[1], "adjoint step")
        return (None, None, None, None, None, None, None, *ubar, *fbbar, kcbar, bbar)


def rollout(grid: Grid, u0: List[torch.Tensor], fb: Optional[List[torch.Tensor]], kc: torch.Tensor,
            body0: torch.Tensor, nsteps: int, ckpt_every: int = 1, coupling=None,
            scheme: Optional[str] = None, cfl=None):
    """Differentiable rollout; returns (u_final list, body_final, F history (S, 3), p_final).
    coupling = (max_iters, tol) runs strongly coupled steps (Alg. 1 with
    N = max_iters), differentiated through their coupling fixed points.
    scheme ("fe", "rk2", "rk3") runs explicit Runge-Kutta steps; cfl =
    (cfl, dt_max) takes each step's size from the CFL rule at the state
    entering it (the sizes are recorded and replayed by the backward pass;
    they are not differentiated)."""
    if fb is None:
        fb = grid.zeros_u()
    nd = grid.dim
    if coupling is not None:
        coupling = (int(coupling[0]), float(coupling[1]))
    if cfl is not None:
        cfl = (float(cfl[0]), float(cfl[1]))
    outs = _Rollout.apply(grid, int(nsteps), int(max(1, ckpt_every)), coupling, scheme, cfl, nd,
                          *u0, *fb, kc, body0)
    return list(outs[:nd]), outs[nd], outs[nd + 1], outs[nd + 2]


class _WallShear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid: Grid, u0: torch.Tensor):
        ctx.grid = grid
        ctx.shape = u0.shape
        return grid.loss_wall_shear(u0.detach().contiguous())[0]

    @staticmethod
    def backward(ctx, g):
        grid = ctx.grid
        ubar = torch.zeros(ctx.shape, dtype=grid.dtype, device=grid.device)
        dummy = torch.zeros(ctx.shape, dtype=grid.dtype, device=grid.device)
        grid.loss_wall_shear(dummy, ubar)
        return None, ubar * g.to(ubar.dtype)


def wall_shear(grid: Grid, u0: torch.Tensor) -> torch.Tensor:
    """Mean wall shear stress of the streamwise velocity (two walls normal to y)."""
    return _WallShear.apply(grid, u0)


class _RmsLift(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid: Grid, Fh: torch.Tensor, u_ref: float, diameter: float):
        Fc = Fh.detach().contiguous()
        dF = torch.zeros_like(Fc)
        J = grid.loss_rms_lift(Fc.view(-1), 3, 1, u_ref, diameter, dF.view(-1))
        ctx.save_for_backward(dF)
        return J[0]

    @staticmethod
    def backward(ctx, g):
        (dF,) = ctx.saved_tensors
        return None, dF * g, None, None


def rms_lift(grid: Grid, Fh: torch.Tensor, u_ref: float = 1.0, diameter: float = 1.0) -> torch.Tensor:
    """sqrt(mean C_L^2) of a force history (S, 3), C_L = 2 F_y / (rho U^2 D)."""
    return _RmsLift.apply(grid, Fh, u_ref, diameter)
