"""torch.autograd.Function around a run of ADER-DG steps with receivers.

``seismograms(solver, u0, params, dt, steps)`` runs ``steps`` FP64 steps of
the solver's PDE from ``u0`` with the step size held fixed and returns the
receiver samples after every step, ``[steps, nrec, nvar]``.  Its backward is
the library's hand-written discrete adjoint (``adg_step_adjoint_kept`` and
``adg_sample_receivers_adjoint``), run in reverse over the steps with
time-step checkpointing: the forward pass keeps the state every ``every``
steps; the backward pass recomputes one segment from its checkpoint with
``adg_run_keep``, which keeps per step what that step's adjoint reads of
its forward predictor, then runs the adjoint steps of that segment
backwards from those buffers.  The forward pass runs its last segment with
``adg_run_keep`` already, so that the backward pass starts without a
recomputation; the segments are laid out from the end (the first one takes
the remainder of ``steps`` / ``every``), so that this kept segment is a
whole one.  Memory: ceil(steps / every) checkpoints plus ``every``
keep buffers (``Solver.keep_size()`` doubles each), the latter held from
the forward pass on.

Gradients flow to ``u0`` and ``params``.  The step size is not
differentiated (it is an input, as in a run with a frozen dt).  Available
for the PDEs the adjoint is built for (elasticity, the advection test PDE).
"""
from __future__ import annotations

import math

import torch

from . import adg


def _segments(steps: int, every: int):
    """Checkpoint segment bounds [0, b_1, ..., steps]: segments of ``every``
    steps counted from the end, the first one the remainder."""
    if steps <= 0:
        return [0]
    nseg = math.ceil(steps / every)
    return [0] + [steps - (nseg - k) * every for k in range(1, nseg)] + [steps]


def _time_nodes(t0: float, dt: float, steps: int):
    """t^n as the device clock accumulates it (t <- t + dt in float64)."""
    ts = [t0]
    t = t0
    for _ in range(steps):
        t = t + dt
        ts.append(t)
    return ts


class _SeismogramRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, params, solver, t0, dt, steps, every):
        if solver.nrec == 0:
            raise ValueError("set receivers on the solver first")
        if solver.cfg.precision != adg.FP64:
            # the library's adjoint is that of the FP64 step
            raise ValueError("seismograms() needs an FP64 solver (the adjoint is that of the FP64 step)")
        prm = params.detach().contiguous() if params is not None else None
        Q = u0.detach().contiguous().clone()
        clock = torch.tensor([t0, dt], dtype=torch.float64, device=Q.device)
        out = torch.empty((steps, solver.nrec, solver.nvar), dtype=torch.float64, device=Q.device)
        ckpts = [Q.clone()]
        last_keeps = None
        bounds = _segments(steps, every)
        nseg = len(bounds) - 1
        for seg in range(nseg):
            # one checkpoint segment (fused corrector/predictor kernels where built)
            n0, n1 = bounds[seg], bounds[seg + 1]
            if seg + 1 < nseg:
                solver.run(Q, prm, clock, n1 - n0, out[n0:n1])
                # (the last segment's start state is not needed: it is kept)
                ckpts.append(Q.clone() if seg + 2 < nseg else None)
            else:
                # the last segment keeps what its adjoint steps read
                last_keeps = torch.empty((n1 - n0, solver.keep_size()), dtype=torch.float64, device=Q.device)
                solver.run_keep(Q, prm, clock, n1 - n0, last_keeps, out[n0:n1])
        ctx.solver, ctx.t0, ctx.dt, ctx.steps, ctx.every = solver, t0, dt, steps, every
        ctx.ckpts = ckpts
        ctx.last_keeps = last_keeps
        ctx.prm = prm
        ctx.has_params = params is not None
        return out

    @staticmethod
    def backward(ctx, gout):
        s, dt, steps, every = ctx.solver, ctx.dt, ctx.steps, ctx.every
        if ctx.ckpts is None:
            raise RuntimeError("the checkpointed adjoint runs once per forward pass (it consumes its checkpoints)")
        prm = ctx.prm
        dev = ctx.ckpts[0].device
        gout = gout.detach().to(torch.float64).contiguous()
        lam = torch.zeros_like(ctx.ckpts[0])
        g = torch.zeros_like(prm) if (prm is not None and s.nparam > 0) else None
        ts = _time_nodes(ctx.t0, dt, steps)
        clocks = torch.tensor([[ts[n], dt] for n in range(steps)], dtype=torch.float64, device=dev)
        bounds = _segments(steps, every)
        nseg = len(bounds) - 1
        keep_n = s.keep_size()
        for seg in reversed(range(nseg)):
            n0, n1 = bounds[seg], bounds[seg + 1]
            if seg == nseg - 1 and ctx.last_keeps is not None:
                keeps, ctx.last_keeps = ctx.last_keeps, None  # kept by the forward pass
            else:
                # recompute steps n0 .. n1-1 from the checkpoint (advanced in
                # place: it is not needed again), keeping what each step's
                # adjoint reads
                Q = ctx.ckpts[seg]
                clock = clocks[n0].clone()
                keeps = torch.empty((n1 - n0, keep_n), dtype=torch.float64, device=dev)
                s.run_keep(Q, prm, clock, n1 - n0, keeps)
                del Q
            ctx.ckpts[seg] = None
            for n in reversed(range(n0, n1)):
                # out[n] samples u^{n+1}; the step n maps u^n to u^{n+1}
                s.sample_receivers_adjoint(gout[n], lam)
                s.step_adjoint_kept(prm, clocks[n], keeps[n - n0], lam, g)
            del keeps
        ctx.ckpts = None
        gu0 = lam
        gp = g if ctx.has_params else None
        return gu0, gp, None, None, None, None, None


def seismograms(solver, u0: torch.Tensor, params, dt: float, steps: int, t0: float = 0.0,
                every: int | None = None) -> torch.Tensor:
    """Receiver samples [steps, nrec, nvar] after each of ``steps`` fixed-dt
    steps from ``u0``; differentiable in ``u0`` and ``params``.  ``every``:
    checkpoint interval (default ceil(sqrt(steps)))."""
    if every is None:
        every = max(1, math.ceil(math.sqrt(steps)))
    return _SeismogramRun.apply(u0, params, solver, float(t0), float(dt), int(steps), int(every))
