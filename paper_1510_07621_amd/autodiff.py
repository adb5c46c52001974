"""Gradients through the P3M force and the kick-drift-kick leapfrog.

``force(plan, pos, mass)`` is the P3M force as a differentiable function of
the positions; its backward is the library's force adjoint
(``p3m_force_vjp``). ``leapfrog(plan, pos, mom, mass, dt, box, steps)`` runs
``steps`` kick-drift-kick steps with the library's calls (the first half-kick
and the drift fused into one pass, then the force and the second half-kick)
and is differentiable in the initial positions and momenta; its
backward runs the transposed steps with the force adjoint and the drift
transpose, recomputing the trajectory segment by segment from stored
checkpoints (every ``segment`` steps, default ceil(sqrt(steps)), so memory
grows as sqrt(steps) states while the recomputation costs about one extra
forward pass).

The transposed step (static background): with x1 = wrap(x + dt p'/m),
p' = p + (dt/2) F(x), p1 = p' + (dt/2) F(x1),

    x1_bar += VJP_F(x1, (dt/2) p1_bar);  p'_bar = p1_bar + (dt/m) x1_bar;
    x_bar = x1_bar + VJP_F(x, (dt/2) p'_bar);  p_bar = p'_bar.

Consecutive steps meet at the same positions with the same momentum
cotangent, so their two half-step adjoints are taken as one call with dt:
a trajectory of T steps costs T + 1 force adjoints, like its T + 1 forces.
Positions are differentiated through the periodic wrap with slope 1; the
force is not differentiable where a pair crosses the cutoff or a particle a
mesh node plane (measure zero).

Everything runs on the current torch stream through the C ABI; nothing here
computes on the host.
"""
from __future__ import annotations

import math

import torch

from . import binding


class _Force(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, plan, mass):
        ctx.plan = plan
        ctx.mass = mass
        ctx.save_for_backward(pos)
        return plan.force(pos.detach(), mass)

    @staticmethod
    def backward(ctx, force_bar):
        (pos,) = ctx.saved_tensors
        pos_bar = ctx.plan.force_vjp(pos.detach(), ctx.mass, force_bar.contiguous())
        return pos_bar, None, None


def force(plan: "binding.Plan", pos: torch.Tensor, mass) -> torch.Tensor:
    """F = m (a_PP + a_PM) at pos, differentiable in pos (FP64 (3, n))."""
    return _Force.apply(pos, plan, mass)


def _steps(plan, x, p, F, mass, dt, box, k, keep=None):
    """k KDK steps in place on (x, p, F); appends a copy of each new x to keep."""
    for _ in range(k):
        binding.kick_drift(x, p, F, mass, 0.5 * dt, dt, box)   # = kick, then drift
        plan.force(x, mass, out=F)
        binding.kick(p, F, 0.5 * dt)
        if keep is not None:
            keep.append(x.clone())


class _Leapfrog(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mom, plan, mass, dt, box, steps, segment):
        x = pos.detach().clone()
        p = mom.detach().clone()
        F = plan.force(x, mass)
        # checkpoint states (x, p, F) at the start of each segment
        ckpt = []
        for s0 in range(0, steps, segment):
            ckpt.append((x.clone(), p.clone(), F.clone()))
            _steps(plan, x, p, F, mass, dt, box, min(segment, steps - s0))
        ctx.plan, ctx.mass, ctx.dt, ctx.box = plan, mass, dt, box
        ctx.steps, ctx.segment, ctx.ckpt = steps, segment, ckpt
        ctx.x_end = x.clone()
        return x, p

    @staticmethod
    def backward(ctx, x_bar, p_bar):
        plan, mass, dt, box = ctx.plan, ctx.mass, ctx.dt, ctx.box
        xb = (torch.zeros_like(ctx.x_end) if x_bar is None else x_bar).clone().contiguous()
        pb = (torch.zeros_like(ctx.x_end) if p_bar is None else p_bar).clone().contiguous()
        vjp = torch.empty_like(xb)
        # second half kick of the last step
        plan.force_vjp(ctx.x_end, mass, pb, out=vjp)
        binding.kick(xb, vjp, 0.5 * dt)
        for si in range(len(ctx.ckpt) - 1, -1, -1):
            s0 = si * ctx.segment
            k = min(ctx.segment, ctx.steps - s0)
            x, p, F = (t.clone() for t in ctx.ckpt[si])
            xs = [x.clone()]                    # x_{s0} .. x_{s0+k-1}
            _steps(plan, x, p, F, mass, dt, box, k - 1, keep=xs)
            for t in range(k - 1, -1, -1):
                binding.drift_vjp(pb, xb, mass, dt)
                plan.force_vjp(xs[t], mass, pb, out=vjp)
                c = 0.5 * dt if (s0 + t == 0) else dt
                binding.kick(xb, vjp, c)
            ctx.ckpt[si] = None
        return xb, pb, None, None, None, None, None, None


def leapfrog(plan: "binding.Plan", pos: torch.Tensor, mom: torch.Tensor, mass, dt: float,
             box: float, steps: int, segment: int | None = None):
    """(x_T, p_T) after ``steps`` KDK steps from (pos, mom), differentiable in
    both; the plan must have been made with ``Params(adjoint=True)``."""
    steps = int(steps)
    if steps < 1:
        raise ValueError("steps must be >= 1")
    if segment is None:
        segment = max(1, math.ceil(math.sqrt(steps)))
    if int(segment) < 1:
        raise ValueError("segment must be >= 1")
    return _Leapfrog.apply(pos, mom, plan, mass, float(dt), float(box), steps, int(segment))
