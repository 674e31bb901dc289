"""PyTorch autograd over the batched step and rollout (Sec. III-D).

Two differentiable entry points, each a ``torch.autograd.Function`` whose
backward is the library's adjoint kernel (no PyTorch arithmetic on the path):

* :func:`step` -- one backward-Euler step of every world, (q-, u-, ctrl) ->
  (q+, u+, lambda+).  The forward stores the Schur factor at the returned
  iterate (the tape); the backward back-solves it (Eqs. (16)-(19)).
  lambda+ is returned for warm starts and is not differentiable.
* :func:`rollout_loss` -- a T-step spline-driven rollout with the final-xy
  loss, per world.  The forward keeps only the checkpoints the workspace
  holds; the backward recomputes each segment from its checkpoint and runs the
  adjoint steps in reverse.  Upstream cotangents of the per-world losses are
  passed to the kernels as loss weights.
"""
from __future__ import annotations

import torch

from . import Simulator

__all__ = ["step", "rollout_loss"]


class _Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, u, ctrl, sim: Simulator, lam):
        tape = sim.new_tape()
        out = sim.step_forward(q.detach(), u.detach(), lam.detach(),
                               None if ctrl is None else ctrl.detach(), tape=tape)
        ctx.sim = sim
        ctx.has_ctrl = ctrl is not None
        ctx.save_for_backward(q.detach(), u.detach(), None if ctrl is None else ctrl.detach(),
                              out["u"], out["lam"], tape)
        ctx.mark_non_differentiable(out["lam"])
        ctx.info = {k: out[k] for k in ("status", "iters", "n_act", "act_slot", "resnorm")}
        return out["q"], out["u"], out["lam"]

    @staticmethod
    def backward(ctx, gq, gu, _glam):
        q, u, ctrl, un, ln, tape = ctx.saved_tensors
        sim = ctx.sim
        if gq is None:
            gq = torch.zeros_like(q)
        if gu is None:
            gu = torch.zeros_like(u)
        gqp, gup, gc = sim.step_adjoint(q, u, ctrl, un, ln, tape, gq.contiguous(), gu.contiguous())
        return gqp, gup, (gc if ctx.has_ctrl else None), None, None


def step(sim: Simulator, q, u, lam, ctrl=None):
    """Differentiable step: returns (q+, u+, lambda+) as device tensors."""
    return _Step.apply(q, u, ctrl, sim, lam)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, knots, q0, u0, sim: Simulator, basis, T, ckpt_every, loss_body, target):
        ws = sim.new_workspace(T, ckpt_every)
        r = sim.rollout(q0.detach(), u0.detach(), None if knots is None else knots.detach(), basis, T,
                        ckpt_every=ckpt_every, loss_body=loss_body, target=target, phase=1, workspace=ws,
                        grads=False)
        ctx.sim, ctx.T, ctx.ck = sim, T, ckpt_every
        ctx.args = (q0.detach(), u0.detach(), None if knots is None else knots.detach(), basis, loss_body, target)
        ctx.ws = ws
        ctx.knots_shape = None if knots is None else knots.shape
        ctx.status = r["status"]
        return r["loss"]

    @staticmethod
    def backward(ctx, gloss):
        q0, u0, knots, basis, lb, tg = ctx.args
        r = ctx.sim.rollout(q0, u0, knots, basis, ctx.T, ckpt_every=ctx.ck, loss_body=lb, target=tg, phase=2,
                            workspace=ctx.ws, loss_grad=gloss.contiguous())
        ctx.ws = None
        gk = None if knots is None else r["g_knots"].reshape(ctx.knots_shape)
        return gk, r["g_q0"], r["g_u0"], None, None, None, None, None, None


def rollout_loss(sim: Simulator, knots, q0, u0, basis, T: int, ckpt_every: int = 10, loss_body=None,
                 target=None):
    """Per-world final-xy loss of a T-step rollout, differentiable in knots, q0 and u0."""
    return _Rollout.apply(knots, q0, u0, sim, basis, T, ckpt_every, loss_body, target)
