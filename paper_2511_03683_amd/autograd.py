"""torch.autograd.Function wrappers over the C entry points.

CollisionIntegral: I = I[f; |g|^2] with the hand-written reverse kernel
(dL/df and dL/d|g|^2).  RtSolve: f(T) after n RK4 steps with the exact
discrete adjoint, checkpointed every `checkpoint_every` steps inside the
library.  The |g|^2 tensor passed in must hold the plan's current values
(load new values with Plan-level update_g2 first); it is an input so that
autograd can route dL/d|g|^2 to it.
"""
import torch

from . import binding


class CollisionIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g2, plan, nph):
        ctx.plan = plan
        ctx.g2_dtype = g2.dtype
        ctx.save_for_backward(f, nph)
        return binding.collision_integral(plan, f, nph)

    @staticmethod
    def backward(ctx, gI):
        if ctx.needs_input_grad[3]:
            raise NotImplementedError("collision: no gradient with respect to the phonon occupations")
        f, nph = ctx.saved_tensors
        plan = ctx.plan
        want_g2 = ctx.needs_input_grad[1]
        gf, gg2 = binding.collision_vjp(plan, f, nph, gI.contiguous(),
                                        want_f=ctx.needs_input_grad[0],
                                        gg2=True if want_g2 else None)
        # the library accumulates dL/d|g|^2 in FP64; autograd wants g2's dtype
        if gg2 is not None:
            gg2 = gg2.to(ctx.g2_dtype)
        return gf, gg2, None, None


class RtSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, g2, plan, nph, dt_fs, n_steps, checkpoint_every=20, use_graph=False):
        ctx.plan = plan
        ctx.g2_dtype = g2.dtype
        ctx.args = (float(dt_fs), int(n_steps), int(checkpoint_every))
        ctx.save_for_backward(f0, nph)
        fT = f0.detach().clone()
        binding.rt_step(plan, fT, nph, dt_fs, n_steps, use_graph=use_graph)
        return fT

    @staticmethod
    def backward(ctx, gfT):
        if ctx.needs_input_grad[3]:
            raise NotImplementedError("rt_solve: no gradient with respect to the phonon occupations")
        f0, nph = ctx.saved_tensors
        dt, n, ce = ctx.args
        gf0, gg2 = binding.rt_adjoint(ctx.plan, f0, nph, dt, n, ce, gfT.contiguous(),
                                      want_f=True,
                                      gg2=True if ctx.needs_input_grad[1] else None)
        if gg2 is not None:
            gg2 = gg2.to(ctx.g2_dtype)
        return gf0, gg2, None, None, None, None, None, None


def collision(f, g2, plan, nph):
    return CollisionIntegral.apply(f, g2, plan, nph)


def rt_solve(f0, g2, plan, nph, dt_fs, n_steps, checkpoint_every=20, use_graph=False):
    return RtSolve.apply(f0, g2, plan, nph, dt_fs, n_steps, checkpoint_every, use_graph)
