"""torch.autograd.Function wrappers over the C entry points.

CollisionIntegral: I = I[f, N; |g|^2] with the hand-written reverse kernels
(dL/df, dL/d|g|^2 and dL/dN).  RtSolve: f(T) after n RK4 steps in a fixed
bath with the exact discrete adjoint, checkpointed every `checkpoint_every`
steps inside the library.  CoupledSolve: (f(T), N(T)) after n coupled
electron-phonon RK4 steps, with the discrete adjoint of those steps.  The
|g|^2 tensor passed in must hold the plan's current values (load new values
with update_g2 first); it is an input so that autograd can route dL/d|g|^2
to it.
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
        f, nph = ctx.saved_tensors
        plan = ctx.plan
        gI = gI.contiguous()
        want_g2 = ctx.needs_input_grad[1]
        gf, gg2 = None, None
        if ctx.needs_input_grad[0] or want_g2:
            gf, gg2 = binding.collision_vjp(plan, f, nph, gI, want_f=ctx.needs_input_grad[0],
                                            gg2=True if want_g2 else None)
        # the library accumulates dL/d|g|^2 in FP64; autograd wants g2's dtype
        if gg2 is not None:
            gg2 = gg2.to(ctx.g2_dtype)
        gN = None
        if ctx.needs_input_grad[3]:
            if f.dim() == 1:
                gN = binding.collision_vjp_nph(plan, f, nph, gI)
            elif nph.dim() == 3:   # one bath per vector
                gN = torch.stack([binding.collision_vjp_nph(plan, f[b].contiguous(), nph[b].contiguous(),
                                                            gI[b].contiguous()) for b in range(f.shape[0])])
            else:                  # one bath shared by the batch: the vectors' gradients add
                gN = torch.zeros_like(nph)
                for b in range(f.shape[0]):
                    gN += binding.collision_vjp_nph(plan, f[b].contiguous(), nph, gI[b].contiguous())
        return gf, gg2, None, gN


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


class CoupledSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, N0, g2, plan, dt_fs, n_steps, checkpoint_every=20):
        ctx.plan = plan
        ctx.g2_dtype = g2.dtype
        ctx.args = (float(dt_fs), int(n_steps), int(checkpoint_every))
        ctx.save_for_backward(f0, N0)
        fT, NT = f0.detach().clone(), N0.detach().clone()
        binding.rt_step_coupled(plan, fT, NT, dt_fs, n_steps)
        return fT, NT

    @staticmethod
    def backward(ctx, gfT, gNT):
        f0, N0 = ctx.saved_tensors
        dt, n, ce = ctx.args
        gf0, gN0, gg2 = binding.rt_adjoint_coupled(
            ctx.plan, f0, N0, dt, n, ce,
            gfT.contiguous() if gfT is not None else None,
            gNT.contiguous() if gNT is not None else None,
            want_f=ctx.needs_input_grad[0], want_nph=ctx.needs_input_grad[1],
            gg2=True if ctx.needs_input_grad[2] else None)
        if gg2 is not None:
            gg2 = gg2.to(ctx.g2_dtype)
        return gf0, gN0, gg2, None, None, None, None


def collision(f, g2, plan, nph):
    return CollisionIntegral.apply(f, g2, plan, nph)


def rt_solve(f0, g2, plan, nph, dt_fs, n_steps, checkpoint_every=20, use_graph=False):
    return RtSolve.apply(f0, g2, plan, nph, dt_fs, n_steps, checkpoint_every, use_graph)


def coupled_solve(f0, N0, g2, plan, dt_fs, n_steps, checkpoint_every=20):
    return CoupledSolve.apply(f0, N0, g2, plan, dt_fs, n_steps, checkpoint_every)
