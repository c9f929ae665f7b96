"""torch.autograd.Function around the library's forward run and hand-written adjoint.

``evolve(fam, U0, nsteps, dt, checkpoint_every)`` advances U0 by ``nsteps`` FAM
steps with the fixed time step ``dt`` (the time step is a constant of the map,
not a function of the state) and returns U_T.  Its backward pass hands
dJ/dU_T to ``fam_adjoint``, which recomputes the forward from checkpoints and
applies the transposed OE, RK stages and residual on the GPU.  Both passes run
entirely in the HIP library; this module only marshals tensors.
"""
import torch


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, fam, nsteps, dt, checkpoint_every):
        U = U0.detach().clone().contiguous()
        fam.run(U, 0.0, int(nsteps), float(dt))
        ctx.fam = fam
        ctx.nsteps = int(nsteps)
        ctx.dt = float(dt)
        ctx.every = int(checkpoint_every)
        ctx.save_for_backward(U0.detach())
        return U

    @staticmethod
    def backward(ctx, grad_out):
        (U0,) = ctx.saved_tensors
        lam = grad_out.detach().to(dtype=torch.float64).contiguous()
        _, g = ctx.fam.adjoint(U0.contiguous(), ctx.nsteps, ctx.dt, ctx.every, dJdUT=lam)
        return g, None, None, None, None


def evolve(fam, U0, nsteps, dt, checkpoint_every=None):
    """U_T after ``nsteps`` fixed-dt steps, differentiable with respect to U0."""
    if checkpoint_every is None:
        checkpoint_every = max(1, int(round(nsteps ** 0.5)))
    return _Evolve.apply(U0, fam, nsteps, dt, checkpoint_every)
