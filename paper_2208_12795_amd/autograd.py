"""torch.autograd.Function over the float64 particle steps of libetpic.

`particle_steps(e_env, ...)` runs `nsteps` steps from a given particle state
and returns the final velocities [3, N] (float64).  Its backward is the
hand-written adjoint of libetpic (checkpoint every `checkpoint_every` steps,
segments recomputed in the reverse sweep) and returns the gradient with
respect to the complex edge envelope `e_env` (complex128 [N_e]) in PyTorch's
convention for real losses (dL/dRe + j dL/dIm).  Marshalling only: the steps
and their adjoint run in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import etpic as E


class _ParticleSteps(torch.autograd.Function):
    @staticmethod
    def forward(fctx, e_env, ctx, parts, species, b_env, e_dc, b_dc, step0, nsteps, dt, omega, checkpoint_every):
        assert e_env.dtype == torch.complex128 and e_env.is_cuda
        if parts.precision != E.FP64:
            raise ValueError("the differentiable path runs in float64")
        ee = torch.view_as_real(e_env.detach()).contiguous()
        fields = E.Fields(ee, b_env, e_dc, b_dc)
        work = parts.clone()
        nbytes = ctx.adjoint_workspace_bytes(work.n, nsteps, checkpoint_every)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=e_env.device)
        ctx.forward_checkpointed(work, species, fields, step0, nsteps, dt, omega, checkpoint_every, ws)
        fctx.ctx, fctx.species, fctx.fields, fctx.ws = ctx, species, fields, ws
        fctx.meta = (work.n, step0, nsteps, dt, omega, checkpoint_every)
        return work.vel.clone()

    @staticmethod
    def backward(fctx, grad_v):
        n, step0, nsteps, dt, omega, every = fctx.meta
        vbar = grad_v.to(torch.float64).contiguous().clone()
        xbar = torch.zeros_like(vbar)
        grad_e = torch.zeros(fctx.fields.e_env.shape, dtype=torch.float64, device=vbar.device)
        fctx.ctx.backward(n, fctx.species, fctx.fields, step0, nsteps, dt, omega, every, fctx.ws, vbar, xbar, grad_e)
        return (torch.view_as_complex(grad_e), None, None, None, None, None, None, None, None, None, None, None)


def particle_steps(e_env, ctx, parts, species, b_env, b_dc=None, e_dc=None, *, step0=0, nsteps, dt, omega,
                   checkpoint_every=5):
    """Final velocities [3, N] after `nsteps` float64 steps; differentiable in e_env."""
    return _ParticleSteps.apply(e_env, ctx, parts, species, b_env, e_dc, b_dc, step0, nsteps, dt, omega,
                                checkpoint_every)
