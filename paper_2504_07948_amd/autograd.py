"""torch.autograd.Function over the library's ion-coordinate adjoint.

``IonGradFn.apply(ion_xyz, ctx)`` moves the ions of a dmcx Context to
``ion_xyz`` (the library re-evaluates orbitals, inverses and local energies at
the current walkers) and returns per-walker ``(log_psi, v_pot, e_local)``.  The
backward pass calls the library's hand-written reverse-mode adjoint
(dmcx_logpsi_vjp / dmcx_potential_vjp): Eq. 3 of arXiv 2504.07948 with
lambda = an ion coordinate, i.e. the Pulay term through basis, MO
contraction, log-determinant and Jastrow, plus the Hellmann-Feynman term
through V.  E_L is returned as a non-differentiable output.

This module only marshals arguments.  With CUDA tensors every buffer is handed
to the library as a device pointer on the context's stream (the caller keeps
torch's current stream equal to the stream the context was created on), so
nothing crosses to the host; CPU tensors are passed as host buffers.
"""
from __future__ import annotations

import torch

from . import dmcx


def _f64(t):
    return t.detach().to(torch.float64).contiguous()


class IonGradFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ion_xyz, dmc):
        dev = ion_xyz.device
        ion = _f64(ion_xyz)
        mem = dmcx.DMCX_DEVICE if ion.is_cuda else dmcx.DMCX_HOST
        dmc.check(dmcx.dmcx_set_ions(dmc.h, 0, ion.data_ptr(), mem))
        e = torch.empty(dmc.W, dtype=torch.float64, device=dev)
        lp = torch.empty_like(e)
        v = torch.empty_like(e)
        dmc.check(dmcx.dmcx_measure(dmc.h, e.data_ptr(), lp.data_ptr(), None, mem))
        dmc.check(dmcx.dmcx_potential(dmc.h, v.data_ptr(), mem))
        ctx.dmc = dmc
        ctx.keep = ion  # the library reads it in stream order
        ctx.mark_non_differentiable(e)
        return lp, v, e

    @staticmethod
    def backward(ctx, g_lp, g_v, g_e):
        dmc = ctx.dmc
        dev = ctx.keep.device
        mem = dmcx.DMCX_DEVICE if ctx.keep.is_cuda else dmcx.DMCX_HOST
        grad = torch.zeros((dmc.n_atom, 3), dtype=torch.float64, device=dev)
        part = torch.empty_like(grad)
        for g, call in ((g_lp, dmcx.dmcx_logpsi_vjp), (g_v, dmcx.dmcx_potential_vjp)):
            if g is None:
                continue
            gg = _f64(g.to(dev))
            dmc.check(call(dmc.h, gg.data_ptr(), part.data_ptr(), mem))
            grad += part
        return grad.to(ctx.keep.dtype), None
