"""torch.autograd.Function over the library's ion-coordinate adjoint.

``IonGradFn.apply(ion_xyz, ctx)`` moves the ions of a dmcx Context to
``ion_xyz`` (re-evaluating orbitals, inverses and local energies at the
current walkers) and returns per-walker ``(log_psi, v_pot, e_local)``.  The
backward pass calls the library's hand-written reverse-mode adjoint
(dmcx_logpsi_vjp / dmcx_potential_vjp): Eq. 3 of arXiv 2504.07948 with
lambda = an ion coordinate, i.e. the Pulay term through basis, MO
contraction, log-determinant and Jastrow, plus the Hellmann-Feynman term
through V.  E_L is returned as a non-differentiable output.

With walker weights omega and E_L held fixed, the force estimate
F = -<dV/dR> - 2 (<E_L dlnPsi/dR> - <E_L><dlnPsi/dR>) is minus the gradient of
``force_objective(log_psi, v_pot, e_local, omega)``.
"""
from __future__ import annotations

import numpy as np
import torch


class IonGradFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ion_xyz, dmc):
        dmc.set_ions(ion_xyz.detach().to("cpu", torch.float64).numpy())
        e, lp, _ = dmc.measure()
        v = dmc.potential()
        ctx.dmc = dmc
        ctx.device = ion_xyz.device
        out = [torch.from_numpy(a).to(ion_xyz.device) for a in (lp, v, e)]
        ctx.mark_non_differentiable(out[2])
        return out[0], out[1], out[2]

    @staticmethod
    def backward(ctx, g_lp, g_v, g_e):
        dmc = ctx.dmc
        grad = np.zeros((dmc.n_atom, 3))
        if g_lp is not None:
            grad += dmc.logpsi_vjp(g_lp.detach().to("cpu", torch.float64).numpy())
        if g_v is not None:
            grad += dmc.potential_vjp(g_v.detach().to("cpu", torch.float64).numpy())
        return torch.from_numpy(grad).to(ctx.device), None


def force_objective(log_psi, v_pot, e_local, omega):
    """<V> + 2 (<E_L lnPsi> - <E_L><lnPsi>) with E_L and omega constant;
    minus its gradient w.r.t. the ions is the Hellmann-Feynman + Pulay force."""
    wsum = omega.sum()
    e = e_local.detach()
    e_mean = (omega * e).sum() / wsum
    return (omega * v_pot).sum() / wsum + 2.0 * ((omega * (e - e_mean) * log_psi).sum() / wsum)
