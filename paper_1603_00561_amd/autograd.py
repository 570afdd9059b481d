"""torch.autograd wrapper of the HIP library: energies E_CCVV, E_CAVV, E_CCAV
as a differentiable function of B, the orbital energies and s (the active
density Gamma is treated as a constant)."""
from __future__ import annotations

import torch

from . import binding


class DsrgDfEnergy(torch.autograd.Function):
    """forward -> dsrg_df_energy; backward -> dsrg_df_energy_backward, which
    recomputes the integral tiles instead of keeping them from the forward."""

    @staticmethod
    def forward(ctx, B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, precision, terms):
        s_val = float(s.detach().item()) if isinstance(s, torch.Tensor) else float(s)
        E = binding.energy(B_cv.detach(), B_ca.detach(), B_av.detach(), eps_c.detach(),
                           eps_a.detach(), eps_v.detach(), gamma1.detach(), s_val,
                           precision=precision, terms=terms)
        ctx.save_for_backward(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1)
        ctx.s_val, ctx.precision, ctx.terms = s_val, precision, terms
        ctx.s_is_tensor = isinstance(s, torch.Tensor)
        return E

    @staticmethod
    def backward(ctx, gE):
        B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1 = ctx.saved_tensors
        g = binding.energy_backward(B_cv.detach(), B_ca.detach(), B_av.detach(),
                                    eps_c.detach(), eps_a.detach(), eps_v.detach(),
                                    gamma1.detach(), ctx.s_val,
                                    gE.detach().to(torch.float64).contiguous(),
                                    precision=ctx.precision, terms=ctx.terms,
                                    want_energy=False)
        ds = g["ds"].reshape(()) if ctx.s_is_tensor else None
        return (g["dB_cv"], g["dB_ca"], g["dB_av"], g["deps_c"], g["deps_a"], g["deps_v"],
                None, ds, None, None)


def energy(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, precision="fp64", terms="all"):
    """Differentiable [E_CCVV, E_CAVV, E_CCAV] (float64 tensor on the GPU)."""
    return DsrgDfEnergy.apply(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, precision, terms)
