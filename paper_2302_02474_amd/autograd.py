"""The TILD energy as a differentiable function of positions and of the
interaction parameters, for torch.autograd.

E(x, chi, kappa, a) is the bonded + non-bonded mesh energy (Eqs. fh,
HelfandP, bonds); its adjoints come from one call of tild_energy_grad:
dE/dx is minus the exact-gradient force, dE/dchi, dE/dkappa and dE/da are the
k-space sums of the energy's derivative.  Every evaluation runs on the GPU
through the C ABI.
"""

from __future__ import annotations

import torch

from . import Tild


class TildEnergy(torch.autograd.Function):
    """E = TildEnergy.apply(x, chi, kappa, a, ctx) for a Tild context ``ctx``.

    x: (n, 3) CUDA tensor (float32 or float64) in ABI order; chi, kappa, a:
    0-d tensors (or Python floats).  Returns a 0-d float64 tensor on x's device.
    """

    @staticmethod
    def forward(fctx, x, chi, kappa, a, tild: Tild):
        c, k, s = (float(v) for v in (chi, kappa, a))
        tild.set_interaction(c, k, s)
        xs = x.detach().contiguous()
        tild.set_positions(xs)
        gx = torch.empty_like(xs)
        vals, _ = tild.energy_grad(grad_x=gx)
        fctx.save_for_backward(gx)
        fctx.dpar = (vals["dE_dchi"], vals["dE_dkappa"], vals["dE_da"])
        fctx.par_meta = [(t.dtype, t.device) if torch.is_tensor(t) else None for t in (chi, kappa, a)]
        return torch.tensor(vals["E"], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(fctx, g):
        (gx,) = fctx.saved_tensors
        gs = g.to(gx.dtype)
        grads = []
        for d, meta in zip(fctx.dpar, fctx.par_meta):
            grads.append(None if meta is None else (g * d).to(dtype=meta[0], device=meta[1]))
        return (gs * gx, *grads, None)


def tild_energy(x, chi, kappa, a, tild: Tild):
    """Differentiable energy; see TildEnergy."""
    return TildEnergy.apply(x, chi, kappa, a, tild)
