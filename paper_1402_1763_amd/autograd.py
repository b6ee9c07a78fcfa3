"""chi2_K of the messenger Wiener filter as a differentiable torch function.

wiener_chi2(pk, d, wf) returns chi2_K = sum_obs d (d - s_K) / N (one per chain
when wf covers every chain of its sampler), where s_K is
the K-th iterate of the deterministic messenger iteration from s = 0 (the
means of the messenger and signal conditionals, Sec. 3.1) at power spectrum
pk.  Its backward pass runs the library's checkpointed adjoint (one forward
recomputation per checkpoint segment, then the adjoint iteration), giving the
gradients with respect to pk (physical units) and d.  Only argument
marshalling happens here; both passes run in the HIP library.
"""
from __future__ import annotations

import torch

from .binding import WienerFilter


class WienerChi2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pk, d, wf: WienerFilter):
        pk = pk.detach().contiguous()
        d = d.detach().contiguous()
        chi2, _ = wf.forward(d, pk)
        ctx.wf = wf
        ctx.generation = wf.generation
        ctx.save_for_backward(pk, d)
        return chi2

    @staticmethod
    def backward(ctx, grad_out):
        pk, d = ctx.saved_tensors
        wf = ctx.wf
        if wf.generation != ctx.generation:   # checkpoints overwritten since
            wf.forward(d, pk)
        grad_d, grad_pk = wf.backward(d)
        if grad_out.dim() == 1:        # one chi2 per chain
            return grad_out[:, None] * grad_pk, grad_out[:, None, None, None] * grad_d, None
        return grad_out * grad_pk, grad_out * grad_d, None


def wiener_chi2(pk: torch.Tensor, d: torch.Tensor, wf: WienerFilter) -> torch.Tensor:
    return WienerChi2.apply(pk, d, wf)
