"""torch.autograd wrappers around the HIP forward map and its adjoint.

PyTorch's gradient of a real loss with respect to a complex tensor z is
dL/dRe z + i dL/dIm z = 2 dL/dz^*, so the conjugate-Wirtinger atom gradient
returned by the library (eq. atom-wirtinger-gradient convention) is doubled
here.  Only the inputs are saved: the backward pass recomputes the rotated
amplitudes setting batch by setting batch instead of storing B*R*D of them.
"""
from __future__ import annotations

import torch

from . import api


class BornMap(torch.autograd.Function):
    """probs[b, u] = sum_r alpha_r |(V_b psi_r)_u|^2  (per-setting Born probabilities).
    ``unitaries`` (optional) holds the 2x2 matrices of settings codes >= 3."""

    @staticmethod
    def forward(ctx, atoms, weights, settings, handle, path, unitaries):
        inst = api.Instance(atoms.detach().contiguous(), weights.detach().contiguous(), settings, unitaries=unitaries)
        probs, _ = api.qst_forward(handle, [inst], want_probs=True, path=path)
        ctx.save_for_backward(atoms, weights, settings)
        ctx.handle, ctx.path, ctx.unitaries = handle, path, unitaries
        return probs[0]

    @staticmethod
    def backward(ctx, grad_probs):
        atoms, weights, settings = ctx.saved_tensors
        inst = api.Instance(atoms.detach().contiguous(), weights.detach().contiguous(), settings,
                            unitaries=ctx.unitaries)
        _, ag, wg = api.qst_backward(ctx.handle, [inst], grad_p=[grad_probs.contiguous()], path=ctx.path)
        return 2 * ag[0], wg[0], None, None, None, None


class FusedLoss(torch.autograd.Function):
    """Loss (CE or LS on the stacked probabilities) with its gradients from one fused pass.
    ``freqs`` is a dense [B][D] tensor or a CSR triple (rowptr, index, values)."""

    @staticmethod
    def forward(ctx, atoms, weights, settings, freqs, handle, loss, eps, path, unitaries):
        dense = freqs if isinstance(freqs, torch.Tensor) else None
        inst = api.Instance(atoms.detach().contiguous(), weights.detach().contiguous(), settings, dense,
                            unitaries=unitaries, freqs_csr=None if dense is not None else tuple(freqs))
        lt, ag, wg = api.qst_backward(handle, [inst], loss=loss, eps=eps, path=path)
        ctx.save_for_backward(ag[0], wg[0])
        return lt[0]

    @staticmethod
    def backward(ctx, grad_out):
        ag, wg = ctx.saved_tensors
        return 2 * ag * grad_out.to(ag.real.dtype), wg * grad_out, None, None, None, None, None, None, None


def born_map(atoms, weights, settings, handle, path=api.PATH_AUTO, unitaries=None):
    return BornMap.apply(atoms, weights, settings, handle, path, unitaries)


def fused_loss(atoms, weights, settings, freqs, handle, loss=api.LOSS_CE, eps=1e-8, path=api.PATH_AUTO,
               unitaries=None):
    return FusedLoss.apply(atoms, weights, settings, freqs, handle, loss, eps, path, unitaries)
