"""torch.autograd wrapper of the structure-factor score (forward kernel) and
its hand-written adjoint (gradient kernel), plus the on-device refinement
driver.  Marshalling only: all arithmetic runs in libaraullo.so.

Score (built on Eq. (2), the direct Fourier transform, evaluated on spherical
shells |k| = f_w along rotated mesh directions): for each ROI with
orientation q, J(q) = sum_{w,v} (|F_{w,v}(q)| / N_w - T_{w,v})^2 with
F_{w,v} = sum_j exp(-2 pi i f_w (R(q/|q|) n_v) . x_j).
"""
from __future__ import annotations

import torch

from . import native


class SFScore(torch.autograd.Function):
    """J per ROI as a differentiable function of the float32 quaternions."""

    @staticmethod
    def forward(ctx, quats, actx, rel, offsets, phase, directions, freqs, targets):
        q = quats.detach().contiguous()
        score, _ = native.ar_sf_score_grad(actx, rel, offsets, q, phase, directions, freqs, targets, grad=False)
        ctx.actx = actx
        ctx.save_for_backward(q, rel, offsets, phase, directions, freqs, targets)
        return score

    @staticmethod
    def backward(ctx, grad_out):
        q, rel, offsets, phase, directions, freqs, targets = ctx.saved_tensors
        _, g = native.ar_sf_score_grad(ctx.actx, rel, offsets, q, phase, directions, freqs, targets, grad=True)
        return grad_out[:, None] * g, None, None, None, None, None, None, None


def sf_score(actx, quats, rel, offsets, phase, directions, freqs, targets):
    return SFScore.apply(quats, actx, rel, offsets, phase, directions, freqs, targets)


def refine(actx, quats, rel, offsets, phase, directions, freqs, targets, steps: int = 50, a0: float = 0.01):
    """Refine float32 quaternions [n_roi][4] in place on the device; returns the final scores."""
    return native.ar_refine_orientations(actx, rel, offsets, quats, phase, directions, freqs, targets, steps, a0)
