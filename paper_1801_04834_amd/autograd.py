"""torch.autograd.Function over the library's gain-applied correlator and its adjoint.

``gain_correlate(plan, vis0, gains)`` returns V' = g_a conj(g_b) V0 (complex64, visibility
layout [SB, C, B, 4]); its backward calls ``cobalt_apply_gains_adjoint``, so gradients with
respect to the gains come from the hand-written HIP adjoint.  ``vis0`` is the ungained output
of the X stage (``torch.view_as_complex`` of a float plan's visibility tensor) and is treated
as a constant.
"""

from __future__ import annotations

import torch


class GainCorrelate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gains, vis0, plan):
        gains = gains.contiguous()
        vis0 = vis0.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(gains, vis0)
        return plan.apply_gains(vis0, gains)

    @staticmethod
    def backward(ctx, grad_vis):
        gains, vis0 = ctx.saved_tensors
        grad = ctx.plan.apply_gains_adjoint(vis0, gains, grad_vis.contiguous())
        return grad, None, None


def gain_correlate(plan, vis0, gains):
    """Differentiable V' = g_a conj(g_b) V0 on the plan's device."""
    return GainCorrelate.apply(gains, vis0, plan)
