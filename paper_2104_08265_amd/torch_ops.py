"""torch.autograd.Function over the C ABI: differentiable simulation.

forward  -> wct_simulate (mean raster + FFT convolution; fluctuation is off in this mode)
backward -> wct_simulate_backward: the adjoint convolution (correlation with the
            conjugate response spectrum) followed by the per-row gather of
            dL/d(Q, t, p, sigma_t, sigma_p) from the Gaussian-pdf derivatives of the
            clipped bin integrals.  The charge grid is recomputed, never stored.
"""
from __future__ import annotations

import torch

from . import wct


class WctSimulate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, q, t, p, sigma_t, sigma_p, plane, event, depo_id, nsigma, n_events):
        dd = wct.DeviceDepos(q.contiguous(), t.contiguous(), p.contiguous(), sigma_t.contiguous(),
                             sigma_p.contiguous(), plane, event, depo_id)
        o = wct.opts(nsigma, False, n_events, 0)
        wave = plan.simulate(dd, o)
        ctx.plan = plan
        ctx.dd = dd
        ctx.o = o
        return wave

    @staticmethod
    def backward(ctx, gwave):
        gq, gt, gp, gst, gsp = ctx.plan.simulate_backward(ctx.dd, ctx.o, gwave.contiguous())
        return None, gq, gt, gp, gst, gsp, None, None, None, None, None


def simulate(plan, q, t, p, sigma_t, sigma_p, plane=None, event=None, depo_id=None, nsigma=3.0, n_events=1):
    """Differentiable waveform [n_events * wave_elems] from per-row depo parameters."""
    return WctSimulate.apply(plan, q, t, p, sigma_t, sigma_p, plane, event, depo_id, nsigma, n_events)
