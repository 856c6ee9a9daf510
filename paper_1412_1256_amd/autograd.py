"""Differentiation form: calibrated Stokes spectra as a torch.autograd.Function.

Forward: set the learnable window, integrate all frames of ``packed`` and form calibrated Stokes spectra
(Eq. 2 with gains and leakage).  Backward: ``ps_calibrate_backward``, which recomputes the per-frame
transforms instead of storing them.  Complex parameters are complex64 tensors; their gradients follow torch's
convention for real losses (dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import torch

from . import Plan, PolarisError


class StokesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gain_x, gain_y, dterms, taps, plan: Plan, packed, psi: float):
        if taps is not None:
            plan.set_window_taps(taps.detach())
        plan.reset()
        plan.accumulate(packed)
        iquv = plan.stokes(gain_x=None if gain_x is None else gain_x.detach(),
                           gain_y=None if gain_y is None else gain_y.detach(),
                           dterms=None if dterms is None else dterms.detach(), psi=psi)
        ctx.save_for_backward(*(t if t is not None else torch.empty(0) for t in (gain_x, gain_y, dterms, taps)))
        ctx.present = tuple(t is not None for t in (gain_x, gain_y, dterms, taps))
        ctx.plan, ctx.packed, ctx.psi = plan, packed, psi
        ctx.integration = plan.integration_id()
        return iquv

    @staticmethod
    def backward(ctx, g_iquv):
        if ctx.plan.integration_id() != ctx.integration:
            # another forward (or reset, accumulate, new taps) ran on the plan since this node's forward: its
            # accumulators and window are no longer this node's
            raise PolarisError(4, "the plan's integration changed after this forward; run the backward before "
                                  "the next forward on the same plan, or use one plan per forward")
        gx, gy, dt, taps = (t if p else None for t, p in zip(ctx.saved_tensors, ctx.present))
        want = []
        if ctx.needs_input_grad[0]:
            want.append("gain_x")
        if ctx.needs_input_grad[1]:
            want.append("gain_y")
        if ctx.needs_input_grad[2]:
            want.append("dterms")
        if ctx.needs_input_grad[3]:
            want.append("taps")
        out = ctx.plan.calibrate_backward(ctx.packed, g_iquv.contiguous(), gain_x=gx, gain_y=gy, dterms=dt,
                                          psi=ctx.psi, want=tuple(want))
        d_gx = torch.view_as_complex(out["gain_x"]) if "gain_x" in out else None
        d_gy = torch.view_as_complex(out["gain_y"]) if "gain_y" in out else None
        d_dt = torch.view_as_complex(out["dterms"].view(-1, 2, 2)) if "dterms" in out else None
        d_taps = out.get("taps")
        return d_gx, d_gy, d_dt, d_taps, None, None, None


def stokes(plan: Plan, packed, gain_x=None, gain_y=None, dterms=None, taps=None, psi: float = 0.0):
    """Differentiable calibrated Stokes spectra [P][4][C] of one integration of ``packed``."""
    return StokesFn.apply(gain_x, gain_y, dterms, taps, plan, packed, psi)
