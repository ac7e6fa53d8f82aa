"""torch.autograd.Functions over the library: forward = jam_eval_batch,
backward = jam_vjp; the chi^2 of eq. (chi2_dyn), forward = jam_eval_chi2,
backward = jam_vjp_chi2; and the radial anisotropy profile, forward =
jam_beta_logistic, backward = jam_beta_logistic_vjp.

Only the per-bin output v_rms^2 is saved for the backward pass (a few
doubles per model); every other forward intermediate is recomputed inside
jam_vjp, so memory does not grow with the batch beyond the workspace.
PyTorch provides device memory and streams; all arithmetic runs in the
library's kernels.
"""
from __future__ import annotations

import torch

from . import binding


class JamVrms2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, jctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0):
        V, st = jctx.eval_batch(geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
        ctx.jctx = jctx
        ctx.geom_idx = geom_idx
        ctx.has_amp = (lum_I0 is not None, mass_S0 is not None)
        ctx.save_for_backward(inc, mass_scale, m_bh, beta,
                              lum_I0 if lum_I0 is not None else inc.new_empty(0),
                              mass_S0 if mass_S0 is not None else inc.new_empty(0), V)
        ctx.mark_non_differentiable(st)
        return V, st

    @staticmethod
    def backward(ctx, gV, _gst):
        inc, ml, mbh, beta, I0, S0, V = ctx.saved_tensors
        I0 = I0 if ctx.has_amp[0] else None
        S0 = S0 if ctx.has_amp[1] else None
        g = ctx.jctx.vjp(ctx.geom_idx, inc, ml, mbh, beta, I0, S0, V,
                         gV.contiguous().to(torch.float64))
        return (None, None, g["inc"], g["mass_scale"], g["m_bh"], g["beta"],
                g["lum_I0"] if ctx.has_amp[0] else None,
                g["mass_S0"] if ctx.has_amp[1] else None)


def jam_vrms2(jctx: binding.Context, geom_idx, inc, mass_scale, m_bh, beta,
              lum_I0=None, mass_S0=None):
    """Differentiable v_rms^2 per bin (packed) and the per-model status."""
    return JamVrms2.apply(jctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)


class JamChi2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, jctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0):
        c2, V, st = jctx.eval_chi2(geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                                   keep_vrms2=True)
        ctx.jctx = jctx
        ctx.geom_idx = geom_idx
        ctx.has_amp = (lum_I0 is not None, mass_S0 is not None)
        ctx.save_for_backward(inc, mass_scale, m_bh, beta,
                              lum_I0 if lum_I0 is not None else inc.new_empty(0),
                              mass_S0 if mass_S0 is not None else inc.new_empty(0), V)
        ctx.mark_non_differentiable(st)
        return c2, st

    @staticmethod
    def backward(ctx, gc, _gst):
        inc, ml, mbh, beta, I0, S0, V = ctx.saved_tensors
        I0 = I0 if ctx.has_amp[0] else None
        S0 = S0 if ctx.has_amp[1] else None
        g = ctx.jctx.vjp_chi2(ctx.geom_idx, inc, ml, mbh, beta, I0, S0,
                              gc.contiguous().to(torch.float64), vrms2=V)
        return (None, None, g["inc"], g["mass_scale"], g["m_bh"], g["beta"],
                g["lum_I0"] if ctx.has_amp[0] else None,
                g["mass_S0"] if ctx.has_amp[1] else None)


def jam_chi2(jctx: binding.Context, geom_idx, inc, mass_scale, m_bh, beta,
             lum_I0=None, mass_S0=None):
    """Differentiable chi^2 per model (eq. chi2_dyn; kinematics set on the
    context with ``set_kinematics``) and the per-model status."""
    return JamChi2.apply(jctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)


class BetaLogistic(torch.autograd.Function):
    @staticmethod
    def forward(ctx, jctx, geom_idx, prof):
        ctx.jctx = jctx
        ctx.geom_idx = geom_idx
        ctx.save_for_backward(prof)
        return jctx.beta_logistic(geom_idx, prof)

    @staticmethod
    def backward(ctx, gbeta):
        (prof,) = ctx.saved_tensors
        return None, None, ctx.jctx.beta_logistic_vjp(ctx.geom_idx, prof,
                                                      gbeta.contiguous().to(torch.float64))


def beta_logistic(jctx: binding.Context, geom_idx, prof):
    """Differentiable packed beta_k of logistic anisotropy profiles
    prof [n, 4] = (beta_0, beta_inf, r_a, alpha), one per model."""
    return BetaLogistic.apply(jctx, geom_idx, prof)
