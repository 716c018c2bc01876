"""torch.autograd wrappers: each forward calls a transform of the C ABI, each backward its
hand-written adjoint (also a C ABI call), so gradients of losses built from the transforms run
entirely in the library's kernels.

Conventions: maps are real (REAL) or complex (COMPLEX) tensors, coefficients complex128
[nmaps, L*L].  Gradients follow torch's convention for complex tensors; for a linear map M the
backward is M^H applied to the incoming gradient, with the real inner products of the C ABI
(for REAL maps the coefficient arrays are Hermitian and so are their gradients)."""
from __future__ import annotations

import torch

from . import (FP64, REAL, analysis, analysis_adjoint, mw_forward, mw_forward_adjoint, mw_inverse,
               mw_inverse_adjoint, synthesis, synthesis_adjoint)


class MWForward(torch.autograd.Function):
    """f -> flm, the forward MW transform."""

    @staticmethod
    def forward(ctx, f, L, reality=REAL, precision=FP64):
        ctx.args = (L, reality, precision)
        return mw_forward(f.contiguous(), L, reality, precision)

    @staticmethod
    def backward(ctx, g):
        L, reality, precision = ctx.args
        return mw_forward_adjoint(g.contiguous(), L, reality, precision), None, None, None


class MWInverse(torch.autograd.Function):
    """flm -> f, the inverse MW transform."""

    @staticmethod
    def forward(ctx, flm, L, reality=REAL, precision=FP64):
        ctx.args = (L, reality, precision)
        return mw_inverse(flm.contiguous(), L, reality, precision)

    @staticmethod
    def backward(ctx, g):
        L, reality, precision = ctx.args
        return mw_inverse_adjoint(g.contiguous(), L, reality, precision), None, None, None


class Analysis(torch.autograd.Function):
    """f -> (f_wav, f_scal), the axisymmetric wavelet analysis."""

    @staticmethod
    def forward(ctx, f, L, B, J_min, multires=True, reality=REAL, precision=FP64):
        ctx.args = (L, B, J_min, multires, reality, precision)
        return analysis(f.contiguous(), L, B, J_min, multires, reality, precision)

    @staticmethod
    def backward(ctx, g_wav, g_scal):
        L, B, J_min, multires, reality, precision = ctx.args
        g_f = analysis_adjoint(g_wav.contiguous(), g_scal.contiguous(), L, B, J_min, multires, reality,
                               precision)
        return g_f, None, None, None, None, None, None


class Synthesis(torch.autograd.Function):
    """(f_wav, f_scal) -> f, the axisymmetric wavelet synthesis."""

    @staticmethod
    def forward(ctx, f_wav, f_scal, L, B, J_min, multires=True, reality=REAL, precision=FP64):
        ctx.args = (L, B, J_min, multires, reality, precision)
        return synthesis(f_wav.contiguous(), f_scal.contiguous(), L, B, J_min, multires, reality, precision)

    @staticmethod
    def backward(ctx, g):
        L, B, J_min, multires, reality, precision = ctx.args
        g_wav, g_scal = synthesis_adjoint(g.contiguous(), L, B, J_min, multires, reality, precision)
        return g_wav, g_scal, None, None, None, None, None, None


def mw_forward_ad(f, L, reality=REAL, precision=FP64):
    return MWForward.apply(f, L, reality, precision)


def mw_inverse_ad(flm, L, reality=REAL, precision=FP64):
    return MWInverse.apply(flm, L, reality, precision)


def analysis_ad(f, L, B, J_min, multires=True, reality=REAL, precision=FP64):
    return Analysis.apply(f, L, B, J_min, multires, reality, precision)


def synthesis_ad(f_wav, f_scal, L, B, J_min, multires=True, reality=REAL, precision=FP64):
    return Synthesis.apply(f_wav, f_scal, L, B, J_min, multires, reality, precision)
