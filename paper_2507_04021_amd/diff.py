"""Differentiable gains for material learning (autograd around the HIP tape).

The path geometry of a RECORD solve does not depend on the materials, so it
is traced once and reused: each forward fills the tape's coefficient rows
from per-label (eps_r, sigma, S) and reduces them to per-receiver gains; each
backward runs the adjoint kernel and the per-label reduction. Both run in
the library's kernels; this module only wires them into torch.autograd.
"""
from __future__ import annotations

import torch

from . import (DIFFUSE, LOS, RECORD, SPECULAR, SolveResult, material_grad, materials_tensor, solve,
               tape_backward, tape_cfr, tape_cfr_backward, tape_forward, tape_fresnel)


def record(scene, mats, tx, rx, freq, n_rays, K=2, flags=LOS | SPECULAR | DIFFUSE, **kw) -> SolveResult:
    """Trace once and keep the tape (a RECORD solve). The solve's status word
    is fetched without waiting; the first backward (or tape access) on this
    recording raises PcrtError if it reports dropped keys or paths left off
    the tape."""
    res = solve(scene, mats, tx, rx, freq, n_rays, K=K, flags=flags | RECORD, **kw)
    res.fetch_status()
    return res


class MaterialGain(torch.autograd.Function):
    """G_r(materials) on a recorded tape. Input: (n_labels, 3) tensor of
    (eps_r, sigma, S); output: float64 per-receiver gains."""

    @staticmethod
    def forward(ctx, mats, rec):
        m = tape_fresnel(rec, mats.detach())
        g, _, _, _ = tape_forward(rec)
        ctx.rec = rec
        ctx.mats_dev = m
        ctx.shape = mats.shape
        ctx.dtype = mats.dtype
        ctx.device = mats.device
        return g

    @staticmethod
    def backward(ctx, grad_g):
        # the adjoint reads the tape's coefficient rows, which any later
        # forward on the same recording overwrites: restore this forward's
        ctx.rec.check_status()
        tape_fresnel(ctx.rec, ctx.mats_dev)
        tape_backward(ctx.rec, grad_g.detach())
        gm = material_grad(ctx.rec, ctx.mats_dev)
        return gm.to(device=ctx.device, dtype=ctx.dtype).reshape(ctx.shape), None


def gains(mats: torch.Tensor, rec: SolveResult) -> torch.Tensor:
    return MaterialGain.apply(mats, rec)


def db_mse_loss(g: torch.Tensor, target_db: torch.Tensor) -> torch.Tensor:
    """Mean over receivers of (10 log10 G_r - T_r)^2."""
    return torch.mean((10.0 * torch.log10(g) - target_db) ** 2)


class MaterialCfr(torch.autograd.Function):
    """Channel frequency response H(materials) on a recorded tape: input
    (n_labels, 3) tensor of (eps_r, sigma, S); output complex128
    [n_rx, n_freq, 2] (TE, TM) over bandwidth_hz around the solve's
    frequency."""

    @staticmethod
    def forward(ctx, mats, rec, bandwidth_hz, n_freq):
        m = tape_fresnel(rec, mats.detach())
        h = tape_cfr(rec, bandwidth_hz, n_freq)
        ctx.rec, ctx.mats_dev, ctx.bw, ctx.n = rec, m, bandwidth_hz, n_freq
        ctx.shape, ctx.dtype, ctx.device = mats.shape, mats.dtype, mats.device
        return h

    @staticmethod
    def backward(ctx, grad_h):
        # for a real loss torch hands over dL/dRe + j dL/dIm of each sample;
        # the coefficient rows are restored first, as in MaterialGain.backward
        ctx.rec.check_status()
        tape_fresnel(ctx.rec, ctx.mats_dev)
        tape_cfr_backward(ctx.rec, ctx.bw, ctx.n, grad_h.detach())
        gm = material_grad(ctx.rec, ctx.mats_dev)
        return gm.to(device=ctx.device, dtype=ctx.dtype).reshape(ctx.shape), None, None, None


def cfr(mats: torch.Tensor, rec: SolveResult, bandwidth_hz: float = 1.5e9, n_freq: int = 129) -> torch.Tensor:
    return MaterialCfr.apply(mats, rec, bandwidth_hz, n_freq)


def cir_loss(h: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """|h - h_hat|^2 / |h_hat|^2 (Eq. 5) of the impulse responses, evaluated on
    the frequency samples: the inverse DFT is unitary up to one scale, which
    cancels in the ratio (Parseval), so both polarisations' CFRs give it."""
    return torch.sum(torch.abs(h - target) ** 2) / torch.sum(torch.abs(target) ** 2)
