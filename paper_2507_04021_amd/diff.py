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


def fit_per_label(sets, init, iters=300, batch=8, lr=0.05, seed=0):
    """Per-label Fresnel materials fitted through the recorded tapes: Adam on
    the dB MSE over channel sets [(rec, freq, target_db)], the gradient from
    the adjoint kernels. Parameters are kept in range by eps_r = 1 +
    softplus(u), sigma = exp(v), S = sigmoid(w). Returns float64 [n_labels, 3]
    and the loss history."""
    import numpy as np
    init = torch.as_tensor(init, dtype=torch.float64)
    u0 = torch.log(torch.expm1(torch.clamp(init[:, 0] - 1.0, min=1e-3)))
    v0 = torch.log(torch.clamp(init[:, 1], min=1e-9))
    s0 = torch.clamp(init[:, 2], 1e-4, 1 - 1e-4)
    w0 = torch.log(s0 / (1 - s0))
    raw = torch.stack([u0, v0, w0], 1).to("cuda").requires_grad_(True)
    opt = torch.optim.Adam([raw], lr=lr)
    rng = np.random.default_rng(seed)

    def mats_of(r):
        return torch.stack([1.0 + torch.nn.functional.softplus(r[:, 0]), torch.exp(r[:, 1]),
                            torch.sigmoid(r[:, 2])], 1)
    hist = []
    for _ in range(iters):
        idx = rng.choice(len(sets), size=min(batch, len(sets)), replace=False)
        opt.zero_grad()
        m = mats_of(raw)
        loss = sum(db_mse_loss(gains(m, sets[i][0]), sets[i][2]) for i in idx) / len(idx)
        loss.backward()
        opt.step()
        hist.append(loss.detach())
    return mats_of(raw).detach().cpu().numpy(), [float(h) for h in hist]
