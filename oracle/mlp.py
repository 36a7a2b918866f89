"""Reference for the learned material model (TEST INFRASTRUCTURE ONLY).

Only tests, smoke() and bench.py's CPU-baseline leg may import this module.

The model maps an interaction's (material label, incidence cosine, carrier
frequency) to its complex TE/TM reflection coefficients and its scattering
coefficient, replacing the per-label Fresnel model of the field computation:

    x  = [emb[label] (16), cos theta, log10(f / 1 GHz), 0 ... 0]   (32 wide)
    h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), h3 = GELU(W3 h2 + b3)   (64 wide)
    z  = W4 h3 + b4                                                   (5 used of 16)
    Gamma_TE = (z0 + j z1) tanh|.|/|.|,  Gamma_TM = (z2 + j z3) tanh|.|/|.|,
    S = sigmoid(z4)

GELU is the exact form x Phi(x). The tanh-radial map keeps |Gamma| < 1
(a passive surface); the sigmoid keeps S in (0, 1).

precision="fp64": every step in float64 (pinned against torch autograd and
finite differences). precision="kernel": the GPU kernels' rounding points --
inputs, weights and hidden activations (and, in the backward pass, the
pre-activation gradients) rounded to bfloat16, products accumulated in
float32 -- so that both sides take the same quantisation decisions.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID, N_OUT_PAD, N_EMB = 32, 64, 16, 16


def bf16(x):
    """Round float32 values to bfloat16 (nearest even) and back to float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(a), out, a)


def init_params(n_labels: int, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)

    def lin(o, i, fan_in):
        return rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=(o, i))
    W1 = np.zeros((N_HID, N_IN))
    W1[:, :N_EMB + 2] = lin(N_HID, N_EMB + 2, N_EMB + 2)
    W4 = np.zeros((N_OUT_PAD, N_HID))
    W4[:5] = lin(5, N_HID, N_HID) * 0.5
    return dict(emb=rng.normal(0.0, 0.5, size=(n_labels, N_EMB)), W1=W1, b1=np.zeros(N_HID),
                W2=lin(N_HID, N_HID, N_HID), b2=np.zeros(N_HID), W3=lin(N_HID, N_HID, N_HID), b3=np.zeros(N_HID),
                W4=W4, b4=np.zeros(N_OUT_PAD))


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def features(params, labels, cosv, freq):
    n = len(labels)
    x = np.zeros((n, N_IN))
    x[:, :N_EMB] = params["emb"][labels]
    x[:, N_EMB] = cosv
    x[:, N_EMB + 1] = math.log10(freq / 1e9)
    return x


def _radial(u, v):
    """(u + j v) tanh(r)/r and its partial derivatives."""
    r = np.sqrt(u * u + v * v)
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    g = np.where(small, 1.0 - r * r / 3.0, np.tanh(rs) / rs)
    # g'(r)/r = (r sech^2 r - tanh r) / r^3, series -2/3 near 0
    sech2 = 1.0 / np.cosh(rs) ** 2
    gp_over_r = np.where(small, -2.0 / 3.0, (rs * sech2 - np.tanh(rs)) / rs ** 3)
    re, im = u * g, v * g
    # d re/du = g + u^2 g'/r, d re/dv = u v g'/r, d im/du = u v g'/r, d im/dv = g + v^2 g'/r
    return re, im, (g + u * u * gp_over_r, u * v * gp_over_r, u * v * gp_over_r, g + v * v * gp_over_r)


def forward(params, labels, cosv, freq, precision="fp64", keep=False):
    """Returns out[n, 5] = (Gamma_TE re, im, Gamma_TM re, im, S) (and the cache)."""
    kern = precision == "kernel"
    rq = (lambda a: bf16(a).astype(np.float64)) if kern else (lambda a: a)
    acc = (lambda a, b: (a.astype(np.float32) @ b.astype(np.float32)).astype(np.float64)) if kern else np.matmul
    x = rq(features(params, labels, cosv, freq))
    W = [rq(params[k]) for k in ("W1", "W2", "W3", "W4")]
    b = [params[k] for k in ("b1", "b2", "b3", "b4")]
    hs, zs = [x], []
    h = x
    for i in range(3):
        z = acc(h, W[i].T) + b[i]
        zs.append(z)
        h = rq(gelu(z))
        hs.append(h)
    z4 = acc(h, W[3].T) + b[3]
    te_re, te_im, dte = _radial(z4[:, 0], z4[:, 1])
    tm_re, tm_im, dtm = _radial(z4[:, 2], z4[:, 3])
    S = 1.0 / (1.0 + np.exp(-z4[:, 4]))
    out = np.stack([te_re, te_im, tm_re, tm_im, S], 1)
    if keep:
        return out, dict(hs=hs, zs=zs, z4=z4, W=W, dte=dte, dtm=dtm, S=S, labels=np.asarray(labels))
    return out


def backward(params, labels, cosv, freq, g_out, precision="fp64", magnitudes=False):
    """Gradients of sum(g_out * out) with respect to every parameter.

    magnitudes=True also returns, per gradient element, the sum of the
    absolute values of the terms it adds up (|dz|^T |h| for a weight, sum
    |dz| for a bias, the rows' sum |dz| |W| for an embedding entry): the
    scale against which rounding differences of those terms are judged."""
    kern = precision == "kernel"
    rq = (lambda a: bf16(a).astype(np.float64)) if kern else (lambda a: a)
    acc = (lambda a, b: (a.astype(np.float32) @ b.astype(np.float32)).astype(np.float64)) if kern else np.matmul
    _, c = forward(params, labels, cosv, freq, precision, keep=True)
    g = np.asarray(g_out, np.float64)
    dz4 = np.zeros((len(labels), N_OUT_PAD))
    a, bb, cc, d = c["dte"]
    dz4[:, 0] = g[:, 0] * a + g[:, 1] * cc
    dz4[:, 1] = g[:, 0] * bb + g[:, 1] * d
    a, bb, cc, d = c["dtm"]
    dz4[:, 2] = g[:, 2] * a + g[:, 3] * cc
    dz4[:, 3] = g[:, 2] * bb + g[:, 3] * d
    dz4[:, 4] = g[:, 4] * c["S"] * (1.0 - c["S"])
    grads, mags = {}, {}
    dz = rq(dz4)
    W, hs, zs = c["W"], c["hs"], c["zs"]
    for i in (3, 2, 1, 0):
        grads["W%d" % (i + 1)] = acc(dz.T, hs[i])
        grads["b%d" % (i + 1)] = dz.sum(0)
        if magnitudes:
            mags["W%d" % (i + 1)] = np.abs(dz).T @ np.abs(hs[i])
            mags["b%d" % (i + 1)] = np.abs(dz).sum(0)
        dh = acc(dz, W[i])
        if i == 0:
            if magnitudes:
                memb = np.zeros_like(params["emb"])
                np.add.at(memb, c["labels"], (np.abs(dz) @ np.abs(W[0]))[:, :N_EMB])
                mags["emb"] = memb
            break
        dz = rq(dh * gelu_grad(zs[i - 1]))
    demb = np.zeros_like(params["emb"])
    np.add.at(demb, c["labels"], dh[:, :N_EMB])
    grads["emb"] = demb
    grads["W1"][:, N_EMB + 2:] = 0.0
    grads["W4"][5:] = 0.0
    grads["b4"][5:] = 0.0
    return (grads, mags) if magnitudes else grads
