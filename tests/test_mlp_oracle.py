"""Pins for the learned-material reference (oracle/mlp.py): library routines
(torch's bfloat16 conversion, linear layers, exact GELU, autograd), closed
forms of the output map, and finite differences."""
import math

import numpy as np
import torch

from oracle import mlp as R


def _torch_forward(params, labels, cosv, freq):
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in params.items()}
    x = torch.zeros(len(labels), R.N_IN, dtype=torch.float64)
    x = x.index_put((torch.arange(len(labels))[:, None], torch.arange(R.N_EMB)[None, :]),
                    P["emb"][torch.as_tensor(labels)])
    x[:, R.N_EMB] = torch.as_tensor(cosv)
    x[:, R.N_EMB + 1] = math.log10(freq / 1e9)
    h = x
    for i in (1, 2, 3):
        h = torch.nn.functional.gelu(torch.nn.functional.linear(h, P["W%d" % i], P["b%d" % i]), approximate="none")
    z = torch.nn.functional.linear(h, P["W4"], P["b4"])
    outs = []
    for a in (0, 2):
        zc = torch.complex(z[:, a], z[:, a + 1])
        r = torch.abs(zc)
        g = zc * torch.tanh(r) / r
        outs += [g.real, g.imag]
    outs.append(torch.sigmoid(z[:, 4]))
    return torch.stack(outs, 1), P


def _data(n=300, seed=1):
    rng = np.random.default_rng(seed)
    params = R.init_params(6, seed=seed)
    for k in ("b1", "b2", "b3"):
        params[k] = rng.normal(0, 0.2, size=params[k].shape)
    params["b4"][:5] = rng.normal(0, 0.3, size=5)
    labels = rng.integers(0, 6, n)
    cosv = rng.uniform(0.0, 1.0, n)
    return params, labels, cosv


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 20000), rng.normal(0, 1e-3, 20000)]).astype(np.float32)
    # exact ties between two bfloat16 values round to even
    ties = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)], np.float32)
    x = np.concatenate([x, ties])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(R.bf16(x), ref)


def test_forward_matches_library_layers():
    params, labels, cosv = _data()
    for f in (3.5e9, 28e9):
        out = R.forward(params, labels, cosv, f)
        ref, _ = _torch_forward(params, labels, cosv, f)
        assert np.allclose(out, ref.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_output_map_closed_form():
    rng = np.random.default_rng(3)
    u, v = rng.normal(0, 2, 1000), rng.normal(0, 2, 1000)
    re, im, _ = R._radial(u, v)
    z = u + 1j * v
    g = re + 1j * im
    assert np.allclose(np.abs(g), np.tanh(np.abs(z)), rtol=1e-13)
    assert np.allclose(np.angle(g), np.angle(z), atol=1e-12)
    # the small-|z| branch is continuous with the exact one
    re0, im0, d0 = R._radial(np.array([0.99e-4]), np.array([0.0]))
    re1, im1, d1 = R._radial(np.array([1.01e-4]), np.array([0.0]))
    assert abs(d0[0][0] - d1[0][0]) < 1e-6


def test_backward_matches_autograd_and_fd():
    params, labels, cosv = _data(200, seed=4)
    f = 28e9
    g_out = np.random.default_rng(5).normal(size=(200, 5))
    grads = R.backward(params, labels, cosv, f, g_out)
    ref, P = _torch_forward(params, labels, cosv, f)
    (ref * torch.tensor(g_out)).sum().backward()
    for k, v in P.items():
        want = v.grad.numpy().copy()
        if k == "W1":
            want[:, R.N_EMB + 2:] = 0
        if k in ("W4", "b4"):
            want[5:] = 0
        assert np.allclose(grads[k], want, rtol=1e-10, atol=1e-12), k
    # finite differences on a few entries
    for k, idx in (("W2", (3, 7)), ("emb", (2, 5)), ("b3", (11,)), ("W4", (4, 9))):
        h = 1e-6
        pp = {a: b.copy() for a, b in params.items()}
        pn = {a: b.copy() for a, b in params.items()}
        pp[k][idx] += h
        pn[k][idx] -= h
        fd = ((R.forward(pp, labels, cosv, f) - R.forward(pn, labels, cosv, f)) * g_out).sum() / (2 * h)
        assert abs(fd - grads[k][idx]) < 1e-6 * max(1.0, abs(fd))


def test_kernel_precision_is_close_to_fp64():
    params, labels, cosv = _data(500, seed=6)
    a = R.forward(params, labels, cosv, 3.5e9)
    b = R.forward(params, labels, cosv, 3.5e9, precision="kernel")
    assert np.max(np.abs(a - b)) < 3e-2 and np.mean(np.abs(a - b)) < 3e-3
