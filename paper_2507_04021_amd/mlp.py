"""Learned material model on the GPU: parameters, kernel calls, training.

The network (declared in include/pcrt.h) maps each interaction slot's
(material label, incidence cosine, log10 frequency) to (Gamma_TE, Gamma_TM, S).
Its forward and backward passes are the library's BF16 MFMA kernels; this
module keeps FP32 master parameters in torch (plumbing for the optimiser),
packs them for the kernels, and wires them to the recorded tapes:

    tape slots -> MLP forward -> coefficient rows -> tape forward -> G
    dL/dG -> tape backward -> adjoint rows -> MLP backward -> parameter grads
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import Mlp, _check, _ptr, _stream, lib, tape, tape_backward, tape_forward

N_IN, N_HID, N_OUT, N_EMB = 32, 64, 16, 16
SHAPES = dict(W1=(N_HID, N_IN), W2=(N_HID, N_HID), W3=(N_HID, N_HID), W4=(N_OUT, N_HID))
BIAS = dict(b1=N_HID, b2=N_HID, b3=N_HID, b4=N_OUT)


def init_params(n_labels: int, seed: int = 0) -> dict:
    """Seeded initial parameters (float64 numpy). W1 columns 18.. and W4 rows
    5.. are structural zeros (padding) and stay zero under training."""
    rng = np.random.default_rng(seed)

    def lin(o, i, fan_in):
        return rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=(o, i))
    W1 = np.zeros((N_HID, N_IN))
    W1[:, :N_EMB + 2] = lin(N_HID, N_EMB + 2, N_EMB + 2)
    W4 = np.zeros((N_OUT, N_HID))
    W4[:5] = lin(5, N_HID, N_HID) * 0.5
    return dict(emb=rng.normal(0.0, 0.5, size=(n_labels, N_EMB)), W1=W1, b1=np.zeros(N_HID),
                W2=lin(N_HID, N_HID, N_HID), b2=np.zeros(N_HID), W3=lin(N_HID, N_HID, N_HID), b3=np.zeros(N_HID),
                W4=W4, b4=np.zeros(N_OUT))


class MaterialMLP:
    def __init__(self, params: dict, device="cuda"):
        self.device = torch.device(device)
        self.p = {k: torch.tensor(np.asarray(v), dtype=torch.float32, device=self.device) for k, v in params.items()}
        self.n_labels = self.p["emb"].shape[0]
        self._ws = None
        self.pack()

    def pack(self):
        """bf16 weight bits and fp32 biases in the kernels' packed layout."""
        w = torch.cat([self.p[k].reshape(-1) for k in ("W1", "W2", "W3", "W4")])
        self.w_bits = w.to(torch.bfloat16).view(torch.int16).contiguous()
        self.b_all = torch.cat([self.p[k] for k in ("b1", "b2", "b3", "b4")]).contiguous()
        self.emb = self.p["emb"].contiguous()
        self.net = Mlp(self.w_bits.data_ptr(), self.b_all.data_ptr(), self.emb.data_ptr(), self.n_labels)

    def forward_rows(self, label, cosv, freq, out):
        """out[n, 8] (tape coefficient rows) for int16 labels and float cosines."""
        L = lib()
        n = label.numel()
        _check(L.pcrt_mlp_forward(ctypes.byref(self.net), n, _ptr(label), _ptr(cosv),
                                  ctypes.c_float(math.log10(freq / 1e9)), _ptr(out), _stream()), L)
        return out

    def backward_rows(self, label, cosv, freq, g_out):
        """Parameter gradients (dict of float32 tensors) of sum(g_out . out)."""
        L = lib()
        n = label.numel()
        nb = ctypes.c_size_t(0)
        _check(L.pcrt_mlp_workspace_size(n, self.n_labels, ctypes.byref(nb)), L)
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        gw = torch.empty(sum(a * b for a, b in SHAPES.values()), dtype=torch.float32, device=self.device)
        gb = torch.empty(sum(BIAS.values()), dtype=torch.float32, device=self.device)
        ge = torch.empty(self.n_labels, N_EMB, dtype=torch.float32, device=self.device)
        _check(L.pcrt_mlp_backward(ctypes.byref(self.net), n, _ptr(label), _ptr(cosv),
                                   ctypes.c_float(math.log10(freq / 1e9)), _ptr(g_out), _ptr(self._ws),
                                   self._ws.numel(), _ptr(gw), _ptr(gb), _ptr(ge), _stream()), L)
        out, o = {"emb": ge}, 0
        for k, (a, b) in SHAPES.items():
            out[k] = gw[o:o + a * b].reshape(a, b)
            o += a * b
        o = 0
        for k, m in BIAS.items():
            out[k] = gb[o:o + m]
            o += m
        return out

    def gains(self, rec, freq):
        """Per-receiver gains of a recorded tape with the network's coefficients."""
        t = tape(rec)
        self.forward_rows(t["label"], t["cos"], freq, t["coef"])
        return tape_forward(rec)[0]

    def loss_and_grads(self, rec, freq, target_db):
        """dB MSE of one recorded channel set and its parameter gradients."""
        t = tape(rec)
        self.forward_rows(t["label"], t["cos"], freq, t["coef"])
        g = tape_forward(rec)[0].detach().requires_grad_(True)
        loss = torch.mean((10.0 * torch.log10(g) - target_db) ** 2)
        (dl_dg,) = torch.autograd.grad(loss, g)
        tape_backward(rec, dl_dg)
        return loss.detach(), self.backward_rows(t["label"], t["cos"], freq, t["adj"])


def train(mlp: MaterialMLP, sets, iters=300, batch=16, lr=3e-3, seed=0, log_every=0):
    """Adam on the dB MSE over channel sets [(rec, freq, target_db)]."""
    params = [mlp.p[k] for k in mlp.p]
    for q in params:
        q.requires_grad_(False)
    opt = torch.optim.Adam(params, lr=lr)
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        idx = rng.choice(len(sets), size=min(batch, len(sets)), replace=False)
        acc = {k: torch.zeros_like(v) for k, v in mlp.p.items()}
        tot = torch.zeros((), dtype=torch.float64, device=mlp.device)  # read once per iteration: no sync per set
        for i in idx:
            rec, f, tgt = sets[i]
            loss, g = mlp.loss_and_grads(rec, f, tgt)
            tot += loss
            for k in acc:
                acc[k] += g[k]
        for k, v in mlp.p.items():
            v.grad = acc[k] / len(idx)
        opt.step()
        mlp.pack()
        hist.append(float(tot) / len(idx))
        if log_every and it % log_every == 0:
            print("iter %d loss %.4f" % (it, hist[-1]), flush=True)
    return hist


def db_error(g, target_db):
    return torch.abs(10.0 * torch.log10(g) - target_db)
