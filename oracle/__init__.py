"""CPU oracle for point-cloud radio ray tracing (FP64, brute force).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports, links or calls it, and the two share no code: the only thing both
sides consume is the seeded input generators' output.

The C source (pcrt_oracle.c) states the method step by step; this module only
builds it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcrt_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

LOS, SPECULAR, DIFFUSE, TRACE, AVERAGE, DPS_LAUNCH, POLARIZED = 1, 2, 4, 8, 16, 32, 64
DEFAULT_THR = dict(eps_tie=1e-4, eps_self=1e-3, t_a_deg=1.0, t_d=0.01, kappa=10)
C0 = 299792458.0


def build(force: bool = True) -> str:
    """Compile the oracle into liborc.so (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _radius(scene):
    """The disk radius as the FP32 value both implementations read."""
    return ctypes.c_double(float(np.float32(scene.radius)))


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(shape) if shape is not None else a


def fib_dirs(n_budget: int, ids=None) -> np.ndarray:
    ids = np.arange(n_budget, dtype=np.int64) if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    out = np.empty((ids.size, 3), np.float32)
    L = _load()
    L.orc_fib_dirs(ctypes.c_int64(n_budget), _p(ids), ctypes.c_int64(ids.size), _p(out))
    return out


def fresnel(eps_r: float, sigma: float, freq: float, cosv):
    """Returns (Gamma_TE, Gamma_TM, dGamma_TE/deta, dGamma_TM/deta) as complex arrays."""
    c = np.ascontiguousarray(np.atleast_1d(cosv), dtype=np.float64)
    out = np.empty((c.size, 8), np.float64)
    _load().orc_fresnel(ctypes.c_double(eps_r), ctypes.c_double(sigma), ctypes.c_double(freq),
                        ctypes.c_int64(c.size), _p(c), _p(out))
    z = out[:, 0::2] + 1j * out[:, 1::2]
    return z[:, 0], z[:, 1], z[:, 2], z[:, 3]


def nearest(scene, o, d, excl=None, t_lo=1e-3, t_hi=np.inf, eps_tie=1e-4):
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    n = o.shape[0]
    excl = np.full(n, -1, np.int64) if excl is None else np.ascontiguousarray(excl, np.int64)
    oid = np.empty(n, np.int64)
    ot = np.empty(n, np.float64)
    oq = np.empty((n, 3), np.float64)
    rc = _load().orc_nearest_batch(ctypes.c_int64(scene.n), _p(scene.pos), _p(scene.normal),
                                   _radius(scene), ctypes.c_int64(n), _p(o), _p(d), _p(excl),
                                   ctypes.c_double(t_lo), ctypes.c_double(t_hi), ctypes.c_double(eps_tie),
                                   _p(oid), _p(ot), _p(oq))
    if rc:
        raise ValueError("oracle nearest: bad scene (%d)" % rc)
    return oid, ot, oq


def average(scene, o, d, rho, lambda_d, excl=None, eps_self=1e-3, eps_tie=1e-4):
    """Nearest disk, then the weighted average over its point set (voxel edge rho).
    Returns (id int64[n], t float64[n], normal float64[n, 3] facing the ray)."""
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    n = o.shape[0]
    excl = np.full(n, -1, np.int64) if excl is None else np.ascontiguousarray(excl, np.int64)
    oid = np.empty(n, np.int64)
    ot = np.empty(n, np.float64)
    on = np.empty((n, 3), np.float64)
    rc = _load().orc_average_batch(ctypes.c_int64(scene.n), _p(scene.pos), _p(scene.normal), _radius(scene),
                                   ctypes.c_double(float(np.float32(rho))), ctypes.c_double(lambda_d),
                                   ctypes.c_int64(n), _p(o), _p(d), _p(excl), ctypes.c_double(eps_self),
                                   ctypes.c_double(eps_tie), _p(oid), _p(ot), _p(on))
    if rc:
        raise ValueError("oracle average: bad scene (%d)" % rc)
    return oid, ot, on


def visibility(scene, rho, rx, eps_self=1e-3):
    """Point sets of voxel edge rho: (reception points float32[n_sets, 3],
    visibility uint8[n_rx, n_sets] from the receivers rx)."""
    rx = _f32(rx).reshape(-1, 3)
    L = _load()
    ns = ctypes.c_int64(0)
    args = (ctypes.c_int64(scene.n), _p(scene.pos), _p(scene.normal), _radius(scene),
            ctypes.c_double(float(np.float32(rho))), ctypes.c_int32(rx.shape[0]), _p(rx), ctypes.c_double(eps_self),
            ctypes.byref(ns))
    if L.orc_visibility(*args, None, None):
        raise ValueError("oracle visibility: bad scene")
    recv = np.empty((ns.value, 3), np.float32)
    vis = np.empty((rx.shape[0], ns.value), np.uint8)
    if L.orc_visibility(*args, _p(recv), _p(vis)):
        raise ValueError("oracle visibility: bad scene")
    return recv, vis


def occluded(scene, a, b, excl=None, eps_self=1e-3):
    a = np.ascontiguousarray(a, np.float64).reshape(-1, 3)
    b = np.ascontiguousarray(b, np.float64).reshape(-1, 3)
    n = a.shape[0]
    excl = np.full(n, -1, np.int64) if excl is None else np.ascontiguousarray(excl, np.int64)
    out = np.empty(n, np.uint8)
    rc = _load().orc_occluded_batch(ctypes.c_int64(scene.n), _p(scene.pos), _p(scene.normal),
                                    _radius(scene), ctypes.c_int64(n), _p(a), _p(b), _p(excl),
                                    ctypes.c_double(eps_self), _p(out))
    if rc:
        raise ValueError("oracle occluded: bad scene (%d)" % rc)
    return out.astype(bool)


@dataclass
class Solution:
    seq: np.ndarray          # int64[n_trace, K]
    rec: np.ndarray          # float64[n_trace, K, 5]: x, y, z, L, cos
    dvis: np.ndarray | None  # bool[n_trace, K, n_rx]
    keys: list               # list of tuples of surface labels
    key_rep: np.ndarray      # int64[n_keys]
    spec_valid: np.ndarray   # bool[n_keys, n_rx]
    spec_len: np.ndarray     # float64[n_keys, n_rx]
    spec_amp: np.ndarray     # complex128[n_keys, n_rx, 2] (TE, TM)
    spec_hid: np.ndarray     # int64[n_keys, n_rx, K]
    G_los: np.ndarray
    G_spec: np.ndarray
    G_diff: np.ndarray
    G: np.ndarray
    h_te: np.ndarray
    h_tm: np.ndarray
    jac: np.ndarray | None   # float64[n_rx, n_labels, 3]: dG/d(eps_r, sigma, S)
    cfr: np.ndarray | None = None  # complex128[n_rx, n_freq, 2]: channel frequency response (TE, TM)
    dpow: np.ndarray | None = None  # float64[n_trace, K, n_rx]: lit connections' power, occluded or not

    def paths(self, r: int):
        """{key: (length, a_TE, a_TM)} of the valid specular paths at receiver r."""
        out = {}
        for i, k in enumerate(self.keys):
            if self.spec_valid[i, r]:
                out[k] = (self.spec_len[i, r], self.spec_amp[i, r, 0], self.spec_amp[i, r, 1])
        return out


def solve(scene, mats, tx, rx, freq, n_budget, ray_ids=None, K=2, flags=LOS | SPECULAR,
          thr=None, want_dvis=False, want_jac=False, cfr=None, average=None, dps_launch=None,
          want_dpow=False, pol=None) -> Solution:
    """Full FP64 solve for one transmitter. mats: float64[n_labels, 3] (eps_r, sigma, S).

    average = (rho, lambda_d): every interaction is the weighted average over
    the intersected disks of the hit disk's point set (voxels of edge rho).

    dps_launch = rho: ray j goes from the transmitter towards the reception
    point of point set j (ray_ids are set indices, n_budget the set count),
    and a (key, receiver) pair is a specular candidate only where the
    receiver sees the reception point of the set its representative ends in.
    Diffuse paths are then one per unique (labels before the last interaction,
    point set of the last), gated the same way, each standing for an area
    rho^2 around its representative's interaction.

    cfr = (bandwidth_hz, n_freq): also the channel frequency response, every
    path's centre-frequency amplitudes times exp(-j 2 pi (f_n - freq) L / c0)
    at n_freq equally spaced frequencies f_n spanning bandwidth_hz around freq.

    pol = (pol_tx, pol_rx): the polarised (Jones-vector) field of line-of-sight
    and specular paths for these transmit and receive polarisation vectors;
    every path's one complex amplitude is reported in both channels (no
    diffuse paths, Jacobian or frequency response in this mode)."""
    th = dict(DEFAULT_THR)
    if thr:
        th.update(thr)
    rho, lam = (float(np.float32(average[0])), float(average[1])) if average else (0.0, 0.0)
    if average:
        flags |= AVERAGE
    if dps_launch:
        if average and float(np.float32(dps_launch)) != rho:
            raise ValueError("one voxel edge for averaging and launch")
        rho = float(np.float32(dps_launch))
        flags |= DPS_LAUNCH
    ptx, prx = (np.asarray(pol[0], np.float64), np.asarray(pol[1], np.float64)) if pol else (np.zeros(3), np.zeros(3))
    if pol:
        flags |= POLARIZED
    thr_arr = np.array([th["eps_tie"], th["eps_self"], th["t_a_deg"], th["t_d"], th["kappa"], rho, lam,
                        *ptx, *prx], np.float64)
    mats = np.ascontiguousarray(mats, np.float64).reshape(-1, 3)
    n_labels = mats.shape[0]
    eps_r = np.ascontiguousarray(mats[:, 0])
    sig = np.ascontiguousarray(mats[:, 1])
    sca = np.ascontiguousarray(mats[:, 2])
    tx = _f32(tx, (3,))
    rx = _f32(rx).reshape(-1, 3)
    n_rx = rx.shape[0]
    ids = np.arange(n_budget, dtype=np.int64) if ray_ids is None else np.ascontiguousarray(ray_ids, np.int64)
    nt = ids.size
    seq = np.empty((nt, K), np.int64)
    rec = np.empty((nt, K, 5), np.float64)
    dvis = np.empty((nt, K, n_rx), np.uint8) if want_dvis else None
    dpow = np.zeros((nt, K, n_rx), np.float64) if want_dpow else None
    cap = max(1, nt * K) if flags & SPECULAR else 1
    keys = np.empty((cap, K), np.uint32)
    klen = np.empty(cap, np.int32)
    krep = np.empty(cap, np.int64)
    nk = ctypes.c_int64(0)
    sv = np.empty((cap, n_rx), np.uint8)
    sl = np.empty((cap, n_rx), np.float64)
    sa = np.empty((cap, n_rx, 4), np.float64)
    sh = np.empty((cap, n_rx, K), np.int64)
    orx = np.empty((n_rx, 8), np.float64)
    jac = np.empty((n_rx, n_labels, 3), np.float64) if want_jac else None
    n_freq, bw = (int(cfr[1]), float(cfr[0])) if cfr else (0, 0.0)
    ocfr = np.empty((n_rx, max(n_freq, 1), 4), np.float64) if cfr else None
    rc = _load().orc_solve(
        ctypes.c_int64(scene.n), _p(scene.pos), _p(scene.normal), _p(scene.material), _p(scene.surface),
        _radius(scene), ctypes.c_int32(n_labels), _p(eps_r), _p(sig), _p(sca),
        _p(tx), ctypes.c_int32(n_rx), _p(rx), ctypes.c_double(freq), ctypes.c_int64(n_budget),
        ctypes.c_int64(nt), _p(ids), ctypes.c_int32(K), ctypes.c_int32(flags), _p(thr_arr),
        _p(seq), _p(rec), _p(dvis), _p(dpow), ctypes.c_int64(cap), _p(keys), _p(klen), _p(krep), ctypes.byref(nk),
        _p(sv), _p(sl), _p(sa), _p(sh), _p(orx), _p(jac), ctypes.c_int32(n_freq), ctypes.c_double(bw),
        _p(ocfr))
    if rc:
        raise ValueError("oracle solve failed (%d)" % rc)
    n = nk.value
    key_list = [tuple(int(x) for x in keys[i, :klen[i]]) for i in range(n)]
    amp = sa[:n, :, 0::2] + 1j * sa[:n, :, 1::2]
    return Solution(seq, rec, dvis.astype(bool) if dvis is not None else None, key_list, krep[:n].copy(),
                    sv[:n].astype(bool), sl[:n].copy(), amp, sh[:n].copy(), orx[:, 0].copy(), orx[:, 1].copy(),
                    orx[:, 2].copy(), orx[:, 3].copy(), orx[:, 4] + 1j * orx[:, 5], orx[:, 6] + 1j * orx[:, 7],
                    jac, (ocfr[..., 0::2] + 1j * ocfr[..., 1::2]) if cfr else None, dpow)


def trace(scene, tx, n_budget, ray_ids=None, K=2, thr=None, average=None):
    """Interaction sequences (int64[n, K]) and records (x, y, z, L, cos) only."""
    n_labels = int(np.max(scene.material)) + 1
    sol = solve(scene, np.ones((n_labels, 3)), tx, np.zeros((0, 3), np.float32), 1e9, n_budget, ray_ids=ray_ids,
                K=K, flags=TRACE, thr=thr, average=average)
    return sol.seq, sol.rec


def wavelength(freq: float) -> float:
    return C0 / freq
