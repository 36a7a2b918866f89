"""Single-bounce edge diffraction, FP64 reference (numpy + scipy's Fresnel integrals).

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU leg may use
it; the GPU library never does, and the two share no code.

The paper computes a diffracted path per edge by minimising the path length
on the edge and checking that the edge point sees both ends (Sec. II-B.3); its
field comes from the EM back end. The field here is the uniform geometrical
theory of diffraction for a wedge (Kouyoumjian and Pathak, Proc. IEEE 1974),
with the face reflection coefficients of Luebbers (IEEE Trans. AP 1984) in the
two reflection terms for lossy faces. Notation: the edge unit vector e, face 0
and face n of the wedge, the exterior angle n*pi, angles phi measured from
face 0 through the exterior in the plane normal to the edge, phi' of the
source and phi of the observer, beta0 the angle between the incident ray and
the edge, s' and s the distances from the edge point to source and observer.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import fresnel as _fresnel

from . import C0, occluded, fresnel as _fresnel_coef


def transition(x):
    """F(x) = 2j sqrt(x) e^{jx} int_{sqrt(x)}^inf e^{-j t^2} dt, x >= 0."""
    x = np.asarray(x, np.float64)
    z = np.sqrt(2.0 * x / np.pi)
    S, C = _fresnel(z)
    tail = np.sqrt(np.pi / 2.0) * ((0.5 - C) - 1j * (0.5 - S))
    return 2j * np.sqrt(x) * np.exp(1j * x) * tail


def _a(beta, n, sign):
    """a^{+-}(beta) = 2 cos^2((2 n pi N - beta) / 2), N the integer nearest to
    satisfying 2 pi n N - beta = +-pi."""
    N = np.round((beta + sign * np.pi) / (2.0 * np.pi * n))
    return 2.0 * np.cos((2.0 * n * np.pi * N - beta) / 2.0) ** 2, N


def _term(beta, n, kL, sign):
    """cot((pi + sign beta) / (2n)) F(kL a^{sign}(beta)), with its finite limit
    at the shadow and reflection boundaries (where the cotangent's pole and the
    zero of F meet)."""
    a, N = _a(beta, n, sign)
    eps = np.pi + sign * beta - 2.0 * np.pi * n * N
    if abs(eps) < 1e-9:
        return n * (math.sqrt(2.0 * np.pi * kL) * np.sign(eps) - 2.0 * kL * eps * np.exp(1j * np.pi / 4.0)) * \
            np.exp(1j * np.pi / 4.0)
    return (1.0 / np.tan((np.pi + sign * beta) / (2.0 * n))) * transition(kL * a)


def coefficient(n, k, L, phi, phip, sin_b0, r0, rn):
    """Wedge diffraction coefficient with face reflection coefficients r0
    (face 0, taken at grazing angle phi') and rn (face n, at n pi - phi):
    r0 = rn = -1 gives the soft (Dirichlet) and +1 the hard (Neumann)
    coefficient of a perfectly conducting wedge."""
    kL = k * L
    bm, bp = phi - phip, phi + phip
    s = (_term(bm, n, kL, +1) + _term(bm, n, kL, -1)
         + r0 * _term(bp, n, kL, -1) + rn * _term(bp, n, kL, +1))
    return -np.exp(-1j * np.pi / 4.0) / (2.0 * n * math.sqrt(2.0 * np.pi * k) * sin_b0) * s


def edge_point(a, b, p, q):
    """The point of segment ab that minimises |p - D| + |D - q| (straight line
    of the two points' distances unfolded about the edge), as a fraction t."""
    a, b, p, q = (np.asarray(v, np.float64) for v in (a, b, p, q))
    ev = b - a
    l2 = ev @ ev
    tp, tq = (p - a) @ ev / l2, (q - a) @ ev / l2
    dp = np.linalg.norm(p - (a + tp * ev))
    dq = np.linalg.norm(q - (a + tq * ev))
    if dp + dq == 0.0:
        return None
    return tp + (tq - tp) * dp / (dp + dq)


def wedge_frame(e, n0, n1):
    """In-face unit vectors t0, t1 (perpendicular to the edge, pointing into
    each face) and the exterior angle factor n."""
    t0 = np.cross(n0, e)
    t0 /= np.linalg.norm(t0)
    if t0 @ n1 > 0:
        t0 = -t0
    t1 = np.cross(n1, e)
    t1 /= np.linalg.norm(t1)
    if t1 @ n0 > 0:
        t1 = -t1
    alpha = math.acos(max(-1.0, min(1.0, float(t0 @ t1))))
    return t0, t1, (2.0 * np.pi - alpha) / np.pi


def angle(v, e, t0, n0):
    """Angle of direction v about the edge from face 0 through the exterior, in [0, 2 pi)."""
    w = v - (v @ e) * e
    ph = math.atan2(float(w @ n0), float(w @ t0))
    return ph + 2.0 * np.pi if ph < 0 else ph


def diffraction(scene, edges, mats, tx, rx, freq, eps_self=1e-3, trim=None):
    """Per receiver: (G, h_te, h_tm) of the single-bounce diffracted paths over
    all edges, summed in edge order, and the per-(receiver, edge) amplitudes
    (complex [n_rx, n_edges, 2], 0 where there is no path).

    edges: float [n_edges, 12] rows (a xyz, b xyz, n0 xyz, n1 xyz) with outward
    face normals, plus int labels [n_edges, 2] in mats' rows (face 0, face n):
    pass (rows, labels). trim: length cut from the edge end of both visibility
    segments (default twice the disk radius: the faces' own disks meet there)."""
    rows, labels = edges
    rows = np.asarray(rows, np.float64).reshape(-1, 12)
    labels = np.asarray(labels, np.int64).reshape(-1, 2)
    mats = np.asarray(mats, np.float64).reshape(-1, 3)
    tx = np.asarray(tx, np.float32).astype(np.float64)
    rx = np.asarray(rx, np.float32).astype(np.float64).reshape(-1, 3)
    k = 2.0 * np.pi * freq / C0
    lam = C0 / freq
    trim = 2.0 * float(np.float32(scene.radius)) if trim is None else trim
    amp = np.zeros((len(rx), len(rows), 2), np.complex128)
    for i, row in enumerate(rows):
        a, b, n0, n1 = row[0:3], row[3:6], row[6:9], row[9:12]
        n0, n1 = n0 / np.linalg.norm(n0), n1 / np.linalg.norm(n1)
        e = (b - a) / np.linalg.norm(b - a)
        t0, _, n = wedge_frame(e, n0, n1)
        for r, q in enumerate(rx):
            t = edge_point(a, b, tx, q)
            if t is None or not (0.0 < t < 1.0):
                continue
            D = a + t * (b - a)
            sp, s = np.linalg.norm(tx - D), np.linalg.norm(q - D)
            phip, phi = angle(tx - D, e, t0, n0), angle(q - D, e, t0, n0)
            if not (0.0 < phip < n * np.pi and 0.0 < phi < n * np.pi):
                continue
            # both ends see the edge point (segments cut short by trim at the edge)
            ui, uo = (tx - D) / sp, (q - D) / s
            if occluded(scene, tx, D + trim * ui, eps_self=eps_self)[0]:
                continue
            if occluded(scene, q, D + trim * uo, eps_self=eps_self)[0]:
                continue
            sin_b0 = np.linalg.norm(np.cross(ui, e))
            L = s * sp * sin_b0 ** 2 / (s + sp)
            m0, mn = mats[labels[i, 0]], mats[labels[i, 1]]
            g0te, g0tm, _, _ = _fresnel_coef(m0[0], m0[1], freq, [math.sin(phip)])
            gnte, gntm, _, _ = _fresnel_coef(mn[0], mn[1], freq, [math.sin(n * np.pi - phi)])
            d_te = coefficient(n, k, L, phi, phip, sin_b0, g0te[0], gnte[0])
            d_tm = coefficient(n, k, L, phi, phip, sin_b0, g0tm[0], gntm[0])
            base = lam / (4.0 * np.pi) / sp * math.sqrt(sp / (s * (s + sp))) * np.exp(-1j * k * (sp + s))
            amp[r, i, 0] = base * d_te
            amp[r, i, 1] = base * d_tm
    G = np.zeros(len(rx))
    h_te = np.zeros(len(rx), np.complex128)
    h_tm = np.zeros(len(rx), np.complex128)
    for r in range(len(rx)):
        for i in range(len(rows)):
            a_te, a_tm = amp[r, i]
            G[r] += 0.5 * (abs(a_te) ** 2 + abs(a_tm) ** 2)
            h_te[r] += a_te
            h_tm[r] += a_tm
    return G, h_te, h_tm, amp
