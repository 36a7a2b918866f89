"""Independent references used by both the oracle pins and the GPU tests.

Maxwell boundary conditions solved as linear systems (Fresnel) and the image
method on the box room's exact planes (specular paths). Neither retypes the
oracle's or the kernels' formulas.
"""
import itertools
import math

import numpy as np

from paper_2507_04021_amd import scenes

C0 = 299792458.0
EPS0 = 8.8541878128e-12

def fresnel_bc(eps_r, sigma, freq, c):
    """Reflection coefficients from the tangential-field boundary conditions.

    Unknowns (reflected, transmitted) for a unit incident wave, solved with a
    generic linear solver. The transmitted normal wavenumber (in units of k0)
    is the root of eta - sin^2 that decays into the medium (Im <= 0 for the
    e^{+j omega t} convention).
    """
    eta = eps_r - 1j * sigma / (2 * math.pi * freq * EPS0)
    kz = np.sqrt(complex(eta - (1 - c * c)))
    if kz.imag > 0 or (kz.imag == 0 and kz.real < 0):
        kz = -kz
    # TE: E_i + E_r = E_t ; (E_i - E_r) c = kz E_t
    A = np.array([[1.0, -1.0], [-c, -kz]], dtype=complex)
    te = np.linalg.solve(A, np.array([-1.0, -c], dtype=complex))[0]
    # TM (H transverse): H_i + H_r = H_t ; (H_i - H_r) c = (kz / eta) H_t
    B = np.array([[1.0, -1.0], [-c, -kz / eta]], dtype=complex)
    tm = np.linalg.solve(B, np.array([-1.0, -c], dtype=complex))[0]
    return te, tm


ROOM = (6.0, 4.0, 3.0)
FACE_PLANE = {0: (0, 0.0), 1: (0, 6.0), 2: (1, 0.0), 3: (1, 4.0), 4: (2, 0.0), 5: (2, 3.0)}
SURF_MAT_FOUR = {0: 0, 1: 0, 2: 0, 3: 0, 4: 2, 5: 0, 6: 1, 7: 3}


def _surface_labels(face, x, margin):
    """Possible surface labels of a point on a face of the box room.

    Returns (labels, inside). A point within `margin` of a window/door border
    can be hit on either side of it (disks overlap the border), so both labels
    are possible there; elsewhere the label is unique.
    """
    ax = FACE_PLANE[face][0]
    others = [a for a in range(3) if a != ax]
    inside = all(0.0 < x[a] < ROOM[a] for a in others)
    labels = {face}
    for sub, spec in ((6, scenes.BOX_WINDOW), (7, scenes.BOX_DOOR)):
        if spec["face"] != face:
            continue
        u, v = x[others[0]], x[others[1]]
        lo_u, hi_u = spec["u"]
        lo_v, hi_v = spec["v"]
        if lo_u <= u <= hi_u and lo_v <= v <= hi_v:
            labels = {sub}
        near = (lo_u - margin <= u <= hi_u + margin and lo_v - margin <= v <= hi_v + margin
                and not (lo_u + margin < u < hi_u - margin and lo_v + margin < v < hi_v - margin))
        # borders on the room's own edges (door sill on the floor) are not label borders
        if near and not (sub == 7 and v < lo_v + margin and lo_u + margin < u < hi_u - margin):
            labels = {face, sub}
    return sorted(labels), inside


def image_method_room(tx, rx, K, mats, freq, margin=0.08):
    """All specular paths of the empty box room by the image method.

    Returns a list of (candidate keys, L, {key: (a_TE, a_TM)}): one entry per
    geometric path; more than one candidate key only where a reflection point
    sits on a window/door border.
    """
    lam = C0 / freq
    k0 = 2 * math.pi / lam
    tx = np.asarray(tx, np.float32).astype(float)  # the FP32 inputs both sides read
    rx = np.asarray(rx, np.float32).astype(float)
    out = []
    for k in range(1, K + 1):
        for faces in itertools.product(range(6), repeat=k):
            if any(faces[i] == faces[i + 1] for i in range(k - 1)):
                continue
            imgs = [tx]
            for f in faces:
                ax, val = FACE_PLANE[f]
                q = imgs[-1].copy()
                q[ax] = 2 * val - q[ax]
                imgs.append(q)
            pts = [None] * (k + 2)
            pts[0], pts[k + 1] = tx, rx
            cur, ok = rx, True
            for m in range(k, 0, -1):
                ax, val = FACE_PLANE[faces[m - 1]]
                seg = imgs[m] - cur
                if seg[ax] == 0:
                    ok = False
                    break
                s = (val - cur[ax]) / seg[ax]
                if not (0 < s < 1):
                    ok = False
                    break
                cur = cur + s * seg
                pts[m] = cur
            if not ok:
                continue
            options, good = [], True
            for m in range(1, k + 1):
                labs, inside = _surface_labels(faces[m - 1], pts[m], margin)
                if not inside:
                    good = False
                    break
                options.append(labs)
            if not good:
                continue
            L = sum(np.linalg.norm(pts[m + 1] - pts[m]) for m in range(k + 1))
            cos_m = []
            for m in range(1, k + 1):
                u = (pts[m] - pts[m - 1]) / np.linalg.norm(pts[m] - pts[m - 1])
                cos_m.append(abs(u[FACE_PLANE[faces[m - 1]][0]]))
            amps = {}
            for key in itertools.product(*options):
                ate = atm = lam / (4 * math.pi) / L * np.exp(-1j * k0 * L)
                for m in range(k):
                    e, s_, S = mats[SURF_MAT_FOUR[key[m]]]
                    te, tm = fresnel_bc(e, s_, freq, cos_m[m])
                    R = math.sqrt(1 - S * S)
                    ate, atm = ate * R * te, atm * R * tm
                amps[key] = (ate, atm)
            out.append((sorted(amps), L, amps))
    return out


