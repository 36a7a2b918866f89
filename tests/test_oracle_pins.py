"""Pins for the CPU oracle: closed forms, independent derivations, invariants.

Nothing here retypes the oracle's formulas. Each expected value comes from a
different route: Maxwell boundary conditions solved as a linear system
(Fresnel), the image method on the room's exact planes (specular paths),
numerical quadrature (diffuse ray-tube normalisation), hand-built tiny scenes
(nearest-hit rule), symmetry (reciprocity, permutation invariance) and finite
differences (gradient).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2507_04021_amd import scenes

C0 = 299792458.0
EPS0 = 8.8541878128e-12
LOS, SPEC, DIFF = 1, 2, 4


from refs import FACE_PLANE, ROOM, fresnel_bc, image_method_room  # noqa: E402


@pytest.fixture(scope="module")
def room_holefree():
    # 10 cm grid, radius just above spacing/sqrt(2): no gaps between disks
    return scenes.box_room(spacing=0.1, radius=0.0708)


# ------------------------------------------------------------------- Fresnel
@pytest.mark.parametrize("eps_r,sigma,freq", [(5.0, 0.1, 3.5e9), (2.0, 0.01, 3.5e9), (6.3, 0.3, 28e9),
                                              (1.0, 1e7, 3.5e9), (3.0, 0.0, 28e9)])
def test_fresnel_matches_boundary_conditions(orc, eps_r, sigma, freq):
    cs = np.linspace(0.01, 1.0, 37)
    gte, gtm, _, _ = orc.fresnel(eps_r, sigma, freq, cs)
    for i, c in enumerate(cs):
        te, tm = fresnel_bc(eps_r, sigma, freq, c)
        assert abs(gte[i] - te) < 1e-12 * max(1, abs(te))
        assert abs(gtm[i] - tm) < 1e-12 * max(1, abs(tm))


def test_fresnel_special_cases(orc):
    f = 3.5e9
    # perfect conductor limit: TE -> -1, TM -> +1 at every angle
    gte, gtm, _, _ = orc.fresnel(1.0, 1e15, f, [0.2, 0.7, 1.0])
    assert np.allclose(gte, -1, atol=1e-5) and np.allclose(gtm, 1, atol=1e-5)
    # normal incidence on a lossless dielectric: TM = -TE = (sqrt(eps)-1)/(sqrt(eps)+1)
    eps = 4.0
    gte, gtm, _, _ = orc.fresnel(eps, 0.0, f, [1.0])
    ref = (math.sqrt(eps) - 1) / (math.sqrt(eps) + 1)
    assert abs(gtm[0] - ref) < 1e-14 and abs(gte[0] + ref) < 1e-14
    # Brewster angle: tan(theta_B) = sqrt(eps) -> Gamma_TM = 0
    cb = 1 / math.sqrt(1 + eps)
    _, gtm, _, _ = orc.fresnel(eps, 0.0, f, [cb])
    assert abs(gtm[0]) < 1e-14
    # grazing incidence: both -> -1
    gte, gtm, _, _ = orc.fresnel(5.0, 0.1, f, [1e-9])
    assert abs(gte[0] + 1) < 1e-8 and abs(gtm[0] + 1) < 1e-7
    # lossless, below the critical value of eta: |Gamma| = 1
    gte, gtm, _, _ = orc.fresnel(0.25, 0.0, f, [0.3])
    assert abs(abs(gte[0]) - 1) < 1e-14 and abs(abs(gtm[0]) - 1) < 1e-14


def test_fresnel_derivative_against_complex_fd(orc):
    """dGamma/deta from the oracle vs finite differences of the linear-solve
    coefficients along the real and the imaginary eta axis."""
    f = 28e9
    w_e0 = 2 * math.pi * f * EPS0
    for eps, sig in ((5.0, 0.5), (2.0, 0.01), (6.3, 0.3)):
        for c in (0.1, 0.5, 0.93):
            _, _, dte, dtm = orc.fresnel(eps, sig, f, [c])
            h = 1e-6
            # d/d eps_r  (d eta = +h)
            tp, mp = fresnel_bc(eps + h, sig, f, c)
            tn, mn = fresnel_bc(eps - h, sig, f, c)
            assert abs((tp - tn) / (2 * h) - dte[0]) < 1e-6 * max(1, abs(dte[0]))
            assert abs((mp - mn) / (2 * h) - dtm[0]) < 1e-6 * max(1, abs(dtm[0]))
            # d/d sigma  (d eta = -j h / (omega eps0))
            hs = h * w_e0
            tp, mp = fresnel_bc(eps, sig + hs, f, c)
            tn, mn = fresnel_bc(eps, sig - hs, f, c)
            assert abs((tp - tn) / (2 * h) - dte[0] * -1j) < 1e-6 * max(1, abs(dte[0]))
            assert abs((mp - mn) / (2 * h) - dtm[0] * -1j) < 1e-6 * max(1, abs(dtm[0]))


# -------------------------------------------------------- launch directions
def test_fibonacci_sphere_properties(orc):
    N = 20000
    d = orc.fib_dirs(N).astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    # uniform on the sphere: each z-band of height h holds a fraction h/2 of the rays
    for lo, hi in ((-1, -0.5), (-0.1, 0.3), (0.7, 1.0)):
        frac = np.mean((d[:, 2] > lo) & (d[:, 2] <= hi))
        assert abs(frac - (hi - lo) / 2) <= 1.5 / N
    # no direction is preferred: the mean vector vanishes
    assert np.linalg.norm(d.mean(0)) < 1e-3
    # a subset returns exactly the rows of the full set
    ids = np.array([0, 17, 9999, N - 1])
    assert np.array_equal(orc.fib_dirs(N, ids), orc.fib_dirs(N)[ids])


# --------------------------------------------------- nearest-hit definition
def _disks(centers, normals, r):
    c = np.asarray(centers, float)
    n = np.asarray(normals, float)
    m = len(c)
    return scenes.Scene(c.astype(np.float32), n.astype(np.float32), np.zeros(m, np.uint16),
                        np.arange(m, dtype=np.uint32), r, 1, m)


def test_nearest_basic_cases(orc):
    up = [0, 0, 1]
    s = _disks([[0, 0, 1], [0, 0, 2], [0, 0, 3]], [up, up, [0, 0, -1]], 0.2)
    ids, t, q = orc.nearest(s, [[0, 0, 0]] * 4, [[0, 0, 1]] * 4, excl=[-1, 0, 1, 2], t_lo=1e-3)
    assert list(ids) == [0, 1, 0, 0]
    assert np.allclose(t, [1, 2, 1, 1])
    # two-sided: from above, moving down, the z=3 disk (normal -z) is hit first
    ids, t, _ = orc.nearest(s, [[0, 0, 5]], [[0, 0, -1]])
    assert ids[0] == 2 and abs(t[0] - 2) < 1e-12
    # the t_lo window skips a disk that is too close to the origin
    ids, _, _ = orc.nearest(s, [[0, 0, 0.9995]], [[0, 0, 1]], t_lo=1e-3)
    assert ids[0] == 1
    # rim is inclusive, just outside the rim misses; a parallel ray misses
    ids, _, _ = orc.nearest(s, [[0.2, 0, 0], [0.2000001, 0, 0]], [[0, 0, 1], [0, 0, 1]])
    assert ids[0] == 0 and ids[1] == 1 or ids[1] == -1
    ids, _, _ = orc.nearest(s, [[-1, 0, 1]], [[1, 0, 0]])
    assert ids[0] == -1


def test_nearest_tie_rule(orc):
    up = [0, 0, 1]
    # coplanar overlapping disks: same t, the centre closer to the hit point wins
    s = _disks([[0, 0, 1], [0.1, 0, 1]], [up, up], 0.15)
    ids, _, _ = orc.nearest(s, [[0.03, 0, 0], [0.08, 0, 0]], [[0, 0, 1]] * 2)
    assert list(ids) == [0, 1]
    # equidistant centres: the smaller index wins, whatever the storage order
    # (coordinates exactly representable in FP32)
    s1 = _disks([[0, 0, 1], [0.125, 0, 1]], [up, up], 0.15)
    ids, _, _ = orc.nearest(s1, [[0.0625, 0, 0]], [[0, 0, 1]])
    assert ids[0] == 0
    s2 = _disks([[0.125, 0, 1], [0, 0, 1]], [up, up], 0.15)
    ids, _, _ = orc.nearest(s2, [[0.0625, 0, 0]], [[0, 0, 1]])
    assert ids[0] == 0
    # inside the tie window (2^-15 m apart) the centre distance decides, not t
    s3 = _disks([[0.125, 0, 1.0], [0, 0, 1.0 + 2.0 ** -15]], [up, up], 0.15)
    ids, t, _ = orc.nearest(s3, [[0.0234375, 0, 0]], [[0, 0, 1]], eps_tie=1e-4)
    assert ids[0] == 1 and t[0] == 1.0 + 2.0 ** -15
    # outside the window (2^-12 m apart) the nearer disk wins
    s4 = _disks([[0.125, 0, 1.0], [0, 0, 1.0 + 2.0 ** -12]], [up, up], 0.15)
    ids, _, _ = orc.nearest(s4, [[0.02, 0, 0]], [[0, 0, 1]], eps_tie=1e-4)
    assert ids[0] == 0


def test_occluded_definition(orc):
    up = [0, 0, 1]
    s = _disks([[0, 0, 1], [5, 5, 5]], [up, up], 0.2)
    occ = orc.occluded(s, [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0.9995]],
                       [[0, 0, 2], [0, 0, 2], [0, 0, 1.0005], [0, 0, 2]], excl=[-1, 0, -1, -1])
    # blocked; own disk excluded; end within eps_self of the disk; start within eps_self
    assert list(occ) == [True, False, False, False]


# ------------------------------------------------------- bounce loop (mirror law)
def test_trace_mirror_law_in_room(orc, room_holefree):
    """First hit = the wall the ray leaves the room through (slab method on the
    exact planes); the second segment obeys the mirror law; lengths add up."""
    s = room_holefree
    N = 4000
    tx = np.array(scenes.BOX_TX)
    sol = orc.solve(s, scenes.box_room_materials(), tx, [scenes.BOX_RX], 3.5e9, N, K=2, flags=SPEC)
    d = orc.fib_dirs(N).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    checked = 0
    for j in range(N):
        # exit plane of the box by the slab method
        tmin, face = np.inf, -1
        for f, (ax, val) in FACE_PLANE.items():
            if d[j, ax] == 0:
                continue
            t = (val - tx[ax]) / d[j, ax]
            if 0 < t < tmin:
                tmin, face = t, f
        x1 = tx + tmin * d[j]
        others = [a for a in range(3) if a != FACE_PLANE[face][0]]
        if any(min(x1[a], ROOM[a] - x1[a]) < 0.15 for a in others):
            continue  # near an edge: overhanging disks of the next face may be hit first
        assert sol.seq[j, 0] >= 0
        hit_face = FACE_PLANE[face]
        assert abs(sol.rec[j, 0, hit_face[0]] - hit_face[1]) < 1e-9
        assert np.allclose(sol.rec[j, 0, :3], x1, atol=1e-9)
        assert abs(sol.rec[j, 0, 3] - tmin) < 1e-9
        assert abs(sol.rec[j, 0, 4] - abs(d[j, hit_face[0]])) < 1e-12
        if sol.seq[j, 1] >= 0:
            u = sol.rec[j, 1, :3] - sol.rec[j, 0, :3]
            seg = np.linalg.norm(u)
            refl = d[j].copy()
            refl[hit_face[0]] *= -1
            assert np.allclose(u / seg, refl, atol=1e-9)
            assert abs(sol.rec[j, 1, 3] - (tmin + seg)) < 1e-9
        checked += 1
    assert checked > N // 2


# ------------------------------------------------- line of sight (closed form)
def test_los_free_space_gain(orc, room_holefree):
    f = 3.5e9
    lam = C0 / f
    rxs = np.array([scenes.BOX_RX, [3.0, 2.0, 2.0], [0.5, 3.5, 0.3]], np.float32)
    sol = orc.solve(room_holefree, scenes.box_room_materials(), scenes.BOX_TX, rxs, f, 16, K=1, flags=LOS)
    for r in range(3):
        dist = np.linalg.norm(rxs[r].astype(float) - np.array(scenes.BOX_TX, np.float32).astype(float))
        assert abs(sol.G_los[r] / (lam / (4 * math.pi * dist)) ** 2 - 1) < 1e-13
        ph = np.exp(-1j * 2 * math.pi / lam * dist) * lam / (4 * math.pi * dist)
        assert abs(sol.h_te[r] - ph) < 1e-13 * abs(ph)
    # tiny box-room LOS: d = 4.482186966 m, G = (lambda/4 pi d)^2
    assert abs(np.linalg.norm(np.subtract(scenes.BOX_RX, scenes.BOX_TX)) - 4.482186966) < 1e-8
    # blocked LOS gives nothing
    wall = scenes.plane_patch(-1, 1, -1, 1, 0.1, 0.0708, z=1.0)
    sol = orc.solve(wall, np.array([[5.0, 0.1, 0.0]]), [0, 0, 0], [[0, 0, 2.0]], f, 16, K=1, flags=LOS)
    assert sol.G_los[0] == 0.0


# -------------------------------------- single reflection vs the image method
def test_single_reflection_image_method(orc):
    f = 3.5e9
    lam = C0 / f
    floor = scenes.plane_patch(-1, 7, -1, 5, 0.1, 0.0708, z=0.0, material=0, surface=0)
    mats = np.array([[2.0, 0.01, 0.0]])
    tx = np.array(scenes.BOX_TX, np.float32).astype(float)  # the FP32 inputs both sides read
    rx = np.array(scenes.BOX_RX, np.float32).astype(float)
    sol = orc.solve(floor, mats, tx, [rx], f, 4000, K=1, flags=SPEC)
    paths = sol.paths(0)
    assert list(paths) == [(0,)]
    L, ate, atm = paths[(0,)]
    img = tx * np.array([1, 1, -1])
    Lref = np.linalg.norm(rx - img)
    assert abs(L - Lref) < 1e-9 and abs(Lref - 5.223983155) < 1e-7
    c = (tx[2] + rx[2]) / Lref
    te, tm = fresnel_bc(2.0, 0.01, f, c)
    base = lam / (4 * math.pi) / Lref * np.exp(-1j * 2 * math.pi / lam * Lref)
    assert abs(ate - base * te) < 1e-9 * abs(base)
    assert abs(atm - base * tm) < 1e-9 * abs(base)


# ------------------------------------------------ box room: full enumeration
@pytest.mark.parametrize("K", [2, 3])
def test_box_room_specular_set_and_gain(orc, room_holefree, K):
    f = 3.5e9
    mats = scenes.box_room_materials()
    ref = image_method_room(scenes.BOX_TX, scenes.BOX_RX, K, mats, f)
    n_rays = 20000 if K == 2 else 30000
    sol = orc.solve(room_holefree, mats, scenes.BOX_TX, [scenes.BOX_RX], f, n_rays, K=K, flags=LOS | SPEC)
    got = sol.paths(0)
    by_order = [sum(1 for c in ref if len(c[0][0]) == o) for o in range(1, K + 1)]
    assert by_order[:2] == [6, 18]  # 6 first-order, 18 of 30 second-order orderings
    if K == 3:
        assert by_order[2] == 36
    n_amb = sum(len(c[0]) > 1 for c in ref)
    assert n_amb <= (1 if K == 2 else 8)
    lam = C0 / f
    tx32 = np.float32(scenes.BOX_TX).astype(float)
    rx32 = np.float32(scenes.BOX_RX).astype(float)
    g_ref = (lam / (4 * math.pi * np.linalg.norm(rx32 - tx32))) ** 2
    matched = set()
    for cands, L, amps in ref:
        hits = [c for c in cands if c in got]
        assert len(hits) == 1, (cands, hits)  # exactly one label choice is found valid
        key = hits[0]
        matched.add(key)
        gl, gte, gtm = got[key]
        ate, atm = amps[key]
        assert abs(gl - L) < 1e-9
        assert abs(gte - ate) < 1e-8 * abs(ate) + 1e-15
        assert abs(gtm - atm) < 1e-8 * abs(atm) + 1e-15
        g_ref += 0.5 * (abs(ate) ** 2 + abs(atm) ** 2)
    assert matched == set(got)  # no valid path that the image method does not know
    assert abs(sol.G[0] / g_ref - 1) < 1e-12


def test_reciprocity(orc, room_holefree):
    f = 3.5e9
    mats = scenes.box_room_materials()
    ta, tb = (1.51, 3.46, 2.02), (2.3, 2.42, 1.26)
    # a pair whose reflection points avoid every window/door border (no label ties)
    assert all(len(c[0]) == 1 for c in image_method_room(ta, tb, 2, mats, f))
    a = orc.solve(room_holefree, mats, ta, [tb], f, 20000, K=2, flags=LOS | SPEC)
    b = orc.solve(room_holefree, mats, tb, [ta], f, 20000, K=2, flags=LOS | SPEC)
    assert len(a.paths(0)) >= 20
    pa, pb = a.paths(0), b.paths(0)
    assert {k[::-1] for k in pa} == set(pb)
    for k, (L, te, tm) in pa.items():
        L2, te2, tm2 = pb[k[::-1]]
        assert abs(L - L2) < 1e-9
        assert abs(te - te2) < 1e-9 * abs(te) and abs(tm - tm2) < 1e-9 * abs(tm)
    assert abs(a.G[0] / b.G[0] - 1) < 1e-10
    assert abs(a.h_te[0] - b.h_te[0]) < 1e-9 * abs(a.h_te[0])


# --------------------------------------- diffuse ray-tube vs quadrature
def _lambert_integral(center, R, tx, rx, weight=lambda c: 1.0):
    """Integral over a horizontal disk of cos_i cos_s / (pi r_i^2 r_s^2) * weight(cos_i)."""
    cx, cy, cz = center

    def f(rho, phi):
        x, y = cx + rho * math.cos(phi), cy + rho * math.sin(phi)
        vi = np.array([x - tx[0], y - tx[1], cz - tx[2]])
        vs = np.array([rx[0] - x, rx[1] - y, rx[2] - cz])
        ri, rs = np.linalg.norm(vi), np.linalg.norm(vs)
        ci, cs = abs(vi[2]) / ri, abs(vs[2]) / rs
        return ci * cs / (math.pi * ri * ri * rs * rs) * weight(ci) * rho

    val, _ = integrate.dblquad(f, 0, 2 * math.pi, 0, R, epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("case", ["unit_reflectance", "concrete"])
def test_diffuse_ray_tube_matches_quadrature(orc, case):
    f = 3.5e9
    lam = C0 / f
    tx, rx = (0.0, 0.0, 1.0), (2.0, 0.0, 1.0)
    disk = scenes.single_disk((1.0, 0.0, 0.0), (0, 0, 1), 3.0)
    N = 400000
    ids = np.arange(N // 2, N)  # the downward half of the sphere
    if case == "unit_reflectance":
        # eta = 0: |Gamma_TE| = |Gamma_TM| = 1 at every angle
        mats = np.array([[0.0, 0.0, 1.0]])
        weight = lambda c: 1.0
    else:
        mats = np.array([[5.0, 0.1, 1.0]])

        def weight(c):
            te, tm = fresnel_bc(5.0, 0.1, f, c)
            return 0.5 * (abs(te) ** 2 + abs(tm) ** 2)
    sol = orc.solve(disk, mats, tx, [rx], f, N, ray_ids=ids, K=1, flags=DIFF)
    I = _lambert_integral((1.0, 0.0, 0.0), 3.0, tx, rx, weight)
    g_ref = (lam / (4 * math.pi)) ** 2 * I
    assert abs(sol.G_diff[0] / g_ref - 1) < 2e-4
    # S = 0: no diffuse power at all
    sol0 = orc.solve(disk, np.array([[5.0, 0.1, 0.0]]), tx, [rx], f, 2000, K=1, flags=DIFF)
    assert sol0.G_diff[0] == 0.0


def test_connection_power_output_sums_to_the_diffuse_gain(orc, room_holefree):
    """The per-connection power output prices every lit connection whether
    or not it is occluded; over the visible ones it sums to G_diff, and it is
    positive wherever a connection is visible."""
    mats = scenes.box_room_materials(scatter=0.3)
    rx = np.array([scenes.BOX_RX, [2.0, 3.0, 2.0]], np.float32)
    sol = orc.solve(room_holefree, mats, scenes.BOX_TX, rx, 3.5e9, 500, K=3, flags=DIFF, want_dvis=True,
                    want_dpow=True)
    assert np.all(sol.dpow[sol.dvis] > 0)
    assert np.allclose((sol.dpow * sol.dvis).sum(axis=(0, 1)), sol.G_diff, rtol=1e-12, atol=0)
    assert np.all(sol.dpow[sol.seq < 0] == 0)


def test_scattering_removes_specular(orc):
    floor = scenes.plane_patch(-1, 7, -1, 5, 0.1, 0.0708)
    sol = orc.solve(floor, np.array([[2.0, 0.01, 1.0]]), scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 2000, K=1,
                    flags=SPEC)
    assert sol.spec_valid.sum() == 1 and sol.G_spec[0] == 0.0  # R = sqrt(1 - S^2) = 0


# ------------------------------------------------------- invariants
def test_permutation_invariance_random(orc):
    s = scenes.random_disks(400, seed=3, extent=1.5, radius=0.25)
    rng = np.random.default_rng(5)
    perm = rng.permutation(s.n)
    mats = np.array([[3.0, 0.1, 0.2], [5.0, 0.5, 0.2], [2.0, 0.01, 0.2]])
    rx = [[0.3, -0.2, 0.1], [-0.5, 0.4, -0.3]]
    a = orc.solve(s, mats, [0, 0, 0], rx, 28e9, 3000, K=4, flags=LOS | SPEC | DIFF)
    b = orc.solve(s.permuted(perm), mats, [0, 0, 0], rx, 28e9, 3000, K=4, flags=LOS | SPEC | DIFF)
    remap = np.where(b.seq >= 0, perm[np.maximum(b.seq, 0)], -1)
    assert np.array_equal(a.seq, remap)
    assert np.allclose(a.G, b.G, rtol=1e-12)


def test_permutation_invariance_coplanar_room(orc):
    """The box room is full of exact coplanar overlaps; the tie rule must not
    depend on the storage order."""
    s = scenes.box_room(spacing=0.1, radius=0.09)
    perm = np.random.default_rng(11).permutation(s.n)
    mats = scenes.box_room_materials()
    a = orc.solve(s, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 3000, K=3, flags=SPEC)
    b = orc.solve(s.permuted(perm), mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 3000, K=3, flags=SPEC)
    remap = np.where(b.seq >= 0, perm[np.maximum(b.seq, 0)], -1)
    assert np.array_equal(a.seq, remap)
    assert a.G[0] == pytest.approx(b.G[0], rel=1e-12)


# ------------------------------------------------------------ gradient
def test_gradient_matches_finite_differences(orc, room_holefree):
    s = scenes.box_room(spacing=0.1, radius=0.0708, labels="surface")
    mats = scenes.box_room_materials("surface", scatter=0.3)
    rx = np.array([scenes.BOX_RX, [2.0, 3.0, 2.0]], np.float32)
    kw = dict(K=2, flags=LOS | SPEC | DIFF)
    base = orc.solve(s, mats, scenes.BOX_TX, rx, 3.5e9, 1500, want_jac=True, **kw)
    assert base.G_diff.min() > 0 and base.G_spec.min() > 0
    for lab in range(8):
        for p, rel in ((0, 1e-5), (1, 1e-4), (2, 1e-4)):
            h = rel * mats[lab, p]
            mp, mn = mats.copy(), mats.copy()
            mp[lab, p] += h
            mn[lab, p] -= h
            gp = orc.solve(s, mp, scenes.BOX_TX, rx, 3.5e9, 1500, **kw).G
            gn = orc.solve(s, mn, scenes.BOX_TX, rx, 3.5e9, 1500, **kw).G
            fd = (gp - gn) / (2 * h)
            an = base.jac[:, lab, p]
            scale = np.abs(base.G).max() * 1e-7 + np.abs(an)
            assert np.all(np.abs(fd - an) <= 2e-5 * scale), (lab, p, fd, an)


def test_gradient_of_the_reception_point_launch_matches_finite_differences(orc):
    """The analytic Jacobian with the paper's launch (rays towards the point
    sets' reception points, candidates gated by the visibility matrix, voxel
    diffuse paths of area rho^2) against central differences of G."""
    s = scenes.box_room(spacing=0.1, radius=0.0708, labels="surface")
    mats = scenes.box_room_materials("surface", scatter=0.3)
    rx = np.array([scenes.BOX_RX, [2.0, 3.0, 2.0]], np.float32)
    rho = 0.25
    n_sets = int(np.unique(np.floor(s.pos.astype(np.float64) / np.float64(np.float32(rho))), axis=0).shape[0])
    kw = dict(K=2, flags=LOS | SPEC | DIFF, dps_launch=rho)
    base = orc.solve(s, mats, scenes.BOX_TX, rx, 3.5e9, n_sets, want_jac=True, **kw)
    assert base.G_diff.min() > 0 and base.G_spec.min() > 0
    for lab in range(8):
        for p, rel in ((0, 1e-5), (1, 1e-4), (2, 1e-4)):
            h = rel * mats[lab, p]
            mp, mn = mats.copy(), mats.copy()
            mp[lab, p] += h
            mn[lab, p] -= h
            gp = orc.solve(s, mp, scenes.BOX_TX, rx, 3.5e9, n_sets, **kw).G
            gn = orc.solve(s, mn, scenes.BOX_TX, rx, 3.5e9, n_sets, **kw).G
            fd = (gp - gn) / (2 * h)
            an = base.jac[:, lab, p]
            # the differences' rounding: a few ulp of G over 2h
            floor = 8 * np.finfo(float).eps * np.abs(base.G).max() / (2 * h)
            assert np.all(np.abs(fd - an) <= 2e-5 * np.abs(an) + floor), (lab, p, fd, an)


def _lambert_integral_vertical(tx, rx, x0, zc, R, weight):
    """Integral over the vertical disk x = x0 (centre (x0, 0, zc), radius R) of
    cos_i cos_s / (pi r_i^2 r_s^2) * weight(point)."""

    def f(rho, phi):
        p = np.array([x0, rho * math.cos(phi), zc + rho * math.sin(phi)])
        vi, vs = p - np.asarray(tx), np.asarray(rx) - p
        ri, rs = np.linalg.norm(vi), np.linalg.norm(vs)
        return abs(vi[0]) / ri * abs(vs[0]) / rs / (math.pi * ri * ri * rs * rs) * weight(p) * rho

    val, _ = integrate.dblquad(f, 0, 2 * math.pi, 0, R, epsabs=1e-14, epsrel=1e-11)
    return val


def test_diffuse_after_specular_bounce_matches_image_quadrature(orc):
    """Mirror floor (S = 0) + vertical scatterer (S = 1, |Gamma| = 1).

    Scattered power = direct illumination of the scatterer + illumination via
    the floor, i.e. from the image transmitter below the floor, weighted by the
    floor's Fresnel power reflectance at the incidence angle of that image ray.
    """
    f = 3.5e9
    lam = C0 / f
    tx, rx = (0.0, 0.0, 1.0), (1.0, 0.5, 2.0)
    wall = scenes.single_disk((3.0, 0.0, 1.5), (-1, 0, 0), 1.0, material=1, surface=1)
    # one radius per scene: the floor is a hole-free grid of unit disks
    floor_disks = [scenes.single_disk((x, y, 0.0), (0, 0, 1), 1.0) for x in np.arange(-7.0, 9.0, 1.2)
                   for y in np.arange(-8.0, 8.01, 1.2)]
    sc = scenes.concat(floor_disks + [wall])
    mats = np.array([[5.0, 0.1, 0.0], [0.0, 0.0, 1.0]])
    N = 400000
    sol = orc.solve(sc, mats, tx, [rx], f, N, K=2, flags=DIFF)
    tx32, rx32 = np.float32(tx).astype(float), np.float32(rx).astype(float)
    img = tx32 * np.array([1, 1, -1])

    def via_floor(p):
        u = p - img
        c = abs(u[2]) / np.linalg.norm(u)
        te, tm = fresnel_bc(5.0, 0.1, f, c)
        # the image ray must cross the floor inside the disk-covered square
        s = img[2] / (img[2] - p[2])
        xf, yf = img[0] + s * u[0], img[1] + s * u[1]
        return 0.5 * (abs(te) ** 2 + abs(tm) ** 2) if (-7.0 <= xf <= 8.0 and -8.0 <= yf <= 8.0) else 0.0

    direct = _lambert_integral_vertical(tx32, rx32, 3.0, 1.5, 1.0, lambda p: 1.0)
    via = _lambert_integral_vertical(img, rx32, 3.0, 1.5, 1.0, via_floor)
    g_ref = (lam / (4 * math.pi)) ** 2 * (direct + via)
    assert via > 0.05 * direct
    assert abs(sol.G_diff[0] / g_ref - 1) < 1e-3


def test_diffuse_phase_uses_unfolded_length(orc):
    """One ray onto a scattering floor: the connection's phase is the phase of
    the geometric length TX -> hit -> RX."""
    f = 28e9
    lam = C0 / f
    floor = scenes.single_disk((0.0, 0.0, 0.0), (0, 0, 1), 5.0)
    N = 1000
    j = 700  # a downward ray
    d = orc.fib_dirs(N, [j])[0].astype(float)
    tx, rx = np.array([0.0, 0.0, 1.0]), np.float32([0.7, -0.4, 1.3]).astype(float)
    sol = orc.solve(floor, np.array([[5.0, 0.1, 1.0]]), tx, [rx], f, N, ray_ids=[j], K=1, flags=DIFF)
    d /= np.linalg.norm(d)
    hit = tx + d * (1.0 / -d[2])
    L = np.linalg.norm(hit - tx) + np.linalg.norm(rx - hit)
    assert abs(sol.h_te[0]) > 0 and abs(sol.h_tm[0]) > 0
    # remove the Fresnel phase at the scatter point, then only propagation remains
    cos_i = -d[2]
    te, tm = fresnel_bc(5.0, 0.1, f, cos_i)
    assert abs(np.angle(sol.h_te[0] / te * np.exp(1j * 2 * math.pi / lam * L))) < 1e-9
    assert abs(np.angle(sol.h_tm[0] / tm * np.exp(1j * 2 * math.pi / lam * L))) < 1e-9


# ------------------------------- channel frequency / impulse response (CFR)
# CFR reading: each path's centre-frequency amplitudes times
# exp(-j 2 pi (f_n - f_c) L / c0) at n_freq equally spaced samples spanning
# the bandwidth (the paper's learning experiment: 129 samples over 1.5 GHz at
# 8 GHz, the CIR being the inverse DFT of those samples).
def _cfr_freqs(fc, bw, n):
    return fc + (np.arange(n) - 0.5 * (n - 1)) * bw / (n - 1)


def test_cfr_centre_sample_is_the_coherent_field(orc, room_holefree):
    """At the centre sample every path's weight is exactly 1, so it is the
    solve's own coherent sum h_TE, h_TM (all three path kinds)."""
    rxs = np.array([scenes.BOX_RX, [3.0, 2.0, 2.0]], np.float32)
    sol = orc.solve(room_holefree, scenes.box_room_materials(scatter=0.3), scenes.BOX_TX, rxs, 8e9, 400, K=2,
                    flags=LOS | SPEC | DIFF, cfr=(1.5e9, 129))
    assert sol.cfr.shape == (2, 129, 2)
    np.testing.assert_array_equal(sol.cfr[:, 64, 0], sol.h_te)
    np.testing.assert_array_equal(sol.cfr[:, 64, 1], sol.h_tm)
    # off-centre samples differ (the paths have different delays)
    assert np.all(np.abs(sol.cfr[:, 0, 0] - sol.h_te) > 1e-3 * np.abs(sol.h_te))


def test_cfr_line_of_sight_is_free_space_at_each_frequency(orc, room_holefree):
    """One path: lambda_c / (4 pi d) exp(-j 2 pi f_n d / c0) -- the phase
    follows each sample frequency, the amplitude stays at the centre's."""
    fc, bw, n = 8e9, 1.5e9, 129
    rx = np.array([[3.0, 2.0, 2.0]], np.float32)
    sol = orc.solve(room_holefree, scenes.box_room_materials(), scenes.BOX_TX, rx, fc, 16, K=1, flags=LOS,
                    cfr=(bw, n))
    d = np.linalg.norm(rx[0].astype(float) - np.array(scenes.BOX_TX, np.float32).astype(float))
    lam = C0 / fc
    ref = lam / (4 * math.pi * d) * np.exp(-1j * 2 * math.pi * _cfr_freqs(fc, bw, n) * d / C0)
    np.testing.assert_allclose(sol.cfr[0, :, 0], ref, rtol=0, atol=1e-12 * abs(ref[0]))
    np.testing.assert_allclose(sol.cfr[0, :, 1], ref, rtol=0, atol=1e-12 * abs(ref[0]))


def test_cfr_impulse_response_peaks_at_the_path_delays(orc):
    """Line of sight plus one floor reflection: the inverse DFT of the 129
    samples peaks at bins tau * N * bw / (N - 1) of the two path delays
    (a wrong phase sign would put them at N minus that)."""
    fc, bw, n = 8e9, 1.5e9, 129
    floor = scenes.plane_patch(-1, 7, -1, 5, 0.1, 0.0708, z=0.0, material=0, surface=0)
    tx = np.array([1.0, 1.0, 1.5], np.float32)
    rx = np.array([4.0, 2.5, 1.2], np.float32)
    sol = orc.solve(floor, np.array([[2.0, 0.01, 0.0]]), tx, [rx], fc, 4000, K=1, flags=LOS | SPEC, cfr=(bw, n))
    taus = [np.linalg.norm(rx.astype(float) - tx.astype(float)) / C0,
            np.linalg.norm(rx.astype(float) - tx.astype(float) * np.array([1, 1, -1])) / C0]
    h = np.fft.ifft(sol.cfr[0, :, 0])
    top = sorted(np.argsort(np.abs(h))[-2:])
    want = sorted(int(round(t * n * bw / (n - 1))) % n for t in taus)
    assert top == want, (top, want)


# ------------------------------------- point-set averaging (Sec. II-C, Eq. 3-4)
RHO, LAM, RP = 0.0625, 100.0, 0.015


def _disks(centres, normals, radius=RP):
    return scenes.concat([scenes.single_disk(c, n, radius) for c, n in zip(centres, normals)])


def _f(v):
    """The FP64 value of an FP32 input, as the oracle reads it."""
    return np.asarray(v, np.float32).astype(np.float64)


def test_average_two_stacked_disks_closed_form(orc):
    """Two +z disks in one voxel, the ray straight down through the upper centre:
    t = (t_A + w_B t_B) / (1 + w_B) with w_B = exp(-a^2/(2 r^2)) exp(-lambda dz),
    a = the in-plane offset of B's centre, dz = the depth between the two hits."""
    pa, pb = _f([0.02, 0.02, 0.03]), _f([0.03, 0.02, 0.02])
    s = _disks([pa, pb], [[0, 0, 1], [0, 0, 1]])
    o = np.array([pa[0], pa[1], 1.0])
    i, t, n = orc.average(s, o, [0, 0, -1], RHO, LAM)
    ta, tb = 1.0 - pa[2], 1.0 - pb[2]
    a2 = (pa[0] - pb[0]) ** 2 + (pa[1] - pb[1]) ** 2
    r = float(np.float32(RP))
    wb = math.exp(-a2 / (2 * r * r)) * math.exp(-LAM * (tb - ta))
    assert i[0] == 0
    assert t[0] == pytest.approx((ta + wb * tb) / (1 + wb), rel=1e-13)
    assert np.allclose(n[0], [0, 0, 1], atol=1e-15)


def test_average_large_lambda_keeps_the_nearest_member(orc):
    pa, pb = _f([0.02, 0.02, 0.03]), _f([0.03, 0.02, 0.02])
    s = _disks([pa, pb], [[0, 0, 1], [0, 0, 1]])
    _, t, _ = orc.average(s, [pa[0], pa[1], 1.0], [0, 0, -1], RHO, 1e6)
    assert t[0] == 1.0 - pa[2]


def test_average_tilted_pair_and_flipped_member_reflect_like_the_plane(orc):
    """Members tilted by +-20 deg about x at one centre average to the +z normal,
    also when one of them is stored facing away from the ray (two-sided disks)."""
    c = _f([0.03, 0.03, 0.03])
    th = math.radians(20.0)
    n1 = [0.0, math.sin(th), math.cos(th)]
    for n2 in ([0.0, -math.sin(th), math.cos(th)], [0.0, math.sin(th), -math.cos(th)]):
        s = _disks([c, c], [n1, n2])
        _, t, n = orc.average(s, [c[0], c[1], 1.0], [0, 0, -1], RHO, LAM)
        assert t[0] == pytest.approx(1.0 - c[2], rel=1e-14)
        assert np.allclose(n[0], [0, 0, 1], atol=1e-7)


def test_average_uses_the_voxel_of_the_hit_disk_only(orc):
    """B overlaps A's footprint from across the voxel boundary x = rho: it is no
    member of A's set. Moved inside the voxel, it changes the average."""
    pa = _f([0.04, 0.03, 0.03])
    r = 0.03
    o = [0.05, 0.03, 1.0]
    for xb, member in ((0.065, False), (0.060, True)):
        pb = _f([xb, 0.03, 0.025])
        s = _disks([pa, pb], [[0, 0, 1], [0, 0, 1]], radius=r)
        i, t, _ = orc.average(s, o, [0, 0, -1], RHO, LAM)
        assert i[0] == 0
        if member:
            assert t[0] > 1.0 - pa[2] + 1e-6
        else:
            assert t[0] == pytest.approx(1.0 - pa[2], rel=1e-14)


def test_average_with_single_point_sets_is_the_nearest_hit(orc):
    """Voxels far smaller than the spacing: every set holds one disk, so the full
    solve with averaging reproduces the plain solve."""
    s = scenes.random_disks(400, seed=11, extent=1.5, radius=0.2)
    mats = np.array([[3.0, 0.1, 0.3], [5.0, 0.5, 0.2], [2.0, 0.01, 0.5]])
    rx = np.array([[0.3, -0.2, 0.1], [-0.5, 0.4, -0.3]], np.float32)
    a = orc.solve(s, mats, [0, 0, 0], rx, 3.5e9, 500, K=3, flags=LOS | SPEC | DIFF)
    b = orc.solve(s, mats, [0, 0, 0], rx, 3.5e9, 500, K=3, flags=LOS | SPEC | DIFF, average=(1e-4, LAM))
    assert np.array_equal(a.seq, b.seq)
    assert np.allclose(a.rec, b.rec, rtol=1e-12, atol=1e-12, equal_nan=True)
    assert np.allclose(a.G, b.G, rtol=1e-10)


def test_average_on_exact_planes_keeps_the_specular_paths(orc, room_holefree):
    """Noise-free room: every point set lies in one face plane with that face's
    normal, so averaged interactions and averaged validation planes are the
    exact face planes and the specular paths are those of the plain solve."""
    mats = scenes.box_room_materials()
    tx, rx = [1.5, 1.2, 1.4], np.array([[4.2, 2.9, 1.1], [0.8, 3.1, 2.0]], np.float32)
    a = orc.solve(room_holefree, mats, tx, rx, 3.5e9, 3000, K=2, flags=SPEC)
    b = orc.solve(room_holefree, mats, tx, rx, 3.5e9, 3000, K=2, flags=SPEC, average=(0.25, 100.0))
    for r in range(len(rx)):
        pa, pb = a.paths(r), b.paths(r)
        assert set(pa) == set(pb) and len(pa) >= 5
        for key in pa:
            assert pb[key][0] == pytest.approx(pa[key][0], rel=1e-9)



# ------------------------------------ visibility matrix (Sec. II-A, II-B)
def test_reception_points_are_set_means(orc):
    s = scenes.random_disks(3000, seed=21, extent=1.0, radius=0.05)
    recv, vis = orc.visibility(s, 0.5, [[0.0, 0.0, 0.0]])
    p = s.pos.astype(np.float64)
    v = np.floor(p / np.float64(np.float32(0.5)))
    keys, inv = np.unique(v, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    mean = np.stack([np.bincount(inv, weights=p[:, k]) for k in range(3)], 1) / np.bincount(inv)[:, None]
    assert recv.shape == (len(keys), 3) and vis.shape == (1, len(keys))
    assert np.allclose(recv, mean.astype(np.float32), rtol=0, atol=2e-7)


def test_visibility_behind_a_blocker_closed_form(orc):
    """A floor patch at z = 0 and one blocking disk (z = 0.5) under a receiver at
    z = 1, all disks of radius 0.15: a reception point is hidden iff the segment
    crosses z = 0.5 within 0.15 of the blocker's centre (points clear of the rim)."""
    R = 0.15
    floor = scenes.plane_patch(0.0, 1.2, 0.0, 1.2, 0.1, R)
    sc = scenes.concat([floor, scenes.single_disk([0.6, 0.6, 0.5], [0, 0, 1], R)])
    rx = np.array([[0.5, 0.5, 1.0]], np.float32)
    recv, vis = orc.visibility(sc, 0.25, rx)
    mid = rx[0].astype(np.float64) + 0.5 * (recv.astype(np.float64) - rx[0])
    dist = np.linalg.norm(mid[:, :2] - [0.6, 0.6], axis=1)
    on_floor = np.abs(recv[:, 2]) < 1e-6
    sel = on_floor & (np.abs(dist - R) > 1e-3)
    assert sel.sum() >= 20
    assert np.array_equal(vis[0, sel].astype(bool), dist[sel] > R)
    assert (dist[sel] <= R).any() and (dist[sel] > R).any()


def test_visibility_ignores_the_own_set_only(orc):
    """A disk 2 cm above a reception point on the segment towards the receiver:
    no occluder while it belongs to the same voxel, an occluder once it sits in
    the voxel above."""
    base = [scenes.single_disk([0.10 + 0.01 * i, 0.10, 0.05], [0, 0, 1], 0.02) for i in range(3)]
    rx = np.array([[0.11, 0.10, 1.0]], np.float32)
    for z, visible in ((0.07, True), (0.13, False)):
        sc = scenes.concat(base + [scenes.single_disk([0.11, 0.10, z], [0, 0, 1], 0.02)])
        recv, vis = orc.visibility(sc, 0.125, rx)
        j = int(np.argmin(np.abs(recv[:, 2] - 0.05) + np.abs(recv[:, 0] - 0.11)))
        assert bool(vis[0, j]) == visible


# ------------------------------- launch at the reception points (Sec. II-B)
def test_dps_launch_hits_the_reception_points(orc):
    """Flat, hole-free floor under the transmitter: the ray towards a set's
    reception point meets the floor exactly there (the mean of coplanar
    centres lies on the plane)."""
    floor = scenes.plane_patch(0.0, 2.0, 0.0, 2.0, 0.05, 0.04)
    recv, _ = orc.visibility(floor, 0.0625, [[1.0, 1.0, 1.0]])
    ns = len(recv)
    sol = orc.solve(floor, np.array([[5.0, 0.1, 0.0]]), [1.0, 1.0, 1.0], np.zeros((1, 3), np.float32), 3.5e9, ns,
                    K=1, flags=SPEC, dps_launch=0.0625)
    hit = sol.seq[:, 0] >= 0
    assert hit.all()
    err = np.abs(sol.rec[:, 0, :3] - recv.astype(np.float64)).max()
    assert err < 1e-6  # FP32 direction rounding over ~1.4 m


def test_dps_launch_gates_specular_candidates(orc):
    """One-bounce floor path TX -> (1.25, 1, 0) -> RX. The key's representative
    is the ray of set 0 (reception point near the origin); a small disk on the
    segment from RX to that reception point, far from the path, removes the
    candidate in this mode."""
    floor = scenes.plane_patch(0.0, 2.0, 0.0, 2.0, 0.05, 0.04)
    tx, rx = np.array([1.0, 1.0, 1.0], np.float32), np.array([[1.5, 1.0, 1.0]], np.float32)
    mats = np.array([[5.0, 0.1, 0.0], [3.0, 0.1, 0.0]])
    recv0, _ = orc.visibility(floor, 0.0625, rx)
    c0 = recv0[0].astype(np.float64)
    mid = 0.5 * (rx[0] + c0)
    axis = (c0 - rx[0]) / np.linalg.norm(c0 - rx[0])
    blocker = scenes.single_disk(mid, axis, 0.04, material=1, surface=1)
    for sc, expect in ((floor, True), (scenes.concat([floor, blocker]), False)):
        recv, vis = orc.visibility(sc, 0.0625, rx)
        sol = orc.solve(sc, mats, tx, rx, 3.5e9, len(recv), K=1, flags=SPEC, dps_launch=0.0625)
        assert sol.key_rep[sol.keys.index((0,))] == 0
        assert bool(vis[0, 0]) == expect
        assert ((0,) in sol.paths(0)) == expect


def test_voxel_diffuse_converges_to_the_lambertian_integral(orc):
    """Reception-point launch over a flat, hole-free 2 x 2 m floor, one
    interaction: each point set (voxel of edge rho) gives one diffuse path
    standing for an area rho^2 (Sec. II-B.4), so the total diffuse power is a
    midpoint-rule sum over the voxels. As rho halves it must converge, with
    error falling as rho^2, to the integral over the floor of the Lambertian
    scattered power (lambda/4 pi)^2 S^2 |Gamma|^2 cos_i cos_s / (pi r_i^2 r_s^2)
    dA, evaluated here by adaptive quadrature with boundary-condition Fresnel
    weights. A wrong area power, a dropped cosine or pi, or the wrong length
    in the spreading changes the limit."""
    h = 1.0 / 32  # grid spacing: every voxel edge below is a multiple, so each set's mean is its voxel centre
    floor = scenes.plane_patch(0.0, 2.0, 0.0, 2.0, h, 0.72 * h)
    tx, rx = np.array([1.0, 1.0, 1.0], np.float32), np.array([[1.5, 1.0, 1.0]], np.float32)
    freq, eps_r, sigma, S = 3.5e9, 5.0, 0.1, 0.4
    lam = C0 / freq
    t64, r64 = tx.astype(np.float64), rx[0].astype(np.float64)

    def integrand(y, x):
        vi, vs = np.array([x, y, 0.0]) - t64, r64 - np.array([x, y, 0.0])
        ri, rs = np.linalg.norm(vi), np.linalg.norm(vs)
        ci, cs = -vi[2] / ri, vs[2] / rs
        te, tm = fresnel_bc(eps_r, sigma, freq, ci)
        return ci * cs / (math.pi * ri * ri * rs * rs) * 0.5 * (abs(te) ** 2 + abs(tm) ** 2)
    I, _ = integrate.dblquad(integrand, 0.0, 2.0, 0.0, 2.0, epsabs=1e-14, epsrel=1e-11)
    g_ref = (lam / (4 * math.pi)) ** 2 * S ** 2 * I
    G = []
    for rho in (0.25, 0.125, 0.0625):
        recv, vis = orc.visibility(floor, rho, rx)
        assert vis.all() and len(recv) == round(2.0 / rho) ** 2
        sol = orc.solve(floor, np.array([[eps_r, sigma, S]]), tx, rx, freq, len(recv), K=1, flags=DIFF,
                        dps_launch=rho)
        assert sol.G_spec[0] == 0.0 and sol.G_los[0] == 0.0
        G.append(sol.G_diff[0])
    err = np.array(G) / g_ref - 1
    assert abs(err[0]) < 1e-2
    assert 3.6 < err[0] / err[1] < 4.4 and 3.6 < err[1] / err[2] < 4.4  # second-order convergence
    rich = (4 * G[2] - G[1]) / 3  # Richardson limit of the midpoint sums
    assert abs(rich / g_ref - 1) < 1e-5


# --------------------------------------- edge diffraction (Sec. II-B.3, UTD)
def test_diffraction_point_obeys_kellers_cone():
    """The edge point found by unfolding makes equal angles with the edge for
    the incident and diffracted rays, and no sampled edge point is shorter."""
    from oracle import diffraction as dif
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        p, q = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        t = dif.edge_point(a, b, p, q)
        D = a + t * (b - a)
        e = (b - a) / np.linalg.norm(b - a)
        assert (D - p) @ e / np.linalg.norm(D - p) == pytest.approx((q - D) @ e / np.linalg.norm(q - D), abs=1e-12)
        ts = np.linspace(t - 0.5, t + 0.5, 2001)
        L = [np.linalg.norm(p - (a + s * (b - a))) + np.linalg.norm(q - (a + s * (b - a))) for s in ts]
        assert min(L) >= np.linalg.norm(p - D) + np.linalg.norm(q - D) - 1e-12


@pytest.mark.parametrize("n", [1.5, 2.0, 1.75])
def test_diffraction_coefficient_far_from_boundaries_is_kellers(n):
    """For large kL away from the shadow and reflection boundaries every
    transition function tends to one, and the perfectly conducting wedge
    coefficient is Keller's: e^{-j pi/4} sin(pi/n) / (n sqrt(2 pi k) sin b0)
    [1/(cos(pi/n) - cos((phi - phi')/n)) -+ 1/(cos(pi/n) - cos((phi + phi')/n))]."""
    from oracle import diffraction as dif
    k, L, sb = 50.0, 2e5, 0.8
    for phip, phi in ((0.4, 0.9 * n * np.pi), (0.7 * n * np.pi, 0.3)):
        for r in (-1.0, 1.0):
            d = dif.coefficient(n, k, L, phi, phip, sb, r, r)
            g = (1 / (np.cos(np.pi / n) - np.cos((phi - phip) / n))
                 + r / (np.cos(np.pi / n) - np.cos((phi + phip) / n)))
            keller = np.exp(-1j * np.pi / 4) * np.sin(np.pi / n) / (n * np.sqrt(2 * np.pi * k) * sb) * g
            assert abs(d - keller) <= 1e-4 * abs(keller)


@pytest.mark.parametrize("r", [-1.0, 1.0])
def test_half_plane_total_field_is_continuous_at_the_boundaries(r):
    """Half-plane (n = 2), perfectly conducting, normal incidence: the incident
    field vanishes across phi = pi + phi' and the reflected one across
    phi = pi - phi'; geometric optics plus the diffracted field stays
    continuous there."""
    from oracle import diffraction as dif
    k, sp, s, phip = 2 * np.pi / 0.1, 3.0, 2.0, np.radians(50.0)
    S = sp * np.array([np.cos(phip), np.sin(phip)])
    Si = sp * np.array([np.cos(phip), -np.sin(phip)])  # image in face 0

    def total(phi):
        O = s * np.array([np.cos(phi), np.sin(phi)])
        u = 0j
        if phi < np.pi + phip:
            R = np.linalg.norm(S - O)
            u += np.exp(-1j * k * R) / R
        if phi < np.pi - phip:
            R = np.linalg.norm(Si - O)
            u += r * np.exp(-1j * k * R) / R
        L = s * sp / (s + sp)
        d = dif.coefficient(2.0, k, L, phi, phip, 1.0, r, r)
        return u + np.exp(-1j * k * sp) / sp * d * np.sqrt(sp / (s * (s + sp))) * np.exp(-1j * k * s)

    # the one-sided limits at each boundary, from a Richardson step on the
    # difference across it (the fields vary smoothly away from the boundary)
    for bnd in (np.pi + phip, np.pi - phip):
        go_jump = 1.0 / (sp + s)  # the geometric-optics term that switches off there (|field| ~ 1/(s + s'))
        J = lambda d: total(bnd - d) - total(bnd + d)  # noqa: E731
        J0 = 2 * J(1e-4) - J(2e-4)
        assert abs(J0) <= 1e-3 * go_jump


# ------------------ validation thresholds t_a, t_d and kappa retries (Table I)
VAL_TX = np.array([0.0, 0.0, 1.0], np.float32)
VAL_RX = np.array([[2.0, 0.0, 1.0]], np.float32)
VAL_N = 20000


def _representative_ray(orc, sc, at_x):
    i = int(np.argmin(np.linalg.norm(sc.pos[:, :2] - np.array([at_x, 0.0]), axis=1)))
    dirs = orc.fib_dirs(VAL_N).astype(np.float64)
    ids, _, q = orc.nearest(sc, np.tile(VAL_TX.astype(np.float64), (VAL_N, 1)), dirs)
    js = np.nonzero(ids == i)[0]
    assert js.size
    return i, int(js[np.argmin(np.linalg.norm(q[js] - sc.pos[i].astype(np.float64), axis=1))])


def _image_length(p, n, tx, rx):
    """Reflection path length over the infinite plane (p, n): |rx - image(tx)|."""
    n = n / np.linalg.norm(n)
    img = tx - 2.0 * ((tx - p) @ n) * n
    return float(np.linalg.norm(rx - img))


@pytest.mark.parametrize("alter,thr,expect", [
    # plane offsets: the validation hit lies dz from the refined plane (t_d = 0.01 m)
    (("offset", 0.005, 1.3), {}, "own"),
    (("offset", 0.015, 1.3), {}, "retry"),
    (("offset", 0.015, 1.3), dict(kappa=0), "none"),
    (("offset", 0.015, 1.3), dict(kappa=1), "retry"),
    (("offset", 0.015, 1.3), dict(t_d=0.02), "own"),
    # tilts about y (t_a = 1 degree): the hit's normal differs by the tilt
    (("tilt", 0.5, 1.3), {}, "own"),
    (("tilt", 1.5, 1.3), {}, "retry"),
    (("tilt", 1.5, 1.3), dict(kappa=0), "none"),
    (("tilt", 1.5, 1.3), dict(t_a_deg=2.0), "own"),
    # a 0.5 degree tilt 1.5 m away: the angle passes, the plane distance (13 mm) does not
    (("tilt", 0.5, 2.5), {}, "retry"),
    (("tilt", 0.5, 2.5), dict(kappa=0), "none"),
])
def test_validation_thresholds_and_retries(orc, alter, thr, expect):
    """Table I thresholds on a hand-built floor. The refinement plane is the
    representative ray's disk, altered here (lifted by dz or tilted); the
    validation ray then meets a flat floor disk. Accepted ("own"): the path
    length is the image-method length over the altered disk's plane.
    Rejected with retries left ("retry"): that plane is replaced by the hit
    disk's (the flat floor) and the path is the flat image path, 2 sqrt 2 m.
    Rejected with kappa = 0 ("none"): no path. A retry rule that re-solves on
    the same plane, an off-by-one in the retry count, t_a read in radians or
    the distance taken from the hit's own plane each fail a case."""
    kind, v, at_x = alter
    sc = scenes.plane_patch(-1.0, 3.0, -1.0, 1.0, 0.05, 0.036)
    i, j = _representative_ray(orc, sc, at_x)
    if kind == "offset":
        sc.pos[i, 2] = v
    else:
        a = math.radians(v)
        sc.normal[i] = [math.sin(a), 0.0, math.cos(a)]
    mats = np.array([[5.0, 0.1, 0.0]])
    f = 3.5e9
    sol = orc.solve(sc, mats, VAL_TX, VAL_RX, f, VAL_N, ray_ids=[j], K=1, flags=SPEC, thr=thr)
    assert sol.seq[0, 0] == i and sol.keys == [(0,)]
    paths = sol.paths(0)
    tx, rx = VAL_TX.astype(np.float64), VAL_RX[0].astype(np.float64)
    if expect == "none":
        assert paths == {}
        return
    if expect == "own":
        L_ref = _image_length(sc.pos[i].astype(np.float64), sc.normal[i].astype(np.float64), tx, rx)
        assert abs(L_ref - 2 * math.sqrt(2)) > 1e-3  # distinguishable from the flat path
    else:
        L_ref = 2 * math.sqrt(2)
    L, ate, atm = paths[(0,)]
    assert abs(L - L_ref) < 1e-9
    # amplitude: boundary-condition Fresnel at the refined plane's incidence cosine
    n = np.array([0.0, 0.0, 1.0]) if expect == "retry" else sc.normal[i].astype(np.float64)
    n /= np.linalg.norm(n)
    p = np.array([0.0, 0.0, 0.0]) if expect == "retry" else sc.pos[i].astype(np.float64)
    img = tx - 2.0 * ((tx - p) @ n) * n
    u = (rx - img) / np.linalg.norm(rx - img)
    te, tm = fresnel_bc(5.0, 0.1, f, abs(u @ n))
    lam = C0 / f
    base = lam / (4 * math.pi) / L_ref * np.exp(-1j * 2 * math.pi / lam * L_ref)
    assert abs(ate - base * te) < 1e-9 * abs(base) and abs(atm - base * tm) < 1e-9 * abs(base)


# --------- diffraction assembly: continuity with the oracle's own GO paths
def _side_limit(x, y, deg=3):
    """Value at 0 of a cubic least-squares fit of complex samples y(x)."""
    return np.polyval(np.polyfit(x, y.real, deg), 0.0) + 1j * np.polyval(np.polyfit(x, y.imag, deg), 0.0)


@pytest.mark.parametrize("mat", ["pec", "concrete"])
@pytest.mark.parametrize("phip_deg,boundary", [(50, "shadow"), (50, "refl0"), (310, "refln"), (310, "shadow"),
                                               (35, "refl0"), (325, "refln")])
def test_diffraction_assembly_continuous_with_the_oracle_paths(orc, mat, phip_deg, boundary):
    """A half-plane of disks (z = 0, x < 0, edge along y) and receivers on a
    1.5 m circle around the edge point, across the incident shadow boundary
    and the reflection boundaries of the top (face 0) and bottom (face n)
    faces. The oracle's own line-of-sight and specular paths (pinned above)
    switch on or off at the boundary; with diffraction() added the field is
    continuous there. The one-sided limits come from cubic fits over samples
    0.02-0.08 rad from the boundary (outside the disks' jagged rim), and their
    difference must be below 0.5 % of the switching path's own jump. The
    field model (lambda/4 pi, the spherical spreading factor, the TE-soft /
    TM-hard mapping, face n's coefficient at n pi - phi) all enter the
    cancellation. The edge is a wedge of interior angle 2e-4 rad (normals
    cannot state a zero-thickness plate's side)."""
    from oracle import diffraction as dif
    plate = scenes.plane_patch(-3.0, 0.0, -2.0, 2.0, 0.02, 0.0144)
    mats = np.array([[1.0, 1e7, 0.0]]) if mat == "pec" else np.array([[5.0, 0.1, 0.0]])
    f, sp, s = 3.5e9, 1.5, 1.5
    dl = 1e-4
    edges = (np.array([[0.0, -1.9, 0.0, 0.0, 1.9, 0.0, math.sin(dl), 0.0, math.cos(dl), math.sin(dl), 0.0,
                        -math.cos(dl)]]), np.array([[0, 0]]))
    phip = math.radians(phip_deg)
    dirv = lambda ph: np.array([-math.cos(ph), 0.0, math.sin(ph)])  # noqa: E731  (angle from face 0)
    tx = (sp * dirv(phip)).astype(np.float32)
    bnd = dict(shadow=(math.pi + phip) % (2 * math.pi), refl0=math.pi - phip, refln=3 * math.pi - phip)[boundary]
    d = np.array([0.02, 0.03, 0.04, 0.05, 0.06, 0.07, 0.08])
    rx = np.array([s * dirv(p) for p in np.concatenate([bnd - d[::-1], bnd + d])], np.float32)
    los = orc.solve(plate, mats, tx, rx, f, 4000, K=1, flags=LOS)
    spec = orc.solve(plate, mats, tx, rx, f, 4000, K=1, flags=SPEC)
    _, hte, htm, _ = dif.diffraction(plate, edges, mats, tx, rx, f)
    m = len(d)
    lit_first = boundary != "refln" if boundary != "shadow" else phip_deg < 180
    switching = los if boundary == "shadow" else spec
    g_sw = switching.G_los if boundary == "shadow" else switching.G_spec
    assert np.all((g_sw[:m] > 0) == lit_first) and np.all((g_sw[m:] > 0) != lit_first)
    other_g = spec.G_spec if boundary == "shadow" else los.G_los
    assert np.all(other_g > 0) or np.all(other_g == 0)  # the other path type does not switch here
    for go, hd in ((switching.h_te, hte), (switching.h_tm, htm)):
        jump = _side_limit(-d[::-1], go[:m] + hd[:m]) - _side_limit(d, go[m:] + hd[m:])
        go_jump = _side_limit(-d[::-1], go[:m]) - _side_limit(d, go[m:])
        assert abs(go_jump) > 1e-4
        assert abs(jump) <= 5e-3 * abs(go_jump), (abs(jump), abs(go_jump))


# ------------------ polarised field (Jones vectors) of line-of-sight and specular paths
POL_FLOOR = dict(x0=-3.0, x1=6.0, y0=-3.0, y1=3.0, spacing=0.05, radius=0.036)
PEC = (1.0, 1e12, 0.0)  # conductivity high enough that 1/sqrt|eta| ~ 4e-7


def _floor():
    f = POL_FLOOR
    return scenes.plane_patch(f["x0"], f["x1"], f["y0"], f["y1"], f["spacing"], f["radius"])


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def _transverse(p, d):
    p = np.asarray(p, float)
    return p - (p @ d) * d


def _floor_path(orc, mat, tx, rx, pol, f=3.5e9, N=2000):
    sol = orc.solve(_floor(), np.array([mat]), tx, [rx], f, N, K=1, flags=LOS | SPEC, pol=pol)
    paths = sol.paths(0)
    assert list(paths) == [(0,)]
    L, ate, atm = paths[(0,)]
    assert ate == atm  # one amplitude, reported in both channels
    tx, rx = np.asarray(tx, float), np.asarray(rx, float)
    img = tx * np.array([1, 1, -1])
    assert abs(L - np.linalg.norm(rx - img)) < 1e-9
    lam = C0 / f
    # the amplitude over the scalar free-space factor of the unfolded path
    return ate / (lam / (4 * math.pi) / L * np.exp(-2j * math.pi / lam * L)), sol


@pytest.mark.parametrize("mat", [PEC, (5.0, 0.1, 0.0), (5.0, 0.1, 0.3)])
@pytest.mark.parametrize("p", [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, 0, 1), (0.3, -0.8, 0.5)])
def test_polarized_normal_incidence_scales_the_field_by_the_normal_coefficient(orc, mat, p):
    """TX straight above RX over a flat floor: the specular path meets the floor
    at normal incidence, where TE and TM are the same wave. The received field
    is the transmitted one (transverse part of the dipole) times
    (1 - sqrt eta) / (1 + sqrt eta) and R = sqrt(1 - S^2), whatever the
    polarisation; for a conductor that is -1: the field reverses."""
    tx, rx = [0.0, 0.0, 1.0], [0.0, 0.0, 2.0]
    pol = (_unit(p), _unit(p))
    ratio, sol = _floor_path(orc, mat, tx, rx, pol)
    eta = mat[0] - 1j * mat[1] / (2 * math.pi * 3.5e9 * EPS0)
    gamma = (1 - np.sqrt(eta)) / (1 + np.sqrt(eta))
    d = np.array([0.0, 0.0, -1.0])
    proj = _transverse(pol[0], d) @ _transverse(pol[1], d)
    expect = math.sqrt(1 - mat[2] ** 2) * gamma * proj
    assert abs(ratio - expect) < 1e-9 * max(1.0, abs(expect))
    if mat is PEC and proj > 0.5:
        assert abs(ratio / proj + 1.0) < 1e-5
    # line of sight: the dipole pattern on both ends, free space in between
    lam = C0 / 3.5e9
    a_los = lam / (4 * math.pi) * np.exp(-2j * math.pi / lam) * proj
    assert abs(sol.G_los[0] - abs(a_los) ** 2) < 1e-12 * abs(a_los) ** 2 + 1e-30


@pytest.mark.parametrize("mat", [(5.0, 0.1, 0.0), (2.5, 0.02, 0.3), (6.3, 0.3, 0.0)])
@pytest.mark.parametrize("rx_x", [2.0, 3.5, 0.75])
def test_polarized_oblique_te_and_tm_from_boundary_conditions(orc, mat, rx_x):
    """One oblique bounce in the x-z plane. TE: dipoles along y (normal to the
    plane of incidence) receive Gamma_TE of the tangential-field boundary
    conditions. TM: vertical dipoles; the incident magnetic field points along
    d_in x E_0 and is scaled by the magnetic-field coefficient of the same
    boundary conditions, and the reflected electric field is H x d_out
    (plane wave, E = Z H x k)."""
    tx, rx = np.array([0.0, 0.0, 1.0]), np.array([rx_x, 0.0, 1.0])
    xr = np.array([rx_x / 2, 0.0, 0.0])  # reflection point (equal heights)
    din, dout = _unit(xr - tx), _unit(rx - xr)
    c = abs(din[2])
    te_bc, tm_bc = fresnel_bc(mat[0], mat[1], 3.5e9, c)
    R = math.sqrt(1 - mat[2] ** 2)
    y = np.array([0.0, 1.0, 0.0])
    ratio_te, _ = _floor_path(orc, mat, tx, rx, (y, y))
    assert abs(ratio_te - R * te_bc) < 1e-9
    z = np.array([0.0, 0.0, 1.0])
    ratio_tm, _ = _floor_path(orc, mat, tx, rx, (z, z))
    e0 = _transverse(z, din)
    e_ref = R * tm_bc * np.cross(np.cross(din, e0), dout)
    expect = e_ref @ _transverse(z, dout)
    assert abs(ratio_tm - expect) < 1e-9 * max(1.0, abs(expect))


def test_polarized_brewster_angle_reflects_no_tm(orc):
    """Lossless floor (eps_r = 4) at the Brewster angle atan 2: the vertical
    dipoles' TM wave is not reflected, the TE wave is."""
    tx, rx = [0.0, 0.0, 1.0], [4.0, 0.0, 1.0]
    mat = (4.0, 0.0, 0.0)
    z, y = np.array([0.0, 0.0, 1.0]), np.array([0.0, 1.0, 0.0])
    r_tm, _ = _floor_path(orc, mat, tx, rx, (z, z))
    r_te, _ = _floor_path(orc, mat, tx, rx, (y, y))
    assert abs(r_tm) < 1e-12 and abs(r_te) > 0.3


@pytest.mark.parametrize("rx", [(2.0, 0.0, 1.0), (3.0, 1.0, 0.5), (0.4, -0.3, 2.5)])
def test_polarized_conductor_cancels_the_tangential_field(orc, rx):
    """On a conductor the tangential electric field vanishes: for any incident
    polarisation, the incident field plus the reflected one (read back as its
    x, y, z components through three receive polarisations) has no component
    in the floor's plane, and the reflected field is transverse to d_out."""
    tx = np.array([0.0, 0.0, 1.0])
    rx = np.asarray(rx, np.float32).astype(float)
    ex = np.eye(3)
    for p in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, -0.2, 0.8]):
        e_k = np.array([_floor_path(orc, PEC, tx, rx, (_unit(p), ex[c]))[0] for c in range(3)])
        t = rx[2] / (tx[2] + rx[2])
        xr = rx + t * (tx * np.array([1, 1, -1]) - rx)  # where the unfolded line meets z = 0
        din, dout = _unit(xr - tx), _unit(rx - xr)
        e0 = _transverse(_unit(p), din)
        tot = e0 + e_k
        assert np.abs(tot[:2]).max() < 1e-5 * np.linalg.norm(e0)
        assert abs(e_k @ dout) < 1e-9


def test_polarized_conducting_room_paths_are_mirror_images(orc, room_holefree):
    """All-conducting hole-free room, paths up to two reflections: a conductor
    maps a field E to 2 (E.n) n - E (tangential part reversed, normal part
    kept), so every path's field is the product of those mirror maps over its
    walls, applied to the transmit dipole's transverse field; the received
    amplitude is its projection on the receive dipole. Paths come from the
    image method on the exact planes."""
    f = 3.5e9
    lam = C0 / f
    mats = np.tile(PEC, (4, 1))
    p_tx, p_rx = _unit([0.3, 0.5, 0.8]), _unit([-0.6, 0.2, 0.7])
    sol = orc.solve(room_holefree, mats, scenes.BOX_TX, [scenes.BOX_RX], f, 20000, K=2, flags=SPEC,
                    pol=(p_tx, p_rx))
    got = sol.paths(0)
    face_of = {0: 0, 1: 1, 2: 2, 3: 3, 4: 4, 5: 5, 6: scenes.BOX_WINDOW["face"], 7: scenes.BOX_DOOR["face"]}
    tx = np.asarray(scenes.BOX_TX, np.float32).astype(float)
    rx = np.asarray(scenes.BOX_RX, np.float32).astype(float)
    checked = 0
    for key, (L, ate, atm) in got.items():
        faces = [face_of[s] for s in key]
        imgs = [tx]
        for fc in faces:
            ax, val = FACE_PLANE[fc]
            q = imgs[-1].copy()
            q[ax] = 2 * val - q[ax]
            imgs.append(q)
        pts = [None] * (len(faces) + 2)
        pts[0], pts[-1] = tx, rx
        cur = rx
        for m in range(len(faces), 0, -1):
            ax, val = FACE_PLANE[faces[m - 1]]
            seg = imgs[m] - cur
            cur = cur + (val - cur[ax]) / seg[ax] * seg
            pts[m] = cur
        assert abs(L - np.linalg.norm(rx - imgs[-1])) < 1e-9
        e = _transverse(p_tx, _unit(pts[1] - pts[0]))
        for fc in faces:
            n = np.zeros(3)
            n[FACE_PLANE[fc][0]] = 1.0
            e = 2 * (e @ n) * n - e
        a_exp = lam / (4 * math.pi) / L * np.exp(-2j * math.pi / lam * L) * (
            e @ _transverse(p_rx, _unit(pts[-1] - pts[-2])))
        assert ate == atm
        assert abs(ate - a_exp) < 1e-5 * np.linalg.norm(e) * lam / (4 * math.pi) / L
        checked += 1
    assert checked >= 20


def test_polarized_two_lossy_bounces_keep_te_and_tm_apart(orc):
    """Floor (z = 0) then ceiling (z = 2), lossy and different, with TX and RX
    in the plane y = 0: both planes of incidence are that plane, so a wave
    normal to it stays TE (Gamma_TE of each bounce, from the boundary
    conditions, multiplies) and vertical dipoles stay TM, the magnetic-field
    relation of the single bounce applied at each reflection with complex
    fields in between."""
    f = 3.5e9
    lam = C0 / f
    floor = scenes.plane_patch(-1.0, 5.0, -2.0, 2.0, 0.05, 0.036, z=0.0, material=0, surface=0)
    ceil = scenes.plane_patch(-1.0, 5.0, -2.0, 2.0, 0.05, 0.036, z=2.0, material=1, surface=1)
    sc = scenes.concat([floor, ceil])
    mats = np.array([[5.0, 0.1, 0.2], [3.0, 0.5, 0.0]])
    tx, rx = np.array([0.0, 0.0, 0.5]), np.array([3.0, 0.0, 1.5])
    i1 = tx * np.array([1, 1, -1])           # image in the floor
    i2 = np.array([i1[0], i1[1], 4.0 - i1[2]])  # then in the ceiling
    p2 = rx + (2.0 - rx[2]) / (i2[2] - rx[2]) * (i2 - rx)
    p1 = p2 + (0.0 - p2[2]) / (i1[2] - p2[2]) * (i1 - p2)
    d0, d1, d2 = _unit(p1 - tx), _unit(p2 - p1), _unit(rx - p2)
    L = np.linalg.norm(rx - i2)
    base = lam / (4 * math.pi) / L * np.exp(-2j * math.pi / lam * L)
    R1 = math.sqrt(1 - 0.2 ** 2)
    te1, tm1 = fresnel_bc(5.0, 0.1, f, abs(d0[2]))
    te2, tm2 = fresnel_bc(3.0, 0.5, f, abs(d1[2]))
    y, z = np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])
    for pol, expect in (((y, y), R1 * te1 * te2),):
        sol = orc.solve(sc, mats, tx, [rx], f, 4000, K=2, flags=SPEC, pol=pol)
        L_got, a, _ = sol.paths(0)[(0, 1)]
        assert abs(L_got - L) < 1e-9
        assert abs(a / base - expect) < 1e-9
    e0 = _transverse(z, d0)
    e1 = R1 * tm1 * np.cross(np.cross(d0, e0), d1)
    e2 = tm2 * np.cross(np.cross(d1, e1), d2)
    sol = orc.solve(sc, mats, tx, [rx], f, 4000, K=2, flags=SPEC, pol=(z, z))
    _, a, _ = sol.paths(0)[(0, 1)]
    expect = e2 @ _transverse(z, d2)
    assert abs(a / base - expect) < 1e-9 * max(1.0, abs(expect))
