"""Polarised field (Jones vectors, the POLARIZED solve flag) of line-of-sight
and specular paths: GPU library against the CPU oracle, through the C ABI.

Bars:
  - specular (receiver, key) path sets identical on the box room; at the
    office scale a symmetric difference <= 0.1 % of the union;
  - path lengths within 1e-6 (box room) and 2e-6 (office);
  - complex amplitudes within 1e-4 of the path's scale lambda / (4 pi L)
    |pol_tx| |pol_rx| (plus, at 28 GHz, the phase of a 4 um FP32 path-length
    error): the bar is on that scale rather than relative to |a| because a
    projection on the receive polarisation can make a path's amplitude
    arbitrarily small;
  - per-receiver G within 1e-4 relative; coherent h within 1e-4 of the sum
    of the path scales.
"""
import math
import sys

import numpy as np
import pytest

from paper_2507_04021_amd import scenes

pytestmark = pytest.mark.gpu
C0 = 299792458.0
LOS, SPEC, DIFF, REC = 1, 2, 4, 8


def step(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    import paper_2507_04021_amd as P
    P.lib()  # raises if the library is not built: no fallback
    return P


@pytest.fixture(scope="module")
def box(P):
    s = scenes.box_room()
    step("box room scene build")
    return s, P.Scene.from_scene(s)


def gpu_paths(P, res, scene):
    pth = P.paths(res)
    out = {}
    for q in range(pth["n_keys"]):
        key = tuple(int(scene.surface[i]) for i in pth["key_seq"][q, :int(pth["key_len"][q])])
        for r in np.nonzero(pth["valid"][q])[0]:
            out[(int(r), key)] = (float(pth["length"][q, r]), complex(pth["amp_te"][q, r]),
                                  complex(pth["amp_tm"][q, r]))
    return out, pth


def oracle_paths(sol, n_rx):
    return {(r, key): v for r in range(n_rx) for key, v in sol.paths(r).items()}


POLS = [((0, 0, 1), (0, 0, 1)), ((0, 1, 0), (1, 0, 0)), ((0.3, -0.5, 0.8), (0.6, 0.2, -0.4))]


@pytest.mark.parametrize("pol", POLS)
def test_polarized_box_room_matches_the_oracle(P, orc, box, pol):
    """Tiny room, 10k rays, K = 3, 3.5 GHz, line of sight + specular, three
    polarisation pairs (co-polar vertical, crossed horizontal, oblique)."""
    s, sg = box
    f = 3.5e9
    mats = scenes.box_room_materials()
    step("box room polarised %s" % (pol,))
    r = P.solve(sg, mats, scenes.BOX_TX, [scenes.BOX_RX], f, 10000, K=3, flags=LOS | SPEC | REC, pol=pol)
    ref = orc.solve(s, mats, scenes.BOX_TX, [scenes.BOX_RX], f, 10000, K=3, flags=LOS | SPEC, pol=pol)
    gp, _ = gpu_paths(P, r, s)
    op = oracle_paths(ref, 1)
    assert len(op) >= 40
    # a reflection point exactly on the door's (or window's) edge may take either
    # label, FP32 and FP64 deciding differently: such a path may appear under the
    # other label on the other side, with the same length (box-room convention)
    edge = ({2, 7}, {1, 6})
    g_only, o_only = set(gp) - set(op), set(op) - set(gp)
    for k in list(g_only):
        for m in list(o_only):
            if m[0] == k[0] and len(m[1]) == len(k[1]) and abs(gp[k][0] - op[m][0]) <= 1e-6 * op[m][0] and all(
                    a == b or {a, b} in edge for a, b in zip(k[1], m[1])):
                g_only.discard(k)
                o_only.discard(m)
                break
    assert not g_only and not o_only, (g_only, o_only)
    assert len(set(gp) ^ set(op)) <= 2
    scale_pol = np.linalg.norm(pol[0]) * np.linalg.norm(pol[1])
    lam = C0 / f
    amp_sum = 0.0
    for k, (L, a, a2) in op.items():
        if k not in gp:
            continue
        gl, ga, ga2 = gp[k]
        assert a == a2 and ga == ga2  # one amplitude in both channels
        assert abs(gl - L) <= 1e-6 * L
        scale = lam / (4 * math.pi * L) * scale_pol
        amp_sum += scale
        assert abs(ga - a) <= 1e-4 * scale, (k, ga, a)
    # gains and coherent sums, less the edge-tied paths (priced by each side's own amplitude)
    un_g = sum(abs(gp[k][1]) ** 2 for k in set(gp) - set(op))
    un_o = sum(abs(op[k][1]) ** 2 for k in set(op) - set(gp))
    assert abs((r.gain.cpu().numpy()[0] - un_g) / (ref.G[0] - un_o) - 1) < 1e-4
    assert abs(r.parts.cpu().numpy()[0, 0] - ref.G_los[0]) <= 1e-4 * ref.G_los[0] + 1e-30
    h = r.h_te.cpu().numpy()[0]
    h2 = r.h_tm.cpu().numpy()[0]
    assert np.array_equal(h, h2)
    d_los = np.linalg.norm(np.float32(scenes.BOX_RX).astype(float) - np.float32(scenes.BOX_TX).astype(float))
    amp_sum += lam / (4 * math.pi * d_los) * scale_pol
    h_g = complex(*h) - sum(gp[k][1] for k in set(gp) - set(op))
    h_o = ref.h_te[0] - sum(op[k][1] for k in set(op) - set(gp))
    assert abs(h_g - h_o) <= 1e-4 * amp_sum


def test_polarized_office_full_size_specular_paths(P, orc):
    """The bench's office (2^20 rays, K = 5, 64 RX, 28 GHz) with vertical
    dipoles: every valid specular path and 24 rejected keys re-derived by the
    oracle from their representative rays."""
    s = scenes.office(seed=2507)
    rx = scenes.office_rx()
    step("office scene build (%d points)" % s.n)
    sg = P.Scene.from_scene(s, leaf_size=2, width=4)
    N, f = 1 << 20, 28e9
    pol = ((0, 0, 1), (0, 0, 1))
    step("office full solve, polarised, RECORD")
    r = P.solve(sg, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, rx, f, N, K=5, flags=LOS | SPEC | REC, pol=pol)
    gp, pth = gpu_paths(P, r, s)
    valid_keys = np.where(pth["valid"].any(1))[0]
    others = np.random.default_rng(0).choice(np.where(~pth["valid"].any(1))[0], 24, replace=False)
    reps = np.unique(pth["key_ray"][np.concatenate([valid_keys, others])].astype(np.int64))
    step("oracle on %d representative rays" % reps.size)
    ref = orc.solve(s, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, rx, f, N, ray_ids=reps, K=5, flags=SPEC, pol=pol)
    op = oracle_paths(ref, len(rx))
    sel = {tuple(int(s.surface[i]) for i in pth["key_seq"][q, :pth["key_len"][q]]) for q in
           np.concatenate([valid_keys, others])}
    g_sel = {k for k in gp if k[1] in sel}
    o_sel = {k for k in op if k[1] in sel}
    assert len(g_sel) >= 20
    step("paths: %d gpu, %d oracle, %d in one set only" % (len(g_sel), len(o_sel), len(g_sel ^ o_sel)))
    assert len(g_sel ^ o_sel) <= 0.001 * len(g_sel | o_sel)
    lam = C0 / f
    k0 = 2 * math.pi / lam
    for k in g_sel & o_sel:
        (gl, ga, _), (L, a, _) = gp[k], op[k]
        assert abs(gl - L) <= 2e-6 * L
        assert abs(ga - a) <= (1e-4 + k0 * 4e-6) * lam / (4 * math.pi * L), (k, ga, a)


def test_polarized_refusals(P, box):
    """Diffuse paths and the tape are outside the polarised mode; the
    polarisation vectors must be finite."""
    s, sg = box
    mats = scenes.box_room_materials()
    pol = ((0, 0, 1), (0, 0, 1))
    with pytest.raises(P.PcrtError) as e:
        P.solve(sg, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 1000, K=2, flags=LOS | SPEC | DIFF, pol=pol)
    assert e.value.code == -4
    r = P.solve(sg, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 1000, K=2, flags=LOS | SPEC | REC, pol=pol)
    with pytest.raises(P.PcrtError) as e:
        P.tape(r)
    assert e.value.code == -4
    with pytest.raises(P.PcrtError) as e:
        P.solve(sg, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 1000, K=2, flags=LOS | SPEC,
                pol=((0, 0, float("nan")), (0, 0, 1)))
    assert e.value.code == -1


def test_polarized_field_is_bilinear_in_the_polarisations(P, box):
    """Doubling pol_tx and tripling pol_rx multiplies every amplitude by 6
    (the gain by 36); swapping two receive polarisations' roles adds their
    fields: h(p + q) = h(p) + h(q)."""
    s, sg = box
    mats = scenes.box_room_materials()
    args = (sg, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 4000)
    p, q = np.array([0.3, -0.5, 0.8]), np.array([0.6, 0.2, -0.4])
    t = np.array([0.1, 0.9, 0.2])
    a = P.solve(*args, K=2, flags=LOS | SPEC, pol=(t, p))
    b = P.solve(*args, K=2, flags=LOS | SPEC, pol=(2 * t, 3 * p))
    assert abs(b.gain.cpu().numpy()[0] / a.gain.cpu().numpy()[0] - 36.0) < 1e-5
    c = P.solve(*args, K=2, flags=LOS | SPEC, pol=(t, q))
    d = P.solve(*args, K=2, flags=LOS | SPEC, pol=(t, p + q))
    ha, hc, hd = (complex(*x.h_te.cpu().numpy()[0]) for x in (a, c, d))
    assert abs(hd - (ha + hc)) <= 1e-5 * (abs(ha) + abs(hc))
