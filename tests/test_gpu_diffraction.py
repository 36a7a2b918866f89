"""Single-bounce edge diffraction (Sec. II-B.3): GPU library vs the FP64
oracle, through the C ABI.

Bars: the set of (receiver, edge) pairs with a path is identical except where
an FP32 visibility walk and the FP64 test disagree at a disk rim (>= 99 % of
pairs); on pairs both keep, the complex amplitudes agree to 1e-5 relative
(both evaluate the geometry and the coefficient in FP64 from the same FP32
inputs; the GPU stores each amplitude in FP32); per-receiver sums follow.
"""
import sys

import numpy as np
import pytest

from paper_2507_04021_amd import scenes

pytestmark = pytest.mark.gpu


def step(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    import paper_2507_04021_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def small_office():
    return scenes.office(target_points=60000)


@pytest.mark.parametrize("freq,width", [(3.5e9, 4), (28e9, 2), (3.5e9, 8)])
def test_diffraction_matches_oracle(P, small_office, freq, width):
    from oracle import diffraction as dif
    sc = small_office
    edges = scenes.office_edges(sc)
    rx = scenes.office_rx()[::2]
    step("diffraction f=%g width=%d" % (freq, width))
    sg = P.Scene.from_scene(sc, leaf_size=2, width=width)
    out, amp = P.diffraction(sg, edges, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, rx, freq, want_pairs=True)
    G, hte, htm, ref = dif.diffraction(sc, edges, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, rx, freq)
    has_g, has_o = np.abs(amp[..., 0]) > 0, np.abs(ref[..., 0]) > 0
    assert has_o.sum() >= 50
    assert (has_g == has_o).mean() >= 0.99
    both = has_g & has_o
    err = np.abs(amp[both] - ref[both]) / np.abs(ref[both])
    assert err.max() <= 1e-5
    o = out.cpu().numpy()
    same_rx = np.all(has_g == has_o, 1)
    assert same_rx.sum() >= len(rx) // 2
    assert np.allclose(o[same_rx, 0], G[same_rx], rtol=1e-4)
    assert np.allclose(o[same_rx, 1] + 1j * o[same_rx, 2], hte[same_rx], rtol=1e-4, atol=1e-6 * np.abs(hte).max())


def test_diffraction_errors(P, small_office):
    step("diffraction errors")
    sg = P.Scene.from_scene(small_office)
    edges = scenes.office_edges(small_office)
    with pytest.raises(P.PcrtError) as e:
        P.diffraction(sg, edges, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, scenes.office_rx()[:2], -1.0)
    assert e.value.code == -1
