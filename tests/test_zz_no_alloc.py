"""pcrt_diffraction_noalloc (the variant for callers that cannot allocate)
against pcrt_diffraction with a caller workspace, through the C ABI: the same
kernels on the same inputs, so outputs must be bitwise identical, on two
calls in a row (the second smaller, so stale scratch contents would show),
with and without the per-pair amplitude output."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2507_04021_amd import scenes

pytestmark = pytest.mark.gpu


def step(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    import paper_2507_04021_amd as P
    sc = scenes.office(target_points=60000)
    sg = P.Scene.from_scene(sc, leaf_size=2, width=4)
    return torch, P, sc, sg


def _both(torch, P, sg, edges_t, n_e, rx, freq, want_pairs):
    L = P.lib()
    dev = sg.device
    mats = P.materials_tensor(scenes.OFFICE_MATERIALS, dev)
    rx_t = torch.as_tensor(np.ascontiguousarray(rx, np.float32), device=dev)
    n_rx = rx_t.shape[0]
    txa = (ctypes.c_float * 3)(*[float(v) for v in scenes.OFFICE_TX])
    nb = ctypes.c_size_t(0)
    assert L.pcrt_diffraction_workspace_size(sg.handle, n_e, n_rx, ctypes.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    out_a = torch.full((n_rx, 5), float("nan"), dtype=torch.float64, device=dev)
    out_b = torch.full((n_rx, 5), float("nan"), dtype=torch.float64, device=dev)
    pa = torch.full((n_rx, n_e, 4), float("nan"), dtype=torch.float32, device=dev) if want_pairs else None
    pb = torch.full((n_rx, n_e, 4), float("nan"), dtype=torch.float32, device=dev) if want_pairs else None
    s = P._stream()
    step("pcrt_diffraction n_edges=%d n_rx=%d pairs=%s" % (n_e, n_rx, want_pairs))
    assert L.pcrt_diffraction(sg.handle, P._ptr(edges_t), n_e, P._ptr(mats), mats.shape[0], txa, P._ptr(rx_t), n_rx,
                              freq, 0.0, P._ptr(ws), ws.numel(), P._ptr(out_a), P._ptr(pa), s) == 0, \
        L.pcrt_last_error()
    step("pcrt_diffraction_noalloc n_edges=%d n_rx=%d pairs=%s" % (n_e, n_rx, want_pairs))
    assert L.pcrt_diffraction_noalloc(sg.handle, P._ptr(edges_t), n_e, P._ptr(mats), mats.shape[0], txa,
                                      P._ptr(rx_t), n_rx, freq, 0.0, P._ptr(out_b), P._ptr(pb), s) == 0, \
        L.pcrt_last_error()
    torch.cuda.synchronize()
    return out_a, out_b, pa, pb


@pytest.mark.parametrize("want_pairs", [False, True])
def test_noalloc_equals_workspace_variant_twice(env, want_pairs):
    torch, P, sc, sg = env
    rows, labels = scenes.office_edges(sc)
    rx = scenes.office_rx()
    big_t, big_n = P.edges_tensor(rows, labels, sg.device)
    small_t, small_n = P.edges_tensor(rows[::3], labels[::3], sg.device)
    for edges_t, n_e, r, f in ((big_t, big_n, rx, 28e9), (small_t, small_n, rx[::5], 3.5e9)):
        a, b, pa, pb = _both(torch, P, sg, edges_t, n_e, r, f, want_pairs)
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
        assert float(a[:, 0].sum()) > 0.0  # some diffracted power reaches the receivers
        if want_pairs:
            assert torch.equal(pa, pb)


def test_noalloc_refuses_beyond_its_scratch(env):
    """A request whose scratch exceeds the fixed 16 MiB is refused on the host
    (before any device work); given pair_amp, only the stack spill counts."""
    torch, P, sc, sg = env
    L = P.lib()
    rows, labels = scenes.office_edges(sc)
    edges_t, n_e = P.edges_tensor(rows, labels, sg.device)
    n_rx = 8192  # 8192 x 160 pairs: 21 MB of amplitudes alone
    nb = ctypes.c_size_t(0)
    assert L.pcrt_diffraction_workspace_size(sg.handle, n_e, n_rx, ctypes.byref(nb)) == 0
    assert nb.value > (16 << 20)
    rx_t = torch.zeros(n_rx, 3, dtype=torch.float32, device=sg.device)
    out = torch.empty(n_rx, 5, dtype=torch.float64, device=sg.device)
    mats = P.materials_tensor(scenes.OFFICE_MATERIALS, sg.device)
    txa = (ctypes.c_float * 3)(*[float(v) for v in scenes.OFFICE_TX])
    step("pcrt_diffraction_noalloc refusal n_rx=%d" % n_rx)
    st = L.pcrt_diffraction_noalloc(sg.handle, P._ptr(edges_t), n_e, P._ptr(mats), mats.shape[0], txa,
                                    P._ptr(rx_t), n_rx, 28e9, 0.0, P._ptr(out), None, P._stream())
    assert st == -4 and b"16777216" in L.pcrt_last_error()
