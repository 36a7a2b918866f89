"""C ABI of libpcrt on the CPU: the library loads, exports every function that
include/pcrt.h declares, and rejects bad arguments on the host before any
device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2507_04021_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcrt.h")
EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = -1, -2, -3, -4


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pcrt_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libpcrt.so is not built; run __graft_entry__.build()")
    return P.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("pcrt_scene_create", "pcrt_solve", "pcrt_solve_workspace_size", "pcrt_paths_copy",
              "pcrt_raygen", "pcrt_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    if os.path.exists(P.LIB_COUNT_PATH):
        Lc = P.lib("count")
        assert not [n for n in declared_functions() if not hasattr(Lc, n)]


def test_version(L):
    assert b"gfx950" in L.pcrt_version()


def test_scene_argument_errors(L):
    nb = ctypes.c_size_t(0)
    assert L.pcrt_scene_workspace_size(0, None, ctypes.byref(nb)) == EINVAL
    assert b"n_points" in L.pcrt_last_error()
    assert L.pcrt_scene_workspace_size(10, None, None) == EINVAL
    assert L.pcrt_scene_workspace_size(1 << 28, None, ctypes.byref(nb)) == EUNSUPPORTED
    # node and disk arrays are addressed with 32-bit byte offsets: at most 2^26 points
    assert L.pcrt_scene_workspace_size((1 << 26) + 1, None, ctypes.byref(nb)) == EUNSUPPORTED
    assert b"2^26" in L.pcrt_last_error()
    assert L.pcrt_scene_workspace_size(1 << 26, None, ctypes.byref(nb)) == 0
    assert L.pcrt_scene_workspace_size(1000, None, ctypes.byref(nb)) == 0 and nb.value > 1000 * 64
    o = P.BvhOpts(4, 2, 1)
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == 0
    binary = nb.value
    for w in (4, 8):  # wide nodes add their own array (32 W bytes per binary internal node) and build buffers
        o = P.BvhOpts(4, w, 1)
        assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == 0
        assert nb.value >= binary + 999 * 32 * w
    for w in (1, 3, 16):
        o = P.BvhOpts(4, w)
        assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == EUNSUPPORTED
        assert b"width" in L.pcrt_last_error()
    o = P.BvhOpts(9, 2)
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == EUNSUPPORTED
    o = P.BvhOpts(4, 2, 3)  # builders are 1 (radix tree) and 2 (clustering)
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == EUNSUPPORTED
    o = P.BvhOpts(4, 2, 2)  # the clustering build needs its own buffers
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(o), ctypes.byref(nb)) == 0 and nb.value > binary
    h = ctypes.c_void_p()
    fake = 0x1000  # never dereferenced: argument checks run first
    pts = P.Points(fake, fake, fake, fake, 10, 0.0)
    assert L.pcrt_scene_create(ctypes.byref(pts), None, ctypes.c_void_p(fake), 1 << 20, None,
                               ctypes.byref(h)) == EINVAL
    assert b"disk_radius" in L.pcrt_last_error()
    pts = P.Points(fake, None, fake, fake, 10, 0.1)
    assert L.pcrt_scene_create(ctypes.byref(pts), None, ctypes.c_void_p(fake), 1 << 20, None,
                               ctypes.byref(h)) == EINVAL
    pts = P.Points(fake, fake, fake, fake, 0, 0.1)
    assert L.pcrt_scene_create(ctypes.byref(pts), None, ctypes.c_void_p(fake), 1 << 20, None,
                               ctypes.byref(h)) == EINVAL
    pts = P.Points(fake, fake, fake, fake, 10, 0.1)
    opts = P.BvhOpts(9, 0)
    assert L.pcrt_scene_create(ctypes.byref(pts), ctypes.byref(opts), ctypes.c_void_p(fake), 1 << 20, None,
                               ctypes.byref(h)) == EUNSUPPORTED
    opts = P.BvhOpts(4, 3)  # widths are 2, 4 or 8
    assert L.pcrt_scene_create(ctypes.byref(pts), ctypes.byref(opts), ctypes.c_void_p(fake), 1 << 20, None,
                               ctypes.byref(h)) == EUNSUPPORTED
    # workspace too small: the required size is in the message
    assert L.pcrt_scene_create(ctypes.byref(pts), None, ctypes.c_void_p(fake), 16, None,
                               ctypes.byref(h)) == ENOMEM
    assert b"need" in L.pcrt_last_error()
    # point sets: a negative or non-finite voxel edge is refused; a positive one adds 44+ bytes per point
    for bad in (-0.1, float("nan"), float("inf")):
        opts = P.BvhOpts(4, 4, 2, bad)
        assert L.pcrt_scene_create(ctypes.byref(pts), ctypes.byref(opts), ctypes.c_void_p(fake), 1 << 30, None,
                                   ctypes.byref(h)) == EINVAL
        assert b"dps_voxel" in L.pcrt_last_error()
    plain, sets = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(P.BvhOpts(4, 4, 2)), ctypes.byref(plain)) == 0
    assert L.pcrt_scene_workspace_size(1000, ctypes.byref(P.BvhOpts(4, 4, 2, 0.0625)), ctypes.byref(sets)) == 0
    assert sets.value >= plain.value + 1000 * 44


def test_solve_argument_errors(L):
    p = P.SolveParams()
    assert L.pcrt_solve(None, None, 0, ctypes.byref(p), None, 0, None, None) == EINVAL
    nb = ctypes.c_size_t(0)
    assert L.pcrt_solve_workspace_size(None, ctypes.byref(p), ctypes.byref(nb)) == EINVAL
    assert L.pcrt_raygen(0, None, 10, None, None) == EINVAL
    ms = (ctypes.c_double * 6)()
    assert L.pcrt_stage_times(ms, 6) == EINVAL
    assert L.pcrt_scene_get_info(None, None) == EINVAL
    assert L.pcrt_reception_points(None, None, None) == EINVAL
    assert L.pcrt_visibility_workspace_size(None, ctypes.byref(nb)) == EINVAL
    assert L.pcrt_visibility(None, None, 1, 0.0, None, 0, None, None) == EINVAL
    assert L.pcrt_diffraction_workspace_size(None, 1, 1, ctypes.byref(nb)) == EINVAL
    assert L.pcrt_diffraction(None, None, 1, None, 1, None, None, 1, 1e9, 0.0, None, 0, None, None, None) == EINVAL
    assert L.pcrt_tape_cfr(None, ctypes.byref(p), None, 1.5e9, 129, None, None) == EINVAL
    assert L.pcrt_tape_cfr_backward(None, ctypes.byref(p), None, 1.5e9, 129, None, None) == EINVAL
    assert L.pcrt_last_error()  # an explanation is always set on failure


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    """No silent fallback: a missing build raises on use."""
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(P, "_libs", {})
    with pytest.raises(ImportError):
        P.lib()


STRUCTS = [("pcrt_points", "Points"), ("pcrt_bvh_opts", "BvhOpts"), ("pcrt_scene_info", "SceneInfo"),
           ("pcrt_thresholds", "Thresholds"), ("pcrt_solve_params", "SolveParams"), ("pcrt_batch_item", "BatchItem"),
           ("pcrt_tuning", "Tuning"), ("pcrt_mlp", "Mlp"), ("pcrt_tape", "Tape"), ("pcrt_outputs", "Outputs"),
           ("pcrt_edge", "Edge")]


def test_binding_structs_match_the_header(tmp_path):
    """Size and every field offset of the binding's ctypes mirrors equal what a
    C compiler makes of include/pcrt.h."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pcrt.h"', "int main(void) {"]
    for cname, pname in STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in getattr(P, pname)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, pname in STRUCTS:
        cls = getattr(P, pname)
        assert int(got["%s size" % cname]) == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert int(got["%s %s" % (cname, f[0])]) == getattr(cls, f[0]).offset, (cname, f[0])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching the GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_status_poll_decodes_every_bit(L):
    """pcrt_status_poll: host-only decoding of the device status word."""
    EOVERFLOW = -5
    c = (ctypes.c_uint64 * 16)()
    assert L.pcrt_status_poll(c) == 0
    assert L.pcrt_status_poll(None) == EINVAL
    c[6] = 1
    assert L.pcrt_status_poll(c) == EOVERFLOW and b"key table" in L.pcrt_last_error()
    c[6] = 4
    assert L.pcrt_status_poll(c) == EOVERFLOW and b"key_capacity" in L.pcrt_last_error()
    c[6] = 2
    assert L.pcrt_status_poll(c) == EINVAL and b"material label" in L.pcrt_last_error()
    c[6] = 7  # every condition is named; the invalid label decides the code
    assert L.pcrt_status_poll(c) == EINVAL
    msg = L.pcrt_last_error()
    assert b"key table" in msg and b"key_capacity" in msg and b"material label" in msg
    c[6] = 0
    c[0] = 123  # other counters are not status
    assert L.pcrt_status_poll(c) == 0
