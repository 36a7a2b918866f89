"""Build libpcrt.so for gfx950 with hipcc (one object per source, in parallel)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpcrt.so")
# same sources with node-visit / disk-test counters compiled in (measurement only)
LIB_COUNT = os.path.join(HERE, "libpcrt_count.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["api.cpp", "bvh.hip", "trace.hip", "specular.hip", "specular_pol.hip", "field.hip", "tape.hip", "mlp.hip", "sort.hip", "dps.hip", "visibility.hip", "diffraction.hip"]
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC,
    # packed FP32 instructions are kept off for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a multiply and an add fuse only within one source expression, so the
    # rounding of every result follows the source and not the inlining and
    # common-subexpression choices around it (outputs do not move when
    # unrelated code changes; measured at the same speed)
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


def _compile(job) -> str:
    src, variant = job
    obj = os.path.join(BUILD, variant, os.path.splitext(src)[0] + ".o")
    extra = ["-DPCRT_COUNT_VISITS=1"] if variant == "count" else []
    cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def _link(objs, out):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "--offload-arch=" + ARCH, "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    variants = ("prod", "count")
    for v in variants:
        os.makedirs(os.path.join(BUILD, v), exist_ok=True)
    jobs = [(s, v) for v in variants for s in SOURCES]
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, jobs))
    n = len(SOURCES)
    _link(objs[:n], LIB)
    _link(objs[n:], LIB_COUNT)
    if verbose:
        print("built", LIB, LIB_COUNT)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
