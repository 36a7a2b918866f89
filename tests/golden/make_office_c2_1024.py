"""Writes office_c2_1024.npz: the oracle's answer for 1024 stratified rays of
the paper-scale office workload (999 312 noisy points, 2^20-ray budget,
K = 5, 64 receivers, 28 GHz, line of sight + specular + diffuse).

Calls only oracle/ (and the seeded scene generator for its inputs); nothing
here touches the GPU library. Run from the repository root:

    python tests/golden/make_office_c2_1024.py

It takes on the order of ten minutes on 8 cores (brute force over every disk
for every query). Stored: the scene's fingerprint, the ray ids, per-ray
interaction sequences and records, diffuse visibility and per-connection
power (lit connections, occluded or not), the unique specular keys with their
representatives, every valid (key, receiver) path (length, hit disks, TE/TM
amplitudes), and the per-receiver gains and coherent fields."""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_04021_amd import scenes  # noqa: E402

N_RAYS, N_SAMPLE, K, FREQ = 1 << 20, 1024, 5, 28e9
OUT = os.path.join(HERE, "office_c2_1024.npz")


def scene_fingerprint(s):
    h = hashlib.sha1()
    for a in (s.pos, s.normal, s.material, s.surface):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.float32(s.radius).tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    s = scenes.office(seed=2507)
    rx = scenes.office_rx()
    ids = scenes.stratified_ray_ids(N_RAYS, N_SAMPLE)
    print("office: %d points; oracle on %d rays x %d receivers ..." % (s.n, ids.size, len(rx)), flush=True)
    sol = oracle.solve(s, scenes.OFFICE_MATERIALS, scenes.OFFICE_TX, rx, FREQ, N_RAYS, ray_ids=ids, K=K,
                       flags=oracle.LOS | oracle.SPECULAR | oracle.DIFFUSE, want_dvis=True, want_dpow=True)
    nk = len(sol.keys)
    keys = np.full((nk, K), -1, np.int64)
    for i, k in enumerate(sol.keys):
        keys[i, :len(k)] = k
    kv, rv = np.nonzero(sol.spec_valid)
    np.savez_compressed(
        OUT, scene_sha1=scene_fingerprint(s), n_points=s.n, n_rays=N_RAYS, K=K, freq=FREQ, ray_ids=ids,
        tx=np.float32(scenes.OFFICE_TX), rx=rx, materials=scenes.OFFICE_MATERIALS,
        seq=sol.seq.astype(np.int32), rec=sol.rec, dvis=np.packbits(sol.dvis.reshape(-1)),
        dvis_shape=np.array(sol.dvis.shape), dpow=sol.dpow.astype(np.float64), keys=keys, key_rep=sol.key_rep,
        path_key=kv, path_rx=rv, path_len=sol.spec_len[kv, rv], path_amp=sol.spec_amp[kv, rv],
        path_hid=sol.spec_hid[kv, rv], G_los=sol.G_los, G_spec=sol.G_spec, G_diff=sol.G_diff, G=sol.G,
        h_te=sol.h_te, h_tm=sol.h_tm)
    print("wrote %s: %d keys, %d valid specular paths, %d visible diffuse connections (%.0f s)"
          % (OUT, nk, kv.size, int(sol.dvis.sum()), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
