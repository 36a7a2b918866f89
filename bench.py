#!/usr/bin/env python3
"""Benchmark of the point-cloud radio ray tracer on one MI355X.

Step = one full scene solve of the paper-scale synthetic office: ~1M noisy
points, 2^20 Fibonacci rays from one transmitter, up to 5 interactions,
64 receivers, 28 GHz, line of sight + specular + diffuse. Inputs (scene,
hierarchy, receivers, materials) are resident on the GPU before the timed
region; the hierarchy build is reported separately.

Prints one JSON line (metric, value = rays*interactions/s, ms_per_step, the
dominant kernel's roofline, the oracle's CPU baseline on a bounded sample).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays·interactions/s and ms per scene solve (1M pts, 5 bounces); grad-step ms"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak (counts packed dual issue)
# the same chip without packed FP32 (disabled in this build): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_NONPACKED_PEAK_TFLOPS = 78.6

# Headline FLOP model (coarse, fixed before any kernel was written): 15 FP32
# operations per child-box slab test, 25 per ray-disk test. The roofline
# fraction of the bench line is this model's FLOPs per launch over the launch
# time, against the published FP32 vector peak.
COARSE_OPS_BOX, COARSE_OPS_DISK = 15, 25


def coarse_flops(cnt, stage, width):
    return cnt[stage + "_nodes"] * width * COARSE_OPS_BOX + cnt[stage + "_disks"] * COARSE_OPS_DISK


# Per-operation FP32 count of the kernels as written (add, mul, min, max,
# compare = 1, a fused multiply-add = 2, as in the FLOP convention), reported
# beside it against the non-packed peak:
#   node visit, width W: W slab tests (per box 6 x (subtract, multiply),
#     6 min/max per axis pair, 6 min/max to combine, 1 compare = 25) and the
#     compares that order the entered children (1 for W = 2; sorting
#     networks of 5 and 19 comparators for W = 4, 8)
#   disk test: plane hit (two dot products, |a| test, divide), hit point,
#     squared distance, radius and t-window compares -> 32
#   visible diffuse connection: distance, cosine, ray-tube amplitude, phase,
#     two complex products, FP64 accumulation -> 60
ORDER_OPS = {2: 1, 4: 5, 8: 19}
OPS_DISK, OPS_DIFFUSE_PATH = 32, 60


def ops_node(width):
    return 25 * width + ORDER_OPS[width]

# HBM traffic of one launch of each traversal kernel on this workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel
# calibration (read x 2.00, write x 1.00), and its L2 hit rate (TCC_HIT /
# (TCC_HIT + TCC_MISS)), with the hash of the sources the measured kernel was
# built from; a figure is reported only while its sources still match.
_CSRC = "paper_2507_04021_amd/csrc/"
TRAFFIC = {
    "k_diffuse": {"bytes": 2047087526, "l2_hit_rate": 0.980,
                  "sources": tuple(_CSRC + f for f in ("common.h", "internal.h", "field.hip", "bvh.hip")),
                  "src_sha256": "8410874cea60a1f9076e51a0a325025136d300afe9d5737e5ef95dd3495685a0"},
    "k_trace": {"bytes": 10116536819, "l2_hit_rate": 0.505,
                "sources": tuple(_CSRC + f for f in ("common.h", "internal.h", "trace.hip", "bvh.hip")),
                "src_sha256": "fb739f401a6570b72102c2dfbef48612751ed02a815505ef5542482615c18322"},
    "k_refine": {"bytes": 10320811085, "l2_hit_rate": 0.481,
                 "sources": tuple(_CSRC + f for f in ("common.h", "internal.h", "refine.h", "specular.hip", "bvh.hip")),
                 "src_sha256": "edccdd494dc47c62a96fff9d50eb96697bc8eab3ad0248d8cfa0917d7e0f6162"},
}


def measured_traffic(kname):
    t = TRAFFIC.get(kname)
    if t and t["src_sha256"] == source_sha256(t["sources"]):
        return t["bytes"], t["l2_hit_rate"]
    return None, None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def office_inputs():
    from paper_2507_04021_amd import scenes
    sc = scenes.office(seed=2507)
    return sc, scenes.office_rx(), np.asarray(scenes.OFFICE_TX, np.float32), scenes.OFFICE_MATERIALS


def algorithmic_bytes(cnt, K, n_rx, stage, width=2):
    """Bytes the method gathers in one launch of a stage's kernel.

    Traversal: per node visited, 32 W bytes of width W for the closest-hit
    walks (7 W floats + pad) and, for the any-hit walks of the diffuse
    connections, 16 + 16 W bytes (the compact node, 16 + 12 W, and its W
    child references; binary nodes: 64 B); 32 B per disk tested (counted by
    the instrumented build). Streams: the trace kernel writes a 48 B record
    per interaction; the diffuse kernel reads every record slot's packed copy
    (32 B) and its index (4 B) once per receiver and writes 40 B of FP64
    partial sums per (ray chunk of 256, receiver).
    """
    nb = 32 * width
    if stage == "trace":
        return cnt["trace_nodes"] * nb + cnt["trace_disks"] * 32 + cnt["interactions"] * 48
    if stage == "diffuse":
        nq = 16 + 16 * width if width > 2 else 64
        chunks = (cnt["rays"] + 255) // 256
        return (cnt["diffuse_nodes"] * nq + cnt["diffuse_disks"] * 32 + chunks * 256 * K * n_rx * 36
                + chunks * n_rx * 40)
    if stage == "refine":
        return cnt["refine_nodes"] * nb + cnt["refine_disks"] * 32
    return 0


def algorithmic_flops(cnt, stage, width=2):
    """FP32 operations one launch of a stage's kernel must perform (counts
    from the instrumented build)."""
    nodes, disks = cnt[stage + "_nodes"], cnt[stage + "_disks"]
    extra = cnt["diffuse"] * OPS_DIFFUSE_PATH if stage == "diffuse" else 0
    return nodes * ops_node(width) + disks * OPS_DISK + extra


def source_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def timed(fn, reps, warm=1):
    """Median device-synchronised wall ms of fn() over reps calls."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def batch_workload(reps):
    """256 transmitter poses along a robot trajectory in the tiny box room,
    ray counts uniform in [2^16, 2^20], K = 2, one graph launch per batch;
    BVH builder, leaf size, node width and rays per wavefront fetch picked by
    the autotuner."""
    import torch
    import paper_2507_04021_amd as P
    from paper_2507_04021_amd import scenes
    s = scenes.box_room()
    mats = scenes.box_room_materials()
    tx, n = scenes.trajectory(seed=4021, n=256)
    choice, rows = P.autotune(s, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 1 << 20, K=2, flags=P.LOS | P.SPECULAR,
                              leaf_sizes=(1, 2, 4, 8), widths=(2, 4, 8), wave_rays=(64, 128, 256), builders=(1, 2),
                              reps=3, cache_path=os.path.join(tempfile.gettempdir(), "pcrt_bench_tuning.json"))
    sg = P.Scene.from_scene(s, leaf_size=choice["leaf_size"], width=choice["width"], builder=choice["builder"])
    graph = P.BatchGraph(sg, mats, tx, n, [scenes.BOX_RX], 3.5e9, K=2, flags=P.LOS | P.SPECULAR,
                         wave_rays=choice["wave_rays"])
    ms = timed(lambda: graph.launch(), reps)
    inter = int(graph.out["counters"][0].item())
    return dict(workload="box room, 256 poses, %d rays total (2^16..2^20 each), K=2, 1 RX, 3.5 GHz, LOS+specular, "
                         "one HIP graph launch" % int(n.sum()),
                batch_ms=ms, ms_per_config=ms / 256, rays_interactions_per_s=inter / (ms / 1e3),
                autotune=choice, autotune_table=rows)


def grad_workload(reps):
    """Material gradient on the box-room geometry with one label per surface
    (8 labels x (eps_r, sigma, S)), 10^4 rays, K = 2, loss = MSE of per-RX
    gain in dB against targets from hidden materials. grad-step = RECORD
    solve + tape forward + loss + backward; train-iter = the same without the
    solve (geometry reused)."""
    import torch
    import paper_2507_04021_amd as P
    from paper_2507_04021_amd import diff, scenes
    s = scenes.box_room(labels="surface")
    sg = P.Scene.from_scene(s)
    rx = np.array([scenes.BOX_RX, [2.0, 3.0, 2.0], [4.5, 0.7, 0.9], [1.5, 2.5, 1.0]], np.float32)
    truth = scenes.hidden_materials(7, 8)
    flags = P.LOS | P.SPECULAR
    target = 10 * torch.log10(P.solve(sg, truth, scenes.BOX_TX, rx, 3.5e9, 10000, K=2, flags=flags).gain)
    guess = torch.tensor(np.tile([5.0, 0.1, 0.0], (8, 1)), dtype=torch.float64, device="cuda", requires_grad=True)
    state = {}

    def step(with_solve):
        if with_solve or "rec" not in state:
            state["rec"] = diff.record(sg, guess.detach(), scenes.BOX_TX, rx, 3.5e9, 10000, K=2, flags=flags)
        guess.grad = None
        loss = diff.db_mse_loss(diff.gains(guess, state["rec"]), target)
        loss.backward()
    return dict(workload="box room, 8 surface labels x 3 parameters, 10^4 rays, K=2, 4 RX, 3.5 GHz, LOS+specular",
                grad_step_ms=timed(lambda: step(True), reps), train_iter_ms=timed(lambda: step(False), reps))


def cir_workload(iters):
    """Material learning from impulse responses (Sec. III-B on a synthetic
    scene): box room, one label per surface (8 labels x (eps_r, sigma, S)),
    1 TX + 6 RX at seeded random positions (seed 5), 6000 rays, K = 2,
    LOS + specular + diffuse, CFR of 129 samples over 1.5 GHz at 8 GHz;
    targets from hidden materials (seed 7, S in [0.1, 0.5]) through the same
    recorded geometry. Adam, lr 0.01, parameters kept in range by sigmoids
    (eps_r in (1, 11), sigma in (0, 1) S/m, S in (0, 1)); each iteration
    draws one receiver at random (seed 0) and minimises Eq. 5 on its CIR.
    Reports the CFR forward / backward kernel times, the iteration time, the
    loss over all receivers before and after, and the recovered parameters'
    mean relative errors (sigma alone is poorly determined where
    sigma / (omega eps0) << eps_r; eta_rel_err is the error of the complex
    permittivity itself)."""
    import torch
    import paper_2507_04021_amd as P
    from paper_2507_04021_amd import diff, scenes
    fc, bw, nf = 8e9, 1.5e9, 129
    s = scenes.box_room(labels="surface")
    sg = P.Scene.from_scene(s)
    tx, rx = scenes.random_links(5, 1, 6)
    tx, rx = tx[0], rx[0]
    truth = scenes.hidden_materials(7, 8, scatter=(0.1, 0.5))
    flags = P.LOS | P.SPECULAR | P.DIFFUSE
    rec = diff.record(sg, np.tile([5.0, 0.1, 0.3], (8, 1)), tx, rx, fc, 6000, K=2, flags=flags)
    with torch.no_grad():
        target = diff.cfr(torch.tensor(truth, dtype=torch.float64, device="cuda"), rec, bw, nf).clone()
    raw = torch.zeros(8, 3, dtype=torch.float64, device="cuda", requires_grad=True)

    def mats_of(raw):
        return torch.stack([1 + 10 * torch.sigmoid(raw[:, 0]), torch.sigmoid(raw[:, 1] - 2.0),
                            torch.sigmoid(raw[:, 2] - 1.0)], 1)

    def full_loss():
        with torch.no_grad():
            return float(diff.cir_loss(diff.cfr(mats_of(raw), rec, bw, nf), target))
    P.tape_fresnel(rec, mats_of(raw).detach())
    fwd_ms = timed(lambda: P.tape_cfr(rec, bw, nf), 5)
    g = torch.ones(rx.shape[0], nf, 2, dtype=torch.complex128, device="cuda")
    bwd_ms = timed(lambda: P.tape_cfr_backward(rec, bw, nf, g), 5)
    loss0 = full_loss()
    opt = torch.optim.Adam([raw], lr=0.01)
    pick = np.random.default_rng(0).integers(0, rx.shape[0], iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        opt.zero_grad()
        r = int(pick[it])
        loss = diff.cir_loss(diff.cfr(mats_of(raw), rec, bw, nf)[r], target[r])
        loss.backward()
        opt.step()
    torch.cuda.synchronize()
    iter_ms = (time.perf_counter() - t0) * 1e3 / iters
    m = mats_of(raw).detach().cpu().numpy()
    rel = np.abs(m - truth) / np.abs(truth)
    we0 = 2 * np.pi * fc * 8.8541878128e-12  # eta = eps_r - j sigma / (omega eps0)
    eta_l, eta_t = m[:, 0] - 1j * m[:, 1] / we0, truth[:, 0] - 1j * truth[:, 1] / we0
    return dict(workload="box room, 8 surface labels x 3 parameters, 1 TX + 6 RX (seed 5), 6000 rays, K=2, "
                         "LOS+specular+diffuse, CFR 129 samples over 1.5 GHz at 8 GHz; Adam lr 0.01, %d iterations, "
                         "one random RX per iteration" % iters,
                cfr_forward_ms=fwd_ms, cfr_backward_ms=bwd_ms, train_iter_ms=iter_ms, loss_first=loss0,
                loss_last=full_loss(), eps_r_rel_err=float(rel[:, 0].mean()), sigma_rel_err=float(rel[:, 1].mean()),
                eta_rel_err=float(np.mean(np.abs(eta_l - eta_t) / np.abs(eta_t))),
                scatter_rel_err=float(rel[:, 2].mean()))


def dps_workload(sc, rx, tx, mats, rays, reps, leaf, width, builder):
    """The office solve with the paper's point-set parameters (Table I: voxel
    0.0625 m, point radius 0.015 m, depth attenuation 100 /m): weighted-average
    interactions against plain nearest-disk interactions on the same scene."""
    import dataclasses
    import torch
    import paper_2507_04021_amd as P
    sc15 = dataclasses.replace(sc, radius=0.015)
    scene = P.Scene.from_scene(sc15, leaf_size=leaf, width=width, builder=builder, dps_voxel=0.0625)
    dev = torch.device("cuda")
    mats_t = P.materials_tensor(mats, dev)
    rx_t = torch.as_tensor(rx, device=dev)
    out = {}
    for name, fl in (("average", P.LOS | P.SPECULAR | P.DIFFUSE | P.AVERAGE), ("plain", P.LOS | P.SPECULAR | P.DIFFUSE)):
        res = P.solve(scene, mats_t, tx, rx_t, 28e9, rays, K=5, flags=fl, lambda_d=100.0)
        o = dict(gain=res.gain, h_te=res.h_te, h_tm=res.h_tm, parts=res.parts, seq=None, counters=res.counters)
        torch.cuda.synchronize()
        stage = {k: 0.0 for k in P.STAGES}
        t0 = time.perf_counter()
        for _ in range(reps):
            P.solve(scene, mats_t, tx, rx_t, 28e9, rays, K=5, flags=fl | P.TIMING, ws=res.ws, out=o, lambda_d=100.0)
            for k, v in P.stage_times().items():
                stage[k] += v
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        cnt = {k: int(o["counters"][i].item()) for k, i in P.CNT.items()}
        out[name] = dict(ms_per_solve=ms, stage_ms={k: v / reps for k, v in stage.items()},
                         counts={k: cnt[k] for k in ("interactions", "keys", "candidates", "specular", "diffuse")},
                         gain_db_mean=float(10 * torch.log10(o["gain"]).mean().item()))
    # visibility matrix: every receiver against every set's reception point
    vis = P.visibility(scene, rx_t)
    nb = ctypes.c_size_t(0)
    P.lib().pcrt_visibility_workspace_size(scene.handle, ctypes.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        P.visibility(scene, rx_t, ws=ws, out=vis)
    e1.record()
    torch.cuda.synchronize()
    vms = e0.elapsed_time(e1) / reps
    n_seg = len(rx) * scene.info["n_point_sets"]
    out["visibility_matrix"] = dict(ms=vms, segments=n_seg, segments_per_s=n_seg / (vms / 1e3),
                                    visible_fraction=float(vis.float().mean().item()))
    # the paper's launch: one ray per set towards its reception point, candidates gated by the matrix
    ns = scene.info["n_point_sets"]
    fl = P.LOS | P.SPECULAR | P.DIFFUSE | P.AVERAGE | P.DPS_LAUNCH
    res = P.solve(scene, mats_t, tx, rx_t, 28e9, ns, K=5, flags=fl, lambda_d=100.0, dps_vis=vis)
    o = dict(gain=res.gain, h_te=res.h_te, h_tm=res.h_tm, parts=res.parts, seq=None, counters=res.counters)
    torch.cuda.synchronize()
    stage = {k: 0.0 for k in P.STAGES}
    t0 = time.perf_counter()
    for _ in range(reps):
        P.solve(scene, mats_t, tx, rx_t, 28e9, ns, K=5, flags=fl | P.TIMING, ws=res.ws, out=o, lambda_d=100.0,
                dps_vis=vis)
        for k, v in P.stage_times().items():
            stage[k] += v
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    cnt = {k: int(o["counters"][i].item()) for k, i in P.CNT.items()}
    out["reception_point_launch"] = dict(
        workload="%d rays (one per set), K=5, 64 RX, LOS+specular+diffuse, averaged interactions, candidates "
                 "gated by the visibility matrix, diffuse paths deduplicated per voxel (area rho^2)" % ns,
        ms_per_solve=ms, stage_ms={k: v / reps for k, v in stage.items()},
        counts={k: cnt[k] for k in ("interactions", "keys", "candidates", "specular", "diffuse")})
    return dict(workload="office as above with point radius 0.015 m, voxel 0.0625 m, lambda_d 100 /m, %d rays, "
                         "K=5, 64 RX, LOS+specular+diffuse" % rays,
                n_point_sets=scene.info["n_point_sets"], build_ms=scene.info["build_ms"], **out)


def diffraction_workload(sc, rx, tx, mats, reps, leaf, width, builder):
    """Single-bounce edge diffraction over the office furniture's 160 convex
    edges to the 64 receivers (one HIP-event-timed call per repetition)."""
    import torch
    import paper_2507_04021_amd as P
    from paper_2507_04021_amd import scenes
    scene = P.Scene.from_scene(sc, leaf_size=leaf, width=width, builder=builder)
    rows, labels = scenes.office_edges(sc)
    e_t = P.edges_tensor(rows, labels)
    mats_t = P.materials_tensor(mats)
    rx_t = torch.as_tensor(rx, device="cuda")
    out, _ = P.diffraction(scene, e_t, mats_t, tx, rx_t, 28e9)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        out, _ = P.diffraction(scene, e_t, mats_t, tx, rx_t, 28e9)
    e1.record()
    torch.cuda.synchronize()
    _, amp = P.diffraction(scene, e_t, mats_t, tx, rx_t, 28e9, want_pairs=True)
    o = out.cpu().numpy()
    return dict(workload="office furniture, %d convex edges x %d RX, 28 GHz, UTD wedge coefficient" % (len(rows), len(rx)),
                ms=e0.elapsed_time(e1) / reps, pairs=len(rows) * len(rx),
                paths=int((np.abs(amp[..., 0]) > 0).sum()),
                gain_db_mean=float(np.mean(10 * np.log10(np.maximum(o[:, 0], 1e-30)))))


def mlp_workload(iters):
    """Learned materials: box room with one label per surface (8 labels);
    512 channel sets, 256 at 3.5 GHz and 256 at 28 GHz, each 1 TX + 8 RX at
    seeded random positions (seed 11); targets from hidden per-label
    materials (seed 7). 448 sets train the network through their recorded
    tapes (Adam, 8 sets per iteration), 64 are held out. Reports the held-out
    mean |dG| in dB for the nominal per-label Fresnel model (the method
    without the learned part), for the per-label Fresnel model fitted
    through the same tapes by the gradient kernels (300 Adam iterations of 8
    sets), and for the trained network, the training
    iteration time, and the BF16 MFMA forward / backward kernels' throughput
    on 2^20 interaction rows."""
    import torch
    import paper_2507_04021_amd as P
    from paper_2507_04021_amd import diff, mlp as M, scenes
    s = scenes.box_room(labels="surface")
    sg = P.Scene.from_scene(s)
    truth = scenes.hidden_materials(7, 8, scatter=(0.1, 0.5))
    nominal = scenes.box_room_materials("surface", scatter=0.2)
    n_sets, rays, flags = 512, 3000, P.LOS | P.SPECULAR | P.DIFFUSE
    tx, rx = scenes.random_links(11, n_sets, 8)
    sets = []
    t0 = time.perf_counter()
    for i in range(n_sets):
        f = 3.5e9 if i < n_sets // 2 else 28e9
        tgt = 10 * torch.log10(P.solve(sg, truth, tx[i], rx[i], f, rays, K=2, flags=flags).gain)
        sets.append((diff.record(sg, nominal, tx[i], rx[i], f, rays, K=2, flags=flags), f, tgt))
    torch.cuda.synchronize()
    rec_s = time.perf_counter() - t0
    order = np.random.default_rng(11).permutation(n_sets)
    train_sets, held = [sets[i] for i in order[:448]], [sets[i] for i in order[448:]]
    net = M.MaterialMLP(M.init_params(8, seed=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = M.train(net, train_sets, iters=iters, batch=8, lr=5e-3)
    torch.cuda.synchronize()
    iter_ms = (time.perf_counter() - t0) * 1e3 / iters
    e_mlp = float(torch.cat([M.db_error(net.gains(r, f), t) for r, f, t in held]).mean())
    e_nom = []
    for r, f, t in held:
        P.tape_fresnel(r, nominal)
        e_nom.append(M.db_error(P.tape_forward(r)[0], t))
    e_nom = float(torch.cat(e_nom).mean())
    # the per-label Fresnel model fitted through the same tapes (the gradient kernels), judged the same way
    t0 = time.perf_counter()
    fitted, fit_hist = diff.fit_per_label(train_sets, nominal, iters=iters, batch=8, lr=0.05)
    fit_s = time.perf_counter() - t0
    e_fit = []
    for r, f, t in held:
        P.tape_fresnel(r, fitted)
        e_fit.append(M.db_error(P.tape_forward(r)[0], t))
    e_fit = float(torch.cat(e_fit).mean())
    out = dict(workload="box room, 8 surface labels, 512 channel sets (256 at 3.5 GHz, 256 at 28 GHz), 1 TX + 8 RX "
                        "each, %d rays, K=2, LOS+specular+diffuse; 448 train / 64 held out" % rays,
               record_s=rec_s, train_iters=iters, train_iter_ms=iter_ms, loss_first=hist[0], loss_last=hist[-1],
               heldout_db_error_nominal=e_nom, heldout_db_error_mlp=e_mlp, heldout_db_error_fitted_per_label=e_fit,
               fitted_per_label_s=fit_s, fitted_loss_last=fit_hist[-1],
               fitted_materials_max_rel_err=float(np.max(np.abs(fitted[:, :2] - truth[:, :2]) / truth[:, :2])))
    out.update(mlp_kernels(net, 1 << 20, reps=5))
    return out


def mlp_kernels(net, n, reps):
    """Throughput of the BF16 MFMA forward and backward kernels on n seeded
    interaction rows (8 labels, 28 GHz)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(3)
    lab = torch.randint(0, 8, (n,), device="cuda", generator=g).to(torch.int16)
    cs = torch.rand(n, device="cuda", generator=g)
    out = torch.empty(n, 8, device="cuda")
    g_out = torch.randn(n, 8, device="cuda", generator=g)
    f_ms = timed(lambda: net.forward_rows(lab, cs, 28e9, out), reps)
    b_ms = timed(lambda: net.backward_rows(lab, cs, 28e9, g_out), reps)
    # per row: forward 2 x (32x64 + 64x64 + 64x64 + 64x16) flops; backward =
    # forward recompute + input-gradient chain + weight gradients (3 x forward)
    fw = 2 * (32 * 64 + 64 * 64 + 64 * 64 + 64 * 16)
    return dict(mlp_forward_ms_1M_rows=f_ms, mlp_backward_ms_1M_rows=b_ms,
                mlp_forward_tflops=fw * n / (f_ms / 1e3) / 1e12, mlp_backward_tflops=3 * fw * n / (b_ms / 1e3) / 1e12,
                mfma_bf16_peak_tflops=2500.0)


def cpu_baseline(sc, rx, tx, mats, n_budget, K, n_sample):
    import oracle
    from paper_2507_04021_amd import scenes
    oracle.build(force=False)
    ids = scenes.stratified_ray_ids(n_budget, n_sample)
    t0 = time.perf_counter()
    sol = oracle.solve(sc, mats, tx, rx, 28e9, n_budget, ray_ids=ids, K=K, flags=7)
    dt = time.perf_counter() - t0
    inter = int((sol.seq >= 0).sum())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=inter / dt, unit="rays·interactions/s", cores=cores, kind="oracle",
                sample="%d stratified rays of 2^20 (all 64 RX, LOS+specular+diffuse, K=%d): %d interactions "
                       "in %.1f s" % (n_sample, K, inter, dt), wall_s=dt,
                # the whole 2^20-ray solve at the sample's time per ray (approximate: the bounce loop and the
                # diffuse connections scale with the rays; the specular refinement grows more slowly, since
                # rays share keys)
                extrapolated_full_solve_s=dt * n_budget / n_sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--leaf", type=int, default=2)
    ap.add_argument("--width", type=int, default=4, help="BVH node width (2, 4, 8)")
    ap.add_argument("--builder", type=int, default=0, help="BVH builder: 0 default, 1 radix tree, 2 clustering")
    ap.add_argument("--rays", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--mlp-iters", type=int, default=300)
    ap.add_argument("--cir-iters", type=int, default=5000, help="Adam iterations of the impulse-response learning (the paper runs 5000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batch and gradient workloads")
    ap.add_argument("--mlp-kernels-only", action="store_true",
                    help="only time the MLP forward / backward kernels on 2^20 rows (profiling)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates the profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (rays would shard by "
              "strided ranges with one all-reduce of per-receiver sums; not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_04021_amd as P

    if args.mlp_kernels_only:
        from paper_2507_04021_amd import mlp as M
        print(json.dumps(mlp_kernels(M.MaterialMLP(M.init_params(8, seed=0)), 1 << 20, reps=max(3, args.steps))),
              flush=True)
        return
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    K, freq = 5, 28e9
    flags = P.LOS | P.SPECULAR | P.DIFFUSE
    sc, rx, tx, mats = office_inputs()
    log("office scene: %d points, %d surfaces" % (sc.n, sc.n_surfaces))
    dev = torch.device("cuda")
    scene = P.Scene.from_scene(sc, leaf_size=args.leaf, width=args.width, builder=args.builder)
    torch.cuda.synchronize()
    log("hierarchy:", scene.info)
    mats_t = P.materials_tensor(mats, dev)
    rx_t = torch.as_tensor(rx, device=dev)
    res = P.solve(scene, mats_t, tx, rx_t, freq, args.rays, K=K, flags=flags)
    ws = res.ws
    out = dict(gain=res.gain, h_te=res.h_te, h_tm=res.h_tm, parts=res.parts, seq=None, counters=res.counters)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        P.solve(scene, mats_t, tx, rx_t, freq, args.rays, K=K, flags=flags, ws=ws, out=out)
    torch.cuda.synchronize()
    log("warmup done")

    stage_sum = {k: 0.0 for k in P.STAGES}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.solve(scene, mats_t, tx, rx_t, freq, args.rays, K=K, flags=flags | P.TIMING, ws=ws, out=out)
        st = P.stage_times()  # waits for this step's last event
        for k, v in st.items():
            stage_sum[k] += v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cnt = {k: int(out["counters"][i].item()) for k, i in P.CNT.items()}
    stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
    log("stages ms:", {k: round(v, 3) for k, v in stage_ms.items()})
    log("counters:", cnt)
    value = cnt["interactions"] / (ms / 1e3)

    # algorithmic bytes from one instrumented solve (same inputs, same results)
    P.use_counting(True)
    scene_c = P.Scene.from_scene(sc, leaf_size=args.leaf, width=args.width, builder=args.builder)
    rc = P.solve(scene_c, mats_t, tx, rx_t, freq, args.rays, K=K, flags=flags)
    torch.cuda.synchronize()
    ccnt = {k: int(rc.counters[i].item()) for k, i in P.CNT.items()}
    P.use_counting(False)
    del scene_c, rc
    dom = max(("trace", "refine", "diffuse"), key=lambda k: stage_ms[k])
    kname = {"trace": "k_trace", "refine": "k_refine", "diffuse": "k_diffuse"}[dom]
    nbytes = algorithmic_bytes(ccnt, K, len(rx), dom, args.width)
    launch_s = stage_ms[dom] / 1e3
    flops = coarse_flops(ccnt, dom, args.width)
    achieved = flops / launch_s / 1e12
    op_flops = algorithmic_flops(ccnt, dom, args.width)
    traffic, l2_hit = measured_traffic(kname)
    stage_traffic = {}
    for st, kn in (("trace", "k_trace"), ("refine", "k_refine"), ("diffuse", "k_diffuse")):
        b, h = measured_traffic(kn)
        stage_traffic[st] = None if b is None else {
            "bytes": b, "GBs": b / (stage_ms[st] / 1e3) / 1e9,
            "hbm_frac": b / (stage_ms[st] / 1e3) / 1e9 / HBM_PEAK_GBS, "l2_hit_rate": h}
    log("visit counters:", {k: ccnt[k] for k in ccnt if "nodes" in k or "disks" in k})

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays·interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "office 12x8x3 m, 20 boxes, %d noisy points (5 mm, 3 deg), 8 materials, 1 TX, 64 RX, "
                        "%d rays, K=5, 28 GHz, LOS+specular+diffuse" % (sc.n, args.rays),
            "leaf_size": args.leaf,
            "bvh_width": args.width,
            "bvh_builder": scene.info["builder"],
        },
        "roofline": {
            "bound": "alu",
            "kernel": kname,
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "flop_model": "%d per child-box slab test, %d per ray-disk test (instrumented visit counts)"
                          % (COARSE_OPS_BOX, COARSE_OPS_DISK),
            "algorithmic_flops_per_launch": flops,
            "launch_ms": stage_ms[dom],
            # the kernels' own per-operation count against the non-packed FP32 rate
            "op_count_flops_per_launch": op_flops,
            "op_count_tflops": op_flops / launch_s / 1e12,
            "op_count_frac_nonpacked": op_flops / launch_s / 1e12 / FP32_NONPACKED_PEAK_TFLOPS,
            # HBM: measured bytes per launch (profiler counters) over the live launch time
            "hbm_GBs": traffic / launch_s / 1e9 if traffic else None,
            "hbm_frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "l2_hit_rate": l2_hit,
            # the bytes the walks gather (nodes, disks, records), served almost entirely by the caches
            "gathered_bytes_per_launch": nbytes,
            "gather_GBs_cache_served": nbytes / launch_s / 1e9,
        },
        "stage_ms": stage_ms,
        # measured L2-to-memory traffic of each traversal kernel over its live launch time
        "stage_traffic": stage_traffic,
        "bvh_build_ms": scene.info["build_ms"],
        "counts": {k: cnt[k] for k in ("rays", "interactions", "segments", "keys", "candidates", "specular",
                                       "diffuse", "tie_spill", "status")},
        "shadow_segments_per_s": cnt["segments"] / (ms / 1e3),
    }
    if not args.no_extras:
        log("batch workload...")
        line["batch"] = batch_workload(max(3, args.steps // 2))
        log("gradient workload...")
        line["grad"] = grad_workload(max(5, args.steps))
        log("learned-material workload...")
        line["mlp"] = mlp_workload(args.mlp_iters)
        log("impulse-response learning workload...")
        line["cir"] = cir_workload(args.cir_iters)
        log("edge diffraction workload...")
        line["diffraction"] = diffraction_workload(sc, rx, tx, mats, max(3, args.steps // 2), args.leaf, args.width,
                                                   args.builder)
        log("point-set averaging workload...")
        line["dps"] = dps_workload(sc, rx, tx, mats, args.rays, max(3, args.steps // 2), args.leaf, args.width,
                                   args.builder)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on %d rays..." % args.cpu_sample)
        line["cpu_baseline"] = cpu_baseline(sc, rx, tx, mats, args.rays, K, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
