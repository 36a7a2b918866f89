"""Batched transmitters in one launch sequence, HIP-graph replay, autotuner."""
import numpy as np
import pytest

from paper_2507_04021_amd import scenes

pytestmark = pytest.mark.gpu
LOS, SPEC, DIFF = 1, 2, 4


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2507_04021_amd as P
    s = scenes.box_room()
    return torch, P, s, P.Scene.from_scene(s)


@pytest.mark.parametrize("flags", [LOS | SPEC, LOS | SPEC | DIFF])
def test_batch_equals_single_solves(env, flags):
    """Each item reduces over its own fixed chunks, so a batched item is
    bitwise equal to the same transmitter solved alone."""
    torch, P, s, sg = env
    tx, n = scenes.trajectory(seed=4021, n=7, min_rays=300, max_rays=5000)
    rx = np.array([scenes.BOX_RX, [2.5, 2.0, 2.2]], np.float32)
    mats = scenes.box_room_materials(scatter=0.3 if flags & DIFF else 0.0)
    print("[gpu-test] batch of %d items, flags %d" % (len(n), flags), flush=True)
    b = P.solve_batch(sg, mats, tx, n, rx, 3.5e9, K=2, flags=flags)
    g = b.gain.cpu().numpy()
    assert b.counter("rays") == int(n.sum())
    for i in range(len(n)):
        r = P.solve(sg, mats, tx[i], rx, 3.5e9, int(n[i]), K=2, flags=flags)
        assert np.array_equal(r.gain.cpu().numpy(), g[i]), i
        assert np.array_equal(r.h_te.cpu().numpy(), b.h_te.cpu().numpy()[i]), i


def test_batch_matches_oracle(env, orc):
    torch, P, s, sg = env
    tx, n = scenes.trajectory(seed=5, n=3, min_rays=2000, max_rays=4000)
    mats = scenes.box_room_materials()
    print("[gpu-test] batch vs oracle", flush=True)
    b = P.solve_batch(sg, mats, tx, n, [scenes.BOX_RX], 3.5e9, K=2, flags=LOS | SPEC)
    for i in range(3):
        ref = orc.solve(s, mats, tx[i], [scenes.BOX_RX], 3.5e9, int(n[i]), K=2, flags=LOS | SPEC)
        assert abs(b.gain.cpu().numpy()[i, 0] / ref.G[0] - 1) < 1e-4


def test_graph_replays_match_eager(env):
    torch, P, s, sg = env
    tx, n = scenes.trajectory(seed=4021, n=16, min_rays=1000, max_rays=8000)
    rx = [scenes.BOX_RX]
    mats = scenes.box_room_materials()
    print("[gpu-test] graph capture", flush=True)
    eager = P.solve_batch(sg, mats, tx, n, rx, 3.5e9, K=2, flags=LOS | SPEC)
    ref = eager.gain.clone()
    graph = P.BatchGraph(sg, mats, tx, n, rx, 3.5e9, K=2, flags=LOS | SPEC)
    for rep in range(3):
        print("[gpu-test] graph replay %d" % rep, flush=True)
        out = graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(out["gain"], ref), rep
        # eager work and a synchronisation between replays
        other = P.solve(sg, mats, tx[rep], rx, 3.5e9, 3000, K=2, flags=LOS | SPEC)
        torch.cuda.synchronize()
        assert other.gain.item() > 0
    # new materials written in place are picked up by the next replay
    mats2 = scenes.box_room_materials()
    mats2[0, 0] = 7.5
    graph.mats.copy_(P.materials_tensor(mats2))
    out = graph.launch()
    torch.cuda.synchronize()
    eager2 = P.solve_batch(sg, mats2, tx, n, rx, 3.5e9, K=2, flags=LOS | SPEC)
    assert torch.equal(out["gain"], eager2.gain)
    assert not torch.equal(out["gain"], ref)


def test_wave_rays_does_not_change_results(env):
    torch, P, s, sg = env
    mats = scenes.box_room_materials(scatter=0.3)
    outs = [P.solve(sg, mats, scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 9000, K=3, flags=LOS | SPEC | DIFF,
                    wave_rays=w).gain for w in (64, 128, 512)]
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_autotune_sweep(env, tmp_path):
    torch, P, s, sg = env
    print("[gpu-test] autotune", flush=True)
    choice, rows = P.autotune(s, scenes.box_room_materials(), scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 20000, K=2,
                              leaf_sizes=(1, 4), widths=(2, 8), wave_rays=(64, 256), reps=2,
                              cache_path=str(tmp_path / "tune.json"))
    assert len(rows) == 8 and all(r["ms"] > 0 for r in rows)
    assert {(r["leaf_size"], r["width"]) for r in rows} == {(1, 2), (1, 8), (4, 2), (4, 8)}
    assert choice["ms"] == min(r["ms"] for r in rows)
    again, rows2 = P.autotune(s, scenes.box_room_materials(), scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 20000, K=2,
                              leaf_sizes=(1, 4), widths=(2, 8), wave_rays=(64, 256), reps=2,
                              cache_path=str(tmp_path / "tune.json"))
    assert rows2 is None and again == choice  # the stored choice is reused for the same candidates
    # other candidates are another key: a fresh sweep over them
    other, rows3 = P.autotune(s, scenes.box_room_materials(), scenes.BOX_TX, [scenes.BOX_RX], 3.5e9, 20000, K=2,
                              leaf_sizes=(2,), widths=(4,), wave_rays=(64,), reps=1,
                              cache_path=str(tmp_path / "tune.json"))
    assert rows3 is not None and len(rows3) == 1 and (other["leaf_size"], other["width"]) == (2, 4)
