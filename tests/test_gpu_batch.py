"""Batched serving: a batch step equals the single-map calls bit for bit, and
the single-map calls equal the oracle (needs an MI355X)."""
import os
import tempfile

import numpy as np
import pytest
import torch

from conftest import params
from parity_util import compare_2d, compare_voxels, Pair
from synth import scenegen

pytestmark = pytest.mark.gpu

SHAPES = [(48, 40, 20, 0.5), (64, 64, 32, 0.4), (30, 34, 96, 0.1), (40, 24, 48, 0.25),
          (16, 16, 16, 0.5)]


def _cloud(rng, n, radius):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-12
    p = d * (radius * rng.uniform(size=(n, 1)) ** 0.5)
    p[rng.uniform(size=n) < 0.05] = np.nan
    return torch.as_tensor(p.astype(np.float32), device="cuda")


def _snapshot(m):
    from paper_2109_13176_amd import gvom
    lut, data, n, origin = m.export_voxels()
    out = m.export_2d()
    torch.cuda.synchronize()
    k = n
    return (lut.cpu().numpy().copy(), data[:k].cpu().numpy().copy(), origin.copy(),
            {key: v.cpu().numpy().copy() for key, v in out.items()})


def _steps(seed, n_steps):
    rng = np.random.default_rng(seed)
    plan = []
    pos = [np.zeros(3) for _ in SHAPES]
    for s in range(n_steps):
        step = []
        for i, (nx, ny, nz, res) in enumerate(SHAPES):
            pos[i] = pos[i] + rng.uniform(-1.5, 1.5, 3) * res * np.array([2, 2, 1])
            ang = rng.uniform(-np.pi, np.pi, 3) * np.array([1, 0.1, 0.1])
            pose = scenegen.pose12(scenegen.rot_zyx(*ang), pos[i])
            n = 0 if (i == 4 and s == 1) else int(rng.integers(500, 6000))
            step.append((_cloud(rng, n, 0.7 * max(nx, ny, nz) * res), pose,
                         1 if (s + i) % 3 else 0))
        plan.append(step)
    return plan


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_maps(graph):
    from paper_2109_13176_amd import gvom
    ps = [params(*sh) for sh in SHAPES]
    bmaps = [gvom.VoxelMap(p) for p in ps]
    smaps = [gvom.VoxelMap(p) for p in ps]
    # half the batch's maps take the 16-pixel surface tiles (the single maps
    # keep 32): results must not depend on the tile
    for i in range(1, len(bmaps), 2):
        assert gvom.map_set_tuning(bmaps[i].h, surface_tile=16) == 0
    batch = gvom.MapBatch(bmaps)
    batch.set_graph(graph)
    try:
        for s, step in enumerate(_steps(11, 4)):
            xyzs = [x for x, _, _ in step]
            poses = [p for _, p, _ in step]
            flags = [f | gvom.MAP_FIRING(1) for _, _, f in step]
            # the first step recentres every map so the sensors are inside
            if s == 0:
                flags = [f | gvom.MAP_RECENTER for f in flags]
            voxels = [(i + s) % 2 == 0 for i in range(len(SHAPES))]
            batch.step(xyzs, poses, flags, voxels)
            lat = batch.latency_ms()
            assert np.isfinite(lat).all() and (lat > 0).all()
            for i, m in enumerate(smaps):
                st = gvom.map_insert_scan(m.h, xyzs[i] if xyzs[i].shape[0] else None, poses[i],
                                          flags[i])
                assert st == 0
            for i in range(len(SHAPES)):
                a = _snapshot(bmaps[i])
                b = _snapshot(smaps[i])
                assert (a[0] == b[0]).all() and (a[1] == b[1]).all() and (a[2] == b[2]).all()
                for k in a[3]:
                    assert (a[3][k].view(np.uint8) == b[3][k].view(np.uint8)).all(), (s, i, k)
                sa, sb = bmaps[i].stats(), smaps[i].stats()
                sa.pop("n_pass_updates"), sb.pop("n_pass_updates")  # work-order dependent
                assert sa == sb, (sa, sb)
    finally:
        batch.close()
        for m in bmaps + smaps:
            m.close()


def test_batch_matches_oracle_on_scenes():
    """Two 16-beam scenes of different maps in one batch, checked against the oracle."""
    from paper_2109_13176_amd import gvom
    ws = [scenegen.single_scan_16beam(seed=s) for s in (21, 22)]
    pairs = [Pair(w["params"]) for w in ws]
    batch = gvom.MapBatch([p.g for p in pairs])
    try:
        xyzs = [w["scans"][0].cuda() for w in ws]
        batch.step(xyzs, [w["poses"][0] for w in ws], [gvom.MAP_FIRING(16)] * 2, [True, True])
        for p, w in zip(pairs, ws):
            assert p.o.insert_scan(w["scans"][0].numpy(), w["poses"][0], 0) == 0
            compare_voxels(p)
            compare_2d(p)
    finally:
        batch.close()
        for p in pairs:
            p.close()


def test_autotune_cache_and_results_unchanged():
    from paper_2109_13176_amd import gvom
    ps = [params(*sh) for sh in SHAPES[:3]]
    maps = [gvom.VoxelMap(p) for p in ps]
    ref = [gvom.VoxelMap(p) for p in ps]
    batch = gvom.MapBatch(maps)
    step = _steps(5, 1)[0][:3]
    xyzs = [x for x, _, _ in step]
    poses = [p for _, p, _ in step]
    flags = [gvom.MAP_RECENTER] * 3
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.txt")
        t1 = batch.autotune(xyzs, poses, flags, cache)
        assert t1["seg_len"] in (6, 8, 16) and t1["trace_waves_per_cu"] in (16, 28)
        assert t1["surface_tile"] in (16, 32)
        assert os.path.exists(cache) and open(cache).read().count("\n") == 1
        t2 = batch.autotune(xyzs, poses, flags, cache)  # served from the cache
        assert t2 == t1 and open(cache).read().count("\n") == 1
    batch.step(xyzs, poses, flags, [True] * 3)
    for i, m in enumerate(ref):
        gvom.map_insert_scan(m.h, xyzs[i], poses[i], flags[i])
        a, b = _snapshot(maps[i]), _snapshot(m)
        assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    batch.close()
    for m in maps + ref:
        m.close()


def test_batch_rejects_bad_requests_without_change():
    from paper_2109_13176_amd import gvom
    ps = [params(*sh) for sh in SHAPES[:2]]
    maps = [gvom.VoxelMap(p) for p in ps]
    batch = gvom.MapBatch(maps)
    rng = np.random.default_rng(0)
    xyzs = [_cloud(rng, 100, 3.0), _cloud(rng, 100, 3.0)]
    good = scenegen.pose12(np.eye(3), [0.1, 0.2, 0.0])
    batch.step(xyzs, [good, good], [1, 1])
    before = [_snapshot(m)[0] for m in maps]
    bad = good.copy()
    bad[2] = np.nan
    with pytest.raises(RuntimeError):
        batch.step(xyzs, [good, bad], [1, 1])   # second map's pose is invalid
    with pytest.raises(RuntimeError):
        batch.step(xyzs, [good, good], [1, 3])  # distinct counting is refused in batches
    after = [_snapshot(m)[0] for m in maps]
    assert all((a == b).all() for a, b in zip(before, after))
    with pytest.raises(RuntimeError):
        gvom.MapBatch([maps[0], maps[0]])
    batch.close()
    for m in maps:
        m.close()
