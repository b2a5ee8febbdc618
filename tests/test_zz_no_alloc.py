"""map_insert_scan_static (the insert that allocates nothing) against
map_insert_scan (needs an MI355X): two maps fed the same scans, one through
each entry point, compared bit for bit after each of two calls in a row (the
second with a smaller scan), then the capacity and flag errors."""
import numpy as np
import pytest
import torch

from synth import scenegen

pytestmark = pytest.mark.gpu


def _state(m):
    from paper_2109_13176_amd import gvom
    lut, data, n_occ, origin = m.export_voxels()
    out = m.export_2d()
    torch.cuda.synchronize()
    st = {k: v for k, v in m.stats().items() if k != "n_pass_updates"}
    return (lut.cpu().numpy().copy(), data[:n_occ].cpu().numpy().copy(), np.asarray(origin).copy(),
            {k: v.cpu().numpy().copy() for k, v in out.items()}, st)


def _same(a, b):
    assert np.array_equal(a[0], b[0]), "lookup table"
    assert np.array_equal(a[1], b[1]), "data array"
    assert np.array_equal(a[2], b[2]), "origin"
    for k in a[3]:
        assert np.array_equal(a[3][k].view(np.uint8), b[3][k].view(np.uint8)), k
    assert a[4] == b[4], (a[4], b[4])


def test_static_insert_equals_map_insert_scan():
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=2, device="cuda")
    ref, sta = gvom.VoxelMap(seq["params"]), gvom.VoxelMap(seq["params"])
    fl = gvom.MAP_RECENTER | gvom.MAP_FIRING(64)
    try:
        for k, n in ((0, 131072), (1, 40000)):  # the second call is smaller
            xyz = seq["scans"][k][:n].contiguous()
            print(f"static insert: scan {k}, {n} points", flush=True)
            ref.insert(xyz, seq["poses"][k], fl)
            assert gvom.map_insert_scan_static(sta.h, xyz, seq["poses"][k], fl) == 0
            _same(_state(ref), _state(sta))
    finally:
        ref.close()
        sta.close()


def test_static_insert_errors_leave_map_unchanged():
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=1, device="cuda")
    m = gvom.VoxelMap(seq["params"])
    try:
        fl = gvom.MAP_RECENTER | gvom.MAP_FIRING(64)
        assert gvom.map_insert_scan_static(m.h, seq["scans"][0], seq["poses"][0], fl) == 0
        before = _state(m)
        big = torch.zeros((3_000_000, 3), dtype=torch.float32, device="cuda")
        assert gvom.map_insert_scan_static(m.h, big, seq["poses"][0], fl) == gvom.MAP_E_CAPACITY
        assert gvom.map_insert_scan_static(m.h, seq["scans"][0], seq["poses"][0],
                                           fl | gvom.MAP_STATS_DISTINCT) == gvom.MAP_E_INVALID
        _same(before, _state(m))
        assert gvom.map_sync(m.h) == 0
    finally:
        m.close()
