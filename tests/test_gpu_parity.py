"""HIP path vs oracle, element by element, on seeded inputs (needs an MI355X)."""
import math

import numpy as np
import pytest
import torch

import oracle
from conftest import params
from parity_util import Pair, compare_all, compare_2d, compare_voxels
from synth import scenegen

pytestmark = pytest.mark.gpu


def _rot(yaw, pitch, roll):
    return scenegen.rot_zyx(yaw, pitch, roll)


def _cloud(rng, n, radius):
    """Points in a ball of `radius` around the sensor (sensor frame), 5% NaN."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-12
    p = d * (radius * rng.uniform(size=(n, 1)) ** 0.5)
    p[rng.uniform(size=n) < 0.05] = np.nan
    return p.astype(np.float32)


@pytest.mark.parametrize("seg_len", [3, 8])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 257, 3001])
def test_ragged_clouds_tiny_map(n, seg_len):
    rng = np.random.default_rng(100 + n)
    pair = Pair(params(16, 16, 16, 0.5, szv=7), seg_len)
    try:
        pose = scenegen.pose12(_rot(0.3, 0.1, -0.2), [0.7, -0.4, 0.25])
        assert pair.insert(_cloud(rng, n, 6.0), pose, 0) == 0
        compare_all(pair, distinct=False)
    finally:
        pair.close()


@pytest.mark.parametrize("dims", [(16, 16, 16, 0.5), (18, 10, 12, 0.25), (40, 26, 7, 0.3),
                                  (32, 32, 64, 0.2), (30, 34, 96, 0.1), (20, 22, 128, 0.15),
                                  (24, 24, 48, 0.4)])
@pytest.mark.parametrize("seg_len", [3, 8])
def test_shapes_and_distinct_counts(dims, seg_len):
    nx, ny, nz, res = dims
    rng = np.random.default_rng(nx * 1000 + nz)
    pair = Pair(params(nx, ny, nz, res), seg_len)
    try:
        for k in range(3):
            ang = rng.uniform(-np.pi, np.pi, 3) * np.array([1, 0.3, 0.3])
            pose = scenegen.pose12(_rot(*ang), rng.uniform(-1, 1, 3) * res * 3)
            pts = _cloud(rng, 4000, 0.6 * max(nx, ny, nz) * res)
            assert pair.insert(pts, pose, 2) == 0  # MAP_STATS_DISTINCT
            compare_all(pair, distinct=True)
    finally:
        pair.close()


@pytest.mark.parametrize("corner", [(1, 1, 1), (62, 1, 30), (1, 62, 16), (62, 62, 2), (32, 32, 16)])
@pytest.mark.parametrize("distinct", [False, True])
def test_sensor_box_near_window_edges(corner, distinct):
    """The segmented traversal sums the passes next to the sensor on chip (a
    17 x 17 x 9 box moved inside the window): with the sensor one voxel from
    a corner of a 64 x 64 x 32 window the box is clamped on every axis.  Two
    dense scans per placement, no recentring, every count against the
    oracle."""
    rng = np.random.default_rng(7000 + 97 * corner[0] + 13 * corner[1] + corner[2])
    res = 0.25
    pair = Pair(params(64, 64, 32, res, szv=16))
    try:
        org = pair.g.origin()
        t = [(corner[k] + int(org[k]) + 0.5) * res for k in range(3)]
        for k in range(2):
            pose = scenegen.pose12(_rot(*(rng.uniform(-np.pi, np.pi, 3) * [1, 0.2, 0.2])), t)
            pts = _cloud(rng, 6000, 9.0)
            assert pair.insert(pts, pose, 2 if distinct else 0) == 0
            compare_all(pair, distinct=distinct)
    finally:
        pair.close()


def test_table_export_reuses_2d_export_ranks():
    """After a 2D export the table export reuses the per-column ranks the
    column pass wrote; a second table export, or one after another insert,
    counts again.  Every table against the oracle."""
    rng = np.random.default_rng(4242)
    pair = Pair(params(40, 36, 20, 0.3))
    try:
        for k in range(3):
            pose = scenegen.pose12(_rot(rng.uniform(-np.pi, np.pi), 0.05, -0.03),
                                   rng.uniform(-1, 1, 3) * 0.6)
            assert pair.insert(_cloud(rng, 5000, 8.0), pose, 1) == 0  # MAP_RECENTER
            if k == 1:
                compare_voxels(pair)      # no 2D export since the insert: counted here
            compare_2d(pair)              # writes the ranks
            compare_voxels(pair)          # reuses them
            compare_voxels(pair)          # the scan consumed them: counted again
    finally:
        pair.close()


@pytest.mark.parametrize("seg_len", [3, 8])
def test_single_scan_16beam_scene(seg_len):
    w = scenegen.single_scan_16beam(seed=1)
    pair = Pair(w["params"], seg_len)
    try:
        assert pair.insert(w["scans"][0], w["poses"][0], 2, firing=16) == 0
        n, g, o = compare_all(pair, distinct=True)
        assert n > 1000
        f = g["flags"]
        assert (f & 4).any() and (f & 8).any() and (f & 16).any()
    finally:
        pair.close()


def test_firing_hint_does_not_change_results():
    w = scenegen.single_scan_16beam(seed=5)
    outs = []
    for fw in (0, 16, 32):
        pair = Pair(w["params"])
        pair.insert(w["scans"][0], w["poses"][0], 0, firing=fw)
        lut, data, n_occ, _ = pair.g.export_voxels()
        o2 = pair.g.export_2d()
        outs.append((lut.cpu().numpy().copy(), data[:n_occ].cpu().numpy().copy(),
                     {k: v.cpu().numpy().copy() for k, v in o2.items()}))
        pair.close()
    for lut, data, o2 in outs[1:]:
        assert (lut == outs[0][0]).all() and (data == outs[0][1]).all()
        for k in o2:
            assert (o2[k].view(np.uint8) == outs[0][2][k].view(np.uint8)).all(), k


@pytest.mark.parametrize("seg_len", [3, 8])
def test_moving_window_sequence(seg_len):
    """Recentring every scan: scrolls in x, y and z (toroidal wrap), one jump
    larger than the window (full clear), general rotations."""
    rng = np.random.default_rng(7)
    p = params(48, 40, 20, 0.5, szv=8)
    pair = Pair(p, seg_len)
    try:
        pos = np.zeros(3)
        for k in range(14):
            if k == 9:
                pos = pos + np.array([40.0, -3.0, 0.0])  # leaves the window entirely
            else:
                pos = pos + rng.uniform(-1.6, 1.6, 3) * np.array([1, 1, 0.6])
            ang = rng.uniform(-np.pi, np.pi, 3) * np.array([1, 0.15, 0.15])
            pose = scenegen.pose12(_rot(*ang), pos)
            pts = _cloud(rng, 3000, 14.0)
            fl = 1 if k % 4 != 3 else 0  # some inserts without recentring
            st = pair.insert(pts, pose, fl)
            assert st in (0, -3)
            if st == 0:
                compare_all(pair)
    finally:
        pair.close()


def _import_both(pair, cols, nz):
    """Hand-filled voxel states pushed into both maps through the import calls."""
    nx, ny = pair.params["nx"], pair.params["ny"]
    V = nx * ny * nz
    lut = np.full(V, -1, np.int32)
    data = []
    for (x, y), vox in cols.items():
        for z, (h, pz, mq) in vox.items():
            i = (x * ny + y) * nz + z
            if h > 0:
                lut[i] = len(data)
                data.append((h, pz, mq))
            else:
                lut[i] = -1 - pz
    data = np.array(data, np.int32).reshape(-1, 3)
    origin = np.array([-5, 7, -3], np.int32)
    from paper_2109_13176_amd import gvom
    s = gvom.map_import_voxels(pair.g.h, torch.as_tensor(lut, device="cuda"),
                               torch.as_tensor(data, device="cuda"), origin)
    assert s == 0
    assert pair.o.import_voxels(lut, data, origin) == 0


def test_import_column_rules_and_negative_search():
    nz, Q = 32, 65536
    p = params(40, 36, nz, 0.4)
    pair = Pair(p)
    try:
        rng = np.random.default_rng(3)
        cols = {}
        base = lambda z: (z - 3) * Q + 1234  # noqa: E731  (world z; origin z = -3)
        for x in range(40):
            for y in range(36):
                if rng.uniform() < 0.45:
                    continue  # unobserved column
                g = int(rng.integers(2, 6)) if x < 20 else int(rng.integers(8, 11))
                vox = {g: (int(rng.integers(1, 9)), int(rng.integers(0, 5)), base(g))}
                for z in range(g + 1, min(nz, g + 9)):
                    r = rng.uniform()
                    if r < 0.2:
                        vox[z] = (int(rng.integers(1, 12)), int(rng.integers(0, 12)), base(z))
                    elif r < 0.4:
                        vox[z] = (0, int(rng.integers(1, 40)), 0)
                cols[(x, y)] = vox
        # exact equality case of the density rule
        cols[(0, 0)] = {2: (3, 0, base(2)), 4: (5, 5, base(4))}
        _import_both(pair, cols, nz)
        compare_voxels(pair)
        g, o = compare_2d(pair)
        assert (g["flags"] & 16).any() and (g["flags"] & 4).any() and (g["flags"] & 8).any()
        assert g["flags"][0, 0] & 8
    finally:
        pair.close()


def test_export_capacity_and_import_roundtrip():
    from paper_2109_13176_amd import gvom
    w = scenegen.single_scan_16beam(seed=2)
    pair = Pair(w["params"])
    try:
        pair.insert(w["scans"][0], w["poses"][0], 0, firing=16)
        lut, data, n_occ, origin = pair.g.export_voxels()
        M = n_occ
        full = data[:M].clone()
        lut2, data2, n2, _ = pair.g.export_voxels(cap=M // 2)
        torch.cuda.synchronize()
        assert n2 == M
        # a truncated export reports the capacity error with the full count,
        # as the oracle does for the same call
        so, _, data_o, n_o, _ = pair.o.export_voxels(cap=M // 2)
        assert so == oracle.E_CAPACITY and n_o == M
        assert pair.g.last_export_status == gvom.MAP_E_CAPACITY
        assert (data2[:M // 2].cpu().numpy() == data_o).all()
        assert (data2[:M // 2] == full[:M // 2]).all()
        assert (lut2 == lut).all()
        # resume: a fresh map imported from the export equals the original
        other = gvom.VoxelMap(w["params"])
        assert gvom.map_import_voxels(other.h, lut.clone(), full, origin) == 0
        l3, d3, n3, o3 = other.export_voxels()
        torch.cuda.synchronize()
        assert (l3 == lut).all() and (d3[:M] == full).all() and (o3 == origin).all()
        # invalid content is rejected and leaves the map empty
        bad = lut.clone()
        bad[0] = M + 5
        assert gvom.map_import_voxels(other.h, bad, full, origin) == gvom.MAP_E_INVALID
        l4, _, n4, _ = other.export_voxels()
        torch.cuda.synchronize()
        assert n4 == 0
        other.close()
    finally:
        pair.close()


def test_error_paths():
    from paper_2109_13176_amd import gvom
    p = params(16, 16, 16, 0.5)
    m = gvom.VoxelMap(p)
    pts = torch.zeros((4, 3), device="cuda")
    good = scenegen.pose12(np.eye(3), [0.1, 0.2, 0.3])
    assert gvom.map_insert_scan(m.h, pts, good, 0) == 0
    lut0 = m.export_voxels()[0].clone()
    bad = good.copy()
    bad[5] = np.inf
    assert gvom.map_insert_scan(m.h, pts, bad, 0) == gvom.MAP_E_POSE
    far = scenegen.pose12(np.eye(3), [100.0, 0, 0])
    assert gvom.map_insert_scan(m.h, pts, far, 0) == gvom.MAP_E_SENSOR_OUTSIDE
    huge = scenegen.pose12(np.eye(3), [1e6, 0, 0])
    assert gvom.map_insert_scan(m.h, pts, huge, 1) == gvom.MAP_E_RANGE
    assert gvom.map_insert_scan(m.h, pts, good, 4) == gvom.MAP_E_INVALID
    assert gvom.lib().map_insert_scan(m.h, None, 5, good.ctypes.data, 0) == gvom.MAP_E_INVALID
    assert gvom.lib().map_insert_scan(m.h, pts.data_ptr(), -1, good.ctypes.data, 0) == gvom.MAP_E_INVALID
    assert (m.export_voxels()[0] == lut0).all()  # errors left the map unchanged
    assert gvom.map_sync(m.h) == 0
    m.close()
    bp = dict(p)
    bp["fit_n"] = 4
    s, h = gvom.map_create(bp)
    assert s == gvom.MAP_E_INVALID


def test_reset_and_repeat_bit_identical():
    w = scenegen.single_scan_16beam(seed=3)
    from paper_2109_13176_amd import gvom
    m = gvom.VoxelMap(w["params"])
    xyz = w["scans"][0].cuda()
    res = []
    for _ in range(2):
        m.insert(xyz, w["poses"][0], gvom.MAP_FIRING(16))
        m.insert(xyz, w["poses"][0], 0)
        lut, data, n, _ = m.export_voxels()
        res.append((lut.cpu().numpy().copy(), data[:n].cpu().numpy().copy()))
        assert gvom.map_reset(m.h) == 0
    assert (res[0][0] == res[1][0]).all() and (res[0][1] == res[1][1]).all()
    m.close()


def _state(m):
    lut, data, n_occ, origin = m.export_voxels()
    out = m.export_2d()
    torch.cuda.synchronize()
    return (lut.cpu().numpy().copy(), data[:n_occ].cpu().numpy().copy(), origin.copy(),
            {k: v.cpu().numpy().copy() for k, v in out.items()},
            {k: v for k, v in m.stats().items() if k != "n_pass_updates"})


@pytest.mark.parametrize("distinct", [False, True])
def test_tunings_bit_identical(distinct):
    """Results do not depend on the launch tuning: the default (segments of
    8 voxels, 32 waves per CU, 32-pixel surface tiles) and a different one
    (segments of 32 voxels, 8 waves per CU, so other waves share line tables
    and other blocks share the sensor box; 16-pixel surface tiles on
    256-thread blocks) give the same map bit for bit: four scans of
    the 64-beam sequence on the 512 x 512 x 64 window (recentred each scan, so
    the storage offsets move), then a cloud of steep rays."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=4, device="cuda")
    maps = [gvom.VoxelMap(seq["params"]) for _ in range(2)]
    assert gvom.map_set_tuning(maps[1].h, seg_len=32, trace_waves_per_cu=8, surface_tile=16) == 0
    assert gvom.map_get_tuning(maps[1].h)[1]["seg_len"] == 32
    assert gvom.map_get_tuning(maps[1].h)[1]["surface_tile"] == 16
    assert gvom.map_set_tuning(maps[1].h, surface_tile=24) == gvom.MAP_E_INVALID
    rng = np.random.default_rng(3)
    steep = _cloud(rng, 20000, 30.0)
    steep[:, 2] *= 3.0
    fl = gvom.MAP_FIRING(64) | (gvom.MAP_STATS_DISTINCT if distinct else 0)
    try:
        for k in range(5):
            xyz = seq["scans"][k] if k < 4 else torch.as_tensor(steep, device="cuda")
            pose = seq["poses"][k] if k < 4 else seq["poses"][3]
            for m in maps:
                m.insert(xyz.contiguous(), pose, fl | gvom.MAP_RECENTER)
            a, b = _state(maps[0]), _state(maps[1])
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            assert np.array_equal(a[2], b[2])
            for key in a[3]:
                assert np.array_equal(a[3][key].view(np.uint8), b[3][key].view(np.uint8)), key
            assert a[4] == b[4], (a[4], b[4])
    finally:
        for m in maps:
            m.close()


def test_profile_phase_mask():
    """Only the phases in the mask are timed; results do not depend on it."""
    from paper_2109_13176_amd import gvom
    w = scenegen.single_scan_16beam(seed=7)
    m = gvom.VoxelMap(w["params"])
    try:
        xyz = w["scans"][0].cuda()
        trace = 1 << gvom.PROF_PHASES.index("trace")
        assert gvom.map_profile_enable(m.h, trace) == 0
        m.insert(xyz, w["poses"][0], gvom.MAP_RECENTER)
        m.export_2d()
        s, prof = gvom.map_profile_read(m.h)
        assert s == 0 and prof["trace"][1] == 1 and prof["trace"][0] > 0
        assert all(prof[p][1] == 0 for p in gvom.PROF_PHASES if p != "trace")
        assert gvom.map_profile_enable(m.h, True) == 0
        m.insert(xyz, w["poses"][0], 0)
        m.export_2d()
        m.export_voxels()
        s, prof = gvom.map_profile_read(m.h)
        assert all(prof[p][1] == 1 for p in ("rays", "trace", "column", "surface", "lut"))
        assert gvom.map_profile_enable(m.h, 1 << 10) != 0
    finally:
        m.close()


def test_device_memory_limit_forces_oom():
    """An allocation cap simulates an out-of-memory device: map_create and a
    map_insert_scan that must grow its work buffers return MAP_E_OOM, the
    failed insert leaves the map unchanged, and lifting the cap restores
    normal operation."""
    from paper_2109_13176_amd import gvom
    L = gvom.lib()
    p = params(32, 32, 16, 0.5)
    m = gvom.VoxelMap(p)
    try:
        good = scenegen.pose12(np.eye(3), [0.1, 0.2, 0.3])
        small = torch.zeros((8, 3), device="cuda")
        assert gvom.map_insert_scan(m.h, small, good, 0) == 0
        before = m.export_voxels()
        lut0, n0 = before[0].clone(), before[2]
        used = L.map_device_memory_in_use()
        assert used > 0
        assert L.map_set_device_memory_limit(-1) == gvom.MAP_E_INVALID
        assert L.map_set_device_memory_limit(used + 1024) == 0
        s, h = gvom.map_create(params(256, 256, 64, 0.2))
        assert s == gvom.MAP_E_OOM
        # a scan far larger than any before needs bigger work buffers
        rng = np.random.default_rng(5)
        big = torch.as_tensor(rng.uniform(-6, 6, (200000, 3)).astype(np.float32), device="cuda")
        assert gvom.map_insert_scan(m.h, big, good, 0) == gvom.MAP_E_OOM
        after = m.export_voxels()
        assert after[2] == n0 and torch.equal(after[0], lut0)
        assert L.map_set_device_memory_limit(0) == 0
        assert gvom.map_insert_scan(m.h, big, good, 0) == 0
        assert m.export_voxels()[2] > n0
    finally:
        gvom.lib().map_set_device_memory_limit(0)
        m.close()
