"""Pins of the oracle's map buffer and combine step (Sec. III-B, III-D).

The combine is checked against a hand-worked example and against the
accumulating map of the oracle (itself pinned in test_oracle_pins.py): when
every voxel of the final window has stayed inside the window since it first
entered (origins that only grow along each axis), the sum of the per-scan maps
over the windows that held a voxel equals what the accumulating map counted
for it.
"""
import numpy as np

from conftest import params


def _ident(t=(0, 0, 0)):
    pose = np.zeros(12, np.float32)
    pose[[0, 5, 10]] = 1
    pose[[3, 7, 11]] = t
    return pose


def _dense(export, shape):
    s, lut, data, n, origin = export
    assert s == 0
    h = np.where(lut >= 0, data[np.maximum(lut, 0), 0] if n else 0, 0).reshape(shape)
    p = np.where(lut >= 0, data[np.maximum(lut, 0), 1] if n else 0, -1 - lut).reshape(shape)
    q = np.where(lut >= 0, data[np.maximum(lut, 0), 2] if n else 0, 2 ** 31 - 1).reshape(shape)
    return h, p, q, origin


def test_combine_hand_example(orc):
    # window 4 x 6 x 3, lookup index (x * 6 + y) * 3 + z
    P = params(4, 6, 3, 0.5, szv=1)
    V = 4 * 6 * 3
    A = orc.OracleMap(P)
    lut = np.full(V, -1, np.int32)
    lut[58] = 0         # world (3,1,1): hits 2, passes 1, lowest 100
    lut[23] = -1 - 5    # world (1,1,2): 5 misses
    lut[6] = -1 - 7     # world (0,2,0): leaves the combined window (x)
    lut[53] = -1 - 4    # world (2,5,2): leaves the combined window (y)
    assert A.import_voxels(lut, [[2, 1, 100]], [0, 0, 0]) == 0
    B = orc.OracleMap(P)
    lut = np.full(V, -1, np.int32)
    lut[7] = 0          # world (1,1,2): hits 1, passes 2, lowest -7
    lut[42] = 1         # world (3,1,1): hits 1, passes 0, lowest 50
    lut[65] = -1 - 3    # world (4,2,3): outside A's window
    lut[18] = -1 - 2    # world (2,-1,1): outside A's window
    assert B.import_voxels(lut, [[1, 2, -7], [1, 0, 50]], [1, -1, 1]) == 0
    buf = orc.OracleBuffer(P, 4)
    buf.maps = [A.export_voxels()[1:3] + (A.origin(),), B.export_voxels()[1:3] + (B.origin(),)]
    out = orc.OracleMap(P)
    assert buf.combine(out) == 0
    s, lut, data, n, origin = out.export_voxels()
    assert s == 0 and list(origin) == [1, -1, 1] and n == 2
    want = np.full(V, -1, np.int32)
    want[7] = 0         # local (0,2,1) = world (1,1,2)
    want[42] = 1        # local (2,2,0) = world (3,1,1)
    want[65] = -1 - 3   # local (3,3,2) = world (4,2,3)
    want[18] = -1 - 2   # local (1,0,0) = world (2,-1,1)
    assert (lut == want).all(), np.nonzero(lut != want)
    assert data.tolist() == [[1, 7, -7], [3, 1, 50]]


def _scans(seed, k, n=600, spread=3.0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        pts = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
        pts[:, 2] = rng.uniform(-1.5, 0.5, n)
        pts[::11] = np.nan
        out.append(pts)
    return out


def test_combine_single_map_is_that_map(orc):
    P = params(16, 16, 8, 0.5)
    buf = orc.OracleBuffer(P, 3)
    pts = _scans(1, 1)[0]
    assert buf.push(pts, _ident((0.3, -0.4, 0.1)), orc.RECENTER) == 0
    ref = orc.OracleMap(P)
    assert ref.insert_scan(pts, _ident((0.3, -0.4, 0.1)), orc.RECENTER) == 0
    out = orc.OracleMap(P)
    assert buf.combine(out) == 0
    a, b = out.export_voxels(), ref.export_voxels()
    assert (a[1] == b[1]).all() and (a[2] == b[2]).all() and (a[4] == b[4]).all()


def _accumulated(orc, P, scans, poses, flags):
    m = orc.OracleMap(P)
    for pts, pose, f in zip(scans, poses, flags):
        assert m.insert_scan(pts, pose, f) == 0
    return m


def _assert_same(orc, P, buf, ref):
    out = orc.OracleMap(P)
    assert buf.combine(out) == 0
    shape = (P["nx"], P["ny"], P["nz"])
    a = _dense(out.export_voxels(), shape)
    b = _dense(ref.export_voxels(), shape)
    assert (a[3] == b[3]).all(), (a[3], b[3])
    for u, v, name in zip(a[:3], b[:3], ("hits", "passes", "min_qz")):
        assert (u == v).all(), (name, np.argwhere(u != v)[:5])
    ea, eb = out.export_2d(), ref.export_2d()
    for k in ea:
        assert (ea[k].view(np.uint8) == eb[k].view(np.uint8)).all(), k
    return a


def test_combine_static_sensor_equals_accumulated_map(orc):
    P = params(16, 16, 8, 0.5)
    scans = _scans(2, 3)
    pose = _ident((0.2, 0.1, 0.0))
    buf = orc.OracleBuffer(P, 3)
    for s in scans:
        assert buf.push(s, pose, orc.RECENTER) == 0
    ref = _accumulated(orc, P, scans, [pose] * 3, [orc.RECENTER] * 3)
    h, p, _, _ = _assert_same(orc, P, buf, ref)
    assert h.sum() > 100 and p.sum() > 1000


def test_combine_monotonic_motion_equals_accumulated_map(orc):
    # origins grow along x, y and z: a voxel of the last window has been in
    # every window since the first one that held it
    P = params(16, 12, 8, 0.5)
    scans = _scans(3, 5)
    poses = [_ident((0.9 * i, 0.35 * i, 0.3 * i)) for i in range(5)]
    buf = orc.OracleBuffer(P, 5)
    for s, pose in zip(scans, poses):
        assert buf.push(s, pose, orc.RECENTER) == 0
    origins = np.stack([o for _, _, o in buf.maps])
    assert (np.diff(origins, axis=0) >= 0).all() and (origins[-1] != origins[0]).all()
    ref = _accumulated(orc, P, scans, poses, [orc.RECENTER] * 5)
    _assert_same(orc, P, buf, ref)


def test_combine_keeps_only_the_last_depth_maps(orc):
    P = params(16, 12, 8, 0.5)
    scans = _scans(4, 6)
    poses = [_ident((0.7 * i, 0.2 * i, 0.0)) for i in range(6)]
    buf = orc.OracleBuffer(P, 3)
    for s, pose in zip(scans, poses):
        assert buf.push(s, pose, orc.RECENTER) == 0
    assert len(buf.maps) == 3
    ref = _accumulated(orc, P, scans[3:], poses[3:], [orc.RECENTER] * 3)
    _assert_same(orc, P, buf, ref)


def test_combine_second_lidar_shares_the_window(orc):
    P = params(16, 16, 8, 0.5)
    scans = _scans(5, 4)
    vehicle = [_ident((0.8 * i, 0.0, 0.0)) for i in range(2)]
    side = [_ident((0.8 * i + 0.6, 0.5, -0.2)) for i in range(2)]
    order = [(scans[0], vehicle[0], 1), (scans[1], side[0], 0),
             (scans[2], vehicle[1], 1), (scans[3], side[1], 0)]
    buf = orc.OracleBuffer(P, 4)
    for s, pose, f in order:
        assert buf.push(s, pose, f) == 0
    o = [m[2] for m in buf.maps]
    assert (o[0] == o[1]).all() and (o[2] == o[3]).all() and (o[1] != o[2]).any()
    ref = _accumulated(orc, P, [x[0] for x in order], [x[1] for x in order],
                       [x[2] for x in order])
    _assert_same(orc, P, buf, ref)


def test_combine_disjoint_windows_keeps_the_newest(orc):
    P = params(8, 8, 8, 0.5)
    scans = _scans(6, 2, spread=1.8)
    buf = orc.OracleBuffer(P, 2)
    assert buf.push(scans[0], _ident((0, 0, 0)), orc.RECENTER) == 0
    assert buf.push(scans[1], _ident((30.0, 0, 0)), orc.RECENTER) == 0
    ref = _accumulated(orc, P, [scans[1]], [_ident((30.0, 0, 0))], [orc.RECENTER])
    _assert_same(orc, P, buf, ref)


def test_buffer_errors(orc):
    P = params(8, 8, 8, 0.5)
    buf = orc.OracleBuffer(P, 2)
    out = orc.OracleMap(P)
    assert buf.combine(out) == orc.E_INVALID
    pts = _scans(7, 1, spread=1.5)[0]
    assert buf.push(pts, _ident((100.0, 0, 0))) == orc.E_SENSOR_OUT
    bad = _ident()
    bad[2] = np.inf
    assert buf.push(pts, bad, orc.RECENTER) == orc.E_POSE
    assert buf.maps == []
    assert buf.push(np.zeros((0, 3), np.float32), _ident(), orc.RECENTER) == 0
    assert buf.combine(out) == 0
    s, lut, _, n, _ = out.export_voxels()
    assert n == 0 and (lut == -1).all()
