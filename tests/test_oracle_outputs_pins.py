"""Pins of the oracle's voxel-map density export and the planner costmap
(Fig. 1, Sec. IV, Sec. V): hand-worked values, the column density of a
one-voxel band (an independently pinned path), the lookup table's
occupied / passed / unobserved classes, and one-layer weights."""
from fractions import Fraction

import numpy as np

from conftest import params


def _ident(t=(0, 0, 0)):
    pose = np.zeros(12, np.float32)
    pose[[0, 5, 10]] = 1
    pose[[3, 7, 11]] = t
    return pose


def test_density_hand_example(orc):
    P = params(4, 4, 2, 0.5, szv=1)
    m = orc.OracleMap(P)
    lut = np.full(32, -1, np.int32)
    lut[(2 * 4 + 1) * 2 + 0] = 0       # hits 3, passes 1
    lut[(0 * 4 + 3) * 2 + 1] = 1       # hits 1, passes 2
    lut[(3 * 4 + 3) * 2 + 1] = -1 - 5  # passed five times
    assert m.import_voxels(lut, [[3, 1, 0], [1, 2, 0]], [0, 0, 0]) == 0
    d = m.export_density()
    assert d[(2 * 4 + 1) * 2] == np.float32(0.75)
    assert d[(0 * 4 + 3) * 2 + 1] == np.float32(1.0 / 3.0)
    assert d[(3 * 4 + 3) * 2 + 1] == 0.0
    rest = np.ones(32, bool)
    rest[[(2 * 4 + 1) * 2, (0 * 4 + 3) * 2 + 1, (3 * 4 + 3) * 2 + 1]] = False
    assert np.isnan(d[rest]).all()
    assert (d[rest].view(np.uint32) == 0x7FC00000).all()


def test_density_equals_column_density_of_a_one_voxel_band(orc):
    # 0.4 m voxels: band = 1..5 voxels above the ground voxel
    P = params(4, 4, 16, 0.4, szv=4)
    m = orc.OracleMap(P)
    lut = np.full(4 * 4 * 16, -1, np.int32)
    data = []
    cases = [(1, 2, 3, 4), (2, 1, 1, 2), (3, 0, 7, 9)]  # (x, ground z, band hits, band passes)
    for x, zg, h, p in cases:
        base = (x * 4 + 1) * 16
        lut[base + zg] = len(data)
        data.append([1, 0, (zg * 65536)])
        lut[base + zg + 3] = len(data)
        data.append([h, p, (zg + 3) * 65536])
    assert m.import_voxels(lut, data, [0, 0, 0]) == 0
    d = m.export_density().reshape(4, 4, 16)
    col = m.export_2d()["density"]
    for x, zg, h, p in cases:
        assert col[x, 1] == d[x, 1, zg + 3], (x, col[x, 1], d[x, 1, zg + 3])
        assert d[x, 1, zg + 3] == np.float32(float(Fraction(h, h + p)))
        assert d[x, 1, zg] == np.float32(1.0)


def test_density_classes_follow_the_lookup_table(orc):
    rng = np.random.default_rng(21)
    m = orc.OracleMap(params(16, 16, 16, 0.5))
    pts = rng.uniform(-4, 4, (800, 3)).astype(np.float32)
    assert m.insert_scan(pts, _ident((0.2, -0.1, 0.3))) == 0
    s, lut, data, n, _ = m.export_voxels()
    d = m.export_density()
    occ = lut >= 0
    passed = lut <= -2
    unobs = lut == -1
    assert occ.sum() > 50 and passed.sum() > 500 and unobs.sum() > 500
    assert np.isnan(d[unobs]).all() and (d[passed] == 0).all()
    h, p = data[lut[occ], 0], data[lut[occ], 1]
    want = np.array([np.float32(float(Fraction(int(a), int(a + b)))) for a, b in zip(h, p)])
    assert (d[occ] == want).all()
    assert ((d[occ] > 0) & (d[occ] <= 1)).all()


def _layers_by_hand():
    nan = np.float32(np.nan)
    out = {
        "slope": np.array([[0.25, nan, 1.5]], np.float32),
        "rough": np.array([[0.01, 0.2, nan]], np.float32),
        "density": np.array([[nan, 0.6, 0.3]], np.float32),
        # pixel 0: defined, positive + hard; pixel 1: defined, positive + soft;
        # pixel 2: undefined height, negative obstacle
        "flags": np.array([[1 | 2 | 4 | 32, 1 | 2 | 8, 16]], np.uint8),
        "height": np.zeros((1, 3), np.float32),
    }
    return out


def test_costmap_hand_pixels(orc):
    out = _layers_by_hand()
    w = {"slope": 2.0, "rough": 10.0, "density": 5.0, "positive": 1.0, "hard": 100.0,
         "soft": 3.0, "negative": 50.0, "unknown": 7.0}
    cost, mag = orc.costmap(out, w)
    F = lambda v: Fraction(float(np.float32(v)))  # noqa: E731
    want = [
        2 * F(0.25) + 10 * F(0.01) + 1 + 100,
        10 * F(0.2) + 5 * F(0.6) + 1 + 3,
        2 * F(1.5) + 5 * F(0.3) + 50 + 7,
    ]
    for i in range(3):
        assert abs(Fraction(cost[0, i]) - want[i]) <= Fraction(1, 2 ** 40), (i, cost[0, i])
        assert mag[0, i] == cost[0, i]  # every weight and layer is non-negative here


def test_costmap_one_layer_weights_select_that_layer(orc):
    rng = np.random.default_rng(22)
    m = orc.OracleMap(params(32, 32, 16, 0.4))
    pts = rng.uniform(-6, 6, (4000, 3)).astype(np.float32)
    pts[:, 2] = rng.uniform(-2.0, 0.5, 4000)
    assert m.insert_scan(pts, _ident()) == 0
    out = m.export_2d()
    fl = out["flags"]
    expect = {
        "slope": np.nan_to_num(out["slope"], nan=0.0),
        "rough": np.nan_to_num(out["rough"], nan=0.0),
        "density": np.nan_to_num(out["density"], nan=0.0),
        "positive": (fl >> 1) & 1, "hard": (fl >> 2) & 1, "soft": (fl >> 3) & 1,
        "negative": (fl >> 4) & 1, "unknown": 1 - (fl & 1),
    }
    for k, v in expect.items():
        cost, _ = orc.costmap(out, {k: 1.0})
        assert (cost == v.astype(np.float64)).all(), k
        cost3, _ = orc.costmap(out, {k: -3.0})
        assert (cost3 == -3.0 * v.astype(np.float64)).all(), k
    assert ((fl & 1) == 0).any() and ((fl >> 2) & 1).any()
    wa = {"slope": 1.5, "hard": 4.0, "unknown": 0.5}
    wb = {"rough": 20.0, "soft": 2.0, "negative": 9.0, "density": 0.25}
    ca, _ = orc.costmap(out, wa)
    cb, _ = orc.costmap(out, wb)
    cab, _ = orc.costmap(out, {**wa, **wb})
    assert np.allclose(cab, ca + cb, rtol=1e-14, atol=1e-14)
