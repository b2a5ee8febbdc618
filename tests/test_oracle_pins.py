"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
examples (tests/golden), exact rational arithmetic (fractions.Fraction), a
textbook routine (numpy.linalg.lstsq), closed forms and invariants.
"""
import json
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from conftest import params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Q = 65536


# ----------------------------------------------------------------------------
# helpers written from the definitions, independent of the oracle's code


def f32_round(x: Fraction) -> Fraction:
    """Exact round-to-nearest-even of a rational to IEEE binary32 (normal range)."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    m = a * (1 << 23)
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * Fraction(fl) * Fraction(2) ** (e - 23)


def floor_div(a: int, b: int) -> int:
    return a // b


def brute_ray_set(s, p):
    """Voxels v with a non-empty intersection of the per-axis time sets
    {t in [0,1] : floor(X_a(t)/Q) = v_a}; X(t) = s + t (p - s)."""
    lo = [min(floor_div(s[a], Q), floor_div(p[a], Q)) for a in range(3)]
    hi = [max(floor_div(s[a], Q), floor_div(p[a], Q)) for a in range(3)]

    def axis_interval(a, v):
        # returns (lo, lo_closed, hi, hi_closed) within [0, 1] or None
        S, D = s[a], p[a] - s[a]
        if D == 0:
            return (Fraction(0), True, Fraction(1), True) if floor_div(S, Q) == v else None
        # v*Q <= S + t D < (v+1)*Q
        t1 = Fraction(v * Q - S, D)
        t2 = Fraction((v + 1) * Q - S, D)
        if D > 0:
            l, lc, h, hc = t1, True, t2, False
        else:
            l, lc, h, hc = t2, False, t1, True
        if l < 0 or (l == 0 and not lc):
            l, lc = max(l, Fraction(0)), (l < 0) or lc
        if l < 0:
            l, lc = Fraction(0), True
        if h > 1:
            h, hc = Fraction(1), True
        return (l, lc, h, hc)

    out = set()
    for x in range(lo[0], hi[0] + 1):
        for y in range(lo[1], hi[1] + 1):
            for z in range(lo[2], hi[2] + 1):
                ivs = [axis_interval(a, v) for a, v in enumerate((x, y, z))]
                if any(iv is None for iv in ivs):
                    continue
                L, Lc = Fraction(0), True
                H, Hc = Fraction(1), True
                for (l, lc, h, hc) in ivs:
                    if l > L or (l == L and not lc):
                        L, Lc = l, lc
                    if h < H or (h == H and not hc):
                        H, Hc = h, hc
                if L < H or (L == H and Lc and Hc):
                    out.add((x, y, z))
    return out


# ----------------------------------------------------------------------------
# constants (parameters named in III-A and III-D; values are our readings)


@pytest.mark.parametrize("res,n_lo,n_hi,d,tau", [
    (0.4, 1, 5, 12, 81920),
    (0.2, 2, 10, 25, 163840),
    (0.1, 4, 20, 50, 327680),
])
def test_derived_constants(orc, res, n_lo, n_hi, d, tau):
    s, c = orc.derive(params(64, 64, 32, res))
    assert s == 0
    assert c["n_lo"] == n_lo and c["n_hi"] == n_hi
    # 5.0 / float32(0.4) = 12.4999998... rounds to 12; float32(0.2) and (0.1) give 25, 50
    assert c["search_d"] == d
    # floor(0.5 / r * 65536) with r the float32 resolution
    assert c["tau_neg_q"] == int(np.floor(np.float64(np.float32(0.5)) / np.float64(np.float32(res)) * 65536))
    assert abs(c["tau_neg_q"] - tau) <= 1
    assert c["inv_r"] == np.float32(1.0 / np.float64(np.float32(res)))


def test_invalid_params(orc):
    bad = [dict(nx=3), dict(nz=0), dict(nz=129), dict(res_m=0.0), dict(res_m=float("nan")),
           dict(fit_n=4), dict(fit_n=1), dict(dens_den=0), dict(sensor_z_voxel=32),
           dict(obs_max_m=0.1), dict(neg_search_m=0.0)]
    for b in bad:
        p = params(16, 16, 32, 0.4)
        p.update(b)
        s, _ = orc.derive(p)
        assert s == orc.E_INVALID, b


# ----------------------------------------------------------------------------
# III-C transform into the map frame


def test_transform_identity_and_translation(orc):
    rng = np.random.default_rng(0)
    r = np.float32(0.25)
    inv_r = np.float32(4.0)
    for _ in range(200):
        p = rng.uniform(-60, 60, 3).astype(np.float32)
        k = rng.integers(-100, 100, 3)
        pose = np.zeros(12, np.float32)
        pose[[0, 5, 10]] = 1
        ok, q0 = orc.transform_point(pose, inv_r, p)
        assert ok
        exact = [int(np.floor(Fraction(float(v)) * 4 * Q)) for v in p]
        assert list(q0) == exact
        pose[[3, 7, 11]] = (k * r).astype(np.float32)
        ok, q1 = orc.transform_point(pose, inv_r, p)
        assert ok
        # a translation by k voxels shifts the voxel index by exactly k
        assert list((q1 >> 16) - (q0 >> 16)) == list(k)


def test_transform_axis_permutation(orc):
    rng = np.random.default_rng(1)
    inv_r = np.float32(2.0)
    perm = np.zeros(12, np.float32)
    # world x = sensor y, world y = -sensor z, world z = sensor x
    perm[1] = 1
    perm[6] = -1
    perm[8] = 1
    for _ in range(100):
        p = rng.uniform(-30, 30, 3).astype(np.float32)
        ok, q = orc.transform_point(perm, inv_r, p)
        assert ok
        src = [p[1], -p[2], p[0]]
        assert list(q) == [int(np.floor(Fraction(float(v)) * 2 * Q)) for v in src]


def test_transform_general_pose_exact_rounding(orc):
    """fma chain t + R0 x + R1 y + R2 z, each fma rounded once to binary32,
    then u = w * inv_r rounded once, Q = floor(u * 2^16)."""
    rng = np.random.default_rng(2)
    res = np.float32(0.2)
    inv_r = np.float32(1.0 / np.float64(res))
    for _ in range(300):
        ang = rng.uniform(-np.pi, np.pi, 3)
        cz, sz = np.cos(ang[0]), np.sin(ang[0])
        cy, sy = np.cos(ang[1]), np.sin(ang[1])
        Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
        Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
        R = Rz @ Ry
        t = rng.uniform(-200, 200, 3)
        pose = np.concatenate([R, t[:, None]], axis=1).astype(np.float32).reshape(12)
        p = rng.uniform(-80, 80, 3).astype(np.float32)
        ok, q = orc.transform_point(pose, inv_r, p)
        assert ok
        for i in range(3):
            w = Fraction(float(pose[4 * i + 3]))
            for j in range(3):
                w = f32_round(Fraction(float(pose[4 * i + j])) * Fraction(float(p[j])) + w)
            u = f32_round(w * Fraction(float(inv_r)))
            assert q[i] == int(np.floor(u * Q)), (i, pose, p)


def test_transform_skips(orc):
    pose = np.zeros(12, np.float32)
    pose[[0, 5, 10]] = 1
    ok, _ = orc.transform_point(pose, np.float32(1.0), np.array([np.nan, 0, 0], np.float32))
    assert not ok
    ok, _ = orc.transform_point(pose, np.float32(1.0), np.array([32768.0, 0, 0], np.float32))
    assert not ok
    ok, _ = orc.transform_point(pose, np.float32(1.0), np.array([32767.5, 0, 0], np.float32))
    assert ok


# ----------------------------------------------------------------------------
# III-A / III-C ray voxels


def test_ray_worked_examples(orc):
    cases = json.load(open(os.path.join(GOLDEN, "ray_worked_examples.json")))["cases"]
    for c in cases:
        s = [int(round(v * Q)) for v in c["s"]]
        p = [int(round(v * Q)) for v in c["p"]]
        got = orc.ray_voxels(s, p).tolist()
        assert got == c["voxels"], c["name"]


def test_ray_brute_force_membership(orc):
    rnd = random.Random(3)
    for it in range(400):
        # coordinates on a 1/4-voxel lattice make boundary ties frequent
        grid = rnd.choice([Q // 4, Q // 2, Q, 1, 977])
        s = [rnd.randint(-6 * Q // grid, 6 * Q // grid) * grid for _ in range(3)]
        p = [rnd.randint(-6 * Q // grid, 6 * Q // grid) * grid for _ in range(3)]
        if it % 5 == 0:
            p[rnd.randrange(3)] = s[0]  # some axis-aligned / degenerate rays
        seq = [tuple(v) for v in orc.ray_voxels(s, p).tolist()]
        want = brute_ray_set(s, p)
        assert set(seq) == want, (s, p)
        assert len(seq) == len(want)  # distinct
        assert seq[0] == tuple(floor_div(v, Q) for v in s)
        assert seq[-1] == tuple(floor_div(v, Q) for v in p)
        for a in range(3):
            sgn = np.sign(p[a] - s[a])
            steps = [seq[k + 1][a] - seq[k][a] for k in range(len(seq) - 1)]
            assert all(st in (0, sgn) for st in steps)


def test_ray_invariants_long(orc):
    rng = np.random.default_rng(4)
    for _ in range(200):
        s = rng.integers(-300 * Q, 300 * Q, 3)
        p = rng.integers(-300 * Q, 300 * Q, 3)
        seq = orc.ray_voxels(s, p)
        d = np.abs((p >> 16) - (s >> 16))
        # each voxel step moves every axis by at most one; total moves = sum |dv|
        steps = np.abs(np.diff(seq, axis=0))
        assert steps.max(initial=0) <= 1
        assert steps.sum() == d.sum()
        assert (steps.sum(axis=1) >= 1).all()


# ----------------------------------------------------------------------------
# III-A / III-C accumulation of hits and passes


def _fresh(orc, nx=8, ny=8, nz=8, res=0.5, **kw):
    return orc.OracleMap(params(nx, ny, nz, res, **kw))


def _ident(t=(0, 0, 0)):
    pose = np.zeros(12, np.float32)
    pose[[0, 5, 10]] = 1
    pose[[3, 7, 11]] = t
    return pose


def test_insert_matches_brute_force(orc):
    rng = np.random.default_rng(5)
    res = 0.5
    m = _fresh(orc, 8, 8, 8, res)
    origin = m.origin()
    pts = rng.uniform(-4, 4, (60, 3)).astype(np.float32)
    pts = (np.round(pts * 8) / 8).astype(np.float32)  # lattice -> boundary ties
    pts[::7] = np.nan
    assert m.insert_scan(pts, _ident()) == 0
    hits = np.zeros((8, 8, 8), np.int64)
    passes = np.zeros((8, 8, 8), np.int64)
    n_hits = n_pass = 0
    S = [0, 0, 0]
    for p in pts:
        if not np.isfinite(p).all():
            continue
        P = [int(np.floor(Fraction(float(v)) * 2 * Q)) for v in p]
        cells = sorted(brute_ray_set(S, P), key=lambda v: sum(abs(v[a] - S[a] // Q) for a in range(3)))
        end = tuple(v // Q for v in P)
        for c in cells:
            l = [c[a] - origin[a] for a in range(3)]
            if not all(0 <= l[a] < 8 for a in range(3)):
                continue
            if c == end:
                hits[tuple(l)] += 1
                n_hits += 1
            else:
                passes[tuple(l)] += 1
                n_pass += 1
    s, lut, data, n_occ, org = m.export_voxels()
    assert s == 0
    lut = lut.reshape(8, 8, 8)
    got_h = np.where(lut >= 0, data[np.maximum(lut, 0), 0], 0)
    got_p = np.where(lut >= 0, data[np.maximum(lut, 0), 1], -1 - lut)
    assert (got_h == hits).all()
    assert (got_p == passes).all()
    st = m.stats()
    assert st["n_hits"] == n_hits and st["n_pass"] == n_pass
    assert st["n_nonfinite"] == len(pts[::7]) and st["n_points"] == len(pts)
    assert st["n_distinct_pass"] == int((passes > 0).sum())
    assert st["n_distinct_hit"] == int((hits > 0).sum())


def test_insert_order_independent_and_minqz(orc):
    rng = np.random.default_rng(6)
    pts = rng.uniform(-6, 6, (500, 3)).astype(np.float32)
    a = _fresh(orc, 16, 16, 16, 0.5)
    b = _fresh(orc, 16, 16, 16, 0.5)
    a.insert_scan(pts, _ident((0.3, -0.2, 0.1)))
    b.insert_scan(pts[rng.permutation(len(pts))], _ident((0.3, -0.2, 0.1)))
    ea, eb = a.export_voxels(), b.export_voxels()
    assert (ea[1] == eb[1]).all() and (ea[2] == eb[2]).all()
    # minimum return height of each occupied voxel, recomputed from the points
    lut, data, org = ea[1].reshape(16, 16, 16), ea[2], ea[4]
    # identity rotation: w = float32(p + t) (one rounding), u = 2 w exactly
    w = pts + np.array([0.3, -0.2, 0.1], np.float32)
    qs = np.floor(w.astype(np.float64) * 2 * Q).astype(np.int64)
    want = {}
    for q in qs:
        v = tuple(q // Q - org)
        if all(0 <= v[k] < 16 for k in range(3)):
            want[v] = min(want.get(v, 1 << 40), q[2])
    for v, mq in want.items():
        assert lut[v] >= 0 and data[lut[v], 2] == mq


def test_sum_hits_plus_passes_is_path_length(orc):
    rng = np.random.default_rng(7)
    m = _fresh(orc, 16, 16, 16, 0.25)
    pts = rng.uniform(-3, 3, (300, 3)).astype(np.float32)
    m.insert_scan(pts, _ident())
    org = m.origin()
    total = 0
    for p in pts:
        P = np.floor(p.astype(np.float64) * 4 * Q).astype(np.int64)
        seq = orc.ray_voxels([0, 0, 0], P)
        loc = seq - org
        total += int(((loc >= 0) & (loc < 16)).all(axis=1).sum())
    st = m.stats()
    assert st["n_hits"] + st["n_pass"] == total


def test_errors_leave_map_unchanged(orc):
    m = _fresh(orc, 8, 8, 8, 0.5)
    pts = np.array([[1.0, 0.2, -0.3]], np.float32)
    m.insert_scan(pts, _ident())
    before = m.export_voxels()[1].copy()
    bad_pose = _ident()
    bad_pose[4] = np.nan
    assert m.insert_scan(pts, bad_pose) == orc.E_POSE
    assert m.insert_scan(pts, _ident((100.0, 0, 0))) == orc.E_SENSOR_OUT
    assert m.insert_scan(pts, _ident((1e5, 0, 0)), orc.RECENTER) == orc.E_RANGE
    assert (m.export_voxels()[1] == before).all()
    assert m.insert_scan(np.zeros((0, 3), np.float32), _ident()) == 0


def test_recentre_equals_shifted_map_plus_fresh_scan(orc):
    rng = np.random.default_rng(8)
    n = 16
    A = rng.uniform(-3, 3, (400, 3)).astype(np.float32)
    B = rng.uniform(-3, 3, (400, 3)).astype(np.float32)
    t0, t1 = (0.1, 0.2, 0.0), (1.6, -0.9, 0.7)
    m = _fresh(orc, n, n, n, 0.5)
    m.insert_scan(A, _ident(t0), orc.RECENTER)
    _, lutA, dataA, _, oA = m.export_voxels()
    m.insert_scan(np.zeros((0, 3), np.float32), _ident(t1), orc.RECENTER)
    _, lutM, dataM, _, oM = m.export_voxels()
    # the moved map is the old one shifted by the origin change, empty elsewhere
    hA = np.where(lutA >= 0, dataA[np.maximum(lutA, 0), 0], 0).reshape(n, n, n)
    pA = np.where(lutA >= 0, dataA[np.maximum(lutA, 0), 1], -1 - lutA).reshape(n, n, n)
    d = oM - oA
    assert np.abs(d).sum() > 0
    hS = np.zeros_like(hA)
    pS = np.zeros_like(pA)
    for x in range(n):
        for y in range(n):
            for z in range(n):
                ox, oy, oz = x + d[0], y + d[1], z + d[2]
                if 0 <= ox < n and 0 <= oy < n and 0 <= oz < n:
                    hS[x, y, z] = hA[ox, oy, oz]
                    pS[x, y, z] = pA[ox, oy, oz]
    hM = np.where(lutM >= 0, dataM[np.maximum(lutM, 0), 0], 0).reshape(n, n, n)
    pM = np.where(lutM >= 0, dataM[np.maximum(lutM, 0), 1], -1 - lutM).reshape(n, n, n)
    assert (hM == hS).all() and (pM == pS).all()
    # inserting B adds exactly what B alone adds to a fresh map at that origin
    m.insert_scan(B, _ident(t1), orc.RECENTER)
    f = _fresh(orc, n, n, n, 0.5)
    f.insert_scan(B, _ident(t1), orc.RECENTER)
    _, lutB, dataB, _, oB = f.export_voxels()
    _, lutT, dataT, _, oT = m.export_voxels()
    assert (oB == oT).all()
    hB = np.where(lutB >= 0, dataB[np.maximum(lutB, 0), 0], 0).reshape(n, n, n)
    pB = np.where(lutB >= 0, dataB[np.maximum(lutB, 0), 1], -1 - lutB).reshape(n, n, n)
    hT = np.where(lutT >= 0, dataT[np.maximum(lutT, 0), 0], 0).reshape(n, n, n)
    pT = np.where(lutT >= 0, dataT[np.maximum(lutT, 0), 1], -1 - lutT).reshape(n, n, n)
    assert (hT == hS + hB).all() and (pT == pS + pB).all()
    # moving away and back leaves the cells that left the window cleared
    m.insert_scan(np.zeros((0, 3), np.float32), _ident((40.0, 0, 0)), orc.RECENTER)
    assert m.stats()["n_cleared"] == n ** 3
    m.insert_scan(np.zeros((0, 3), np.float32), _ident(t1), orc.RECENTER)
    s, lut, _, n_occ, _ = m.export_voxels()
    assert n_occ == 0 and (lut == -1).all()


# ----------------------------------------------------------------------------
# III-A lookup table


def test_lut_encoding_invariants(orc):
    rng = np.random.default_rng(9)
    m = _fresh(orc, 16, 16, 16, 0.5)
    m.insert_scan(rng.uniform(-4, 4, (700, 3)).astype(np.float32), _ident())
    s, lut, data, n_occ, _ = m.export_voxels()
    occ = lut >= 0
    assert occ.sum() == n_occ
    assert (lut[occ] == np.arange(n_occ)).all()  # ranks 0..M-1 in index order
    assert (data[:, 0] >= 1).all()
    s2, lut2, data2, n2, _ = m.export_voxels(cap=n_occ - 1)
    assert s2 == orc.E_CAPACITY and n2 == n_occ and (lut2 == lut).all()
    assert (data2 == data[:n_occ - 1]).all()


# ----------------------------------------------------------------------------
# III-D height, positive obstacles, density


def _column_map(orc, cols, nz=32, res=0.4, n=4):
    """A map whose voxels are filled by hand: cols = {(x, y): {z: (hits, passes, minqz)}}."""
    m = orc.OracleMap(params(n, n, nz, res))
    V = n * n * nz
    lut = np.full(V, -1, np.int32)
    data = []
    for (x, y), vox in cols.items():
        for z, (h, p, mq) in vox.items():
            i = (x * n + y) * nz + z
            if h > 0:
                lut[i] = len(data)
                data.append((h, p, mq))
            else:
                lut[i] = -1 - p
    assert m.import_voxels(lut, np.array(data, np.int32).reshape(-1, 3), [0, 0, 0]) == 0
    return m


def test_column_rules(orc):
    z0 = 3
    base = lambda z: z * Q + 100  # noqa: E731  (a return inside voxel z)
    cols = {
        # ground only: height defined, no obstacle
        (0, 0): {z0: (4, 0, base(z0))},
        # box face: band voxels returned often -> hard
        (0, 1): {z0: (4, 0, base(z0)), z0 + 1: (9, 1, base(z0 + 1)), z0 + 5: (9, 2, base(z0 + 5))},
        # sparse vegetation: band voxels mostly passed through -> soft
        (0, 2): {z0: (4, 0, base(z0)), z0 + 2: (1, 20, base(z0 + 2))},
        # equality 5 / 10 = threshold 1/2 -> soft; band voxel free with passes ignored
        (0, 3): {z0: (4, 0, base(z0)), z0 + 3: (5, 5, base(z0 + 3)), z0 + 4: (0, 50, 0)},
        # 6 / 10 > 1/2 -> hard
        (1, 0): {z0: (4, 0, base(z0)), z0 + 3: (6, 4, base(z0 + 3))},
        # occupied voxel just above the band (n_hi + 1 = 6) -> no obstacle
        (1, 1): {z0: (4, 0, base(z0)), z0 + 6: (9, 0, base(z0 + 6))},
        # the band is counted from the LOWEST occupied voxel
        (1, 2): {1: (1, 0, base(1)), 7: (9, 0, base(7))},
        # only passes: undefined height
        (1, 3): {z0: (0, 12, 0)},
    }
    m = _column_map(orc, cols)
    out = m.export_2d()
    f, h, d = out["flags"], out["height"], out["density"]
    r = np.float64(np.float32(0.4))
    assert f[0, 0] & 0xF == 1 and np.isnan(d[0, 0])
    assert h[0, 0] == np.float32(base(z0) * r / Q)
    assert f[0, 1] & 0xF == 1 | 2 | 4
    assert d[0, 1] == np.float32(18 / 21)
    assert f[0, 2] & 0xF == 1 | 2 | 8 and d[0, 2] == np.float32(1 / 21)
    assert f[0, 3] & 0xF == 1 | 2 | 8 and d[0, 3] == np.float32(0.5)
    assert f[1, 0] & 0xF == 1 | 2 | 4
    assert f[1, 1] & 0xF == 1
    assert f[1, 2] & 0xF == 1 and h[1, 2] == np.float32(base(1) * r / Q)
    assert f[1, 3] & 0xF == 0 and np.isnan(h[1, 3])
    assert np.isnan(h[2, 2]) and f[2, 2] & 1 == 0
    # undefined floats are the canonical quiet NaN
    assert h.view(np.uint32)[2, 2] == 0x7FC00000
    # hard and soft exclusive, each implies positive
    assert not ((f & 4) & ((f & 8) >> 1)).any()
    assert (((f & 12) > 0) <= ((f & 2) > 0)).all()


# ----------------------------------------------------------------------------
# III-D slope and roughness


def test_flat_plane_slope_zero(orc):
    hq = np.full((9, 11), 5 * Q + 7, np.int32)
    s, r, sd, neg = orc.surface(hq, np.ones_like(hq, np.uint8), 5, 0.4, 12, 81920)
    assert sd.all()
    assert (s == 0).all() and (r == 0).all()


def test_known_pitch_plane(orc):
    # r = 0.5 m, slope m = 1/4: height at pixel centre x is m * x * r metres,
    # i.e. m * x voxels = 16384 * x in Q16 -- exact.
    nx, ny = 12, 10
    hq = (16384 * np.arange(nx)[:, None] + 0 * np.arange(ny)[None, :]).astype(np.int32)
    for fit_n in (3, 5, 7):
        s, r, sd, _ = orc.surface(hq, np.ones_like(hq, np.uint8), fit_n, 0.5, 10, 65536)
        assert sd.all()
        assert (s == np.float32(0.25)).all()
        assert (np.abs(r) <= 1e-12).all()


def test_plane_fit_vs_lstsq(orc):
    rng = np.random.default_rng(10)
    nx, ny, res = 20, 17, 0.2
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    hq = (3000 * X - 1700 * Y + rng.normal(0, 5000, (nx, ny)) + 4 * Q).astype(np.int32)
    defined = (rng.uniform(size=(nx, ny)) > 0.25).astype(np.uint8)
    for fit_n in (3, 5):
        s, r, sd, _ = orc.surface(hq, defined, fit_n, res, 25, 163840)
        h = fit_n // 2
        for i in range(nx):
            for j in range(ny):
                if not defined[i, j]:
                    assert not sd[i, j] and np.isnan(s[i, j])
                    continue
                rows, rhs = [], []
                for dx in range(-h, h + 1):
                    for dy in range(-h, h + 1):
                        x, y = i + dx, j + dy
                        if 0 <= x < nx and 0 <= y < ny and defined[x, y]:
                            rows.append((dx, dy, 1.0))
                            rhs.append(float(int(hq[x, y]) - int(hq[i, j])))
                A = np.array(rows, np.float64)
                b = np.array(rhs)
                if len(rows) < 3 or np.linalg.matrix_rank(A) < 3:
                    assert not sd[i, j]
                    continue
                assert sd[i, j]
                coef, *_ = np.linalg.lstsq(A, b, rcond=None)
                res_ = b - A @ coef
                slope = np.hypot(coef[0], coef[1]) / Q
                rough = (res_ ** 2).mean() * (np.float64(np.float32(res)) / Q) ** 2
                assert abs(s[i, j] - slope) <= 1e-6 * max(slope, 1e-3)
                assert abs(r[i, j] - rough) <= 1e-6 * max(rough, 1e-9)


def test_plane_fit_degenerate(orc):
    # a single defined row: every dy = 0 -> singular normal matrix
    hq = np.zeros((7, 7), np.int32)
    defined = np.zeros((7, 7), np.uint8)
    defined[3, :] = 1
    s, r, sd, _ = orc.surface(hq, defined, 5, 0.4, 12, 81920)
    assert not sd.any()
    # two defined pixels: n < 3
    defined[:] = 0
    defined[3, 3] = defined[3, 4] = 1
    s, r, sd, _ = orc.surface(hq, defined, 5, 0.4, 12, 81920)
    assert not sd.any()
    # corner pixel: window cut at the map edge still fits a plane
    defined[:] = 1
    s, r, sd, _ = orc.surface(hq, defined, 5, 0.4, 12, 81920)
    assert sd[0, 0] and s[0, 0] == 0


# ----------------------------------------------------------------------------
# III-D negative obstacles


def _grid_from_walkthrough(g, h_green):
    res = g["res_m"]
    hq = np.zeros((g["nx"], g["ny"]), np.int32)
    df = np.zeros((g["nx"], g["ny"]), np.uint8)
    for c in g["ground_cells"]:
        h = h_green if c["height_m"] == "H_green" else c["height_m"]
        hq[tuple(c["cell"])] = int(round(h / res * Q))
        df[tuple(c["cell"])] = 1
    return hq, df


def test_negative_walkthrough(orc):
    g = json.load(open(os.path.join(GOLDEN, "negative_search_walkthrough.json")))
    s, c = orc.derive(params(8, 8, 8, g["res_m"], neg_thresh_m=g["neg_thresh_m"],
                             neg_search_m=g["neg_search_m"]))
    for e in g["expect"]:
        hq, df = _grid_from_walkthrough(g, e["H_green"])
        _, _, _, neg = orc.surface(hq, df, 5, g["res_m"], c["search_d"], c["tau_neg_q"])
        assert bool(neg[tuple(g["start"])]) == e["negative"], e["why"]


def _strip(heights):
    """A 3-pixel-wide strip along x; None = unobserved."""
    nx = len(heights)
    hq = np.zeros((nx, 3), np.int32)
    df = np.zeros((nx, 3), np.uint8)
    for i, h in enumerate(heights):
        if h is not None:
            hq[i, :] = int(round(h / 0.4 * Q))
            df[i, :] = 1
    return hq, df


def test_negative_hole_cliff_flat(orc):
    tau = 81920  # 0.5 m at 0.4 m voxels
    # hole: near rim at 0 m, unseen floor, far wall seen lower (-0.8 m)
    hq, df = _strip([0, 0, 0, None, None, None, -0.8, -0.8, 0, 0])
    neg = orc.surface(hq, df, 5, 0.4, 12, tau)[3]
    assert neg[3:6].all()
    assert not neg[df.astype(bool)].any()  # only undefined pixels are flagged
    # gap between two equal heights: not an obstacle
    hq, df = _strip([0, 0, 0, None, None, None, 0.1, 0.1])
    assert not orc.surface(hq, df, 5, 0.4, 12, tau)[3].any()
    # cliff: upper ground, hidden band, lower ground seen further out
    hq, df = _strip([1.5, 1.5, 1.5, None, None, None, None, None, None, 0, 0])
    neg = orc.surface(hq, df, 5, 0.4, 12, tau)[3]
    assert neg[3:9].all()
    # cliff whose lower ground lies beyond the search distance: nothing to compare
    hq, df = _strip([1.5, 1.5] + [None] * 20 + [0])
    neg = orc.surface(hq, df, 5, 0.4, 6, tau)[3]
    # (+x finds nothing within D = 6 pixels, -x only the upper ground)
    assert not neg[2:15].any()


def _cone_bruteforce(hq, df, D, tau):
    nx, ny = hq.shape
    out = np.zeros_like(df)
    for i in range(nx):
        for j in range(ny):
            if df[i, j]:
                continue
            cells = set()
            for dirx, diry in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                for d in range(1, D + 1):
                    ring = set()
                    for e in range(-d, d + 1):
                        x = i + dirx * d + (e if dirx == 0 else 0)
                        y = j + diry * d + (e if diry == 0 else 0)
                        if 0 <= x < nx and 0 <= y < ny and df[x, y]:
                            ring.add((x, y))
                    if ring:
                        cells |= ring
                        break
            if len(cells) >= 2:
                v = [int(hq[c]) for c in cells]
                out[i, j] = max(v) - min(v) > tau
    return out


def test_negative_random_grids_vs_bruteforce(orc):
    rng = np.random.default_rng(11)
    for _ in range(8):
        nx, ny = rng.integers(5, 30, 2)
        hq = rng.integers(-3 * Q, 3 * Q, (nx, ny)).astype(np.int32)
        df = (rng.uniform(size=(nx, ny)) < rng.uniform(0.05, 0.5)).astype(np.uint8)
        D = int(rng.integers(1, 12))
        tau = int(rng.integers(0, 2 * Q))
        neg = orc.surface(hq, df, 3, 0.3, D, tau)[3]
        assert (neg == _cone_bruteforce(hq, df, D, tau)).all()
