"""Pins of the gap-fill surrogate's oracle (a project extension, not in the
paper): the network against torch's float64 convolution (a library routine),
bf16 rounding against torch's bfloat16 conversion, the gradient against
finite differences, and the features and the fallback merge against
hand-worked cases."""
import numpy as np
import pytest
import torch

from conftest import params as map_params

from oracle import sgt, OracleMap

CIN = [16, 32, 32, 32, 32]
COUT = [32, 32, 32, 32, 2]


def _split(p):
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        w = p[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = p[o:o + co]
        o += co
        out.append((w, b))
    assert o == p.size
    return out


def _rand_params(rng, quant=None):
    p = np.zeros(sgt.num_params(), np.float32)
    o = 0
    for ci, co in zip(CIN, COUT):
        n = co * ci * 9
        p[o:o + n] = rng.normal(0, np.sqrt(2.0 / (9 * ci)), n)
        p[o + n:o + n + co] = rng.normal(0, 0.1, co)
        o += n + co
    if quant:
        p = (np.round(p.astype(np.float64) * quant) / quant).astype(np.float32)
    return p


def _bf(t, on):
    return t.float().bfloat16().double() if on else t


def _torch_forward(feat, p, round_bf16):
    x = _bf(torch.from_numpy(feat.astype(np.float64)).permute(2, 0, 1)[None], round_bf16)
    layers = _split(p)
    for l, (w, b) in enumerate(layers):
        wt = _bf(torch.from_numpy(w.astype(np.float64)), round_bf16)
        z = torch.nn.functional.conv2d(x, wt, torch.from_numpy(b.astype(np.float64)), padding=1)
        x = _bf(torch.relu(z), round_bf16) if l < 4 else z
    return x[0].permute(1, 2, 0).numpy()


def test_num_params():
    assert sgt.num_params() == sum(co * ci * 9 + co for ci, co in zip(CIN, COUT)) == 32962


@pytest.mark.parametrize("round_bf16", [False, True])
@pytest.mark.parametrize("shape", [(1, 1), (6, 7), (9, 4)])
def test_forward_equals_library_convolution(round_bf16, shape):
    rng = np.random.default_rng(3 + shape[0])
    H, W = shape
    feat = rng.normal(size=(H, W, 16)).astype(np.float32)
    p = _rand_params(rng)
    ours = sgt.forward(feat, p, round_bf16)
    ref = _torch_forward(feat, p, round_bf16)
    np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_is_nearest_even():
    """Feature values on and next to bf16 rounding ties, pushed through a
    network whose first layer copies input channel 0 (one-hot centre tap) and
    whose later layers pass channel 0 on: the output is bf16(x) for x > 0."""
    base = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                     1.0 + 2.0 ** -9, 3.0, 0.5 + 2.0 ** -10], np.float64)
    feat = np.zeros((1, base.size, 16), np.float32)
    feat[0, :, 0] = base.astype(np.float32)
    p = np.zeros(sgt.num_params(), np.float32)
    o = 0
    for ci, co in zip(CIN, COUT):
        w = np.zeros((co, ci, 3, 3), np.float32)
        w[0, 0, 1, 1] = 1.0
        p[o:o + co * ci * 9] = w.reshape(-1)
        o += co * ci * 9 + co
    out = sgt.forward(feat, p, True)[0, :, 0]
    expect = torch.from_numpy(base.astype(np.float32)).bfloat16().double().numpy()
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6; above a tie rounds up
    np.testing.assert_array_equal(expect[:3], [1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7])
    np.testing.assert_array_equal(out, expect)


def test_gradient_matches_finite_differences():
    """Within one linear region the loss is linear in any single parameter
    (every later layer is linear in it while no ReLU or L1 sign flips), so a
    central difference is exact up to rounding; a step that crosses a kink
    shows up as unequal one-sided differences and is skipped."""
    rng = np.random.default_rng(17)
    H, W = 5, 6
    feat = rng.normal(size=(H, W, 16)).astype(np.float32)
    p = _rand_params(rng, quant=2.0 ** 22)
    out = sgt.forward(feat, p, False)
    label = (out + rng.choice([-1, 1], size=out.shape) * rng.uniform(0.05, 0.5, out.shape))
    label = label.astype(np.float32)
    label[rng.uniform(size=label.shape) < 0.3] = np.nan
    loss, g = sgt.loss_grad(feat, p, label, False)
    valid = ~np.isnan(label)
    assert loss == pytest.approx(np.abs(out - label.astype(np.float64))[valid].mean(), rel=1e-12)
    offs = np.cumsum([0] + [co * ci * 9 + co for ci, co in zip(CIN, COUT)])
    idx = []
    for l in range(5):
        nw = COUT[l] * CIN[l] * 9
        idx += list(rng.choice(nw, 12, replace=False) + offs[l])
        idx += list(rng.choice(COUT[l], 2, replace=False) + offs[l] + nw)
    h = 2.0 ** -20
    checked = 0
    gmax = np.abs(g).max()
    for i in idx:
        vals = []
        for s in (-1, 0, 1):
            q = p.copy()
            q[i] = np.float32(np.float64(p[i]) + s * h)
            assert np.float64(q[i]) == np.float64(p[i]) + s * h  # exact step
            vals.append(sgt.loss_grad(feat, q, label, False)[0])
        fwd, bwd = (vals[2] - vals[1]) / h, (vals[1] - vals[0]) / h
        if abs(fwd - bwd) > 1e-7 * max(abs(fwd), gmax):
            continue  # a kink lies within the step
        fd = (vals[2] - vals[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * gmax), (i, fd, g[i])
        checked += 1
    assert checked >= 0.9 * len(idx)
    # a planted mistake is seen: dropping one bias from the gradient fails the check
    assert abs(g[offs[1] - 1]) > 1e-6 * gmax or abs(g[offs[1] - 2]) > 1e-6 * gmax


def test_fill_hand_cases():
    """Two defined columns in row 1 of a 3 x 14 grid: column 0 (plain 2,
    network 1.9375: error 1/16) and column 2 (plain 1, network 1.03125: error
    1/32); every value is exact in binary, so the tolerance tests are exact."""
    nan = np.nan
    H, W = 3, 14
    ph = np.full((H, W), nan, np.float32)
    pr = np.full((H, W), nan, np.float32)
    ph[1, 0], pr[1, 0] = 2.0, 0.25
    ph[1, 2], pr[1, 2] = 1.0, 0.5
    pred = np.zeros((H, W, 2), np.float32)
    pred[..., 0] = 1.0
    pred[..., 1] = -0.125
    pred[1, 0, 0] = 1.9375
    pred[1, 2, 0] = 1.03125
    pred[0, 3, 1] = 0.75
    oh, orr = sgt.fill(pred, ph, pr, 0.05)
    # defined columns keep the plain values
    assert oh[1, 0] == 2.0 and orr[1, 0] == 0.25 and oh[1, 2] == 1.0 and orr[1, 2] == 0.5
    # (0, 3): window columns 0..8 hold both: mean 3/64 = 0.046875 <= 0.05
    assert oh[0, 3] == 1.0 and orr[0, 3] == 0.75
    # (0, 6): columns 1..11 hold only column 2: 1/32; roughness clamped at 0
    assert oh[0, 6] == 1.0 and orr[0, 6] == 0.0
    # (1, 8): columns 3..13 hold no defined column: stays undefined
    assert np.isnan(oh[1, 8]) and np.isnan(orr[1, 8])
    # (2, 7): columns 2..12, rows clipped: column 2 only
    assert oh[2, 7] == 1.0
    # the bound is inclusive: at tol = 3/64 column (0, 3) is filled, below it not
    oh2, _ = sgt.fill(pred, ph, pr, 0.046875)
    assert oh2[0, 3] == 1.0 and oh2[0, 6] == 1.0
    oh3, orr3 = sgt.fill(pred, ph, pr, 0.046)
    assert np.isnan(oh3[0, 3]) and np.isnan(orr3[0, 3]) and oh3[0, 6] == 1.0
    # a larger error at column 0 rejects every window that contains it
    pred[1, 0, 0] = 1.75
    oh4, _ = sgt.fill(pred, ph, pr, 0.05)
    assert np.isnan(oh4[0, 3]) and np.isnan(oh4[1, 1]) and oh4[0, 6] == 1.0


def test_features_hand_built_map():
    p = map_params(6, 4, 8, 0.5)
    m = OracleMap(p)
    nx, ny, nz = 6, 4, 8
    lut = np.full((nx, ny, nz), -1, np.int32)
    data = []

    def put(x, y, z, h, ps, qz):
        lut[x, y, z] = len(data)
        data.append((h, ps, qz))
    # column (2, 1): voxels z=1 (3 hits, 1 pass) and z=4 (2 hits, 6 passes); 5 passes at z=6
    put(2, 1, 1, 3, 1, 70000)
    put(2, 1, 4, 2, 6, 300000)
    lut[2, 1, 6] = -1 - 5
    # column (4, 3): one voxel, hits 1 passes 0
    put(4, 3, 0, 1, 0, -5000)
    # column (0, 0): passes only
    lut[0, 0, 3] = -1 - 7
    origin = np.array([-3, -2, -1], np.int32)
    assert m.import_voxels(lut.reshape(-1), np.array(data, np.int32), origin) == 0
    plain = m.export_2d()
    sensor = (0.25, -0.5, 1.0)
    f = sgt.features(m, plain, sensor)
    q2m = 0.5 / 65536
    c = f[2, 1]
    assert c[0] == 5 and c[1] == 12 and c[2] == 2 and c[3] == np.float32(2 / 8)
    assert c[4] == plain["height"][2, 1] == np.float32(70000 * q2m) and c[7] == 1
    assert c[5] == np.float32(300000 * q2m)
    assert c[6] == np.float32((70000 + 300000) / 2 * q2m)
    assert c[8] == np.float32(3 / 4)
    assert c[14] == np.float32(1.0 - np.float64(np.float32(70000 * q2m)))
    cx, cy = (-3 + 2 + 0.5) * 0.5 - 0.25, (-2 + 1 + 0.5) * 0.5 + 0.5
    assert c[13] == np.float32(np.hypot(cx, cy)) and c[15] == 0
    d = f[4, 3]
    assert d[0] == 1 and d[1] == 0 and d[2] == 1 and d[5] == d[6] == np.float32(-5000 * q2m)
    assert d[8] == 1.0
    e = f[0, 0]
    assert e[1] == 7 and e[0] == e[2] == e[3] == e[4] == e[7] == e[8] == 0
    # band density and slope come from the plain maps where they are defined
    assert np.array_equal(f[..., 9] != 0, (plain["flags"] & 2) != 0)
    assert np.array_equal(f[..., 12] == 1, (plain["flags"] & 32) != 0)
    # thinning: the column's voxels are gone and only distance and the mask remain
    mask = np.zeros((nx, ny), np.uint8)
    mask[2, 1] = 1
    sgt.thin(m, mask)
    plain2 = m.export_2d()
    assert np.isnan(plain2["height"][2, 1])
    g = sgt.features(m, plain2, sensor, mask)
    assert (g[2, 1, :13] == 0).all() and g[2, 1, 14] == 0 and g[2, 1, 15] == 1
    assert g[2, 1, 13] == c[13]
    assert np.array_equal(g[4, 3], d)
    m.close()
