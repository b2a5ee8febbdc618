"""Gap-fill surrogate on the GPU against its FP64 oracle: features bit for bit,
network output and gradients within the stated tolerances, the fallback merge
bit for bit, and a trained-versus-untrained gain on held-out scenes (needs an
MI355X)."""
import numpy as np
import pytest
import torch

from oracle import sgt as osgt
from oracle import OracleMap
from synth import scenegen

pytestmark = pytest.mark.gpu

CIN = [16, 32, 32, 32, 32]
COUT = [32, 32, 32, 32, 2]


def _params(rng, bias_sd=0.1):
    p = np.zeros(osgt.num_params(), np.float32)
    o = 0
    for ci, co in zip(CIN, COUT):
        n = co * ci * 9
        p[o:o + n] = rng.normal(0, np.sqrt(2.0 / (9 * ci)), n)
        p[o + n:o + n + co] = rng.normal(0, bias_sd, co)
        o += n + co
    return p


def _offsets():
    return np.cumsum([0] + [co * ci * 9 + co for ci, co in zip(CIN, COUT)])


# Tolerance of the network output.  The GPU accumulates in fp32 where the
# oracle accumulates in fp64, and both round every layer input to bf16; an
# activation within the fp32 accumulation error (~1e-6 relative) of a bf16
# rounding boundary can round the other way, which moves it by one bf16 step
# (2^-8 relative) and the output by a small multiple of that step times one
# weight.  The bound is 1e-3 of the output scale (the largest |oracle|).
OUT_TOL = 1e-3


@pytest.mark.parametrize("shape,norm", [((37, 70), False), ((5, 130), True), ((1, 1), False),
                                        ((64, 64), False)])
def test_forward_matches_oracle(shape, norm):
    from paper_2109_13176_amd import gvom
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    net = gvom.Surrogate(H, W, seed=1)
    p = _params(rng)
    net.set_params(p)
    raw = rng.normal(size=(H, W, 16)).astype(np.float32)
    if norm:
        mean = rng.normal(size=16).astype(np.float32)
        std = rng.uniform(0.5, 3.0, 16).astype(np.float32)
        raw = (raw * std + mean).astype(np.float32)
        net.set_norm(mean, std)
        x = ((raw.astype(np.float64) - mean) / std).astype(np.float32)
    else:
        x = raw
    out = net.forward(torch.from_numpy(raw).cuda()).cpu().numpy()
    ref = osgt.forward(x, p, True)
    scale = max(np.abs(ref).max(), 1e-6)
    e = np.abs(out - ref) / scale
    err = e.max()
    print(f"forward {shape}: max error {err:.2e}, 99.9% {np.quantile(e, 0.999):.2e}, "
          f"median {np.median(e):.2e} of scale {scale:.3g}", flush=True)
    assert err <= OUT_TOL
    assert np.array_equal(net.get_params(), p)
    net.close()


def test_gradient_matches_oracle():
    """Labels sit 0.05..0.5 away from the oracle's output, so the L1 sign of
    every entry is the same on both sides; the bound is per layer, relative
    to the layer's largest gradient entry, 1e-3 (fp32 against fp64)."""
    from paper_2109_13176_amd import gvom
    H, W = 37, 70
    rng = np.random.default_rng(5)
    net = gvom.Surrogate(H, W, seed=2)
    p = _params(rng)
    net.set_params(p)
    x = rng.normal(size=(H, W, 16)).astype(np.float32)
    ref_out = osgt.forward(x, p, True)
    label = ref_out + rng.choice([-1, 1], size=ref_out.shape) * rng.uniform(0.05, 0.5, ref_out.shape)
    label = label.astype(np.float32)
    label[rng.uniform(size=label.shape) < 0.3] = np.nan
    loss, g = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(label).cuda(), True)
    ref_loss, ref_g = osgt.loss_grad(x, p, label, True)
    assert loss == pytest.approx(ref_loss, rel=1e-4)
    offs = _offsets()
    for l in range(5):
        a, b = g[offs[l]:offs[l + 1]], ref_g[offs[l]:offs[l + 1]]
        scale = np.abs(b).max()
        err = np.abs(a - b).max() / scale
        print(f"layer {l}: max gradient error {err:.2e} of scale {scale:.3g}", flush=True)
        assert err <= 1e-3, l
    net.close()


def test_adam_step_matches_definition():
    """One Adam step from zero moments moves every weight by lr * g / (|g| + eps)."""
    from paper_2109_13176_amd import gvom
    H, W = 16, 20
    rng = np.random.default_rng(8)
    net = gvom.Surrogate(H, W, seed=3)
    p = _params(rng)
    net.set_params(p)
    x = torch.from_numpy(rng.normal(size=(H, W, 16)).astype(np.float32)).cuda()
    label = torch.from_numpy(rng.normal(size=(H, W, 2)).astype(np.float32)).cuda()
    _, g = net.loss_grad(x, label, True)
    net.adam(1e-3)
    q = net.get_params()
    g64 = g.astype(np.float64)
    expect = p.astype(np.float64) - 1e-3 * g64 / (np.abs(g64) + 1e-8)
    np.testing.assert_allclose(q, expect, rtol=0, atol=2e-6)
    net.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_fill_matches_oracle(seed):
    from paper_2109_13176_amd import gvom
    rng = np.random.default_rng(seed)
    H, W = 45, 77
    ph = rng.normal(0, 2, (H, W)).astype(np.float32)
    pr = rng.uniform(0, 0.1, (H, W)).astype(np.float32)
    ph[rng.uniform(size=(H, W)) < 0.6] = np.nan
    ph[10:30, 20:50] = np.nan             # a large hole: some windows see nothing
    pred = np.stack([ph, pr], 2).astype(np.float32)
    # network error small on the left, large on the right: both outcomes occur
    sigma = np.where(np.arange(W)[None, :] < W // 2, 0.01, 0.1)
    pred[..., 0] = np.where(np.isnan(ph), rng.normal(0, 2, (H, W)), ph + rng.normal(0, 1, (H, W)) * sigma)
    pred[..., 1] = rng.normal(0, 0.05, (H, W))
    pred = pred.astype(np.float32)
    plain = {"height": torch.from_numpy(ph).cuda(), "rough": torch.from_numpy(pr).cuda()}
    for k in ("slope", "density"):
        plain[k] = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    plain["flags"] = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    for tol in (0.05, 0.02):
        gh, gr = gvom.sgt_fill(torch.from_numpy(pred).cuda(), plain, tol)
        oh, orr = osgt.fill(pred, ph, pr, tol)
        assert np.array_equal(gh.cpu().numpy().view(np.uint32), oh.view(np.uint32))
        assert np.array_equal(gr.cpu().numpy().view(np.uint32), orr.view(np.uint32))
        assert (~np.isnan(oh) & np.isnan(ph)).any() and (np.isnan(oh) & np.isnan(ph)).any()


@pytest.mark.parametrize("seed,n_scans", [(31, 1), (32, 3)])
def test_features_match_oracle(seed, n_scans):
    """Features of a thinned map (one scan, or three scans with the window
    scrolled so the storage offsets are not zero) are equal bit for bit,
    except slope and roughness, which follow the plain maps' tolerance."""
    from paper_2109_13176_amd import gvom
    from parity_util import ROUGH_RTOL, SLOPE_RTOL, Pair, compare_2d
    seq = scenegen.surrogate_sequence(seed, n_scans=n_scans, device="cuda")
    if n_scans > 1:   # move far enough between scans to scroll the window
        seq["poses"] = [np.asarray(p, np.float32).copy() for p in seq["poses"]]
        for i, p in enumerate(seq["poses"]):
            p[3] += 3.3 * i
            p[7] -= 2.1 * i
    prm = seq["params"]
    nx, ny = prm["nx"], prm["ny"]
    rng = np.random.default_rng(seed)
    mask = (rng.uniform(size=(nx, ny)) < 0.4).astype(np.uint8)
    pair = Pair(prm)
    try:
        for xyz, pose in zip(seq["scans"], seq["poses"]):
            assert pair.insert(xyz, pose, gvom.MAP_RECENTER) == 0
        thin = torch.from_numpy(mask).cuda()
        assert gvom.sgt_thin(pair.g, thin) == 0
        osgt.thin(pair.o, mask)
        g2d, o2d = compare_2d(pair)
        plain = pair.g.export_2d()
        sensor = np.asarray(seq["poses"][-1], np.float32).reshape(3, 4)[:, 3]
        f = gvom.sgt_features(pair.g, plain, sensor, thin).cpu().numpy()
        of = osgt.features(pair.o, o2d, sensor, mask)
        assert np.array_equal(pair.g.origin(), pair.o.origin())
        exact = [k for k in range(16) if k not in (10, 11)]
        bad = np.argwhere(f[..., exact].view(np.uint32) != of[..., exact].view(np.uint32))
        assert bad.size == 0, (bad[:5], f[tuple(bad[0][:2])], of[tuple(bad[0][:2])])
        r2 = float(np.float32(prm["res_m"])) ** 2
        for k, floor, tol in ((10, 1.0, SLOPE_RTOL), (11, r2, ROUGH_RTOL)):
            dd = np.abs(f[..., k].astype(np.float64) - of[..., k])
            assert (dd <= tol * np.maximum(np.abs(of[..., k]).astype(np.float64), floor)).all(), k
        assert (f[..., 7] == 1).sum() > 100 and (f[..., 15] == 1).sum() > 100
    finally:
        pair.close()


def test_training_gain_on_held_out_scenes():
    """A network trained by the library's own kernels on six sequences fills
    the gaps of two unseen sequences far better than the untrained network,
    and the fallback merge raises coverage while keeping its error small."""
    from paper_2109_13176_amd import gvom, surrogate
    train_ex = [surrogate.Example(scenegen.surrogate_sequence(100 + s, device="cuda"))
                for s in range(6)]
    test_ex = [surrogate.Example(scenegen.surrogate_sequence(900 + s, device="cuda"))
               for s in range(2)]
    H, W = train_ex[0].params["nx"], train_ex[0].params["ny"]
    net = gvom.Surrogate(H, W, seed=7)
    rng = np.random.default_rng(0)
    surrogate.fit_normalisation(net, train_ex, rng)
    before = surrogate.evaluate(net, test_ex, np.random.default_rng(1))
    losses = surrogate.train(net, train_ex, steps=600, lr=2e-3, rng=rng)
    after = surrogate.evaluate(net, test_ex, np.random.default_rng(1))
    print("untrained", before, flush=True)
    print("trained", after, flush=True)
    print("loss first/last 50:", np.mean(losses[:50]), np.mean(losses[-50:]), flush=True)
    assert np.isfinite(losses).all()
    assert np.mean(losses[-50:]) < 0.5 * np.mean(losses[:50])
    assert after["gap_mae_net"] < 0.5 * before["gap_mae_net"]
    assert after["coverage_filled"] > after["coverage_plain"]
    assert after["gap_mae_filled"] < 0.5
    for ex in train_ex + test_ex:
        ex.close()
    net.close()
