"""Voxel-map density export and planner costmap: the HIP path against the
oracle (needs an MI355X).  Density: bit-exact.  Costmap: the GPU adds the
eight weighted terms in binary32 (one rounding per product and per addition,
each at most 2^-24 of a partial sum bounded by the sum of the terms'
magnitudes), so |gpu - oracle| <= 2^-20 * sum |w_k layer_k|."""
import numpy as np
import pytest
import torch

from conftest import params
from parity_util import Pair
from synth import scenegen

pytestmark = pytest.mark.gpu

COST_TOL = 2.0 ** -20


def _cloud(rng, n, radius):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-12
    p = d * (radius * rng.uniform(size=(n, 1)) ** 0.5)
    p[rng.uniform(size=n) < 0.05] = np.nan
    return p.astype(np.float32)


def _compare_density(pair):
    g = pair.g.export_density()
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    o = pair.o.export_density()
    bad = np.nonzero(g.view(np.uint32) != o.view(np.uint32))[0]
    assert bad.size == 0, f"{bad.size} density mismatches, e.g. {bad[:5]}: {g[bad[:5]]} vs {o[bad[:5]]}"
    return g


def _compare_costmap(pair, weights):
    import oracle
    from paper_2109_13176_amd import gvom
    out = pair.g.export_2d()
    cost = pair.g.costmap(weights)
    torch.cuda.synchronize()
    g = cost.cpu().numpy()
    o, mag = oracle.costmap({k: v.cpu().numpy() for k, v in out.items()}, weights)
    err = np.abs(g.astype(np.float64) - o)
    assert (err <= COST_TOL * mag).all(), f"max excess {np.max(err - COST_TOL * mag)}"
    return g


WEIGHTS = [
    {"slope": 2.0, "rough": 40.0, "density": 5.0, "positive": 1.0, "hard": 100.0, "soft": 3.0,
     "negative": 50.0, "unknown": 7.0},
    {"slope": -0.37, "rough": 1e3, "density": 0.1, "hard": 12.5, "unknown": -2.0},
]


@pytest.mark.parametrize("dims", [(16, 16, 16, 0.5), (18, 10, 12, 0.25), (40, 26, 7, 0.3),
                                  (30, 34, 96, 0.1), (20, 22, 128, 0.15), (64, 64, 32, 0.4)])
def test_density_and_costmap_shapes(dims):
    nx, ny, nz, res = dims
    rng = np.random.default_rng(nx * 10 + nz)
    pair = Pair(params(nx, ny, nz, res))
    try:
        for k in range(3):
            ang = rng.uniform(-np.pi, np.pi, 3) * np.array([1, 0.3, 0.3])
            pose = scenegen.pose12(scenegen.rot_zyx(*ang), rng.uniform(-1, 1, 3) * res * 3)
            pts = _cloud(rng, 4000, 0.6 * max(nx, ny, nz) * res)
            assert pair.insert(pts, pose, 1) == 0
            d = _compare_density(pair)
            for w in WEIGHTS:
                _compare_costmap(pair, w)
        assert (d == 0).any() and (d > 0).any() and np.isnan(d).any()
    finally:
        pair.close()


def test_costmap_rejects_non_finite_weights():
    from paper_2109_13176_amd import gvom
    m = gvom.VoxelMap(params(16, 16, 16, 0.5))
    try:
        out = m.export_2d()
        cost = torch.empty_like(out["height"])
        assert gvom.map_costmap(m.h, out, {"slope": float("inf")}, cost) == gvom.MAP_E_INVALID
        assert gvom.map_costmap(m.h, out, {"hard": float("nan")}, cost) == gvom.MAP_E_INVALID
        assert gvom.map_costmap(m.h, out, {"unknown": 1.0}, cost) == 0
        torch.cuda.synchronize()
        assert (cost == 1.0).all()  # an empty map: every height undefined
    finally:
        m.close()


def test_64beam_full_size():
    """Density and costmap of the 512 x 512 x 64 window after three scans of
    the 64-beam sequence (firing width 64, as the benchmark runs it)."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=3, device="cuda")
    pair = Pair(seq["params"])
    try:
        for k in range(3):
            print(f"64-beam scan {k}", flush=True)
            assert pair.insert(seq["scans"][k], seq["poses"][k], gvom.MAP_RECENTER, firing=64) == 0
        d = _compare_density(pair)
        assert (d > 0).sum() > 20000
        c = _compare_costmap(pair, WEIGHTS[0])
        assert (c >= 100).any() and (c < 100).any()
    finally:
        pair.close()
