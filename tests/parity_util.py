"""Helpers for the GPU-vs-oracle parity tests (the comparison rule).

Bit-exact: lookup table, data array, origin, height (value and NaN pattern),
density, flags, counters.  Slope: |g - o| <= 1e-5 max(|o|, 1).  Roughness:
|g - o| <= 1e-5 max(|o|, r^2).  Defined masks must match exactly.
"""
import numpy as np
import torch

import oracle
from paper_2109_13176_amd import gvom

SLOPE_RTOL = 1e-5
ROUGH_RTOL = 1e-5


class Pair:
    """The HIP map and the oracle map, fed the same inputs."""

    def __init__(self, params, seg_len=0):
        self.params = dict(params)
        self.g = gvom.VoxelMap(params)
        if seg_len:
            assert gvom.map_set_tuning(self.g.h, seg_len=seg_len) == 0
        self.o = oracle.OracleMap(params)

    def insert(self, xyz, pose, flags=0, firing=0):
        xyz_np = xyz.detach().cpu().numpy() if isinstance(xyz, torch.Tensor) else np.asarray(xyz, np.float32)
        xyz_d = torch.as_tensor(xyz_np, device="cuda")
        fl = flags | (gvom.MAP_FIRING(firing) if firing else 0)
        sg = gvom.map_insert_scan(self.g.h, xyz_d if len(xyz_np) else None, pose, fl)
        so = self.o.insert_scan(xyz_np, pose, flags & oracle.RECENTER)
        assert sg == so, (sg, so)
        return sg

    def close(self):
        self.g.close()
        self.o.close()


def compare_stats(pair, distinct=False):
    gs = pair.g.stats()
    os_ = pair.o.stats()
    keys = ["n_points", "n_nonfinite", "n_range", "n_hits", "n_pass", "n_cleared"]
    if distinct:
        keys += ["n_distinct_pass", "n_distinct_hit"]
    for k in keys:
        assert gs[k] == os_[k], (k, gs[k], os_[k])
    return gs


def compare_voxels(pair):
    lut, data, n_occ, origin = pair.g.export_voxels()
    torch.cuda.synchronize()
    s, lut_o, data_o, n_o, origin_o = pair.o.export_voxels()
    assert s == 0
    n_g = n_occ
    assert n_g == n_o, (n_g, n_o)
    assert (origin == origin_o).all(), (origin, origin_o)
    lut_g = lut.cpu().numpy()
    bad = np.nonzero(lut_g != lut_o)[0]
    assert bad.size == 0, f"{bad.size} LUT mismatches, first at {bad[:5]}: {lut_g[bad[:5]]} vs {lut_o[bad[:5]]}"
    assert (data[:n_g].cpu().numpy() == data_o).all()
    return n_g


def compare_2d_arrays(g, o, res_m):
    """g, o: dicts of host arrays (height, slope, rough, density, flags)."""
    r2 = float(np.float32(res_m)) ** 2
    fb = np.nonzero(g["flags"] != o["flags"])
    assert fb[0].size == 0, f"{fb[0].size} flag mismatches at {list(zip(*fb))[:5]}: " \
        f"{g['flags'][fb][:5]} vs {o['flags'][fb][:5]}"
    for k in ("height", "density"):
        gb, ob = g[k].view(np.uint32), o[k].view(np.uint32)
        bad = np.nonzero(gb != ob)
        assert bad[0].size == 0, f"{k}: {bad[0].size} mismatches, e.g. {g[k][bad][:5]} vs {o[k][bad][:5]}"
    for k, floor, tol in (("slope", 1.0, SLOPE_RTOL), ("rough", r2, ROUGH_RTOL)):
        gn, on = np.isnan(g[k]), np.isnan(o[k])
        assert (gn == on).all(), f"{k} defined masks differ at {np.argwhere(gn != on)[:5]}"
        d = np.abs(g[k][~on].astype(np.float64) - o[k][~on])
        lim = tol * np.maximum(np.abs(o[k][~on]).astype(np.float64), floor)
        assert (d <= lim).all(), f"{k}: max excess {np.max(d - lim)}"


def host_2d(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


def compare_2d(pair):
    out = pair.g.export_2d()
    torch.cuda.synchronize()
    g = host_2d(out)
    o = pair.o.export_2d()
    compare_2d_arrays(g, o, pair.params["res_m"])
    return g, o


class OracleTrack:
    """The oracle side of a long full-size parity run.

    Inserts run in order on one oracle map.  A 2D export of the oracle map at
    the largest windows takes seconds, so it runs on a worker thread, on a
    fresh oracle map that imports the oracle's own exported state (lookup
    table, data array, origin): the 2D maps are a function of that state.
    Nothing here takes a value from the HIP path.
    """

    def __init__(self, params, workers=8):
        from concurrent.futures import ThreadPoolExecutor
        self.params = dict(params)
        self.o = oracle.OracleMap(params)
        self.pool = ThreadPoolExecutor(max_workers=workers)

    def insert(self, xyz_np, pose, flags):
        return self.o.insert_scan(xyz_np, pose, flags & oracle.RECENTER)

    def voxels(self):
        s, lut, data, n, origin = self.o.export_voxels()
        assert s == oracle.OK
        return lut, np.ascontiguousarray(data), n, origin

    def submit_2d(self, lut, data, origin):
        params = self.params

        def job():
            m = oracle.OracleMap(params)
            try:
                assert m.import_voxels(lut, data, origin) == oracle.OK
                return m.export_2d()
            finally:
                m.close()
        return self.pool.submit(job)

    def close(self):
        self.pool.shutdown(wait=True)
        self.o.close()


def compare_voxel_arrays(gpu_export, lut_o, data_o, n_o, origin_o):
    lut, data, n_g, origin = gpu_export
    assert n_g == n_o, (n_g, n_o)
    assert (origin == origin_o).all(), (origin, origin_o)
    lut_g = lut.cpu().numpy()
    bad = np.nonzero(lut_g != lut_o)[0]
    assert bad.size == 0, f"{bad.size} LUT mismatches, first at {bad[:5]}: {lut_g[bad[:5]]} vs {lut_o[bad[:5]]}"
    assert (data[:n_g].cpu().numpy() == data_o).all()


def compare_all(pair, distinct=False):
    compare_stats(pair, distinct)
    n = compare_voxels(pair)
    g, o = compare_2d(pair)
    return n, g, o
