"""Parity at the benchmark workloads' full sizes (needs an MI355X): the
64-beam sequence on 512 x 512 x 64, a three-lidar frame on 1024 x 1024 x 96,
and batched vehicles of uneven scan sizes, each compared with the oracle
element by element (and, for the batch, with single-map inserts bit for
bit)."""
import numpy as np
import pytest
import torch

from parity_util import Pair, compare_all
from synth import scenegen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("traversal", [2, 1])
def test_64beam_sequence_full_size(traversal):
    """Three consecutive 131,072-point scans, recentred every scan, in the
    launch configuration the benchmark times (firing width 64)."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_scans=3, device="cuda")
    pair = Pair(seq["params"], traversal)
    try:
        for k in range(3):
            print(f"64-beam scan {k}, traversal {traversal}", flush=True)
            assert pair.insert(seq["scans"][k], seq["poses"][k], gvom.MAP_RECENTER,
                               firing=64) == 0
        n, g, o = compare_all(pair)
        assert n > 20000
        assert (g["flags"] & 4).any() and (g["flags"] & 8).any() and (g["flags"] & 16).any()
    finally:
        pair.close()


def test_three_lidar_frame_full_size():
    """One frame of the three-lidar workload on the 1024 x 1024 x 96 window:
    the 128-beam scan recentres, the two 32-beam scans do not."""
    from paper_2109_13176_amd import gvom
    fr = scenegen.multi_lidar_frames(seed=3, n_frames=1, device="cuda")
    pair = Pair(fr["params"])
    try:
        for xyz, pose, fl, fw in zip(fr["scans"], fr["poses"], fr["flags"], fr["firing"]):
            print(f"three-lidar insert of {xyz.shape[0]} points", flush=True)
            assert pair.insert(xyz, pose, fl, firing=fw) == 0
        n, g, o = compare_all(pair)
        assert n > 10000
    finally:
        pair.close()


def test_batched_vehicles_full_size():
    """Three vehicles of the batched workload (scan sizes drawn from 20k to
    330k points, 256 x 256 x 48 or 512 x 512 x 64 grids), two steps: batch
    results equal single-map inserts bit for bit, and the single maps equal
    the oracle."""
    from paper_2109_13176_amd import gvom
    veh = scenegen.batch_of_vehicles(3, 2, device="cuda")
    bmaps = [gvom.VoxelMap(v["params"]) for v in veh]
    pairs = [Pair(v["params"]) for v in veh]
    batch = gvom.MapBatch(bmaps)
    try:
        for k in range(2):
            xyzs = [v["scans"][k].contiguous() for v in veh]
            poses = [v["poses"][k] for v in veh]
            print("batch step", k, [x.shape[0] for x in xyzs], flush=True)
            flags = [gvom.MAP_RECENTER | gvom.MAP_FIRING(v["firing"]) for v in veh]
            batch.step(xyzs, poses, flags, [True] * 3)
            for i, p in enumerate(pairs):
                assert p.insert(xyzs[i], poses[i], gvom.MAP_RECENTER, firing=veh[i]["firing"]) == 0
        for bm, p in zip(bmaps, pairs):
            lut_b, data_b, n_b, org_b = bm.export_voxels()
            lut_s, data_s, n_s, org_s = p.g.export_voxels()
            torch.cuda.synchronize()
            assert int(n_b.item()) == int(n_s.item()) and np.array_equal(org_b, org_s)
            assert torch.equal(lut_b, lut_s)
            k = int(n_s.item())
            assert torch.equal(data_b[:k], data_s[:k])
            ob, os_ = bm.export_2d(), p.g.export_2d()
            for key in ob:
                assert torch.equal(ob[key].view(torch.uint8), os_[key].view(torch.uint8)), key
            compare_all(p)
    finally:
        batch.close()
        for m in bmaps:
            m.close()
        for p in pairs:
            p.close()
