"""Parity at the benchmark workloads' full sizes and lengths (needs an MI355X).

* every scan of the 100-scan 64-beam sequence on 512 x 512 x 64, compared
  after each scan (the benchmark times scans of this same sequence);
* ten consecutive three-lidar frames on 1024 x 1024 x 96, compared after
  each frame (counters after each of the three inserts);
* two autotuned graph steps of all 32 batched vehicles, every map compared
  with its own oracle map after each step.

Each comparison is element by element: lookup table, data array, origin,
counters, height, density and flags bit for bit, slope and roughness within
the stated tolerance.  The launch configuration is the benchmark's (firing
width, default tuning; the batch's autotuned tuning and graph replay).
"""
import numpy as np
import pytest
import torch

import oracle
from parity_util import (OracleTrack, Pair, compare_2d_arrays, compare_all,
                         compare_voxel_arrays, host_2d)
from synth import scenegen

pytestmark = pytest.mark.gpu

STAT_KEYS = ("n_points", "n_nonfinite", "n_range", "n_hits", "n_pass", "n_cleared")


class _Run:
    """State carried from one block of a long sequence to the next."""

    def __init__(self, work, gmap, track):
        self.work, self.g, self.o, self.next = work, gmap, track, 0
        self.flag_counts = np.zeros(3, np.int64)

    def close(self):
        self.g.close()
        self.o.close()


def _stats_equal(gmap, track, what):
    gs, os_ = gmap.stats(), track.o.stats()
    for k in STAT_KEYS:
        assert gs[k] == os_[k], (what, k, gs[k], os_[k])


def _compare_state(run, what, pending):
    """2D export then table export (the benchmark's order: the table export
    reuses the column pass's ranks); the oracle's 2D maps come from a worker."""
    g2d = host_2d(run.g.export_2d())
    gv = run.g.export_voxels()
    lut_o, data_o, n_o, org_o = run.o.voxels()
    compare_voxel_arrays(gv, lut_o, data_o, n_o, org_o)
    pending.append((what, g2d, run.o.submit_2d(lut_o, data_o, org_o)))


def _drain(run, pending):
    res = run.work["params"]["res_m"]
    for what, g2d, fut in pending:
        o2d = fut.result()
        try:
            compare_2d_arrays(g2d, o2d, res)
        except AssertionError as e:
            raise AssertionError(f"{what}: {e}") from None
        fl = g2d["flags"]
        run.flag_counts += [(fl & 4).any(), (fl & 8).any(), (fl & 16).any()]
    pending.clear()


@pytest.fixture(scope="module")
def seq64():
    from paper_2109_13176_amd import gvom
    work = scenegen.sequence_64beam(seed=2, n_scans=100, device="cuda")
    run = _Run(work, gvom.VoxelMap(work["params"]), OracleTrack(work["params"]))
    yield run
    run.close()


@pytest.mark.parametrize("first", [0, 25, 50, 75])
def test_64beam_sequence_every_scan(seq64, first):
    """Scans first .. first+24 of the 100-scan sequence, recentred every scan,
    firing width 64; compared after each scan.  Blocks run in order on one
    map pair (a block run alone first inserts the scans before it)."""
    from paper_2109_13176_amd import gvom
    run, work = seq64, seq64.work
    pending = []
    while run.next < first + 25:
        k = run.next
        print(f"64-beam scan {k}", flush=True)
        xyz = work["scans"][k]
        run.g.insert(xyz, work["poses"][k], gvom.MAP_RECENTER | gvom.MAP_FIRING(64))
        assert run.o.insert(xyz.cpu().numpy(), work["poses"][k], oracle.RECENTER) == 0
        run.next += 1
        if k >= first:
            _stats_equal(run.g, run.o, f"scan {k}")
            _compare_state(run, f"scan {k}", pending)
        if len(pending) >= 8:
            _drain(run, pending)
    _drain(run, pending)
    if first == 75:
        assert run.flag_counts.min() > 0  # hard, soft and negative pixels were seen


@pytest.fixture(scope="module")
def frames3():
    from paper_2109_13176_amd import gvom
    work = scenegen.multi_lidar_frames(seed=3, n_frames=50, n_sim=10, device="cuda")
    run = _Run(work, gvom.VoxelMap(work["params"]), OracleTrack(work["params"]))
    yield run
    run.close()


@pytest.mark.parametrize("first", [0, 5])
def test_three_lidar_frames_each_frame(frames3, first):
    """Frames first .. first+4 of the three-lidar workload: the 128-beam scan
    recentres, the two 32-beam scans do not; counters compared after every
    insert, the whole map after every frame."""
    from paper_2109_13176_amd import gvom
    run, work = frames3, frames3.work
    pending = []
    while run.next < first + 5:
        f = run.next
        for j in range(3):
            i = 3 * f + j
            xyz, pose, fl, fw = work["scans"][i], work["poses"][i], work["flags"][i], work["firing"][i]
            print(f"three-lidar frame {f} insert {j}: {xyz.shape[0]} points", flush=True)
            run.g.insert(xyz, pose, fl | gvom.MAP_FIRING(fw))
            assert run.o.insert(xyz.cpu().numpy(), pose, fl) == 0
            if f >= first:
                _stats_equal(run.g, run.o, f"frame {f} insert {j}")
        run.next += 1
        if f >= first:
            _compare_state(run, f"frame {f}", pending)
    _drain(run, pending)


def test_batched_32_vehicles_autotuned_full_size():
    """All 32 vehicles of the batched workload (scan sizes 20k-330k points,
    256 x 256 x 48 or 512 x 512 x 64 grids): the autotuner picks the tuning,
    then two graph-replayed batch steps; after each step every map's batch
    outputs (2D maps, lookup table, data array, occupied count) equal its own
    oracle map's."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2109_13176_amd import gvom
    veh = scenegen.batch_of_vehicles(32, n_steps=100, n_sim=2, device="cuda")
    maps = [gvom.VoxelMap(v["params"]) for v in veh]
    orcs = [oracle.OracleMap(v["params"]) for v in veh]
    batch = gvom.MapBatch(maps)
    pool = ThreadPoolExecutor(max_workers=8)

    def oracle_step(i, k):
        o = orcs[i]
        assert o.insert_scan(veh[i]["scans"][k].cpu().numpy(), veh[i]["poses"][k],
                             oracle.RECENTER) == 0
        s, lut, data, n, origin = o.export_voxels()
        assert s == oracle.OK
        return lut, np.ascontiguousarray(data), n, origin, o.export_2d()

    try:
        flags = [gvom.MAP_RECENTER | gvom.MAP_FIRING(v["firing"]) for v in veh]
        x0 = [v["scans"][0].contiguous() for v in veh]
        tuned = batch.autotune(x0, [v["poses"][0] for v in veh], flags)
        print("autotuned", tuned, flush=True)
        for k in range(2):
            xyzs = [v["scans"][k].contiguous() for v in veh]
            print("batch step", k, [x.shape[0] for x in xyzs], flush=True)
            futs = [pool.submit(oracle_step, i, k) for i in range(32)]
            batch.step(xyzs, [v["poses"][k] for v in veh], flags, [True] * 32)
            torch.cuda.synchronize()
            for i, (m, fut) in enumerate(zip(maps, futs)):
                lut_o, data_o, n_o, org_o, o2d = fut.result()
                n_g = int(m.n_occ.item())
                compare_voxel_arrays((m.lut, m.data, n_g, m.origin()), lut_o, data_o, n_o, org_o)
                try:
                    compare_2d_arrays(host_2d(m.out2d), o2d, veh[i]["params"]["res_m"])
                except AssertionError as e:
                    raise AssertionError(f"step {k} map {i}: {e}") from None
    finally:
        pool.shutdown(wait=True)
        batch.close()
        for m in maps:
            m.close()
        for o in orcs:
            o.close()


@pytest.mark.parametrize("seg_len", [8, 5])
def test_64beam_scans_segment_lengths(seg_len):
    """The first three scans of the sequence with the default segment length
    and with one that cuts rays at other cells."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=3, device="cuda")
    pair = Pair(seq["params"], seg_len)
    try:
        for k in range(3):
            print(f"64-beam scan {k}, segment length {seg_len}", flush=True)
            assert pair.insert(seq["scans"][k], seq["poses"][k], gvom.MAP_RECENTER,
                               firing=64) == 0
        n, g, o = compare_all(pair)
        assert n > 20000
    finally:
        pair.close()
