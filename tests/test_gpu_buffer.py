"""Map buffer and combine (Sec. III-B, III-C, III-D): the HIP buffer against the
oracle's buffer, element by element on seeded inputs (needs an MI355X)."""
import types

import numpy as np
import pytest
import torch

import oracle
from conftest import params
from parity_util import compare_2d, compare_voxels
from synth import scenegen

pytestmark = pytest.mark.gpu


def _cloud(rng, n, radius):
    """Points in a ball of `radius` around the sensor (sensor frame), 5% NaN."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-12
    p = d * (radius * rng.uniform(size=(n, 1)) ** 0.5)
    p[rng.uniform(size=n) < 0.05] = np.nan
    return p.astype(np.float32)


class BufPair:
    """The HIP buffer + combined map and the oracle's, fed the same scans."""

    def __init__(self, prm, depth, stream=None):
        from paper_2109_13176_amd import gvom
        self.gvom = gvom
        self.params = dict(prm)
        self.g = gvom.ScanBuffer(prm, depth, stream)
        self.gm = gvom.VoxelMap(prm)
        self.o = oracle.OracleBuffer(prm, depth)
        self.om = oracle.OracleMap(prm)
        self.view = types.SimpleNamespace(g=self.gm, o=self.om, params=self.params)

    def push(self, xyz, pose, flags=0, firing=0):
        xyz_np = xyz.detach().cpu().numpy() if isinstance(xyz, torch.Tensor) else xyz
        xyz_d = torch.as_tensor(xyz_np, device="cuda") if len(xyz_np) else None
        fl = flags | (self.gvom.MAP_FIRING(firing) if firing else 0)
        sg = self.gvom.map_buffer_push(self.g.h, xyz_d, pose, fl)
        so = self.o.push(xyz_np, pose, flags & oracle.RECENTER)
        assert sg == so, (sg, so)
        return sg

    def combine(self):
        sg = self.gvom.map_buffer_combine(self.g.h, self.gm.h)
        so = self.o.combine(self.om)
        assert sg == so, (sg, so)
        return sg

    def compare(self):
        n = compare_voxels(self.view)
        compare_2d(self.view)
        return n

    def close(self):
        self.g.close()
        self.gm.close()
        self.o.close()
        self.om.close()


def test_moving_sequence_with_second_lidar_and_eviction():
    rng = np.random.default_rng(11)
    bp = BufPair(params(32, 24, 16, 0.5, szv=6), depth=3)
    try:
        sizes = [3001, 0, 65, 1, 4000, 2500, 257]
        for k, n in enumerate(sizes):
            ang = rng.uniform(-0.4, 0.4, 3) * np.array([1, 0.3, 0.3])
            t = np.array([0.9 * k, -0.4 * k, 0.1 * k]) + rng.uniform(-0.3, 0.3, 3)
            pose = scenegen.pose12(scenegen.rot_zyx(*ang), t)
            recentre = k != 3  # scan 3 is a second lidar sharing scan 2's window
            if not recentre:
                pose = scenegen.pose12(scenegen.rot_zyx(*ang), prev_t + [0.4, 0.3, -0.2])
            print(f"push {k}: {n} points, recentre {recentre}", flush=True)
            assert bp.push(_cloud(rng, n, 7.0), pose, 1 if recentre else 0) == 0
            prev_t = t
            assert bp.g.count() == min(k + 1, 3)
            assert bp.combine() == 0
            bp.compare()
    finally:
        bp.close()


def test_producer_on_its_own_stream():
    """Pushes on a second stream, combine and exports on the output map's
    stream: the events order them."""
    from paper_2109_13176_amd import gvom
    rng = np.random.default_rng(12)
    side = torch.cuda.Stream()
    bp = BufPair(params(40, 40, 24, 0.4), depth=4, stream=side)
    try:
        for k in range(6):
            pose = scenegen.pose12(scenegen.rot_zyx(0.1 * k, 0.02, -0.03), [0.5 * k, 0.2 * k, 0.0])
            pts = _cloud(rng, 6000, 9.0)
            assert bp.push(pts, pose, gvom.MAP_RECENTER) == 0
            assert bp.combine() == 0
            out = bp.gm.export_2d()  # enqueued on the output map's stream
        torch.cuda.synchronize()
        bp.compare()
        assert torch.isfinite(out["height"]).any()
    finally:
        bp.close()


@pytest.mark.parametrize("dims", [(18, 10, 12, 0.25), (40, 26, 7, 0.3), (30, 34, 96, 0.1),
                                  (20, 22, 128, 0.15), (24, 24, 48, 0.4)])
def test_window_shapes(dims):
    nx, ny, nz, res = dims
    rng = np.random.default_rng(nx * 100 + nz)
    bp = BufPair(params(nx, ny, nz, res), depth=2)
    try:
        for k in range(3):
            ang = rng.uniform(-np.pi, np.pi, 3) * np.array([1, 0.3, 0.3])
            pose = scenegen.pose12(scenegen.rot_zyx(*ang), rng.uniform(-1, 1, 3) * res * 4)
            pts = _cloud(rng, 3000, 0.6 * max(nx, ny, nz) * res)
            assert bp.push(pts, pose, 1) == 0
            assert bp.combine() == 0
            bp.compare()
    finally:
        bp.close()


def test_errors_leave_buffer_unchanged():
    from paper_2109_13176_amd import gvom
    rng = np.random.default_rng(13)
    P = params(16, 16, 16, 0.5)
    bp = BufPair(P, depth=2)
    other = gvom.VoxelMap(params(16, 16, 8, 0.5))
    try:
        assert bp.combine() == gvom.MAP_E_INVALID  # nothing buffered yet
        pts = _cloud(rng, 500, 4.0)
        assert bp.push(pts, scenegen.pose12(np.eye(3), [0.2, 0.1, 0.0]), 1) == 0
        bad = scenegen.pose12(np.eye(3), [0.0, 0.0, 0.0])
        bad[1] = np.nan
        assert bp.push(pts, bad, 1) == gvom.MAP_E_POSE
        assert bp.push(pts, scenegen.pose12(np.eye(3), [40.0, 0, 0]), 0) == gvom.MAP_E_SENSOR_OUTSIDE
        assert bp.g.count() == 1
        assert gvom.map_buffer_combine(bp.g.h, other.h) == gvom.MAP_E_INVALID
        assert bp.combine() == 0
        bp.compare()
        assert gvom.map_buffer_reset(bp.g.h) == 0 and bp.g.count() == 0
        assert gvom.map_buffer_combine(bp.g.h, bp.gm.h) == gvom.MAP_E_INVALID
    finally:
        other.close()
        bp.close()


def test_64beam_sequence_full_size():
    """Five 131,072-point scans of the 64-beam sequence on 512 x 512 x 64
    through a buffer of depth 4 (the first scan evicted), in the launch
    configuration of the benchmark (firing width 64)."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=5, device="cuda")
    bp = BufPair(seq["params"], depth=4)
    try:
        for k in range(5):
            print(f"64-beam push {k}", flush=True)
            assert bp.push(seq["scans"][k], seq["poses"][k], gvom.MAP_RECENTER, firing=64) == 0
        st = bp.g.stats()
        assert st["n_points"] == seq["scans"][4].shape[0]
        assert bp.combine() == 0
        n = bp.compare()
        assert n > 20000
    finally:
        bp.close()


@pytest.mark.parametrize("depth", [1, 3])
def test_incremental_and_full_combines_interleaved(depth):
    """Every way a combine can follow the previous one: one push later into
    the same unchanged map (updated in place), several pushes later, no push,
    another output map, an output map changed in between, a window jump; each
    result is compared with the oracle."""
    from paper_2109_13176_amd import gvom
    rng = np.random.default_rng(14 + depth)
    P = params(40, 40, 24, 0.4)
    bp = BufPair(P, depth=depth)
    g2, o2 = gvom.VoxelMap(P), oracle.OracleMap(P)
    view2 = types.SimpleNamespace(g=g2, o=o2, params=bp.params)
    t = [0.0, 0.0, 0.0]

    def push(step=(0.45, 0.2, 0.05), flags=1):
        t[0] += step[0]
        t[1] += step[1]
        t[2] += step[2]
        pose = scenegen.pose12(scenegen.rot_zyx(rng.uniform(-0.5, 0.5), 0.03, -0.02), t)
        assert bp.push(_cloud(rng, 5000, 9.0), pose, flags) == 0

    def combine_second():
        assert gvom.map_buffer_combine(bp.g.h, g2.h) == bp.o.combine(o2) == 0
        compare_voxels(view2)
        compare_2d(view2)

    try:
        for k in range(5):           # first combine in full, then updates, evictions from k = 3
            push()
            assert bp.combine() == 0
            bp.compare()
        push()
        push(flags=0)                # two pushes (a second lidar) before one combine
        assert bp.combine() == 0
        bp.compare()
        assert bp.combine() == 0     # no push since the last combine
        bp.compare()
        push()
        combine_second()             # another output map
        push()
        assert bp.combine() == 0     # the first map was not the last output
        bp.compare()
        push()
        assert bp.combine() == 0     # updated in place again
        bp.compare()
        extra = _cloud(rng, 800, 5.0)
        bp.gm.insert(torch.as_tensor(extra, device="cuda"), scenegen.pose12(np.eye(3), t), 0)
        assert bp.om.insert_scan(extra, scenegen.pose12(np.eye(3), t), 0) == 0
        push()
        assert bp.combine() == 0     # the output map changed in between
        bp.compare()
        push(step=(60.0, -20.0, 1.0))  # the window jumps: every voxel enters
        assert bp.combine() == 0
        bp.compare()
        for k in range(3):
            push()
            assert bp.combine() == 0
            bp.compare()
    finally:
        g2.close()
        o2.close()
        bp.close()


def test_incremental_equals_full_combine_full_size():
    """Thirteen scans of the 64-beam sequence through two buffers of depth
    10, one updating its output map, one combining in full every time: the
    outputs are bit-identical after every step (three evictions), and equal
    the oracle's at the end."""
    from paper_2109_13176_amd import gvom
    seq = scenegen.sequence_64beam(seed=2, n_sim=13, device="cuda")
    prm = seq["params"]
    inc = BufPair(prm, depth=10)
    full = gvom.ScanBuffer(prm, 10)
    full.set_incremental(False)
    fm = gvom.VoxelMap(prm)
    try:
        fl = gvom.MAP_RECENTER | gvom.MAP_FIRING(64)
        for k in range(13):
            print(f"64-beam step {k}", flush=True)
            xyz = seq["scans"][k].contiguous()
            assert gvom.map_buffer_push(inc.g.h, xyz, seq["poses"][k], fl) == 0
            full.push(xyz, seq["poses"][k], fl)
            assert gvom.map_buffer_combine(inc.g.h, inc.gm.h) == 0
            full.combine(fm)
            a = inc.gm.export_voxels()
            lut_a, data_a, n_a = a[0].clone(), a[1].clone(), a[2]
            b = fm.export_voxels()
            assert n_a == b[2] and np.array_equal(a[3], b[3])
            assert torch.equal(lut_a, b[0]) and torch.equal(data_a[:n_a], b[1][:n_a])
            oa, ob = inc.gm.export_2d(), fm.export_2d()
            for key in oa:
                assert torch.equal(oa[key].view(torch.uint8), ob[key].view(torch.uint8)), key
        for k in range(13):
            assert inc.o.push(seq["scans"][k].cpu().numpy(), seq["poses"][k], oracle.RECENTER) == 0
        assert inc.o.combine(inc.om) == 0
        assert inc.compare() > 20000
    finally:
        fm.close()
        full.close()
        inc.close()


def test_three_lidar_frame_full_size():
    """One frame of the three-lidar workload on 1024 x 1024 x 96 through a
    buffer: the 128-beam scan recentres, the two 32-beam scans take its
    window (three maps of one frame, combined)."""
    from paper_2109_13176_amd import gvom
    fr = scenegen.multi_lidar_frames(seed=3, n_sim=1, device="cuda")
    bp = BufPair(fr["params"], depth=3)
    try:
        for xyz, pose, fl, fw in zip(fr["scans"], fr["poses"], fr["flags"], fr["firing"]):
            print(f"three-lidar push of {xyz.shape[0]} points", flush=True)
            assert bp.push(xyz, pose, fl, firing=fw) == 0
        assert bp.g.count() == 3
        assert bp.combine() == 0
        assert bp.compare() > 10000
    finally:
        bp.close()
