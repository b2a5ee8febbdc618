#!/usr/bin/env python3
"""Benchmark of the per-scan voxel-mapping path on one MI355X.

Workload: a seeded 100-scan sequence of 64-beam x 2048-azimuth lidar scans
(131,072 points each, 100 m range, 0.02 m noise) driven along a spline at
4.5 m/s, one scan per 0.1 s, mapped into a 512 x 512 x 64 voxel window at
0.2 m that recentres on the vehicle every scan.  One step = one map update =
map_insert_scan (transform, returns, ray traversal, window scroll) +
map_export_2d (height, obstacles, density, slope, roughness, negative
obstacles) + map_export_voxels (lookup table + data array).  Inputs are
resident in HBM before the timed region.

Prints one JSON line: points/s (value), map updates/s, per-phase kernel
times from HIP events on the library's stream, the roofline of the dominant
kernel, and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lidar points/sec ingested + map updates/sec (64-beam, 512x512x64) on 1 MI355X"
HBM_PEAK_GBS = 8000.0
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s (non-packed)
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2109_13176_amd", "csrc")
# sources of the traversal kernel (k_trace) whose counters are committed
TRACE_SRCS = [os.path.join(CSRC, f)
              for f in ("insert.hip", "insert_body.h", "ray_common.h", "gvom_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def phase_bytes(params, st, n_occ):
    """Algorithmic HBM bytes per launch of each phase."""
    nx, ny, nz = params["nx"], params["ny"], params["nz"]
    V, C, W = nx * ny * nz, nx * ny, (nz + 63) // 64
    return {
        # points read; hits and min height read+write per distinct hit voxel
        "rays": 12 * st["n_points"] + 16 * st["n_distinct_hit"],
        # passes read+write per distinct passed voxel
        "trace": 8 * st["n_distinct_pass"],
        "scroll": 12 * st["n_cleared"],
        # occupancy word, ground-voxel height, outputs (height, density, flags, Q height)
        "column": C * (8 * W + 4 + 13),
        # Q heights + flags in; slope, roughness, flags out
        "surface": C * (4 + 1 + 8 + 1),
        # occupancy (twice), passes of every voxel, lookup table out, data array
        # out, hits + min height of occupied voxels
        "lut": 2 * 8 * C * W + 4 * V + 4 * V + 12 * n_occ + 8 * n_occ,
    }


def read_summary(name):
    """key: value lines of a committed profile summary (None if absent)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.rsplit(":", 1)  # keys may hold a colon ("sha256[:16]")
            out[k.strip()] = v.strip()
    return out


def source_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_line_requests():
    """Atomic line requests per traversal phase (TCC_ATOMIC of the traversal
    and the sensor-box fold) from the committed PMC summary, or None when the
    kernel source changed since the counters were taken."""
    s = read_summary("atomics_seq64.txt")
    if not s or s.get("kernel sources sha256[:16]") != source_sha(TRACE_SRCS):
        return None
    return float(s["line requests per traversal phase"])


def measured_traffic():
    """HBM bytes per launch of the traversal kernel from the committed PMC
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy's counters), or
    None when the kernel source changed since the counters were taken."""
    s = read_summary("trace_seq64_traffic.txt")
    if not s or s.get("kernel sources sha256[:16]") != source_sha(TRACE_SRCS):
        return None
    return float(s["hbm bytes per launch"])


def measured_valu():
    """VALU wave-instructions per launch of the traversal kernel from the
    committed SQ counter summary, or None when the kernel source changed
    since the counters were taken."""
    s = read_summary("trace_seq64_instructions.txt")
    if not s or s.get("kernel sources sha256[:16]") != source_sha(TRACE_SRCS):
        return None
    return float(s["k_trace<false> SQ_INSTS_VALU"])


def calibrate():
    """Reference rates from the library's own calibration kernels
    (map_calib_copy, map_calib_atomic): a plain device copy, the scale for
    the FETCH_SIZE / WRITE_SIZE counters, and scattered int32 atomic adds at
    1, 4, 16 and 64 lanes per 64-byte line on an L2-sized (2 MiB) and an
    HBM-sized (256 MiB) footprint, reported per update and per line request."""
    import torch
    from paper_2109_13176_amd import gvom
    reps = 10

    def timed(fn):
        for _ in range(2):
            assert fn() == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    n = 128 << 20  # int32 elements: 512 MiB per buffer
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: gvom.map_calib_copy(dst, src))
    assert torch.equal(dst, src)
    out = {"kernel_copy": "k_copy_bw", "copy_bytes_per_launch": 2 * n * 4,
           "copy_GBps": 2 * n * 4 / t / 1e9, "kernel_atomic": "k_atomic_peak", "atomics": []}
    del src, dst
    n_waves, per_wave = 16384, 64
    upd = 64 * n_waves * per_wave
    for foot_mib in (2, 256):
        tgt = torch.zeros(foot_mib << 18, dtype=torch.int32, device="cuda")
        for g in (1, 4, 16, 64):
            tgt.zero_()
            ta = timed(lambda: gvom.map_calib_atomic(tgt, n_waves, per_wave, g, seed=7))
            total = int(tgt.sum(dtype=torch.int64))
            assert total == upd * (reps + 2), (total, upd)
            out["atomics"].append({"footprint_MiB": foot_mib, "lanes_per_line": g,
                                   "updates_per_launch": upd,
                                   "line_requests_per_launch": upd // g,
                                   "updates_per_s": upd / ta, "line_requests_per_s": upd / g / ta})
        del tgt
    print(json.dumps(out), flush=True)


def oracle_worker(first, warm, timed):
    """Child process of the CPU baseline: waits for the path prefix of the
    saved sequence on stdin, then times the single-threaded C oracle on scans
    first+warm .. first+warm+timed-1 (each insert + 2D export + table export)
    after `warm` untimed scans before them, and prints one JSON line."""
    import numpy as np
    import oracle
    prefix = sys.stdin.readline().strip()
    if not prefix:
        return
    scans = np.load(prefix + "_scans.npy", mmap_mode="r")
    poses = np.load(prefix + "_poses.npy")
    params = json.loads(open(prefix + "_params.json").read())
    m = oracle.OracleMap(params)
    for k in range(first, first + warm):
        m.insert_scan(np.ascontiguousarray(scans[k]), poses[k], oracle.RECENTER)
    pts = 0
    t0 = time.perf_counter()
    for k in range(first + warm, first + warm + timed):
        m.insert_scan(np.ascontiguousarray(scans[k]), poses[k], oracle.RECENTER)
        m.export_2d()
        m.export_voxels()
        pts += scans.shape[1]
    t1 = time.perf_counter()
    m.close()
    print(json.dumps({"points": pts, "updates": timed, "t0": t0, "t1": t1}), flush=True)


class OracleBaseline:
    """The CPU oracle timed on the GPU host, in processes started before this
    process touches the GPU (a process that has initialised the GPU must not
    fork).  One process alone gives the single-core rate on exactly the
    scans the GPU times; then `procs` processes at once, each on its own
    stretch of the sequence, give the all-core rate (sum of their rates)."""

    def __init__(self, warm, timed, procs, n_scans):
        import subprocess
        self.warm, self.timed, self.n_scans = warm, timed, n_scans
        me = os.path.abspath(__file__)

        def spawn(first):
            return subprocess.Popen([sys.executable, me, "--oracle-worker", str(first), str(warm),
                                     str(timed)], stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                                    text=True)
        self.solo = spawn(0)
        span = warm + timed
        self.firsts = [(j * 5) % max(1, n_scans - span + 1) for j in range(procs)]
        self.group = [spawn(f) for f in self.firsts]

    @staticmethod
    def _collect(procs):
        out = []
        for p in procs:
            line = p.stdout.readline()
            p.wait()
            if not line:
                raise RuntimeError("oracle worker failed")
            out.append(json.loads(line))
        return out

    def run(self, seq):
        import numpy as np
        import tempfile
        shm = "/dev/shm" if os.path.isdir("/dev/shm") else tempfile.gettempdir()
        prefix = os.path.join(shm, f"gvom_bench_{os.getpid()}")
        files = [prefix + s for s in ("_scans.npy", "_poses.npy", "_params.json")]
        try:
            np.save(files[0], np.stack([s.cpu().numpy() for s in seq["scans"][:self.n_scans]]))
            np.save(files[1], np.stack([np.asarray(p, np.float32) for p in seq["poses"][:self.n_scans]]))
            open(files[2], "w").write(json.dumps(seq["params"]))
            self.solo.stdin.write(prefix + "\n")
            self.solo.stdin.flush()
            solo = self._collect([self.solo])[0]
            log(f"oracle, one process: {solo['updates'] / (solo['t1'] - solo['t0']):.2f} updates/s")
            for p in self.group:
                p.stdin.write(prefix + "\n")
                p.stdin.flush()
            grp = self._collect(self.group)
        finally:
            for f in files:
                if os.path.exists(f):
                    os.remove(f)
        one = solo["points"] / (solo["t1"] - solo["t0"])
        rates = [g["points"] / (g["t1"] - g["t0"]) for g in grp]
        upd = [g["updates"] / (g["t1"] - g["t0"]) for g in grp]
        wall = max(g["t1"] for g in grp) - min(g["t0"] for g in grp)
        n = len(grp)
        return {"value": float(sum(rates)), "unit": "points/s", "cores": n, "kind": "oracle",
                "updates_per_s": float(sum(upd)),
                "sample": f"{n} single-threaded oracle processes at once, each timing "
                          f"{self.timed} scans (after {self.warm} untimed) of its own stretch "
                          f"of the 100-scan sequence (first scans {self.firsts}), each scan "
                          f"insert + export_2d + export_voxels; value = sum of their rates "
                          f"(all points over the {wall:.1f} s wall span: "
                          f"{sum(g['points'] for g in grp) / wall:.4g} points/s)",
                "single_core": {"value": one, "unit": "points/s", "cores": 1,
                                "updates_per_s": solo["updates"] / (solo["t1"] - solo["t0"]),
                                "sample": f"scans {self.warm}..{self.warm + self.timed - 1} "
                                          f"after scans 0..{self.warm - 1} untimed: the scans "
                                          f"the GPU's first {self.timed} timed steps process",
                                "seconds": solo["t1"] - solo["t0"]},
                "host": host_info()}

    def close(self):
        for p in [self.solo] + self.group:
            if p.poll() is None:
                try:
                    p.stdin.close()
                except OSError:
                    pass
                p.wait()


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": aff}


def voxel_outputs(args, params, scans, poses, flags):
    """The voxel map's density export (one float per voxel) and the planner
    costmap (weighted sum of the 2D layers), timed with HIP events on the
    map's stream after the warm-up scans."""
    import numpy as np
    import torch
    from paper_2109_13176_amd import gvom
    m = gvom.VoxelMap(params)
    for k in range(args.warmup + 1):
        m.insert(scans[k], poses[k], flags)
    m.export_2d()
    w = {"slope": 2.0, "rough": 40.0, "density": 5.0, "positive": 1.0, "hard": 100.0,
         "soft": 3.0, "negative": 50.0, "unknown": 7.0}
    res = {}
    reps = 20
    for name, fn in (("density", m.export_density), ("costmap", lambda: m.costmap(w))):
        fn()
        # back-to-back launches between one event pair: the queue stays full,
        # so launch gaps do not count
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        res[name + "_us"] = a.elapsed_time(b) * 1e3 / reps
    m.close()
    V = params["nx"] * params["ny"] * params["nz"]
    C = params["nx"] * params["ny"]
    # density reads hits and passes and writes one float per voxel; the
    # costmap reads 4 floats + 1 flag byte and writes 1 float per pixel
    res["density_bytes"] = 12 * V
    res["density_gbps"] = 12 * V / (res["density_us"] * 1e-6) / 1e9
    res["density_frac"] = res["density_gbps"] / HBM_PEAK_GBS
    res["costmap_bytes"] = 21 * C
    res["costmap_gbps"] = 21 * C / (res["costmap_us"] * 1e-6) / 1e9
    return res


def paper_dataflow(args, params, scans, poses, flags, depth=10):
    """The paper's own dataflow (Sec. III-B to III-D) on the same scans: each
    scan becomes a voxel map of its own in a buffer of the last `depth` (one
    second of scans at 10 Hz); map processing combines the buffered maps and
    exports the same outputs as the headline step.  Pushes run on a second
    stream, the combine and the exports on the output map's stream."""
    import numpy as np
    import torch
    from paper_2109_13176_amd import gvom
    W, K = args.warmup, args.steps

    def run(with_events, incremental=True):
        side = torch.cuda.Stream()
        buf = gvom.ScanBuffer(params, depth, side)
        buf.set_incremental(incremental)
        cm = gvom.VoxelMap(params)
        ev = []
        origins = []
        t0 = None
        for k in range(W + K):
            if k == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            timed = with_events and k >= W
            if timed:
                p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                # the push waits for the previous combine; time the push alone
                side.wait_stream(torch.cuda.current_stream())
                p0.record(side)
            buf.push(scans[k], poses[k], flags)
            if timed:
                p1.record(side)
                # the combine waits for the push; time the combine kernel alone
                torch.cuda.current_stream().wait_stream(side)
                c0.record()
            buf.combine(cm)
            if timed:
                c1.record()
                ev.append((p0, p1, c0, c1))
            cm.export_2d()
            cm.export_voxels_async()
            origins.append(cm.origin().copy())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        buf.close()
        cm.close()
        return dt, ev, origins

    t_df, _, _ = run(False)
    _, ev, origins = run(True)
    push_us = float(np.mean([a.elapsed_time(b) for a, b, _, _ in ev])) * 1e3
    upd_us = float(np.mean([c.elapsed_time(d) for _, _, c, d in ev])) * 1e3
    # the paper's combine: every buffered map combined again at every update
    t_full, _, _ = run(False, incremental=False)
    _, ev_full, _ = run(True, incremental=False)
    comb_us = float(np.mean([c.elapsed_time(d) for _, _, c, d in ev_full])) * 1e3
    n = np.array([params["nx"], params["ny"], params["nz"]])
    V = int(n.prod())
    C = int(n[0] * n[1])
    words = (params["nz"] + 63) // 64
    # voxels of the combined window that each buffered window holds, per step
    overlap = []
    for j in range(W, W + K):
        o = origins[j]
        overlap.append(sum(int(np.prod(np.maximum(0, n - np.abs(o - origins[i]))))
                           for i in range(max(0, j - depth + 1), j + 1)))
    ov = float(np.mean(overlap))

    def combine_bytes(distinct_hit):
        # the full combine: lookup tables of the overlapping windows, the data
        # entries of their occupied voxels (at most M per map), the combined
        # state written (hits, passes, lowest return) and its occupancy words
        b = 4 * ov + 12 * depth * distinct_hit + 12 * V + 8 * C * words
        gbps = b / (comb_us * 1e-6) / 1e9
        return {"bytes": b, "us": comb_us, "achieved_gbps": gbps, "peak_gbps": HBM_PEAK_GBS,
                "frac": gbps / HBM_PEAK_GBS, "overlap_voxels": ov}

    return {"depth": depth, "ms_per_step": t_df * 1e3 / K, "updates_per_s": K / t_df,
            "points_per_s": sum(int(scans[k].shape[0]) for k in range(W, W + K)) / t_df,
            "push_us": push_us, "combine_update_us": upd_us,
            "full_combine": {"ms_per_step": t_full * 1e3 / K, "updates_per_s": K / t_full,
                             "combine_us": comb_us},
            "combine_bytes_fn": combine_bytes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=95)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-scans", type=int, default=20,
                    help="scans each oracle process times (after --warmup untimed ones)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes of the all-core figure (0: the usable CPUs, at most 16)")
    ap.add_argument("--oracle-worker", type=int, nargs=3, metavar=("FIRST", "WARM", "TIMED"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--print-sha", action="store_true",
                    help="print the hash of the traversal kernel sources, then exit")
    ap.add_argument("--calibrate", action="store_true",
                    help="measure a plain copy and scattered atomics (profile scaling), then exit")
    ap.add_argument("--c5-train-seqs", type=int, default=100,
                    help="surrogate workload: training sequences of 20 scans (0: timing only)")
    ap.add_argument("--c5-test-seqs", type=int, default=10)
    ap.add_argument("--c5-steps", type=int, default=10000)
    ap.add_argument("--workload", default="seq64", choices=["seq64", "batch32", "surrogate"],
                    help="seq64: the 64-beam 512x512x64 sequence (default); batch32: 32 "
                         "independent maps stepped as one batch; surrogate: the gap-fill "
                         "network on the 512x512 grid (inference and training step)")
    args = ap.parse_args()
    if args.oracle_worker:
        return oracle_worker(*args.oracle_worker)
    if args.print_sha:
        print(source_sha(TRACE_SRCS))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent maps would shard one per GPU with no exchange).", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle's processes start before anything touches the GPU
    baseline = None
    if args.workload == "seq64" and not args.calibrate and not args.no_cpu_baseline:
        procs = args.cpu_procs or min(16, len(os.sched_getaffinity(0)))
        baseline = OracleBaseline(args.warmup, min(args.cpu_scans, args.steps), procs, 100)
    try:
        return bench_main(args, baseline)
    finally:
        if baseline:
            baseline.close()


def bench_main(args, baseline):
    import numpy as np
    import torch
    from paper_2109_13176_amd import gvom
    from synth import scenegen

    torch.cuda.set_device(0)
    if args.calibrate:
        return calibrate()
    if args.workload == "batch32":
        return bench_batch(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    W, K = args.warmup, args.steps
    t0 = time.time()
    # the 100-scan sequence; all of it is simulated when the oracle processes
    # need their own stretches of it
    n_sim = max(W + K, 100) if baseline else W + K
    seq = scenegen.sequence_64beam(seed=2, n_scans=max(100, W + K), n_sim=n_sim, device="cuda")
    params = seq["params"]
    scans = [s.contiguous() for s in seq["scans"]]
    poses = seq["poses"]
    flags = gvom.MAP_RECENTER | gvom.MAP_FIRING(64)
    log(f"generated {len(scans)} scans in {time.time() - t0:.1f} s")

    # untimed pre-pass on a shadow map: distinct voxels touched per scan
    shadow = gvom.VoxelMap(params)
    dstats = []
    for k in range(W + K):
        shadow.insert(scans[k], poses[k], flags | gvom.MAP_STATS_DISTINCT)
        if k >= W:
            dstats.append(shadow.stats())
    shadow.close()
    del shadow

    m = gvom.VoxelMap(params)
    trace_bit = 1 << gvom.PROF_PHASES.index("trace")

    def step(k):
        m.insert(scans[k], poses[k], flags)
        m.export_2d()
        m.export_voxels_async()

    for k in range(W):
        step(k)
    torch.cuda.synchronize()

    # timed region: HIP events only around the dominant kernel (the traversal)
    gvom.map_profile_enable(m.h, trace_bit)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(W, W + K):
        step(k)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    elapsed = t_end - t_start
    s, prof_timed = gvom.map_profile_read(m.h)
    n_occ = int(m.n_occ.item())
    m.close()

    # every phase timed in a second pass over the same scans (fresh map)
    m = gvom.VoxelMap(params)
    for k in range(W):
        step(k)
    gvom.map_profile_enable(m.h, True)
    torch.cuda.synchronize()
    gvom.map_profile_read(m.h)
    for k in range(W, W + K):
        step(k)
    s, prof = gvom.map_profile_read(m.h)
    prof["trace"] = prof_timed["trace"]
    m.close()

    # the same steps on a fresh map with each scan first copied from pinned
    # host memory (the copy is outside the library's boundary: reported, not
    # the value)
    m = gvom.VoxelMap(params)
    for k in range(W):
        step(k)
    host = [scans[k].cpu().pin_memory() for k in range(W, W + K)]
    dev = torch.empty_like(scans[W])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, k in enumerate(range(W, W + K)):
        if host[i].shape != dev.shape:
            dev = torch.empty(host[i].shape, dtype=host[i].dtype, device="cuda")
        dev.copy_(host[i], non_blocking=True)
        m.insert(dev, poses[k], flags)
        m.export_2d()
        m.export_voxels_async()
    torch.cuda.synchronize()
    pcie_elapsed = time.perf_counter() - t0
    m.close()

    # the narrower units: insert alone (points ingested) and insert + 2D
    # export (a map update without the voxel table), each on a fresh map
    def timed(fn):
        mm = gvom.VoxelMap(params)
        for k in range(W):
            fn(mm, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(W, W + K):
            fn(mm, k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mm.close()
        return dt

    t_insert = timed(lambda mm, k: mm.insert(scans[k], poses[k], flags))
    t_insert_2d = timed(lambda mm, k: (mm.insert(scans[k], poses[k], flags), mm.export_2d()))

    dataflow = paper_dataflow(args, params, scans, poses, flags)
    outputs = voxel_outputs(args, params, scans, poses, flags)

    n_points = sum(int(scans[k].shape[0]) for k in range(W, W + K))
    value = n_points / elapsed
    updates = K / elapsed

    avg = {k: float(np.mean([d[k] for d in dstats])) for k in dstats[0]}
    by = phase_bytes(params, avg, n_occ)
    phases = {}
    for p, (ms, cnt) in prof.items():
        if cnt:
            t = ms / cnt
            phases[p] = {"avg_ms": t, "launches": cnt, "bytes": by[p],
                         "gbps": by[p] / (t * 1e-3) / 1e9 if t > 0 else None}
    dom = max(phases, key=lambda p: phases[p]["avg_ms"] * phases[p]["launches"])
    roof = {"kernel": dom, "bound": "hbm", "achieved": phases[dom]["gbps"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": phases[dom]["gbps"] / HBM_PEAK_GBS,
            "traffic": measured_traffic() if dom == "trace" else None}
    if dom == "trace":
        # co-reported atomic roofline: device atomics are charged per line
        # request (TCC_ATOMIC); the peak is the best line-request rate of the
        # library's k_atomic_peak (random lines, HBM-sized footprint)
        t_tr = phases["trace"]["avg_ms"] * 1e-3
        cal = read_summary("calibration_mi355x.txt")
        peak = float(cal["peak atomic line requests per s"]) if cal and "peak atomic line requests per s" in cal else None
        lr = measured_line_requests()
        roof["atomics"] = {"achieved": lr / t_tr if lr else None, "peak": peak,
                           "unit": "line requests/s",
                           "frac": lr / t_tr / peak if (lr and peak) else None,
                           "line_requests_per_launch": lr,
                           "updates_per_launch": avg["n_pass_updates"],
                           "updates_per_s": avg["n_pass_updates"] / t_tr}
        # co-reported issue roofline: the walk is bound by VALU issue; a wave64
        # VALU instruction takes a 16-lane SIMD 4 cycles, 1024 SIMDs at 2.4 GHz
        valu = measured_valu()
        roof["valu_issue"] = {"achieved": valu / t_tr if valu else None, "peak": VALU_ISSUE_PEAK,
                              "unit": "wave instructions/s",
                              "frac": valu / t_tr / VALU_ISSUE_PEAK if valu else None,
                              "valu_per_launch": valu}

    # whole-path HBM fractions with the counted minimum bytes: the ray cast
    # moves 12 N + 16 U_h + 8 U_p, the exports 4 V (table) + 12 M + 17 C
    V = params["nx"] * params["ny"] * params["nz"]
    C = params["nx"] * params["ny"]
    n_scan = n_points / K
    b_rc = 12 * n_scan + 16 * avg["n_distinct_hit"] + 8 * avg["n_distinct_pass"]
    b_ex = 4 * V + 12 * n_occ + 17 * C
    t_rc = t_insert / K
    path_hbm = {"ray_cast": {"bytes": b_rc, "us": t_rc * 1e6,
                             "frac": b_rc / t_rc / (HBM_PEAK_GBS * 1e9)},
                "step": {"bytes": b_rc + b_ex, "us": elapsed / K * 1e6,
                         "frac": (b_rc + b_ex) / (elapsed / K) / (HBM_PEAK_GBS * 1e9)}}

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "64-beam x 2048-azimuth lidar sequence (131,072 points/scan, "
                               "4.5 m/s spline, 0.1 s/scan), 512x512x64 voxels at 0.2 m, "
                               "recentred every scan",
                   "points_per_scan": int(scans[0].shape[0]), "map": [512, 512, 64],
                   "res_m": 0.2, "scans_timed": K},
        "updates_per_s": updates,
        "insert_only_points_per_s": n_points / t_insert,
        "insert_2d_updates_per_s": K / t_insert_2d,
        "pcie_inclusive_points_per_s": n_points / pcie_elapsed,
        "path_hbm": path_hbm,
        "phases": phases,
        "per_scan": {"pass_incidences": avg["n_pass"], "distinct_passed": avg["n_distinct_pass"],
                     "distinct_hit": avg["n_distinct_hit"], "hits": avg["n_hits"],
                     "occupied_voxels_final": n_occ, "cleared": avg["n_cleared"],
                     "pass_updates": avg["n_pass_updates"]},
        "roofline": roof,
    }
    df_hbm = dataflow.pop("combine_bytes_fn")(avg["n_distinct_hit"])
    dataflow["full_combine"]["hbm"] = df_hbm
    out["paper_dataflow"] = dataflow
    out["voxel_outputs"] = outputs
    if baseline:
        out["cpu_baseline"] = baseline.run(seq)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """32 independent maps, uneven scan sizes, one batched step per 0.1 s of
    driving: map updates/s and per-map latency percentiles."""
    import numpy as np
    import torch
    from paper_2109_13176_amd import gvom
    from synth import scenegen

    W, K = min(args.warmup, 3), min(args.steps, 20)
    t0 = time.time()
    veh = scenegen.batch_of_vehicles(32, n_steps=max(100, W + K), n_sim=W + K, device="cuda")
    log(f"generated {32 * (W + K)} scans in {time.time() - t0:.1f} s")
    maps = [gvom.VoxelMap(v["params"]) for v in veh]
    batch = gvom.MapBatch(maps)
    flags = [gvom.MAP_RECENTER | gvom.MAP_FIRING(v["firing"]) for v in veh]

    def inputs(k):
        return [v["scans"][k] for v in veh], [v["poses"][k] for v in veh]

    xs, ps = inputs(0)
    tuning = batch.autotune(xs, ps, flags, os.path.join("/tmp", "gvom_tune_cache.txt"))
    log(f"autotuned: {tuning}")
    for k in range(W):
        xs, ps = inputs(k)
        batch.step(xs, ps, flags, [True] * 32)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(W, W + K):
        xs, ps = inputs(k)
        batch.step(xs, ps, flags, [True] * 32)
        lat.append(batch.latency_ms())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    lat = np.concatenate(lat)
    pts = sum(int(v["scans"][k].shape[0]) for v in veh for k in range(W, W + K))
    out = {"metric": "map updates/s, 32 independent maps batched (C4-type)",
           "value": 32 * K / elapsed, "unit": "map updates/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "32 vehicles, scans of 20k-330k points (log-uniform), grids "
                                  "256x256x48@0.4m or 512x512x64@0.2m, one hipGraph step",
                      "maps": 32},
           "points_per_s": pts / elapsed, "latency_ms_p50": float(np.percentile(lat, 50)),
           "latency_ms_p99": float(np.percentile(lat, 99)), "tuning": tuning}
    batch.close()
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """Gap-fill network on the 512 x 512 grid of the 64-beam workload:
    inference (features -> height / roughness) and one training step
    (forward, masked L1, backward, Adam), features of a thinned single-scan map."""
    import numpy as np
    import torch
    from paper_2109_13176_amd import gvom
    from synth import scenegen

    W, K = max(args.warmup, 3), max(args.steps, 20)
    seq = scenegen.sequence_64beam(seed=2, n_sim=1, device="cuda")
    p = seq["params"]
    H, Wd = p["nx"], p["ny"]
    m = gvom.VoxelMap(p)
    m.insert(seq["scans"][0].contiguous(), seq["poses"][0], gvom.MAP_RECENTER | gvom.MAP_FIRING(64))
    rng = np.random.default_rng(0)
    thin = torch.from_numpy((rng.uniform(size=(H, Wd)) < 0.5).astype(np.uint8)).cuda()
    gvom.sgt_thin(m, thin)
    plain = m.export_2d()
    sensor = np.asarray(seq["poses"][0], np.float32).reshape(3, 4)[:, 3]
    feat = gvom.sgt_features(m, plain, sensor, thin)
    net = gvom.Surrogate(H, Wd, seed=1)
    sums = net.feature_sums(feat)
    n = H * Wd
    mean = sums[:16] / n
    std = np.maximum(np.sqrt(np.maximum(sums[16:] / n - mean ** 2, 0)), 1e-3)
    net.set_norm(mean.astype(np.float32), std.astype(np.float32))
    label = torch.stack([plain["height"], plain["rough"]], 2).contiguous()
    out = torch.empty((H, Wd, 2), dtype=torch.float32, device="cuda")
    for _ in range(W):
        net.forward(feat, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        net.forward(feat, out)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / K * 1e-3
    for _ in range(W):
        net.loss_grad(feat, label)
        net.adam(1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        net.loss_grad(feat, label)
        net.adam(1e-3)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / K
    flop_px = 2 * 9 * (16 * 32 + 3 * 32 * 32 + 32 * 2)
    flops = flop_px * n
    peak = 2500.0  # dense bf16 MFMA, TFLOP/s
    res = {"metric": "gap-fill surrogate inference maps/s (512x512, bf16 MFMA)",
           "value": 1.0 / t_fwd, "unit": "maps/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": t_fwd * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "features of a thinned 64-beam single-scan map, 512x512, "
                                  "conv3x3 16-32-32-32-32-2", "pixels": n},
           "train_step_ms": t_train * 1e3,
           # a training step = forward + weight gradients (as many MACs as
           # the forward) + input gradients (the same, less the first layer,
           # whose input needs none); the loss and Adam are negligible
           "train_tflop_per_s": (3 * flops - 2 * 9 * 16 * 32 * n) / t_train / 1e12,
           "roofline": {"kernel": "forward (5 convolutions)", "bound": "mfma",
                        "achieved": flops / t_fwd / 1e12, "peak": peak, "unit": "TFLOP/s",
                        "frac": flops / t_fwd / 1e12 / peak, "traffic": None,
                        "flop_per_launch": flops}}
    net.close()
    m.close()
    if args.c5_train_seqs > 0:
        res["c5"] = surrogate_c5(args)
    print(json.dumps(res), flush=True)


def surrogate_c5(args):
    """The gap-fill network trained and evaluated at full size: 64-beam
    sequences of 20 scans on 512 x 512 x 64 at 0.2 m (scene seeds 5000.. for
    training, 5900.. held out), each sequence in the window of its middle
    pose; label = plain map of all 20 scans, input = one scan with 30-70 % of
    its columns thinned (fresh mask per step).  Reports the held-out gap
    error and the filled map's error and coverage against the plain map at
    the 0.05 m fallback tolerance."""
    import numpy as np
    from paper_2109_13176_amd import gvom, surrogate
    from synth import scenegen

    t0 = time.time()

    def make(seeds):
        out = []
        for i, s in enumerate(seeds):
            out.append(surrogate.WindowSequence(scenegen.sequence_64beam(seed=s, n_scans=20,
                                                                         device="cuda")))
            if (i + 1) % 10 == 0:
                log(f"c5: {i + 1}/{len(seeds)} sequences ({time.time() - t0:.0f} s)")
        return out

    train = make(range(5000, 5000 + args.c5_train_seqs))
    test = make(range(5900, 5900 + args.c5_test_seqs))
    t_gen = time.time() - t0
    p = train[0].params
    builder = surrogate.InputBuilder(p)
    net = gvom.Surrogate(p["nx"], p["ny"], seed=7)
    rng = np.random.default_rng(0)
    surrogate.fit_normalisation_frames(net, builder, train, rng)
    before = surrogate.evaluate_frames(net, builder, test, np.random.default_rng(1))
    t1 = time.time()
    losses = surrogate.train_frames(net, builder, train, args.c5_steps, 2e-3, rng,
                                    log_every=max(args.c5_steps // 10, 1))
    t_train = time.time() - t1
    after = surrogate.evaluate_frames(net, builder, test, np.random.default_rng(1))
    builder.close()
    net.close()
    return {"train_sequences": len(train), "train_frames": sum(len(w) for w in train),
            "train_steps": args.c5_steps, "heldout_sequences": len(test),
            "loss_first_100": float(np.mean(losses[:100])),
            "loss_last_100": float(np.mean(losses[-100:])),
            "generate_s": t_gen, "train_s": t_train,
            "heldout_untrained": before, "heldout_trained": after}


if __name__ == "__main__":
    main()
