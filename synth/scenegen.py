"""Seeded synthetic off-road scenes and a spinning-lidar simulator.

Input generator only: it draws scenes, trajectories and lidar returns and
holds none of the mapping method's arithmetic.  It stands in for the field
recordings of the paper (Texas A&M RELLIS campus), which are not available.

Scene recipe (all sizes in metres):
  terrain    sum of 6 sinusoids, amplitude 0.3/6 each (|H| <= 0.3), wavelengths
             log-uniform on [3, 20], random directions and phases; optional
             low-frequency relief A sin(2 pi x / L) cos(2 pi y / L) for steep
             terrain;
  boxes      1 x 1 x 2 axis-aligned, base 0.1 below the lowest terrain under them
             (hard positive obstacles);
  vegetation clusters of points uniform in a sphere of radius 1.5 centred
             1.5 above the terrain, each point a small sphere (soft obstacles);
  pits       2 x 2 footprint, flat floor 1 below the terrain at the centre,
             vertical walls (negative obstacles);
  ramps      optional linear rises along x (steps and cliffs of the small
             semantic scenes).
Lidar: beams at fixed elevations, azimuth-major point order (one firing of
all beams per azimuth step), range noise N(0, sigma) along the ray, NaN for
beams with no return within the maximum range.  Points are returned in the
sensor frame as float32 [N, 3].

Random draws use numpy (SeedSequence-spawned streams for scene, trajectory,
noise) so a seed gives the same scene on every device; the ray casting runs
in torch on the requested device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass
class Scene:
    waves: np.ndarray            # [K, 4]: amplitude, kx, ky, phase
    relief: tuple = (0.0, 1.0)   # amplitude, wavelength
    z0: float = 0.0              # constant terrain offset
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))   # xmin..zmax
    pits: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))    # xmin,xmax,ymin,ymax,floor
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # cx,cy,cz,r
    clusters: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))  # cx,cy,cz,R,first idx
    cluster_end: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    ramps: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))   # x0, x1, dz

    # -------------------------------------------------------------- terrain
    def terrain_np(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        h = np.full(np.broadcast(x, y).shape, self.z0)
        for a, kx, ky, ph in self.waves:
            h = h + a * np.sin(kx * x + ky * y + ph)
        A, L = self.relief
        if A:
            h = h + A * np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L)
        for x0, x1, dz in self.ramps:
            h = h + dz * np.clip((x - x0) / (x1 - x0), 0.0, 1.0)
        return h

    def ground_np(self, x, y):
        h = self.terrain_np(x, y)
        for x0, x1, y0, y1, fl in self.pits:
            inside = (x >= x0) & (x < x1) & (y >= y0) & (y < y1)
            h = np.where(inside, fl, h)
        return h


def _torch_ground(scene: Scene, x, y, consts):
    h = torch.full_like(x, scene.z0)
    w = consts["waves"]
    for k in range(w.shape[0]):
        h = h + w[k, 0] * torch.sin(w[k, 1] * x + w[k, 2] * y + w[k, 3])
    A, L = scene.relief
    if A:
        h = h + A * torch.sin(2 * math.pi * x / L) * torch.cos(2 * math.pi * y / L)
    for x0, x1, dz in scene.ramps:
        h = h + dz * torch.clamp((x - x0) / (x1 - x0), 0.0, 1.0)
    for p in consts["pits"]:
        inside = (x >= p[0]) & (x < p[1]) & (y >= p[2]) & (y < p[3])
        h = torch.where(inside, p[4], h)
    return h


def raycast(scene: Scene, origin, dirs: torch.Tensor, max_range: float,
            step: float = 0.2) -> torch.Tensor:
    """Range of the first surface along each unit ray from `origin` (inf if none)."""
    dev, dt = dirs.device, torch.float64
    o = torch.as_tensor(np.asarray(origin, np.float64), device=dev, dtype=dt)
    d = dirs.to(dt)
    consts = {"waves": torch.as_tensor(scene.waves, device=dev, dtype=dt),
              "pits": [torch.as_tensor(p, device=dev, dtype=dt) for p in scene.pits]}
    N = d.shape[0]
    best = torch.full((N,), math.inf, device=dev, dtype=dt)

    # terrain: march, then bisection on the first sign change
    n_steps = int(math.ceil(max_range / step))
    prev_s = torch.zeros(N, device=dev, dtype=dt)
    hit_s = torch.full((N,), math.inf, device=dev, dtype=dt)
    lo = torch.zeros(N, device=dev, dtype=dt)
    chunk = 32
    for s0 in range(1, n_steps + 1, chunk):
        ss = torch.arange(s0, min(s0 + chunk, n_steps + 1), device=dev, dtype=dt) * step
        ss = torch.clamp(ss, max=max_range)
        P = o[None, None, :] + d[:, None, :] * ss[None, :, None]
        f = P[..., 2] - _torch_ground(scene, P[..., 0], P[..., 1], consts)
        below = f <= 0
        first = torch.where(below.any(1), below.float().argmax(1), torch.full((N,), -1, device=dev))
        new = (first >= 0) & torch.isinf(hit_s)
        idx = torch.clamp(first, min=0)
        s_hit = ss[idx]
        s_prev = torch.where(idx > 0, ss[torch.clamp(idx - 1, min=0)], prev_s)
        hit_s = torch.where(new, s_hit, hit_s)
        lo = torch.where(new, s_prev, lo)
        prev_s = ss[-1].expand(N)
        if not torch.isinf(hit_s).any():
            break
    found = ~torch.isinf(hit_s)
    a = torch.where(found, lo, torch.zeros_like(lo))
    b = torch.where(found, hit_s, torch.zeros_like(lo))
    for _ in range(30):
        m = 0.5 * (a + b)
        P = o[None, :] + d * m[:, None]
        f = P[:, 2] - _torch_ground(scene, P[:, 0], P[:, 1], consts)
        a = torch.where(f > 0, m, a)
        b = torch.where(f > 0, b, m)
    best = torch.where(found, b, best)

    # boxes: slab test
    if len(scene.boxes):
        bx = torch.as_tensor(scene.boxes, device=dev, dtype=dt)  # [B, 6]
        inv = 1.0 / torch.where(d.abs() < 1e-12, torch.full_like(d, 1e-12), d)
        t1 = (bx[None, :, 0::2] - o[None, None, :]) * inv[:, None, :]
        t2 = (bx[None, :, 1::2] - o[None, None, :]) * inv[:, None, :]
        tn = torch.minimum(t1, t2).amax(-1)
        tf = torch.maximum(t1, t2).amin(-1)
        ok = (tf >= tn) & (tf > 0)
        tn = torch.where(tn > 0, tn, torch.zeros_like(tn))
        tb = torch.where(ok, tn, torch.full_like(tn, math.inf)).amin(1)
        best = torch.minimum(best, tb)

    # vegetation: per cluster, rays through its bounding sphere test its elements
    if len(scene.clusters):
        sph = torch.as_tensor(scene.spheres, device=dev, dtype=dt)
        for ci, (cx, cy, cz, R, first) in enumerate(scene.clusters):
            last = int(scene.cluster_end[ci])
            c = torch.as_tensor([cx, cy, cz], device=dev, dtype=dt) - o
            tc = d @ c
            dist2 = (c * c).sum() - tc * tc
            rr = R + float(scene.spheres[int(first), 3])
            cand = torch.nonzero((dist2 <= rr * rr) & (tc > -rr)).flatten()
            if cand.numel() == 0:
                continue
            el = sph[int(first):last]
            for k0 in range(0, cand.numel(), 4096):
                ids = cand[k0:k0 + 4096]
                dd = d[ids]
                oc = el[None, :, :3] - o[None, None, :]
                tca = (oc * dd[:, None, :]).sum(-1)
                d2 = (oc * oc).sum(-1) - tca * tca
                r2 = el[None, :, 3] ** 2
                th = torch.sqrt(torch.clamp(r2 - d2, min=0))
                t0 = tca - th
                hit = (d2 <= r2) & (t0 > 0)
                tmin = torch.where(hit, t0, torch.full_like(t0, math.inf)).amin(1)
                best[ids] = torch.minimum(best[ids], tmin)
    best = torch.where(best <= max_range, best, torch.full_like(best, math.inf))
    return best


def lidar_dirs(n_beams: int, el_lo_deg: float, el_hi_deg: float, n_az: int,
               device="cpu") -> torch.Tensor:
    """Unit directions in the sensor frame, azimuth-major: index = az * n_beams + beam."""
    el = torch.linspace(math.radians(el_lo_deg), math.radians(el_hi_deg), n_beams,
                        dtype=torch.float64, device=device)
    az = torch.arange(n_az, dtype=torch.float64, device=device) * (2 * math.pi / n_az)
    E, A = torch.meshgrid(el, az, indexing="xy")  # [n_az, n_beams]
    return torch.stack([torch.cos(E) * torch.cos(A), torch.cos(E) * torch.sin(A),
                        torch.sin(E)], -1).reshape(-1, 3)


def simulate_scan(scene: Scene, R: np.ndarray, t: np.ndarray, dirs_s: torch.Tensor,
                  max_range: float, sigma: float, rng: np.random.Generator) -> torch.Tensor:
    """Returns float32 [N, 3] sensor-frame points (NaN rows for no return)."""
    Rw = torch.as_tensor(R, dtype=torch.float64, device=dirs_s.device)
    dw = dirs_s @ Rw.T
    r = raycast(scene, t, dw, max_range)
    noise = torch.as_tensor(rng.normal(0.0, sigma, r.shape[0]), device=r.device)
    rn = r + noise
    pts = dirs_s * rn[:, None]
    pts = torch.where(torch.isinf(r)[:, None], torch.full_like(pts, float("nan")), pts)
    return pts.to(torch.float32)


# ---------------------------------------------------------------- scenes


def _waves(rng, k=6, amp=0.3):
    lam = np.exp(rng.uniform(np.log(3.0), np.log(20.0), k))
    th = rng.uniform(0, 2 * np.pi, k)
    ph = rng.uniform(0, 2 * np.pi, k)
    kk = 2 * np.pi / lam
    return np.stack([np.full(k, amp / k), kk * np.cos(th), kk * np.sin(th), ph], 1)


def make_scene(seed: int, extent: float, n_boxes: int, n_clusters: int, n_pits: int,
               cluster_points=500, element_r=0.05, relief=(0.0, 1.0), place=None,
               keep_clear=None) -> Scene:
    """Random scene on [-extent/2, extent/2]^2.  `place(rng)` may draw object
    centres; `keep_clear` = (points [M,2], radius) keeps objects off a path."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss.spawn(1)[0])
    sc = Scene(waves=_waves(rng), relief=relief)
    placed = []

    def draw(rad):
        for _ in range(1000):
            c = place(rng) if place else rng.uniform(-extent / 2, extent / 2, 2)
            if any(np.hypot(*(c - q)) < rad + r for q, r in placed):
                continue
            if keep_clear is not None:
                pts, kr = keep_clear
                if np.min(np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1])) < kr + rad:
                    continue
            placed.append((c, rad))
            return c
        raise RuntimeError("could not place object")

    boxes, pits, spheres, clusters, ends = [], [], [], [], []
    for _ in range(n_boxes):
        c = draw(1.0)
        gx, gy = np.meshgrid(np.linspace(c[0] - 0.5, c[0] + 0.5, 5),
                             np.linspace(c[1] - 0.5, c[1] + 0.5, 5))
        base = sc.terrain_np(gx, gy).min() - 0.1
        boxes.append([c[0] - 0.5, c[0] + 0.5, c[1] - 0.5, c[1] + 0.5, base, base + 2.0])
    for _ in range(n_pits):
        c = draw(1.6)
        fl = float(sc.terrain_np(c[0], c[1])) - 1.0
        pits.append([c[0] - 1.0, c[0] + 1.0, c[1] - 1.0, c[1] + 1.0, fl])
    for _ in range(n_clusters):
        c = draw(1.7)
        cz = float(sc.terrain_np(c[0], c[1])) + 1.5
        npts = cluster_points(rng) if callable(cluster_points) else cluster_points
        u = rng.normal(size=(npts, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        rad = 1.5 * rng.uniform(size=npts) ** (1 / 3)
        p = np.array([c[0], c[1], cz]) + u * rad[:, None]
        first = len(spheres)
        spheres.extend([[*q, element_r] for q in p])
        clusters.append([c[0], c[1], cz, 1.5, first])
        ends.append(len(spheres))
    sc.boxes = np.array(boxes, np.float64).reshape(-1, 6)
    sc.pits = np.array(pits, np.float64).reshape(-1, 5)
    sc.spheres = np.array(spheres, np.float64).reshape(-1, 4)
    sc.clusters = np.array(clusters, np.float64).reshape(-1, 5)
    sc.cluster_end = np.array(ends, np.int64)
    return sc


def rot_zyx(yaw, pitch, roll):
    cz, sz = math.cos(yaw), math.sin(yaw)
    cy, sy = math.cos(pitch), math.sin(pitch)
    cx, sx = math.cos(roll), math.sin(roll)
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    return Rz @ Ry @ Rx


def pose12(R, t) -> np.ndarray:
    return np.concatenate([np.asarray(R), np.asarray(t).reshape(3, 1)], 1).astype(np.float32).reshape(12)


def trajectory(scene: Scene, rng, n: int, spacing: float, height: float,
               yaw_noise_deg: float, extent: float):
    """Catmull-Rom spline through random control points, sampled every `spacing`
    metres of arc length.  True pose: yaw along the path, roll and pitch from the
    terrain normal, `height` above the terrain.  Returns (true [(R, t)], mapper
    pose12 list with yaw noise)."""
    length = n * spacing + 10
    k = max(4, int(length / 10) + 4)
    start = rng.uniform(-extent / 8, extent / 8, 2)
    head = rng.uniform(0, 2 * np.pi)
    ctrl = [start - 10 * np.array([math.cos(head), math.sin(head)])]
    for _ in range(k):
        head += rng.normal(0, 0.35)
        ctrl.append(ctrl[-1] + 10 * np.array([math.cos(head), math.sin(head)]))
    ctrl = np.array(ctrl)
    dense = []
    for i in range(1, len(ctrl) - 2):
        p0, p1, p2, p3 = ctrl[i - 1], ctrl[i], ctrl[i + 1], ctrl[i + 2]
        for s in np.linspace(0, 1, 200, endpoint=False):
            dense.append(0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s * s
                                + (-p0 + 3 * p1 - 3 * p2 + p3) * s ** 3))
    dense = np.array(dense)
    seg = np.hypot(*np.diff(dense, axis=0).T)
    arc = np.concatenate([[0], np.cumsum(seg)])
    out_true, out_map = [], []
    for j in range(n):
        a = j * spacing
        i = min(np.searchsorted(arc, a), len(dense) - 2)
        xy = dense[i]
        tang = dense[i + 1] - dense[max(i - 1, 0)]
        yaw = math.atan2(tang[1], tang[0])
        e = 0.05
        gx = (scene.ground_np(xy[0] + e, xy[1]) - scene.ground_np(xy[0] - e, xy[1])) / (2 * e)
        gy = (scene.ground_np(xy[0], xy[1] + e) - scene.ground_np(xy[0], xy[1] - e)) / (2 * e)
        # slope along and across the heading
        along = gx * math.cos(yaw) + gy * math.sin(yaw)
        across = -gx * math.sin(yaw) + gy * math.cos(yaw)
        pitch = -math.atan(along)
        roll = math.atan(across)
        z = float(scene.ground_np(xy[0], xy[1])) + height
        R = rot_zyx(yaw, pitch, roll)
        t = np.array([xy[0], xy[1], z])
        out_true.append((R, t))
        yn = yaw + math.radians(rng.normal(0, yaw_noise_deg))
        out_map.append(pose12(rot_zyx(yn, pitch, roll), t))
    return out_true, out_map, dense


# ---------------------------------------------------------------- workloads


def params_for(nx, ny, nz, res, szv=None):
    return dict(nx=nx, ny=ny, nz=nz, res_m=res, sensor_z_voxel=nz // 2 if szv is None else szv,
                obs_min_m=0.4, obs_max_m=2.0, dens_num=1, dens_den=2, fit_n=5,
                neg_thresh_m=0.5, neg_search_m=5.0)


def single_scan_16beam(seed=1, device="cpu"):
    """16-beam x 1800-azimuth scan (28,800 points, 50 m, sigma 0.02 m), identity pose,
    128 x 128 x 32 map at 0.4 m.  Ground under the sensor at z = -1.5."""
    ss = np.random.SeedSequence(seed)
    r_place, r_noise = [np.random.default_rng(s) for s in ss.spawn(2)]

    def place(rng):
        rad = r_place.uniform(5, 20)
        ang = r_place.uniform(0, 2 * np.pi)
        return np.array([rad * math.cos(ang), rad * math.sin(ang)])

    sc = make_scene(seed, 100.0, 3, 2, 1, place=place)
    sc.z0 = -1.5 - float(sc.terrain_np(0.0, 0.0))
    # re-derive object heights after the terrain shift
    sc = _rebase(sc, sc.z0)
    dirs = lidar_dirs(16, -15.0, 15.0, 1800, device)
    xyz = simulate_scan(sc, np.eye(3), np.zeros(3), dirs, 50.0, 0.02, r_noise)
    pose = pose12(np.eye(3), np.zeros(3))
    return dict(params=params_for(128, 128, 32, 0.4, 16), scans=[xyz], poses=[pose],
                flags=[0], firing=16, scene=sc)


def _rebase(sc: Scene, dz: float) -> Scene:
    """Objects were placed on the unshifted terrain; shift them by dz."""
    if len(sc.boxes):
        sc.boxes[:, 4:6] += dz
    if len(sc.pits):
        sc.pits[:, 4] += dz
    if len(sc.spheres):
        sc.spheres[:, 2] += dz
        sc.clusters[:, 2] += dz
    return sc


def sequence_64beam(seed=2, n_scans=100, device="cpu", n_az=2048, n_beams=64, n_sim=None):
    """64-beam x 2048 scans (131,072 points, 100 m, sigma 0.02 m) along a spline at
    4.5 m/s, one scan per 0.1 s, yaw noise 0.1 deg; 300 x 300 m scene with 40 boxes,
    60 vegetation clusters and 10 pits; 512 x 512 x 64 map at 0.2 m, recentred.
    The scene and trajectory are those of the n_scans-scan sequence; only the first
    n_sim scans (default all) are simulated, so a shorter run sees exactly the
    first scans of the full one."""
    s_traj, s_noise = np.random.SeedSequence(seed).spawn(2)
    r_noise = np.random.default_rng(s_noise)
    base = make_scene(seed + 1000, 300.0, 0, 0, 0)
    _, _, path = trajectory(base, np.random.default_rng(s_traj), n_scans, 0.45, 1.5, 0.1, 300.0)
    sc = make_scene(seed + 1000, 300.0, 40, 60, 10, keep_clear=(path, 3.0))
    true, mapper, _ = trajectory(sc, np.random.default_rng(s_traj), n_scans, 0.45, 1.5, 0.1,
                                 300.0)
    n_sim = n_scans if n_sim is None else min(n_sim, n_scans)
    dirs = lidar_dirs(n_beams, -16.6, 16.6, n_az, device)
    scans = [simulate_scan(sc, R, t, dirs, 100.0, 0.02, r_noise) for R, t in true[:n_sim]]
    return dict(params=params_for(512, 512, 64, 0.2, 32), scans=scans, poses=mapper[:n_sim],
                flags=[1] * n_sim, firing=n_beams, scene=sc)


def multi_lidar_frames(seed=3, n_frames=50, device="cpu", n_sim=None):
    """One 128-beam x 2048 lidar at (0, 0, 1.8) plus two 32-beam x 1024 lidars at
    (+-0.7, 0.9, 1.2) pitched 10 deg down; 12 m/s; dense vegetation (100..2000
    points per cubic metre, element radius 0.02 m); relief keeps slopes below 35 deg;
    1024 x 1024 x 96 map at 0.1 m.  Each frame = three inserts (primary recentres).
    Scene and trajectory are those of n_frames frames; the first n_sim frames
    (default all) are simulated."""
    s_traj, s_noise, s_dens = np.random.SeedSequence(seed).spawn(3)
    r_noise, r_dens = np.random.default_rng(s_noise), np.random.default_rng(s_dens)

    def dens(rng):
        return int(np.exp(r_dens.uniform(np.log(100), np.log(2000))) * (4 / 3) * np.pi * 1.5 ** 3)

    relief = (3.0, 27.0)
    base = make_scene(seed + 1000, 300.0, 0, 0, 0, relief=relief)
    _, _, path = trajectory(base, np.random.default_rng(s_traj), n_frames, 1.2, 0.0, 0.1, 300.0)
    sc = make_scene(seed + 1000, 300.0, 40, 60, 10, cluster_points=dens, element_r=0.02,
                    relief=relief, keep_clear=(path, 3.0))
    true, mapper, _ = trajectory(sc, np.random.default_rng(s_traj), n_frames, 1.2, 0.0, 0.1,
                                 300.0)
    mounts = [(np.eye(3), np.array([0.0, 0.0, 1.8]), 128, -22.5, 22.5, 2048),
              (rot_zyx(0.0, math.radians(10), 0.0), np.array([0.7, 0.9, 1.2]), 32, -16, 16, 1024),
              (rot_zyx(0.0, math.radians(10), 0.0), np.array([-0.7, 0.9, 1.2]), 32, -16, 16, 1024)]
    scans, poses, flags, firing = [], [], [], []
    n_sim = n_frames if n_sim is None else min(n_sim, n_frames)
    for (Rv, tv), pm in zip(true[:n_sim], mapper[:n_sim]):
        Rm = pm.reshape(3, 4)[:, :3].astype(np.float64)
        tm = pm.reshape(3, 4)[:, 3].astype(np.float64)
        for k, (Rs, ts, nb, lo, hi, naz) in enumerate(mounts):
            dirs = lidar_dirs(nb, lo, hi, naz, device)
            scans.append(simulate_scan(sc, Rv @ Rs, Rv @ ts + tv, dirs, 100.0, 0.02, r_noise))
            poses.append(pose12(Rm @ Rs, Rm @ ts + tm))
            flags.append(1 if k == 0 else 0)
            firing.append(nb)
    return dict(params=params_for(1024, 1024, 96, 0.1, 48), scans=scans, poses=poses,
                flags=flags, firing=firing, scene=sc)


def small_random_cloud(seed: int, n: int, extent: float, device="cpu"):
    """Uniform points in a box around the sensor, a fraction non-finite (tests)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-extent, extent, (n, 3)).astype(np.float32)
    p[rng.uniform(size=n) < 0.05] = np.nan
    return torch.as_tensor(p, device=device)


def batch_of_vehicles(n_maps=32, n_steps=100, seed0=400, device="cpu", n_beams=64, n_sim=None):
    """Independent vehicles for batched serving: map i uses scene seed seed0 + i,
    its scan size N_i is drawn log-uniformly in [20k, 330k] points per step
    (n_beams x round(N_i / n_beams) azimuths), its grid uniformly from
    {256 x 256 x 48 at 0.4 m, 512 x 512 x 64 at 0.2 m}; 4.5 m/s, one scan per
    0.1 s, 100 m range, sigma 0.02 m.  Scenes and trajectories are those of
    n_steps steps; the first n_sim steps (default all) are simulated."""
    out = []
    n_sim = n_steps if n_sim is None else min(n_sim, n_steps)
    for i in range(n_maps):
        s_traj, s_noise, s_pick = np.random.SeedSequence(seed0 + i).spawn(3)
        rp = np.random.default_rng(s_pick)
        grid = [(256, 256, 48, 0.4), (512, 512, 64, 0.2)][int(rp.integers(0, 2))]
        base = make_scene(seed0 + i + 1000, 300.0, 0, 0, 0)
        _, _, path = trajectory(base, np.random.default_rng(s_traj), n_steps, 0.45, 1.5, 0.1,
                                300.0)
        sc = make_scene(seed0 + i + 1000, 300.0, 40, 60, 10, keep_clear=(path, 3.0))
        true, mapper, _ = trajectory(sc, np.random.default_rng(s_traj), n_steps, 0.45, 1.5, 0.1,
                                     300.0)
        r_noise = np.random.default_rng(s_noise)
        scans = []
        for (R, t) in true[:n_sim]:
            n_pts = float(np.exp(rp.uniform(np.log(20000), np.log(330000))))
            n_az = max(1, int(round(n_pts / n_beams)))
            dirs = lidar_dirs(n_beams, -16.6, 16.6, n_az, device)
            scans.append(simulate_scan(sc, R, t, dirs, 100.0, 0.02, r_noise))
        out.append(dict(params=params_for(*grid), scans=scans, poses=mapper[:n_sim],
                        firing=n_beams))
    return out


def surrogate_sequence(seed: int, n_scans: int = 20, device="cpu", n_beams=32, n_az=1024):
    """Gap-fill training / evaluation sequence: n_scans scans of a 32-beam x 1024
    lidar (50 m, sigma 0.02 m) along a spline at 4.5 m/s (0.45 m per scan) in a
    150 x 150 m scene with 12 boxes, 20 vegetation clusters and 4 pits;
    128 x 128 x 32 map at 0.4 m.  Scan 0 is the single-frame input, all scans
    together give the dense label."""
    s_traj, s_noise = np.random.SeedSequence(seed).spawn(2)
    r_noise = np.random.default_rng(s_noise)
    base = make_scene(seed + 5000, 150.0, 0, 0, 0)
    _, _, path = trajectory(base, np.random.default_rng(s_traj), n_scans, 0.45, 1.5, 0.1, 150.0)
    sc = make_scene(seed + 5000, 150.0, 12, 20, 4, keep_clear=(path, 3.0))
    true, mapper, _ = trajectory(sc, np.random.default_rng(s_traj), n_scans, 0.45, 1.5, 0.1,
                                 150.0)
    dirs = lidar_dirs(n_beams, -16.6, 16.6, n_az, device)
    scans = [simulate_scan(sc, R, t, dirs, 50.0, 0.02, r_noise) for R, t in true]
    return dict(params=params_for(128, 128, 32, 0.4, 16), scans=scans, poses=mapper,
                firing=n_beams)


# ---------------------------------------------------------------- small semantic scenes


def _window_params(nx, nz, res):
    return params_for(nx, nx, nz, res, nz // 2)


def column_centre_plane(nx=32, nz=16, res=0.5, z0=-1.75, slope_x=0.0):
    """One point at the centre of every column of the initial window (world =
    sensor frame, identity pose) on the plane z = z0 + slope_x * x.  With a
    power-of-two voxel edge and these values every coordinate is exact in
    binary32 and in the Q16 grid."""
    p = _window_params(nx, nz, res)
    i = np.arange(nx)
    c = (i - nx // 2 + 0.5) * res
    X, Y = np.meshgrid(c, c, indexing="ij")
    Z = z0 + slope_x * X
    pts = np.stack([X, Y, Z], -1).reshape(-1, 3).astype(np.float32)
    return dict(params=p, scans=[torch.as_tensor(pts)], poses=[pose12(np.eye(3), np.zeros(3))],
                flags=[0], firing=1)


def semantic_scene(kind: str, device="cpu"):
    """Small ray-cast scenes with one feature each on flat ground 1.5 m below
    the sensor (32-beam lidar, -25..+10 deg, 1800 azimuths, 30 m, sigma 5 mm,
    map 256 x 256 x 32 at 0.2 m in the initial window, no recentring):
      box      a 1 x 1 x 2 m box, front face at x = 7.1, y in [-0.5, 0.5];
      cluster  500 elements (radius 5 cm) uniform in a 1.5 m sphere centred
               at (8, 3) 1.5 m above the ground;
      pit      a 2 x 2 x 1 m pit, x in [4.1, 6.1], y in [-0.9, 1.1];
      downhill the ground drops 1.5 m at x = 8 (cliff); a second scan from
               (20, 0) on the lower ground sees the area the first one could
               not;
      uphill   a ramp rising 1.5 m from x = 6 to x = 7.5 (slope 1).
    Returns the workload dict plus `feature`, the feature's geometry."""
    sc = Scene(waves=np.zeros((0, 4)), z0=-1.5)
    feat = {}
    poses = [pose12(np.eye(3), np.zeros(3))]
    if kind == "box":
        sc.boxes = np.array([[7.1, 8.1, -0.5, 0.5, -1.6, 0.4]])
        feat = dict(x=(7.1, 8.1), y=(-0.5, 0.5))
    elif kind == "cluster":
        rng = np.random.default_rng(11)
        u = rng.normal(size=(500, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        rad = 1.5 * rng.uniform(size=500) ** (1 / 3)
        c = np.array([8.0, 3.0, 0.0])
        sc.spheres = np.concatenate([c + u * rad[:, None], np.full((500, 1), 0.05)], 1)
        sc.clusters = np.array([[8.0, 3.0, 0.0, 1.5, 0]])
        sc.cluster_end = np.array([500], np.int64)
        feat = dict(centre=(8.0, 3.0), radius=1.5)
    elif kind == "pit":
        sc.pits = np.array([[4.1, 6.1, -0.9, 1.1, -2.5]])
        feat = dict(x=(4.1, 6.1), y=(-0.9, 1.1))
    elif kind == "downhill":
        sc.ramps = np.array([[8.0, 8.02, -1.5]])
        poses.append(pose12(rot_zyx(math.pi, 0.0, 0.0), np.array([20.0, 0.0, -1.5])))
        feat = dict(edge=8.0, drop=1.5)
    elif kind == "uphill":
        sc.ramps = np.array([[6.0, 7.5, 1.5]])
        feat = dict(x=(6.0, 7.5), slope=1.0)
    else:
        raise ValueError(kind)
    rng = np.random.default_rng(7)
    dirs = lidar_dirs(32, -25.0, 10.0, 1800, device)
    scans = []
    for p in poses:
        P = p.reshape(3, 4).astype(np.float64)
        scans.append(simulate_scan(sc, P[:, :3], P[:, 3], dirs, 30.0, 0.005, rng))
    return dict(params=_window_params(256, 32, 0.2), scans=scans, poses=poses,
                flags=[0] * len(poses), firing=32, scene=sc, feature=feat)
