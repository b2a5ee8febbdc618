"""TEST INFRASTRUCTURE ONLY: the CPU oracle of the G-VOM per-scan mapping path.

Python wrapper (ctypes + numpy) around ``gvom_oracle.c``, a plain, slow,
single-threaded C statement of what the method computes (arXiv 2109.13176,
Section III).  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It imports nothing
from the HIP library and the HIP library imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gvom_oracle.c")
_SRC_SGT = os.path.join(_HERE, "sgt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID, E_POSE, E_SENSOR_OUT, E_RANGE, E_CAPACITY, E_OOM = 0, -1, -2, -3, -4, -5, -6
RECENTER = 1


def build() -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no SIMD flags)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra", "-fPIC",
           "-shared", "-o", _LIB + ".tmp", _SRC, _SRC_SGT, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("res_m", ctypes.c_float), ("sensor_z_voxel", ctypes.c_int32),
                ("obs_min_m", ctypes.c_float), ("obs_max_m", ctypes.c_float),
                ("dens_num", ctypes.c_int32), ("dens_den", ctypes.c_int32),
                ("fit_n", ctypes.c_int32), ("neg_thresh_m", ctypes.c_float),
                ("neg_search_m", ctypes.c_float)]


class Consts(ctypes.Structure):
    _fields_ = [("inv_r", ctypes.c_float), ("n_lo", ctypes.c_int32), ("n_hi", ctypes.c_int32),
                ("tau_neg_q", ctypes.c_int64), ("search_d", ctypes.c_int32),
                ("half_fit", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_points", "n_nonfinite", "n_range", "n_hits", "n_pass",
                 "n_distinct_pass", "n_distinct_hit", "n_cleared")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_derive.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Consts)]
        L.orc_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(P)]
        L.orc_destroy.argtypes = [P]
        L.orc_destroy.restype = None
        L.orc_reset.argtypes = [P]
        L.orc_insert_scan.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_uint32]
        L.orc_export_2d.argtypes = [P, P, P, P, P, P]
        L.orc_export_voxels.argtypes = [P, P, P, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int64), P]
        L.orc_import_voxels.argtypes = [P, P, P, ctypes.c_int64, P]
        L.orc_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.orc_get_origin.argtypes = [P, P]
        L.orc_combine.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P), P]
        L.orc_export_density.argtypes = [P, P]
        L.orc_costmap.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P]
        L.orc_transform_point.argtypes = [P, ctypes.c_float, P, P]
        L.orc_ray_voxels.argtypes = [P, P, P, ctypes.c_int64]
        L.orc_ray_voxels.restype = ctypes.c_int64
        L.orc_surface.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_float, ctypes.c_int32, ctypes.c_int64,
                                  P, P, P, P]
        L.orc_sgt_num_params.argtypes = []
        L.orc_sgt_num_params.restype = ctypes.c_int64
        L.orc_sgt_forward.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P]
        L.orc_sgt_loss_grad.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32,
                                        P, P]
        L.orc_sgt_fill.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P, P]
        for f in ("orc_sgt_forward", "orc_sgt_loss_grad", "orc_sgt_fill"):
            getattr(L, f).restype = ctypes.c_int32
        for f in ("orc_derive", "orc_create", "orc_reset", "orc_insert_scan", "orc_export_2d",
                  "orc_export_voxels", "orc_import_voxels", "orc_get_stats", "orc_get_origin", "orc_combine",
                  "orc_export_density", "orc_costmap",
                  "orc_transform_point", "orc_surface"):
            getattr(L, f).restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_params(d: dict) -> Params:
    return Params(**{k: d[k] for k, _ in Params._fields_})


def derive(params: dict):
    c = Consts()
    s = lib().orc_derive(ctypes.byref(make_params(params)), ctypes.byref(c))
    return s, {k: getattr(c, k) for k, _ in Consts._fields_}


def transform_point(pose, inv_r: float, p):
    pose = np.ascontiguousarray(pose, dtype=np.float32)
    p = np.ascontiguousarray(p, dtype=np.float32)
    q = np.zeros(3, dtype=np.int32)
    ok = lib().orc_transform_point(_ptr(pose), ctypes.c_float(inv_r), _ptr(p), _ptr(q))
    return bool(ok), q


def ray_voxels(s_q, p_q) -> np.ndarray:
    """Voxel sequence of the ray from Q16 point s_q to Q16 point p_q (unclipped)."""
    s = np.ascontiguousarray(s_q, dtype=np.int32)
    p = np.ascontiguousarray(p_q, dtype=np.int32)
    n = lib().orc_ray_voxels(_ptr(s), _ptr(p), None, 0)
    out = np.zeros((max(n, 1), 3), dtype=np.int32)
    lib().orc_ray_voxels(_ptr(s), _ptr(p), _ptr(out), n)
    return out[:n]


def surface(hq, defined, fit_n: int, res_m: float, search_d: int, tau_neg_q: int):
    """Slope, roughness, slope-defined and negative flags of a height grid (Q16)."""
    hq = np.ascontiguousarray(hq, dtype=np.int32)
    defined = np.ascontiguousarray(defined, dtype=np.uint8)
    nx, ny = hq.shape
    slope = np.zeros((nx, ny), np.float32)
    rough = np.zeros((nx, ny), np.float32)
    sdef = np.zeros((nx, ny), np.uint8)
    neg = np.zeros((nx, ny), np.uint8)
    s = lib().orc_surface(_ptr(hq), _ptr(defined), nx, ny, fit_n, ctypes.c_float(res_m),
                          search_d, tau_neg_q, _ptr(slope), _ptr(rough), _ptr(sdef), _ptr(neg))
    if s:
        raise ValueError(f"orc_surface status {s}")
    return slope, rough, sdef, neg


COST_LAYERS = ("slope", "rough", "density", "positive", "hard", "soft", "negative", "unknown")


def costmap(out2d: dict, weights: dict):
    """Planner costmap of Sec. IV from a 2D export: (cost, magnitude) in double."""
    sl = np.ascontiguousarray(out2d["slope"], dtype=np.float32).reshape(-1)
    ro = np.ascontiguousarray(out2d["rough"], dtype=np.float32).reshape(-1)
    de = np.ascontiguousarray(out2d["density"], dtype=np.float32).reshape(-1)
    fl = np.ascontiguousarray(out2d["flags"], dtype=np.uint8).reshape(-1)
    w = np.array([float(np.float32(weights.get(k, 0.0))) for k in COST_LAYERS], np.float64)
    cost = np.zeros(sl.size, np.float64)
    mag = np.zeros(sl.size, np.float64)
    s = lib().orc_costmap(_ptr(sl), _ptr(ro), _ptr(de), _ptr(fl), sl.size, _ptr(w), _ptr(cost),
                          _ptr(mag))
    if s:
        raise ValueError(f"orc_costmap status {s}")
    shape = np.shape(out2d["slope"])
    return cost.reshape(shape), mag.reshape(shape)


class OracleMap:
    """One map of the oracle; all arrays are host numpy arrays."""

    def __init__(self, params: dict):
        self.params = dict(params)
        h = ctypes.c_void_p()
        s = lib().orc_create(ctypes.byref(make_params(params)), ctypes.byref(h))
        if s:
            raise ValueError(f"orc_create status {s}")
        self._h = h
        self.nx, self.ny, self.nz = params["nx"], params["ny"], params["nz"]

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        return lib().orc_reset(self._h)

    def insert_scan(self, xyz, pose, flags: int = 0) -> int:
        xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
        return lib().orc_insert_scan(self._h, _ptr(xyz), xyz.shape[0], _ptr(pose), flags)

    def export_2d(self) -> dict:
        C = (self.nx, self.ny)
        out = {k: np.zeros(C, np.float32) for k in ("height", "slope", "rough", "density")}
        out["flags"] = np.zeros(C, np.uint8)
        s = lib().orc_export_2d(self._h, _ptr(out["height"]), _ptr(out["slope"]),
                                _ptr(out["rough"]), _ptr(out["density"]), _ptr(out["flags"]))
        if s:
            raise ValueError(f"orc_export_2d status {s}")
        return out

    def export_voxels(self, cap: int | None = None):
        V = self.nx * self.ny * self.nz
        lut = np.zeros(V, np.int32)
        if cap is None:
            cap = V
        data = np.zeros((max(cap, 1), 3), np.int32)
        n = ctypes.c_int64()
        origin = np.zeros(3, np.int32)
        s = lib().orc_export_voxels(self._h, _ptr(lut), _ptr(data), cap, ctypes.byref(n),
                                    _ptr(origin))
        return s, lut, data[:min(n.value, cap)], n.value, origin

    def import_voxels(self, lut, data, origin) -> int:
        lut = np.ascontiguousarray(lut, dtype=np.int32).reshape(-1)
        data = np.ascontiguousarray(data, dtype=np.int32).reshape(-1, 3)
        origin = np.ascontiguousarray(origin, dtype=np.int32).reshape(3)
        return lib().orc_import_voxels(self._h, _ptr(lut), _ptr(data), data.shape[0],
                                       _ptr(origin))

    def export_density(self) -> np.ndarray:
        out = np.zeros(self.nx * self.ny * self.nz, np.float32)
        s = lib().orc_export_density(self._h, _ptr(out))
        if s:
            raise ValueError(f"orc_export_density status {s}")
        return out

    def stats(self) -> dict:
        st = Stats()
        lib().orc_get_stats(self._h, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def origin(self) -> np.ndarray:
        o = np.zeros(3, np.int32)
        lib().orc_get_origin(self._h, _ptr(o))
        return o


class OracleBuffer:
    """The map buffer of Sec. III-B and the combine step of Sec. III-D.

    Pointcloud processing turns each scan into its own voxel map (III-C: a
    fresh window, this scan's hits, misses and lowest returns only), exported
    as (lookup table, data array, origin) and appended to the buffer; the
    buffer keeps the ``depth`` most recent maps.  A scan pushed with RECENTER
    gets a window centred on its sensor; otherwise it takes the window of the
    most recent buffered map (several lidars feeding one map), or the initial
    window while the buffer is empty.  ``combine`` writes the combination of
    the buffered maps into an OracleMap (``orc_combine``).
    """

    def __init__(self, params: dict, depth: int):
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.params = dict(params)
        self.depth = depth
        self.maps = []  # (lut, data, origin), oldest first
        self._scan = OracleMap(params)

    def close(self):
        self._scan.close()

    def push(self, xyz, pose, flags: int = 0) -> int:
        m = self._scan
        m.reset()
        if not (flags & RECENTER) and self.maps:
            V = m.nx * m.ny * m.nz
            s = m.import_voxels(np.full(V, -1, np.int32), np.zeros((0, 3), np.int32),
                                self.maps[-1][2])
            assert s == OK
        s = m.insert_scan(xyz, pose, flags & RECENTER)
        if s:
            return s
        s, lut, data, _, origin = m.export_voxels()
        assert s == OK
        self.maps.append((lut, np.ascontiguousarray(data), origin.copy()))
        if len(self.maps) > self.depth:
            self.maps.pop(0)
        return OK

    def combine(self, out: OracleMap) -> int:
        k = len(self.maps)
        if k == 0:
            return E_INVALID
        P = ctypes.c_void_p
        keep = [d if d.size else np.zeros((1, 3), np.int32) for _, d, _ in self.maps]
        luts = (P * k)(*[lut.ctypes.data for lut, _, _ in self.maps])
        datas = (P * k)(*[d.ctypes.data for d in keep])
        origins = np.ascontiguousarray(np.stack([o for _, _, o in self.maps]), dtype=np.int32)
        return lib().orc_combine(out._h, k, luts, datas, _ptr(origins))
