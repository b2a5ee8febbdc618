"""Thin Python binding of libgvom.so (include/gvom.h), argument marshalling only.

Every function has the name of the C entry point it calls.  Device buffers are
torch CUDA (HIP) tensors; torch supplies device memory and streams, every step
of the mapping path runs in the library's HIP kernels.  There is no CPU path:
if the library is not built, or a tensor is not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgvom.so")

MAP_OK, MAP_E_INVALID, MAP_E_POSE, MAP_E_SENSOR_OUTSIDE = 0, -1, -2, -3
MAP_E_RANGE, MAP_E_CAPACITY, MAP_E_OOM, MAP_E_DEVICE = -4, -5, -6, -7
MAP_RECENTER = 1
MAP_STATS_DISTINCT = 2


def MAP_FIRING(b: int) -> int:
    return (int(b) & 0xFFFF) << 16


class map_params_t(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("res_m", ctypes.c_float), ("sensor_z_voxel", ctypes.c_int32),
                ("obs_min_m", ctypes.c_float), ("obs_max_m", ctypes.c_float),
                ("dens_num", ctypes.c_int32), ("dens_den", ctypes.c_int32),
                ("fit_n", ctypes.c_int32), ("neg_thresh_m", ctypes.c_float),
                ("neg_search_m", ctypes.c_float)]


class map_derived_t(ctypes.Structure):
    _fields_ = [("inv_r", ctypes.c_float), ("n_lo", ctypes.c_int32), ("n_hi", ctypes.c_int32),
                ("tau_neg_q", ctypes.c_int64), ("search_d", ctypes.c_int32),
                ("half_fit", ctypes.c_int32)]


class map_2d_t(ctypes.Structure):
    _fields_ = [("height", ctypes.c_void_p), ("slope", ctypes.c_void_p),
                ("rough", ctypes.c_void_p), ("density", ctypes.c_void_p),
                ("flags", ctypes.c_void_p)]


class map_tuning_t(ctypes.Structure):
    _fields_ = [("seg_len", ctypes.c_int32), ("trace_waves_per_cu", ctypes.c_int32),
                ("surface_tile", ctypes.c_int32)]


COST_LAYERS = ("slope", "rough", "density", "positive", "hard", "soft", "negative", "unknown")


class map_cost_weights_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in COST_LAYERS]


class map_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_points", "n_nonfinite", "n_range", "n_hits", "n_pass",
                 "n_distinct_pass", "n_distinct_hit", "n_cleared", "n_pass_updates")]


EXPORTED = [
    "map_params_validate", "map_create", "map_destroy", "map_reset", "map_insert_scan",
    "map_export_2d", "map_export_voxels", "map_export_voxels_async", "map_import_voxels", "map_get_stats",
    "map_get_origin", "map_sync", "map_status_str", "map_profile_enable", "map_profile_read",
    "map_set_tuning", "map_get_tuning",
    "map_batch_create", "map_batch_destroy", "map_batch_step", "map_batch_latency",
    "map_batch_set_graph", "map_batch_autotune",
    "map_buffer_create", "map_buffer_destroy", "map_buffer_reset", "map_buffer_push",
    "map_buffer_combine", "map_buffer_count", "map_buffer_get_stats",
    "map_export_density", "map_costmap", "map_buffer_set_incremental",
    "sgt_num_params", "sgt_create", "sgt_destroy", "sgt_get_params", "sgt_set_params",
    "sgt_set_norm", "sgt_features", "sgt_thin", "sgt_feature_sums", "sgt_forward",
    "sgt_loss_grad", "sgt_adam", "sgt_fill",
    "map_set_device_memory_limit", "map_device_memory_in_use",
    "map_calib_copy", "map_calib_atomic", "map_insert_scan_static",
]
PROF_PHASES = ("scroll", "rays", "trace", "column", "surface", "lut")

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libgvom.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.map_set_device_memory_limit.argtypes = [I64]
        L.map_device_memory_in_use.argtypes = []
        L.map_device_memory_in_use.restype = I64
        L.map_params_validate.argtypes = [ctypes.POINTER(map_params_t),
                                          ctypes.POINTER(map_derived_t)]
        L.map_create.argtypes = [ctypes.POINTER(map_params_t), P, ctypes.POINTER(P)]
        L.map_destroy.argtypes = [P]
        L.map_reset.argtypes = [P]
        L.map_insert_scan.argtypes = [P, P, I64, P, ctypes.c_uint32]
        L.map_insert_scan_static.argtypes = [P, P, I64, P, ctypes.c_uint32]
        L.map_export_2d.argtypes = [P, ctypes.POINTER(map_2d_t)]
        L.map_export_voxels.argtypes = [P, P, P, I64, P, P]
        L.map_export_voxels_async.argtypes = [P, P, P, I64, P, P]
        L.map_import_voxels.argtypes = [P, P, P, I64, P]
        L.map_get_stats.argtypes = [P, ctypes.POINTER(map_stats_t)]
        L.map_get_origin.argtypes = [P, P]
        L.map_sync.argtypes = [P]
        L.map_set_tuning.argtypes = [P, ctypes.POINTER(map_tuning_t)]
        L.map_get_tuning.argtypes = [P, ctypes.POINTER(map_tuning_t)]
        L.map_batch_create.argtypes = [P, I32, P, ctypes.POINTER(P)]
        L.map_batch_destroy.argtypes = [P]
        L.map_batch_step.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.map_batch_latency.argtypes = [P, P]
        L.map_batch_set_graph.argtypes = [P, I32]
        L.map_batch_autotune.argtypes = [P, P, P, P, P, P, ctypes.c_char_p,
                                         ctypes.POINTER(map_tuning_t)]
        L.map_export_density.argtypes = [P, P]
        L.map_costmap.argtypes = [P, ctypes.POINTER(map_2d_t), ctypes.POINTER(map_cost_weights_t), P]
        L.map_buffer_create.argtypes = [ctypes.POINTER(map_params_t), I32, P, ctypes.POINTER(P)]
        L.map_buffer_destroy.argtypes = [P]
        L.map_buffer_reset.argtypes = [P]
        L.map_buffer_push.argtypes = [P, P, I64, P, ctypes.c_uint32]
        L.map_buffer_combine.argtypes = [P, P]
        L.map_buffer_count.argtypes = [P]
        L.map_buffer_set_incremental.argtypes = [P, I32]
        L.map_buffer_get_stats.argtypes = [P, ctypes.POINTER(map_stats_t)]
        L.sgt_num_params.argtypes = []
        L.sgt_create.argtypes = [I32, I32, ctypes.c_uint64, P, ctypes.POINTER(P)]
        L.sgt_destroy.argtypes = [P]
        L.sgt_get_params.argtypes = [P, P]
        L.sgt_set_params.argtypes = [P, P]
        L.sgt_set_norm.argtypes = [P, P, P]
        L.sgt_features.argtypes = [P, ctypes.POINTER(map_2d_t), P, P, P]
        L.sgt_thin.argtypes = [P, P]
        L.sgt_feature_sums.argtypes = [P, P, P]
        L.sgt_forward.argtypes = [P, P, P]
        L.sgt_loss_grad.argtypes = [P, P, P, P, P]
        L.sgt_adam.argtypes = [P, ctypes.c_float]
        L.sgt_fill.argtypes = [P, ctypes.POINTER(map_2d_t), I32, I32, ctypes.c_float, P, P, P]
        L.map_profile_enable.argtypes = [P, I32]
        L.map_profile_read.argtypes = [P, P, P]
        L.map_calib_copy.argtypes = [P, P, I64, P]
        L.map_calib_atomic.argtypes = [P, I64, I64, I32, I32, ctypes.c_uint32, P]
        L.map_status_str.argtypes = [I32]
        L.map_status_str.restype = ctypes.c_char_p
        for f in EXPORTED:
            if f != "map_status_str":
                getattr(L, f).restype = I32
        L.sgt_num_params.restype = I64
        L.map_device_memory_in_use.restype = I64
        _lib = L
    return _lib


def _dev(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _params(p: dict) -> map_params_t:
    return map_params_t(**{k: p[k] for k, _ in map_params_t._fields_})


def map_status_str(status: int) -> str:
    return lib().map_status_str(status).decode()


def map_params_validate(params: dict):
    d = map_derived_t()
    s = lib().map_params_validate(ctypes.byref(_params(params)), ctypes.byref(d))
    return s, {k: getattr(d, k) for k, _ in map_derived_t._fields_}


def map_create(params: dict, stream=None):
    """Returns (status, handle).  `stream` is a torch.cuda.Stream or None (current)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    s = lib().map_create(ctypes.byref(_params(params)), ctypes.c_void_p(stream.cuda_stream),
                         ctypes.byref(h))
    return s, h


def map_destroy(h) -> int:
    return lib().map_destroy(h)


def map_reset(h) -> int:
    return lib().map_reset(h)


def map_insert_scan(h, xyz, pose, flags: int = 0) -> int:
    import torch
    n = 0 if xyz is None else xyz.shape[0]
    ptr = ctypes.c_void_p(0) if n == 0 else _dev(xyz, torch.float32, "xyz")
    if n and (xyz.dim() != 2 or xyz.shape[1] != 3):
        raise ValueError("xyz must be [n, 3]")
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    return lib().map_insert_scan(h, ptr, n, pose.ctypes.data_as(ctypes.c_void_p), flags)


def map_insert_scan_static(h, xyz, pose, flags: int = 0) -> int:
    """map_insert_scan whose work buffers come from the library's fixed
    per-GPU array (no device allocation)."""
    import torch
    n = 0 if xyz is None else xyz.shape[0]
    ptr = ctypes.c_void_p(0) if n == 0 else _dev(xyz, torch.float32, "xyz")
    if n and (xyz.dim() != 2 or xyz.shape[1] != 3):
        raise ValueError("xyz must be [n, 3]")
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    return lib().map_insert_scan_static(h, ptr, n, pose.ctypes.data_as(ctypes.c_void_p), flags)


def map_export_2d(h, out: dict) -> int:
    import torch
    o = map_2d_t(_dev(out["height"], torch.float32, "height"),
                 _dev(out["slope"], torch.float32, "slope"),
                 _dev(out["rough"], torch.float32, "rough"),
                 _dev(out["density"], torch.float32, "density"),
                 _dev(out["flags"], torch.uint8, "flags"))
    return lib().map_export_2d(h, ctypes.byref(o))


def map_export_voxels(h, lut, data):
    """lut int32[V], data int32[cap, 3] (or None); -> (status, n_occupied, origin).
    Synchronises; status MAP_E_CAPACITY when cap < n_occupied."""
    import torch
    cap = 0 if data is None else data.shape[0]
    dptr = ctypes.c_void_p(0) if data is None else _dev(data, torch.int32, "data")
    origin = np.zeros(3, np.int32)
    n_occ = ctypes.c_int64(-1)
    s = lib().map_export_voxels(h, _dev(lut, torch.int32, "lut"), dptr, cap,
                                ctypes.byref(n_occ), origin.ctypes.data_as(ctypes.c_void_p))
    return s, int(n_occ.value), origin


def map_export_voxels_async(h, lut, data, n_occupied):
    """As map_export_voxels without waiting: n_occupied is a device int64[1]
    tensor written on the stream; -> (status, origin)."""
    import torch
    cap = 0 if data is None else data.shape[0]
    dptr = ctypes.c_void_p(0) if data is None else _dev(data, torch.int32, "data")
    origin = np.zeros(3, np.int32)
    s = lib().map_export_voxels_async(h, _dev(lut, torch.int32, "lut"), dptr, cap,
                                      _dev(n_occupied, torch.int64, "n_occupied"),
                                      origin.ctypes.data_as(ctypes.c_void_p))
    return s, origin


def map_import_voxels(h, lut, data, origin) -> int:
    import torch
    n = 0 if data is None else data.shape[0]
    dptr = ctypes.c_void_p(0) if data is None else _dev(data, torch.int32, "data")
    origin = np.ascontiguousarray(origin, dtype=np.int32).reshape(3)
    return lib().map_import_voxels(h, _dev(lut, torch.int32, "lut"), dptr, n,
                                   origin.ctypes.data_as(ctypes.c_void_p))


def map_export_density(h, density) -> int:
    import torch
    return lib().map_export_density(h, _dev(density, torch.float32, "density"))


def map_costmap(h, out2d: dict, weights: dict, cost) -> int:
    import torch
    w = map_cost_weights_t(*[float(weights.get(k, 0.0)) for k in COST_LAYERS])
    o = _out2d(out2d)
    return lib().map_costmap(h, ctypes.byref(o), ctypes.byref(w), _dev(cost, torch.float32, "cost"))


def map_get_stats(h):
    st = map_stats_t()
    s = lib().map_get_stats(h, ctypes.byref(st))
    return s, {k: getattr(st, k) for k, _ in map_stats_t._fields_}


def map_get_origin(h):
    o = np.zeros(3, np.int32)
    s = lib().map_get_origin(h, o.ctypes.data_as(ctypes.c_void_p))
    return s, o


def map_sync(h) -> int:
    return lib().map_sync(h)


def map_set_tuning(h, seg_len: int = 0, trace_waves_per_cu: int = 0, surface_tile: int = 0) -> int:
    return lib().map_set_tuning(h, ctypes.byref(map_tuning_t(seg_len, trace_waves_per_cu,
                                                             surface_tile)))


def map_get_tuning(h):
    t = map_tuning_t()
    s = lib().map_get_tuning(h, ctypes.byref(t))
    return s, {"seg_len": t.seg_len, "trace_waves_per_cu": t.trace_waves_per_cu,
               "surface_tile": t.surface_tile}


MAP_PROF_ALL = (1 << len(PROF_PHASES)) - 1


def map_profile_enable(h, enable=True) -> int:
    """enable: True (every phase), False, or a mask of phases (bit p = PROF_PHASES[p])."""
    mask = MAP_PROF_ALL if enable is True else (0 if enable is False else int(enable))
    return lib().map_profile_enable(h, mask)


def map_profile_read(h):
    """-> (status, {phase: (total_ms, launches)})"""
    ms = np.zeros(len(PROF_PHASES), np.float64)
    cnt = np.zeros(len(PROF_PHASES), np.int64)
    s = lib().map_profile_read(h, ms.ctypes.data_as(ctypes.c_void_p),
                               cnt.ctypes.data_as(ctypes.c_void_p))
    return s, {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PROF_PHASES)}


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[p if isinstance(p, int) else (p.value or 0)
                                           for p in ptrs])
    return arr


class MapBatch:
    """A batch of VoxelMaps stepped together (map_batch_* calls)."""

    def __init__(self, maps, stream=None):
        """stream: a torch.cuda.Stream, or None for a stream owned by the batch."""
        self.maps = list(maps)
        hs = (ctypes.c_void_p * len(self.maps))(*[m.h.value for m in self.maps])
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(0 if stream is None else stream.cuda_stream)
        s = lib().map_batch_create(hs, len(self.maps), sp, ctypes.byref(h))
        if s != MAP_OK:
            raise RuntimeError(f"map_batch_create: {map_status_str(s)}")
        self.h = h

    def close(self):
        if self.h:
            lib().map_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _inputs(self, xyzs, poses, flags):
        import torch
        k = len(self.maps)
        assert len(xyzs) == k and len(poses) == k and len(flags) == k
        ptrs, ns = [], []
        for x in xyzs:
            if x is None or x.shape[0] == 0:
                ptrs.append(0)
                ns.append(0)
            else:
                ptrs.append(_dev(x, torch.float32, "xyz").value)
                ns.append(int(x.shape[0]))
        xa = _ptr_array(ptrs)
        na = np.ascontiguousarray(ns, dtype=np.int64)
        pa = np.ascontiguousarray(np.stack([np.asarray(p, np.float32).reshape(12) for p in poses]))
        fa = np.ascontiguousarray(flags, dtype=np.uint32)
        outs = (map_2d_t * k)()
        for i, m in enumerate(self.maps):
            o = m.out2d
            outs[i] = map_2d_t(_dev(o["height"]), _dev(o["slope"]), _dev(o["rough"]),
                               _dev(o["density"]), _dev(o["flags"]))
        keep = (xa, na, pa, fa, outs)
        return keep

    def step(self, xyzs, poses, flags, voxels=None):
        """voxels: None, or a list of k booleans (export the lookup table of map i)."""
        k = len(self.maps)
        xa, na, pa, fa, outs = self._inputs(xyzs, poses, flags)
        P = ctypes.c_void_p
        if voxels is None:
            la = da = ca = oa = None
        else:
            lptr, dptr, cap, optr = [], [], [], []
            for i, m in enumerate(self.maps):
                if voxels[i]:
                    V = m.lut.numel()
                    if m.data is None or m.data.shape[0] != V:
                        import torch
                        m.data = torch.empty((V, 3), dtype=torch.int32, device=m.lut.device)
                    lptr.append(m.lut.data_ptr())
                    dptr.append(m.data.data_ptr())
                    cap.append(V)
                    optr.append(m.n_occ.data_ptr())
                else:
                    lptr.append(0)
                    dptr.append(0)
                    cap.append(0)
                    optr.append(0)
            la, da, oa = _ptr_array(lptr), _ptr_array(dptr), _ptr_array(optr)
            ca = np.ascontiguousarray(cap, dtype=np.int64)
        s = lib().map_batch_step(
            self.h, xa, na.ctypes.data_as(P), pa.ctypes.data_as(P), fa.ctypes.data_as(P),
            ctypes.cast(outs, P), la, da, None if ca is None else ca.ctypes.data_as(P), oa)
        if s != MAP_OK:
            raise RuntimeError(f"map_batch_step: {map_status_str(s)}")

    def latency_ms(self):
        ms = np.zeros(len(self.maps), np.float64)
        s = lib().map_batch_latency(self.h, ms.ctypes.data_as(ctypes.c_void_p))
        if s != MAP_OK:
            raise RuntimeError(map_status_str(s))
        return ms

    def set_graph(self, enable: bool):
        return lib().map_batch_set_graph(self.h, 1 if enable else 0)

    def autotune(self, xyzs, poses, flags, cache_path=None):
        xa, na, pa, fa, outs = self._inputs(xyzs, poses, flags)
        P = ctypes.c_void_p
        t = map_tuning_t()
        s = lib().map_batch_autotune(self.h, xa, na.ctypes.data_as(P), pa.ctypes.data_as(P),
                                     fa.ctypes.data_as(P), ctypes.cast(outs, P),
                                     None if cache_path is None else cache_path.encode(),
                                     ctypes.byref(t))
        if s != MAP_OK:
            raise RuntimeError(f"map_batch_autotune: {map_status_str(s)}")
        return {"seg_len": t.seg_len, "trace_waves_per_cu": t.trace_waves_per_cu,
                "surface_tile": t.surface_tile}


class VoxelMap:
    """Owns one map and its export buffers (torch tensors on the current device)."""

    def __init__(self, params: dict, stream=None):
        import torch
        self.params = dict(params)
        s, self.h = map_create(params, stream)
        if s != MAP_OK:
            raise RuntimeError(f"map_create: {map_status_str(s)}")
        nx, ny, nz = params["nx"], params["ny"], params["nz"]
        dev = torch.device("cuda", torch.cuda.current_device())
        self.out2d = {k: torch.empty((nx, ny), dtype=torch.float32, device=dev)
                      for k in ("height", "slope", "rough", "density")}
        self.out2d["flags"] = torch.empty((nx, ny), dtype=torch.uint8, device=dev)
        self.lut = torch.empty(nx * ny * nz, dtype=torch.int32, device=dev)
        self.n_occ = torch.zeros(1, dtype=torch.int64, device=dev)
        self.data = None

    def close(self):
        if self.h:
            map_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what):
        if s != MAP_OK:
            raise RuntimeError(f"{what}: {map_status_str(s)}")

    def insert(self, xyz, pose, flags=0):
        self._check(map_insert_scan(self.h, xyz, pose, flags), "map_insert_scan")

    def export_2d(self):
        self._check(map_export_2d(self.h, self.out2d), "map_export_2d")
        return self.out2d

    def _data_for(self, cap):
        import torch
        if self.data is None or self.data.shape[0] != max(cap, 1):
            self.data = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=self.lut.device)
        return self.data[:cap] if cap else None

    def export_voxels(self, cap: int | None = None):
        """-> (lut, data, n_occupied: int, origin); synchronises.  With a cap
        below the occupied count the status MAP_E_CAPACITY is kept in
        self.last_export_status instead of raising."""
        cap = self.lut.numel() if cap is None else cap
        s, n, origin = map_export_voxels(self.h, self.lut, self._data_for(cap))
        self.last_export_status = s
        if s != MAP_E_CAPACITY:
            self._check(s, "map_export_voxels")
        return self.lut, self.data, n, origin

    def export_voxels_async(self, cap: int | None = None):
        """-> (lut, data, n_occupied device int64[1], origin); no wait."""
        cap = self.lut.numel() if cap is None else cap
        s, origin = map_export_voxels_async(self.h, self.lut, self._data_for(cap), self.n_occ)
        self._check(s, "map_export_voxels_async")
        return self.lut, self.data, self.n_occ, origin

    def export_density(self):
        import torch
        if getattr(self, "density3d", None) is None:
            self.density3d = torch.empty(self.lut.numel(), dtype=torch.float32, device=self.lut.device)
        self._check(map_export_density(self.h, self.density3d), "map_export_density")
        return self.density3d

    def costmap(self, weights: dict, out2d=None):
        import torch
        out2d = self.out2d if out2d is None else out2d
        if getattr(self, "cost", None) is None:
            self.cost = torch.empty_like(self.out2d["height"])
        self._check(map_costmap(self.h, out2d, weights, self.cost), "map_costmap")
        return self.cost

    def stats(self):
        s, st = map_get_stats(self.h)
        self._check(s, "map_get_stats")
        return st

    def origin(self):
        return map_get_origin(self.h)[1]

    def sync(self):
        self._check(map_sync(self.h), "map_sync")


def map_buffer_create(params: dict, depth: int, stream=None):
    """Returns (status, handle).  `stream` is a torch.cuda.Stream or None (current)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    s = lib().map_buffer_create(ctypes.byref(_params(params)), depth,
                                ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
    return s, h


def map_buffer_destroy(h) -> int:
    return lib().map_buffer_destroy(h)


def map_buffer_reset(h) -> int:
    return lib().map_buffer_reset(h)


def map_buffer_push(h, xyz, pose, flags: int = 0) -> int:
    import torch
    n = 0 if xyz is None else xyz.shape[0]
    ptr = ctypes.c_void_p(0) if n == 0 else _dev(xyz, torch.float32, "xyz")
    if n and (xyz.dim() != 2 or xyz.shape[1] != 3):
        raise ValueError("xyz must be [n, 3]")
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    return lib().map_buffer_push(h, ptr, n, pose.ctypes.data_as(ctypes.c_void_p), flags)


def map_buffer_combine(h, out_map) -> int:
    return lib().map_buffer_combine(h, out_map)


def map_buffer_set_incremental(h, enable: bool) -> int:
    return lib().map_buffer_set_incremental(h, 1 if enable else 0)


def map_buffer_count(h) -> int:
    return lib().map_buffer_count(h)


def map_buffer_get_stats(h):
    st = map_stats_t()
    s = lib().map_buffer_get_stats(h, ctypes.byref(st))
    return s, {k: getattr(st, k) for k, _ in map_stats_t._fields_}


class ScanBuffer:
    """Owns a map buffer (the paper's per-scan maps, Sec. III-B); pushes run on
    `stream`, combines on the output map's stream."""

    def __init__(self, params: dict, depth: int, stream=None):
        self.params = dict(params)
        self.depth = depth
        s, self.h = map_buffer_create(params, depth, stream)
        if s != MAP_OK:
            raise RuntimeError(f"map_buffer_create: {map_status_str(s)}")

    def close(self):
        if self.h:
            map_buffer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, xyz, pose, flags=0):
        s = map_buffer_push(self.h, xyz, pose, flags)
        if s != MAP_OK:
            raise RuntimeError(f"map_buffer_push: {map_status_str(s)}")

    def combine(self, out: "VoxelMap"):
        s = map_buffer_combine(self.h, out.h)
        if s != MAP_OK:
            raise RuntimeError(f"map_buffer_combine: {map_status_str(s)}")

    def count(self) -> int:
        return map_buffer_count(self.h)

    def set_incremental(self, enable: bool):
        s = map_buffer_set_incremental(self.h, enable)
        if s != MAP_OK:
            raise RuntimeError(f"map_buffer_set_incremental: {map_status_str(s)}")

    def stats(self):
        s, st = map_buffer_get_stats(self.h)
        if s != MAP_OK:
            raise RuntimeError(f"map_buffer_get_stats: {map_status_str(s)}")
        return st


def _out2d(out):
    import torch
    return map_2d_t(_dev(out["height"], torch.float32), _dev(out["slope"], torch.float32),
                    _dev(out["rough"], torch.float32), _dev(out["density"], torch.float32),
                    _dev(out["flags"], torch.uint8))


class Surrogate:
    """The gap-fill network (sgt_* calls) for H x W maps."""

    N_FEAT = 16

    def __init__(self, H: int, W: int, seed: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.H, self.W = H, W
        h = ctypes.c_void_p()
        s = lib().sgt_create(H, W, seed, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if s != MAP_OK:
            raise RuntimeError(f"sgt_create: {map_status_str(s)}")
        self.h = h
        self.n_params = int(lib().sgt_num_params())

    def close(self):
        if self.h:
            lib().sgt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, s, what):
        if s != MAP_OK:
            raise RuntimeError(f"{what}: {map_status_str(s)}")

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        self._ok(lib().sgt_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), "sgt_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        self._ok(lib().sgt_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), "sgt_set_params")

    def set_norm(self, mean, std):
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        self._ok(lib().sgt_set_norm(self.h, mean.ctypes.data_as(ctypes.c_void_p),
                                    std.ctypes.data_as(ctypes.c_void_p)), "sgt_set_norm")

    def feature_sums(self, feat):
        out = np.zeros(32, np.float64)
        self._ok(lib().sgt_feature_sums(self.h, _dev(feat), out.ctypes.data_as(ctypes.c_void_p)),
                 "sgt_feature_sums")
        return out

    def forward(self, feat, out=None):
        import torch
        if out is None:
            out = torch.empty((self.H, self.W, 2), dtype=torch.float32, device=feat.device)
        self._ok(lib().sgt_forward(self.h, _dev(feat, torch.float32), _dev(out, torch.float32)),
                 "sgt_forward")
        return out

    def loss_grad(self, feat, label, want_grad=False):
        import torch
        loss = ctypes.c_float()
        g = np.zeros(self.n_params, np.float32) if want_grad else None
        self._ok(lib().sgt_loss_grad(self.h, _dev(feat, torch.float32), _dev(label, torch.float32),
                                     ctypes.byref(loss),
                                     None if g is None else g.ctypes.data_as(ctypes.c_void_p)),
                 "sgt_loss_grad")
        return float(loss.value), g

    def adam(self, lr: float):
        self._ok(lib().sgt_adam(self.h, ctypes.c_float(lr)), "sgt_adam")


def sgt_features(vmap, plain, sensor_xyz, thin=None, out=None):
    import torch
    nx, ny = vmap.params["nx"], vmap.params["ny"]
    if out is None:
        out = torch.empty((nx, ny, 16), dtype=torch.float32, device=plain["height"].device)
    sxyz = np.ascontiguousarray(sensor_xyz, dtype=np.float32).reshape(3)
    o = _out2d(plain)
    s = lib().sgt_features(vmap.h, ctypes.byref(o), sxyz.ctypes.data_as(ctypes.c_void_p),
                           ctypes.c_void_p(0) if thin is None else _dev(thin, torch.uint8),
                           _dev(out, torch.float32))
    if s != MAP_OK:
        raise RuntimeError(f"sgt_features: {map_status_str(s)}")
    return out


def sgt_thin(vmap, thin) -> int:
    import torch
    return lib().sgt_thin(vmap.h, _dev(thin, torch.uint8))


def sgt_fill(pred, plain, tol_m: float, stream=None):
    import torch
    H, W = pred.shape[0], pred.shape[1]
    if stream is None:
        stream = torch.cuda.current_stream()
    h = torch.empty((H, W), dtype=torch.float32, device=pred.device)
    r = torch.empty((H, W), dtype=torch.float32, device=pred.device)
    o = _out2d(plain)
    s = lib().sgt_fill(_dev(pred, torch.float32), ctypes.byref(o), H, W, ctypes.c_float(tol_m),
                       _dev(h), _dev(r), ctypes.c_void_p(stream.cuda_stream))
    if s != MAP_OK:
        raise RuntimeError(f"sgt_fill: {map_status_str(s)}")
    return h, r


def map_calib_copy(dst, src, stream=None) -> int:
    """Enqueues the library's plain device copy of src into dst (same size)."""
    import torch
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("map_calib_copy: sizes differ")
    if stream is None:
        stream = torch.cuda.current_stream()
    return lib().map_calib_copy(_dev(dst), _dev(src), dst.numel() * dst.element_size(),
                                ctypes.c_void_p(stream.cuda_stream))


def map_calib_atomic(target, n_waves: int, per_wave: int, lanes_per_line: int,
                     seed: int = 1, stream=None) -> int:
    """Enqueues the library's scattered atomic-add kernel on the int32 target."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return lib().map_calib_atomic(_dev(target, torch.int32), target.numel(), n_waves, per_wave,
                                  lanes_per_line, ctypes.c_uint32(seed),
                                  ctypes.c_void_p(stream.cuda_stream))
