"""TEST INFRASTRUCTURE ONLY: oracle of the gap-fill surrogate (a project
extension, not part of the paper's method).

The network, its loss and gradient and the fallback merge are plain FP64 C
loops in ``sgt_oracle.c``; the per-column features and the column thinning
are written here in numpy over the oracle map's exported voxel state.
"""
from __future__ import annotations

import numpy as np

from . import lib, _ptr, OracleMap

N_FEAT = 16


def num_params() -> int:
    return int(lib().orc_sgt_num_params())


def forward(feat, params, round_bf16: bool = True) -> np.ndarray:
    """Network output [H][W][2] (float64) of normalised features [H][W][16]."""
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float32)
    H, W, C = feat.shape
    assert C == N_FEAT and params.size == num_params()
    out = np.zeros((H, W, 2), np.float64)
    s = lib().orc_sgt_forward(_ptr(feat), H, W, _ptr(params), int(round_bf16), _ptr(out))
    assert s == 0
    return out


def loss_grad(feat, params, label, round_bf16: bool = True):
    """Masked L1 loss and its gradient (float64) with respect to every parameter."""
    import ctypes
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float32)
    label = np.ascontiguousarray(label, dtype=np.float32)
    H, W, _ = feat.shape
    loss = ctypes.c_double()
    grad = np.zeros(num_params(), np.float64)
    s = lib().orc_sgt_loss_grad(_ptr(feat), H, W, _ptr(params), _ptr(label), int(round_bf16),
                                ctypes.byref(loss), _ptr(grad))
    assert s == 0
    return loss.value, grad


def fill(pred, plain_h, plain_r, tol_m: float):
    import ctypes
    pred = np.ascontiguousarray(pred, dtype=np.float32)
    plain_h = np.ascontiguousarray(plain_h, dtype=np.float32)
    plain_r = np.ascontiguousarray(plain_r, dtype=np.float32)
    H, W = plain_h.shape
    oh = np.zeros((H, W), np.float32)
    orr = np.zeros((H, W), np.float32)
    s = lib().orc_sgt_fill(_ptr(pred), _ptr(plain_h), _ptr(plain_r), H, W, ctypes.c_float(tol_m),
                           _ptr(oh), _ptr(orr))
    assert s == 0
    return oh, orr


def thin(omap: OracleMap, mask) -> None:
    """Empties every voxel of the window-local columns where mask[x][y] is set."""
    s, lut, data, n, origin = omap.export_voxels()
    assert s == 0
    nx, ny, nz = omap.nx, omap.ny, omap.nz
    lut = lut.reshape(nx, ny, nz).copy()
    m = np.asarray(mask).reshape(nx, ny).astype(bool)
    lut[m] = -1
    assert omap.import_voxels(lut, data, origin) == 0


def features(omap: OracleMap, plain: dict, sensor_xyz, thin_mask=None) -> np.ndarray:
    """Per-column features [nx][ny][16] (float32) of an oracle map.

    0 sum of hits, 1 sum of passes, 2 occupied voxels, 3 occupied fraction,
    4 ground height (the plain height), 5 lowest return of the highest
    occupied voxel, 6 mean lowest return of the occupied voxels, 7 height
    defined, 8 hits / (hits + passes) of the lowest occupied voxel, 9 band
    density, 10 slope, 11 roughness, 12 slope defined, 13 horizontal distance
    of the column centre to the sensor, 14 sensor height above the ground,
    15 column thinned.  Undefined values are 0; a thinned column keeps only
    13 and 15.  Metres: Q16 heights times res / 65536 in double.
    """
    s, lut, data, n, origin = omap.export_voxels()
    assert s == 0
    nx, ny, nz = omap.nx, omap.ny, omap.nz
    res = float(np.float32(omap.params["res_m"]))
    q2m = res / 65536.0
    lut = lut.reshape(nx, ny, nz).astype(np.int64)
    occ = lut >= 0
    idx = np.where(occ, lut, 0)
    hits = np.where(occ, data[idx, 0] if n else 0, 0).astype(np.int64)
    passes = np.where(occ, data[idx, 1] if n else 0, -1 - lut).astype(np.int64)
    minqz = np.where(occ, data[idx, 2] if n else 0, 0).astype(np.int64)
    f = np.zeros((nx, ny, N_FEAT), np.float64)
    cnt = occ.sum(axis=2)
    f[..., 0] = hits.sum(axis=2)
    f[..., 1] = passes.sum(axis=2)
    f[..., 2] = cnt
    f[..., 3] = cnt.astype(np.float64) / float(nz)
    any_occ = cnt > 0
    top = nz - 1 - np.argmax(occ[:, :, ::-1], axis=2)
    bot = np.argmax(occ, axis=2)
    xi, yi = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    f[..., 5] = np.where(any_occ, minqz[xi, yi, top].astype(np.float64) * q2m, 0.0)
    mean_q = minqz.sum(axis=2).astype(np.float64) / np.maximum(cnt, 1).astype(np.float64)
    f[..., 6] = np.where(any_occ, mean_q * q2m, 0.0)
    hb = hits[xi, yi, bot].astype(np.float64)
    pb = passes[xi, yi, bot].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        f[..., 8] = np.where(any_occ, hb / (hb + pb), 0.0)
    fl = plain["flags"]
    hdef = (fl & 1) != 0
    sx, sy, sz = (float(np.float32(v)) for v in sensor_xyz)
    height = plain["height"].astype(np.float64)
    f[..., 4] = np.where(hdef, height, 0.0)
    f[..., 7] = hdef
    f[..., 14] = np.where(hdef, sz - height, 0.0)
    f[..., 9] = np.where((fl & 2) != 0, plain["density"].astype(np.float64), 0.0)
    sdef = (fl & 32) != 0
    f[..., 10] = np.where(sdef, plain["slope"].astype(np.float64), 0.0)
    f[..., 11] = np.where(sdef, plain["rough"].astype(np.float64), 0.0)
    f[..., 12] = sdef
    cx = ((origin[0] + xi).astype(np.float64) + 0.5) * res - sx
    cy = ((origin[1] + yi).astype(np.float64) + 0.5) * res - sy
    d13 = np.sqrt(cx * cx + cy * cy)
    out = f.astype(np.float32)
    if thin_mask is not None:
        t = np.asarray(thin_mask).reshape(nx, ny).astype(bool)
        out[t] = 0.0
        out[t, 15] = 1.0
    out[..., 13] = d13.astype(np.float32)
    return out
