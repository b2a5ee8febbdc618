"""Training and evaluation driver of the learned gap-fill surrogate (a project
extension next to the paper's plain per-column estimates).

Examples come from the library's own mapper: the dense label is the plain
height and roughness of a map into which a whole sequence of scans was
inserted; the input is a map of the sequence's first scan alone, in the same
window, with a random 30-70 % of its columns emptied (``sgt_thin``) so that
the network sees gaps it has to fill.  Everything numeric runs in the HIP
library (mapping, features, network, loss, gradients, Adam, fallback); this
module only loops over examples and steps.
"""
from __future__ import annotations

import numpy as np

from . import gvom


def _nan_where(t, keep):
    import torch
    return torch.where(keep, t, torch.full_like(t, float("nan")))


class Example:
    """One (input scan, dense label) pair in a fixed map window."""

    def __init__(self, seq: dict):
        import torch
        self.params = seq["params"]
        self.scan = seq["scans"][0].cuda().contiguous()
        self.pose = np.asarray(seq["poses"][0], np.float32)
        self.firing = gvom.MAP_FIRING(seq["firing"])
        self.sensor = self.pose.reshape(3, 4)[:, 3].copy()
        dense = gvom.VoxelMap(self.params)
        dense.insert(self.scan, self.pose, gvom.MAP_RECENTER | self.firing)
        for xyz, pose in zip(seq["scans"][1:], seq["poses"][1:]):
            dense.insert(xyz.cuda().contiguous(), pose, self.firing)
        out = dense.export_2d()
        hdef = (out["flags"] & 1) != 0
        sdef = (out["flags"] & 32) != 0
        self.label = torch.stack([_nan_where(out["height"], hdef), _nan_where(out["rough"], sdef)],
                                 dim=2).contiguous()
        self.origin = dense.origin().copy()
        dense.close()
        self.map = gvom.VoxelMap(self.params)
        nx, ny = self.params["nx"], self.params["ny"]
        self.feat = torch.empty((nx, ny, 16), dtype=torch.float32, device="cuda")
        self.thin = torch.zeros((nx, ny), dtype=torch.uint8, device="cuda")

    def make_input(self, rng: np.random.Generator, frac: float | None = None):
        """Single-scan map with a random fraction of its columns thinned; fills
        self.feat and returns the plain 2D maps of the thinned map."""
        import torch
        nx, ny = self.params["nx"], self.params["ny"]
        if frac is None:
            frac = float(rng.uniform(0.3, 0.7))
        mask = (rng.uniform(size=(nx, ny)) < frac).astype(np.uint8)
        self.thin.copy_(torch.from_numpy(mask))
        st = gvom.map_reset(self.map.h)
        if st != gvom.MAP_OK:
            raise RuntimeError(gvom.map_status_str(st))
        self.map.insert(self.scan, self.pose, gvom.MAP_RECENTER | self.firing)
        if not np.array_equal(self.map.origin(), self.origin):
            raise RuntimeError("input and label windows differ")
        if gvom.sgt_thin(self.map, self.thin) != gvom.MAP_OK:
            raise RuntimeError("sgt_thin failed")
        plain = self.map.export_2d()
        gvom.sgt_features(self.map, plain, self.sensor, self.thin, self.feat)
        return plain

    def close(self):
        self.map.close()


def fit_normalisation(net: gvom.Surrogate, examples, rng, reps: int = 2):
    """Per-feature mean and standard deviation over thinned training inputs."""
    s = np.zeros(32)
    n = 0
    for _ in range(reps):
        for ex in examples:
            ex.make_input(rng)
            s += net.feature_sums(ex.feat)
            n += ex.feat.shape[0] * ex.feat.shape[1]
    mean = s[:16] / n
    var = np.maximum(s[16:] / n - mean ** 2, 0.0)
    std = np.maximum(np.sqrt(var), 1e-3)
    net.set_norm(mean.astype(np.float32), std.astype(np.float32))
    return mean, std


def train(net: gvom.Surrogate, examples, steps: int, lr: float, rng, log_every: int = 0):
    """Adam on the masked L1 loss, one freshly thinned example per step."""
    losses = []
    for it in range(steps):
        ex = examples[it % len(examples)]
        ex.make_input(rng)
        loss, _ = net.loss_grad(ex.feat, ex.label)
        net.adam(lr)
        losses.append(loss)
        if log_every and (it + 1) % log_every == 0:
            print(f"step {it + 1}: loss {np.mean(losses[-log_every:]):.4f}", flush=True)
    return losses


def evaluate(net: gvom.Surrogate, examples, rng, tol_m: float = 0.05, frac: float = 0.5):
    """Height error on the columns that the label defines and the thinned
    single-scan plain map does not (the gaps), for the raw network and for
    the fallback merge, plus the merge's coverage gain."""
    import torch
    err_net, err_fill, n_gap, n_filled, n_plain, n_label = [], [], 0, 0, 0, 0
    for ex in examples:
        plain = ex.make_input(rng, frac)
        pred = net.forward(ex.feat)
        fh, _ = gvom.sgt_fill(pred, plain, tol_m)
        torch.cuda.synchronize()
        lab = ex.label[..., 0]
        ldef = ~torch.isnan(lab)
        pdef = ~torch.isnan(plain["height"])
        gap = ldef & ~pdef
        filled = gap & ~torch.isnan(fh)
        err_net.append((pred[..., 0] - lab)[gap].abs().cpu().numpy())
        err_fill.append((fh - lab)[filled].abs().cpu().numpy())
        n_gap += int(gap.sum())
        n_filled += int(filled.sum())
        n_plain += int((ldef & pdef).sum())
        n_label += int(ldef.sum())
    en = np.concatenate(err_net)
    ef = np.concatenate(err_fill) if n_filled else np.zeros(0)
    return {
        "gap_mae_net": float(en.mean()) if en.size else float("nan"),
        "gap_mae_filled": float(ef.mean()) if ef.size else float("nan"),
        "gaps": n_gap, "filled": n_filled,
        "coverage_plain": n_plain / max(n_label, 1),
        "coverage_filled": (n_plain + n_filled) / max(n_label, 1),
    }


# ---- full-size examples: every scan of a sequence in one fixed window ------


class WindowSequence:
    """A sequence of scans in one fixed map window, the window of its middle
    pose: the dense label is the plain height / roughness of all its scans
    accumulated, and every scan alone is one input frame."""

    def __init__(self, seq: dict):
        import torch
        self.params = seq["params"]
        self.scans = [s.cuda().contiguous() for s in seq["scans"]]
        self.poses = [np.asarray(p, np.float32) for p in seq["poses"]]
        self.firing = gvom.MAP_FIRING(seq["firing"])
        self.mid = len(self.scans) // 2
        dense = gvom.VoxelMap(self.params)
        self._place(dense)
        for xyz, pose in zip(self.scans, self.poses):
            dense.insert(xyz, pose, self.firing)
        out = dense.export_2d()
        hdef = (out["flags"] & 1) != 0
        sdef = (out["flags"] & 32) != 0
        self.label = torch.stack([_nan_where(out["height"], hdef), _nan_where(out["rough"], sdef)],
                                 dim=2).contiguous()
        self.origin = dense.origin().copy()
        dense.close()

    def _place(self, m):
        """Moves m's window onto the middle pose (an insert of no points)."""
        st = gvom.map_insert_scan(m.h, None, self.poses[self.mid], gvom.MAP_RECENTER)
        if st != gvom.MAP_OK:
            raise RuntimeError(gvom.map_status_str(st))

    def __len__(self):
        return len(self.scans)


class InputBuilder:
    """Builds input frames of WindowSequence examples in one reused map:
    scan k alone in the sequence's window, a random fraction of its columns
    thinned; fills self.feat and returns the plain 2D maps of that map."""

    def __init__(self, params: dict):
        import torch
        self.params = params
        self.map = gvom.VoxelMap(params)
        nx, ny = params["nx"], params["ny"]
        self.feat = torch.empty((nx, ny, 16), dtype=torch.float32, device="cuda")
        self.thin = torch.zeros((nx, ny), dtype=torch.uint8, device="cuda")

    def make_input(self, ws: WindowSequence, k: int, rng: np.random.Generator,
                   frac: float | None = None):
        import torch
        nx, ny = self.params["nx"], self.params["ny"]
        if frac is None:
            frac = float(rng.uniform(0.3, 0.7))
        mask = (rng.uniform(size=(nx, ny)) < frac).astype(np.uint8)
        self.thin.copy_(torch.from_numpy(mask))
        st = gvom.map_reset(self.map.h)
        if st != gvom.MAP_OK:
            raise RuntimeError(gvom.map_status_str(st))
        ws._place(self.map)
        self.map.insert(ws.scans[k], ws.poses[k], ws.firing)
        if not np.array_equal(self.map.origin(), ws.origin):
            raise RuntimeError("input and label windows differ")
        if gvom.sgt_thin(self.map, self.thin) != gvom.MAP_OK:
            raise RuntimeError("sgt_thin failed")
        plain = self.map.export_2d()
        sensor = ws.poses[k].reshape(3, 4)[:, 3].copy()
        gvom.sgt_features(self.map, plain, sensor, self.thin, self.feat)
        return plain

    def close(self):
        self.map.close()


def fit_normalisation_frames(net: gvom.Surrogate, builder: InputBuilder, seqs, rng,
                             frames: int = 64):
    """Feature mean and standard deviation over `frames` random input frames."""
    s = np.zeros(32)
    n = 0
    for _ in range(frames):
        ws = seqs[int(rng.integers(len(seqs)))]
        builder.make_input(ws, int(rng.integers(len(ws))), rng)
        s += net.feature_sums(builder.feat)
        n += builder.feat.shape[0] * builder.feat.shape[1]
    mean = s[:16] / n
    std = np.maximum(np.sqrt(np.maximum(s[16:] / n - mean ** 2, 0.0)), 1e-3)
    net.set_norm(mean.astype(np.float32), std.astype(np.float32))
    return mean, std


def train_frames(net: gvom.Surrogate, builder: InputBuilder, seqs, steps: int, lr: float, rng,
                 log_every: int = 0):
    """Adam on the masked L1 loss; each step one random frame (sequence, scan)
    with a fresh thinning mask."""
    losses = []
    for it in range(steps):
        ws = seqs[int(rng.integers(len(seqs)))]
        builder.make_input(ws, int(rng.integers(len(ws))), rng)
        loss, _ = net.loss_grad(builder.feat, ws.label)
        net.adam(lr)
        losses.append(loss)
        if log_every and (it + 1) % log_every == 0:
            print(f"step {it + 1}: loss {np.mean(losses[-log_every:]):.4f}", flush=True)
    return losses


def evaluate_frames(net: gvom.Surrogate, builder: InputBuilder, seqs, rng, tol_m: float = 0.05):
    """Every frame of the held-out sequences, thinned by a random 30-70 %:
    the network's height error on the gaps (label defined, plain map not),
    and, against the label, the error and coverage of the plain map and of
    the filled map (plain where defined, the network where the fallback rule
    accepts it)."""
    import torch
    e_gap, e_fill, e_plainmap, e_filledmap = [], [], [], []
    n_label = n_plain = n_filled = n_gap = 0
    for ws in seqs:
        lab = ws.label[..., 0]
        ldef = ~torch.isnan(lab)
        for k in range(len(ws)):
            plain = builder.make_input(ws, k, rng)
            pred = net.forward(builder.feat)
            fh, _ = gvom.sgt_fill(pred, plain, tol_m)
            pdef = ~torch.isnan(plain["height"])
            gap = ldef & ~pdef
            filled = gap & ~torch.isnan(fh)
            both = ldef & pdef
            e_gap.append((pred[..., 0] - lab)[gap].abs().cpu().numpy())
            e_fill.append((fh - lab)[filled].abs().cpu().numpy())
            e_plainmap.append((plain["height"] - lab)[both].abs().cpu().numpy())
            e_filledmap.append((fh - lab)[ldef & ~torch.isnan(fh)].abs().cpu().numpy())
            n_label += int(ldef.sum())
            n_plain += int(both.sum())
            n_filled += int(filled.sum())
            n_gap += int(gap.sum())
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0)
    eg, ef, ep, em = cat(e_gap), cat(e_fill), cat(e_plainmap), cat(e_filledmap)
    mean = lambda a: float(a.mean()) if a.size else float("nan")
    return {
        "frames": sum(len(ws) for ws in seqs), "tol_m": tol_m,
        "gap_mae_net_m": mean(eg), "gap_mae_filled_m": mean(ef),
        "plain_map_mae_m": mean(ep), "filled_map_mae_m": mean(em),
        "coverage_plain": n_plain / max(n_label, 1),
        "coverage_filled": (n_plain + n_filled) / max(n_label, 1),
        "gap_columns": n_gap, "filled_columns": n_filled,
    }
