"""Small scenes with one feature each, sent through insert and the 2D export,
checked against what the geometry fixes (Sec. III-D, and the step climbs of
Sec. IV-B):

* points at the column centres of a flat plane: slope 0 and roughness 0
  exactly, the plane's height exactly, no obstacle;
* the plane z = x/4 at r = 0.5 m: slope exactly 1/4, roughness 0;
* a ray-cast 1 x 1 x 2 m box: hard exactly on the columns of its visible
  face, nowhere else;
* a sparse vegetation cluster: mostly soft, positive only on its footprint;
* a 2 x 2 x 1 m pit whose floor the lidar cannot see: its interior is
  undefined and flagged negative;
* a 1.5 m cliff seen from above (the downhill climb): the hidden lower
  ground near the far end of the shadow is negative; after a scan from the
  lower ground it is not;
* a ramp rising 1.5 m over 1.5 m (the uphill climb): slope near 1 on the
  ramp, near 0 on the flat.

The `-m "not gpu"` tests run the oracle; the `gpu` tests run the HIP path,
require it to equal the oracle element by element, and apply the same checks
to its output.
"""
import numpy as np
import pytest

import oracle
from synth import scenegen

R = 0.2          # voxel edge of the ray-cast scenes
HALF = 128       # window-local index of world coordinate 0 (256-wide window)


def _col(v):
    """Window-local column of world coordinate v in the ray-cast scenes."""
    return int(np.floor(v / R)) + HALF


def _centres():
    c = (np.arange(256) - HALF + 0.5) * R
    return np.meshgrid(c, c, indexing="ij")


def check_flat(outs, w):
    g = outs[-1]
    d = (g["flags"] & 32) > 0
    assert d.all() and (g["flags"] & 1).all()
    assert (g["slope"] == 0.0).all() and (g["rough"] == 0.0).all()
    assert (g["height"] == np.float32(-1.75)).all()
    assert not (g["flags"] & (2 | 16)).any()


def check_pitched(outs, w):
    g = outs[-1]
    p = w["params"]
    assert ((g["flags"] & 32) > 0).all()
    assert (g["slope"] == 0.25).all() and (g["rough"] == 0.0).all()
    x = (np.arange(p["nx"]) - p["nx"] // 2 + 0.5) * p["res_m"]
    assert (g["height"] == (-1.75 + 0.25 * x)[:, None].astype(np.float32)).all()


def check_box(outs, w):
    fl = outs[-1]["flags"]
    hard = np.argwhere(fl & 4)
    # the visible face x = 7.1, y in [-0.5, 0.5] lies in one column row
    want = [(_col(7.1), _col(y)) for y in (-0.5, -0.3, -0.1, 0.1, 0.3, 0.5)]
    assert sorted(map(tuple, hard.tolist())) == sorted(want)
    assert not (fl & 8).any()


def check_cluster(outs, w):
    fl = outs[-1]["flags"]
    X, Y = _centres()
    foot = np.hypot(X - 8.0, Y - 3.0) <= 1.5 + R
    soft, hard = (fl & 8) > 0, (fl & 4) > 0
    assert not ((fl & 2) > 0)[~foot].any()
    assert soft[foot].sum() >= 30 and soft[foot].sum() > 2 * hard[foot].sum()


def check_pit(outs, w):
    fl = outs[-1]["flags"]
    X, Y = _centres()
    inner = (X > 4.2) & (X < 6.0) & (Y > -0.8) & (Y < 1.0)  # columns wholly inside
    assert not (fl[inner] & 1).any()          # the floor is never seen
    assert ((fl[inner] & 16) > 0).sum() >= 20
    near = (X > 3.1) & (X < 7.1) & (Y > -1.9) & (Y < 2.1)
    assert not ((fl & 16) > 0)[~near].any()


def check_downhill(outs, w):
    # shadow of the edge x = 8 (sensor 1.5 m above the upper ground, drop
    # 1.5 m): lower ground from x = 8 to x = 16 unseen.  Columns within the
    # 5 m search of both the edge and the seen lower ground (11 < x < 13)
    # find both levels.
    first, second = outs[0]["flags"], outs[1]["flags"]
    rows = slice(_col(-4.0), _col(4.0) + 1)
    band = slice(_col(11.2), _col(12.8) + 1)
    assert ((first[band, rows] & 16) > 0).all()
    assert not (first[band, rows] & 1).any()
    shadow = slice(_col(8.2), _col(15.8) + 1)
    assert not (second[shadow, rows] & 16).any()   # the lower ground was seen
    assert (second[shadow, rows] & 1).sum() >= 200


def check_uphill(outs, w):
    g = outs[-1]
    rows = slice(_col(-2.0), _col(2.0) + 1)
    ramp = g["slope"][_col(6.4):_col(7.0) + 1, rows]     # 5 x 5 windows on the ramp only
    assert not np.isnan(ramp).any()
    assert np.abs(ramp - 1.0).max() < 0.15
    flat = g["slope"][_col(2.4):_col(5.0) + 1, rows]
    assert np.nanmax(flat) < 0.05


SCENES = {
    "flat": (lambda: scenegen.column_centre_plane(slope_x=0.0), check_flat),
    "pitched": (lambda: scenegen.column_centre_plane(slope_x=0.25), check_pitched),
    "box": (lambda: scenegen.semantic_scene("box"), check_box),
    "cluster": (lambda: scenegen.semantic_scene("cluster"), check_cluster),
    "pit": (lambda: scenegen.semantic_scene("pit"), check_pit),
    "downhill": (lambda: scenegen.semantic_scene("downhill"), check_downhill),
    "uphill": (lambda: scenegen.semantic_scene("uphill"), check_uphill),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_scene_oracle(name):
    make, check = SCENES[name]
    w = make()
    o = oracle.OracleMap(w["params"])
    outs = []
    try:
        for xyz, pose, fl in zip(w["scans"], w["poses"], w["flags"]):
            assert o.insert_scan(xyz.numpy(), pose, fl) == oracle.OK
            outs.append(o.export_2d())
    finally:
        o.close()
    check(outs, w)


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(SCENES))
def test_scene_hip(name):
    from parity_util import Pair, compare_all
    make, check = SCENES[name]
    w = make()
    pair = Pair(w["params"])
    outs = []
    try:
        for xyz, pose, fl in zip(w["scans"], w["poses"], w["flags"]):
            assert pair.insert(xyz, pose, fl, firing=w["firing"]) == 0
            _, g, _ = compare_all(pair)
            outs.append(g)
    finally:
        pair.close()
    check(outs, w)
