"""Pins of the map-conversion oracle (oracle/maps.py) against closed forms.

A sphere's signed distance field gives occupied voxels exactly where the voxel
centre lies within the radius (centres at integer squared distances, radius^2
not an integer, so no centre is on the boundary); unknown voxels are exactly
those below the minimum weight; the thresholds are inclusive as stated;
NaNs follow the stated rule; updates replace exactly the listed voxels.
"""
import numpy as np

from oracle import maps


def _sphere(n=24, r=7.3, c=(11.5, 12.5, 10.5)):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    dist2 = (x + 0.5 - c[0]) ** 2 + (y + 0.5 - c[1]) ** 2 + (z + 0.5 - c[2]) ** 2
    return (np.sqrt(dist2) - r).astype(np.float32), dist2


def test_sphere_occupancy():
    d, dist2 = _sphere()
    w = np.ones_like(d)
    st = maps.tsdf_states(d, w, 0.0, 0.5)
    assert np.array_equal(st == maps.OCC, dist2 <= 7.3 ** 2)
    assert np.all(st[dist2 > 7.3 ** 2] == maps.FREE)
    # a band of one unit around the surface is also occupied
    st1 = maps.tsdf_states(d, w, 1.0, 0.5)
    assert np.array_equal(st1 == maps.OCC, dist2 <= 8.3 ** 2)


def test_weights_decide_unknown():
    d, _ = _sphere()
    rng = np.random.Generator(np.random.PCG64(3))
    w = rng.uniform(0, 2, d.shape).astype(np.float32)
    st = maps.tsdf_states(d, w, 0.0, 1.0)
    assert np.array_equal(st == maps.UNK, w < 1.0)
    assert np.array_equal(st[w >= 1.0], maps.tsdf_states(d, np.ones_like(d), 0.0, 1.0)[w >= 1.0])


def test_thresholds_inclusive_and_nan():
    d = np.array([0.25, 0.25, 0.2500001, -5, np.nan, 1.0], np.float32)
    w = np.array([1.0, 0.5, 1.0, 1.0, 1.0, np.nan], np.float32)
    st = maps.tsdf_states(d, w, 0.25, 0.5)
    assert st.tolist() == [maps.OCC, maps.OCC, maps.FREE, maps.OCC, maps.FREE, maps.UNK]


def test_updates_and_boxes():
    st = np.zeros((4, 5, 6), np.uint8)
    ids = [0, 6 * 5 * 4 - 1, 7, 6 * 5 * 4, 3]
    new = [2, 1, 2, 1, 9]
    out, skipped = maps.apply_updates(st, ids, new)
    assert skipped == 2
    assert out[0, 0, 0] == 2 and out[3, 4, 5] == 1 and out[0, 1, 1] == 2 and out[0, 0, 3] == 0
    assert out.sum() == 5
    box = np.full((2, 3, 4), 2, np.uint8)
    out2 = maps.apply_box(st, (1, 2, 1), box)
    assert out2[1:3, 2:5, 1:5].min() == 2 and out2.sum() == 2 * box.size
