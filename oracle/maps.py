"""Oracle of the map conversion and map updates (test infrastructure only).

The planners keep a truncated signed distance field; Sec. IV converts it into
the contiguous grid the GPU reads. Reading used here (the paper gives no
rule): a voxel is unknown unless its weight reaches the minimum weight,
occupied when its signed distance is at most the surface threshold (inside
the surface or within the band), free otherwise; comparisons with NaN are
false (a NaN weight is unknown, a NaN distance free). Updates between replans
replace the states of listed voxels; ids outside the grid and states above 2
are skipped. Plain numpy, no blocking; float32 comparisons as given.
"""
from __future__ import annotations

import numpy as np

UNK, FREE, OCC = 0, 1, 2


def tsdf_states(distance, weight, surface_m, min_weight):
    """uint8 states [nz, ny, nx] of a TSDF (float32 distance in metres, float32 weight)."""
    d = np.asarray(distance, dtype=np.float32)
    w = np.asarray(weight, dtype=np.float32)
    known = w >= np.float32(min_weight)            # False for NaN
    occupied = d <= np.float32(surface_m)          # False for NaN
    return np.where(known, np.where(occupied, OCC, FREE), UNK).astype(np.uint8)


def apply_updates(states, voxel_ids, new_states):
    """Copy of `states` with listed voxels replaced; returns (states, number of skipped entries)."""
    out = np.array(states, dtype=np.uint8, copy=True)
    flat = out.reshape(-1)
    skipped = 0
    for i, s in zip(np.asarray(voxel_ids, dtype=np.int64), np.asarray(new_states, dtype=np.int64)):
        if 0 <= i < flat.size and 0 <= s <= 2:
            flat[i] = s
        else:
            skipped += 1
    return out, skipped


def apply_box(states, lo, box_states):
    """Copy of `states` with the box starting at lo = (x, y, z) replaced by box_states [sz, sy, sx]."""
    out = np.array(states, dtype=np.uint8, copy=True)
    sz, sy, sx = box_states.shape
    x, y, z = (int(v) for v in lo)
    out[z:z + sz, y:y + sy, x:x + sx] = box_states
    return out
