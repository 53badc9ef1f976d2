"""Independent double-precision references used to pin the oracle.

Nothing here shares code with the oracle or the GPU library: ray/voxel
intersection is the slab test over every voxel of a micro grid, and the pixel
cell of a voxel centre is found with atan2 in degrees. Each function reports
when its answer is too close to a decision boundary to be compared.
"""
from __future__ import annotations

import math

import numpy as np

UNK, FREE, OCC = 0, 1, 2


def slab_intervals(dims, q, d):
    """Entry/exit parameters of the line q + t d through every voxel (fp64)."""
    nx, ny, nz = dims
    q = np.asarray(q, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    lo_all, hi_all = [], []
    for a, n in enumerate((nx, ny, nz)):
        i = np.arange(n, dtype=np.float64)
        if d[a] != 0.0:
            t1 = (i - q[a]) / d[a]
            t2 = (i + 1.0 - q[a]) / d[a]
            lo, hi = np.minimum(t1, t2), np.maximum(t1, t2)
        else:
            inside = (i <= q[a]) & (q[a] < i + 1.0)
            lo = np.where(inside, -np.inf, np.inf)
            hi = np.where(inside, np.inf, -np.inf)
        lo_all.append(lo)
        hi_all.append(hi)
    # arrays indexed [z][y][x]
    tin = np.maximum(np.maximum(lo_all[2][:, None, None], lo_all[1][None, :, None]), lo_all[0][None, None, :])
    tout = np.minimum(np.minimum(hi_all[2][:, None, None], hi_all[1][None, :, None]), hi_all[0][None, None, :])
    return tin, tout


def ray_reference(states, q, d, rv, eps=1e-4):
    """Voxels the ray must / may visit and the first-hit depth (fp64).

    Returns (must_ids, may_ids, h_ref, h_ambiguous) with linear ids x + nx(y + ny z).
    """
    nz, ny, nx = states.shape
    tin, tout = slab_intervals((nx, ny, nz), q, d)
    entry = np.maximum(tin, 0.0)
    length = tout - entry
    cross = (tout > 0.0)
    solid = cross & (length > eps) & (entry < rv - eps)
    touch = (tout > -eps) & (length > -eps) & (entry < rv + eps)
    occ = states == OCC
    occ_may = touch & occ
    occ_must = solid & occ
    t_occ_may = float(entry[occ_may].min()) if occ_may.any() else math.inf
    t_occ_must = float(entry[occ_must].min()) if occ_must.any() else math.inf
    must = solid & (entry < t_occ_may - eps)
    may = touch & (entry <= t_occ_must + eps)
    ids = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    h_amb = bool(t_occ_may < t_occ_must - eps or abs(t_occ_must - rv) < eps)
    h_ref = t_occ_must if t_occ_must < rv else float(rv)
    return set(ids[must].tolist()), set(ids[may].tolist()), h_ref, h_amb, dict(entry=entry, ids=ids)


def pixel_of(sensor, qa, c0, ix, iy, iz):
    """(in_cell, row, col, ambiguous) of voxel centre (ix,iy,iz) seen from qa, fp64 angles."""
    W, H = sensor.n_az, sensor.n_el
    daz = 360.0 / W
    dl = sensor.fov_v_deg / H
    wb = sensor.w_buf
    r = np.array([ix + 0.5, iy + 0.5, iz + 0.5], dtype=np.float64) - np.asarray(qa, dtype=np.float64)
    rho = math.hypot(r[0], r[1])
    if rho < 1e-6:
        return False, -1, -1, True
    az = math.degrees(math.atan2(r[1], r[0]))
    beta0 = sensor.az_offset_deg + c0 * daz
    rel = (az - beta0) % 360.0
    el = math.degrees(math.atan2(r[2], rho))
    amb = False
    # distance to nearest azimuth boundary, in degrees
    fa = rel / daz
    if abs(fa - round(fa)) * daz < 1e-4 or abs(rel - 360.0) < 1e-4:
        amb = True
    fe = (el + sensor.fov_v_deg / 2.0) / dl
    if abs(fe - round(fe)) * dl < 1e-4:
        amb = True
    if not (0.0 <= rel < wb * daz) or not (-sensor.fov_v_deg / 2.0 <= el < sensor.fov_v_deg / 2.0):
        return False, -1, -1, amb
    col = int(math.floor(fa))
    row = int(math.floor(fe))
    return True, min(row, H - 1), min(col, wb - 1), amb


def observed(sensor, qa, c0, Da, ix, iy, iz, eps=1e-4):
    """(observed, ambiguous) for ancestor at qa with window start c0 and buffer Da (fp64)."""
    inside, row, col, amb = pixel_of(sensor, qa, c0, ix, iy, iz)
    if not inside:
        return False, amb
    r = np.array([ix + 0.5, iy + 0.5, iz + 0.5], dtype=np.float64) - np.asarray(qa, dtype=np.float64)
    rng = float(np.linalg.norm(r))
    D = float(Da[row, col])
    if abs(rng - D) < eps * max(1.0, D):
        amb = True
    return rng <= D, amb


def best_window(bins, w):
    bins = np.asarray(bins, dtype=np.int64)
    B = bins.shape[0]
    ext = np.concatenate([bins, bins[:w]])
    sums = np.array([ext[k:k + w].sum() for k in range(B)])
    k = int(np.flatnonzero(sums == sums.max())[0])
    return int(sums[k]), k
