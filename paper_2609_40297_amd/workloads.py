"""Seeded synthetic workloads: occupancy grids, RRTs of candidate viewpoints, sensors.

This module only draws inputs. It holds none of the gain method's arithmetic
(no ray traversal, projection, window selection or depth buffers), imports
neither the oracle nor the HIP binding, and is the one piece of code that both
of them consume.

The paper evaluates on Voxblox maps of Gazebo worlds and a real patio
(Sec. V, Table I; Sec. VI); those maps are not available, so every map here is
synthetic with the paper's shapes: voxel states {unknown, free, occupied}
(Sec. III-A), a known region that follows the robot's past trajectory, RRT
edges of at most 1.5 m (Table I step sizes), tree sizes 50..3000 (Table II
sizes) and a 5..15 m sensor (Sec. V).

Recipe (numpy PCG64):
  * seed of workload i is 1000*(i+1); sub-streams: +0 map, +1 trajectory,
    +2 arrivals, +100+t tree t.
  * boxes: side per axis U[lo, hi] m, min corner U[0, extent-side]; a voxel is
    occupied in ground truth when its centre lies inside a box.
  * trajectory: random walk of K waypoints starting at a uniform free point
    with z in [1, ext_z-1]; each step has heading U[0, 2pi), length
    U[0.5, 1.5] m, dz U[-0.3, 0.3] m, clamped 1 m inside the borders; a step
    whose sampled segment enters an occupied voxel is redrawn (<= 100 tries).
  * known region: voxels whose centre is within `known_radius` of the
    trajectory polyline keep their ground-truth state; the rest are unknown.
  * RRT: the root is the last waypoint (or, for multi-tree workloads, a uniform
    point inside a uniformly drawn known-free voxel). Repeatedly sample a
    uniform point in the grid, find the nearest node whose depth is below the
    limit (ties: lowest id), steer to at most 1.5 m, accept when the point and
    the edge (sampled every v/4) lie in known-free voxels; ids grow so that
    parent < child.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

UNK, FREE, OCC = 0, 1, 2


@dataclasses.dataclass
class Sensor:
    """Panoramic candidate-ray sensor: n_az columns over 360 deg, n_el rows over fov_v."""
    n_az: int
    n_el: int
    fov_h_deg: float
    fov_v_deg: float
    range_m: float
    yaw_bins: int
    az_offset_deg: float = 0.0

    @property
    def window_bins(self) -> int:
        return int(round(self.yaw_bins * self.fov_h_deg / 360.0))

    @property
    def w_buf(self) -> int:
        return self.n_az * self.window_bins // self.yaw_bins

    @property
    def rays(self) -> int:
        return self.n_az * self.n_el


@dataclasses.dataclass
class Map:
    states: np.ndarray          # uint8 [nz][ny][nx] (x fastest in memory)
    voxel_m: float
    origin_m: np.ndarray        # float32[3]
    seed: int = 0

    @property
    def dims(self):
        nz, ny, nx = self.states.shape
        return nx, ny, nz

    @property
    def extent_m(self):
        nx, ny, nz = self.dims
        return np.array([nx, ny, nz], dtype=np.float64) * self.voxel_m


@dataclasses.dataclass
class Tree:
    pos_m: np.ndarray           # float32[n][3]
    parent: np.ndarray          # int32[n], parent[0] == -1, parent[i] < i
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.parent.shape[0])

    def depth(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.int32)
        for i in range(1, self.n):
            d[i] = d[self.parent[i]] + 1
        return d


@dataclasses.dataclass
class Workload:
    name: str
    map: Map
    trees: List[Tree]
    sensor: Sensor
    extra: Dict = dataclasses.field(default_factory=dict)

    @property
    def rays(self) -> int:
        return sum(t.n for t in self.trees) * self.sensor.rays


# --------------------------------------------------------------------------- maps

def _gt_boxes(rng, dims, v, n_boxes, side_lo, side_hi):
    nx, ny, nz = dims
    ext = np.array([nx, ny, nz], dtype=np.float64) * v
    occ = np.zeros((nz, ny, nx), dtype=bool)
    cx = (np.arange(nx) + 0.5) * v
    cy = (np.arange(ny) + 0.5) * v
    cz = (np.arange(nz) + 0.5) * v
    for _ in range(n_boxes):
        side = rng.uniform(side_lo, side_hi, size=3)
        side = np.minimum(side, ext)
        lo = rng.uniform(0.0, ext - side)
        hi = lo + side
        ix = np.nonzero((cx >= lo[0]) & (cx < hi[0]))[0]
        iy = np.nonzero((cy >= lo[1]) & (cy < hi[1]))[0]
        iz = np.nonzero((cz >= lo[2]) & (cz < hi[2]))[0]
        if ix.size and iy.size and iz.size:
            occ[iz[0]:iz[-1] + 1, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1] = True
    return occ


def _voxel_of(p, v, dims):
    i = np.floor(np.asarray(p, dtype=np.float64) / v).astype(np.int64)
    return i


def _inside(i, dims):
    return all(0 <= int(i[a]) < dims[a] for a in range(3))


def _segment_clear(a, b, v, dims, ok_grid):
    """True when every sample of segment a->b (spacing v/4) lies in a voxel with ok_grid True."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    L = float(np.linalg.norm(b - a))
    n = max(1, int(math.ceil(L / (0.25 * v))))
    s = np.linspace(0.0, 1.0, n + 1)[:, None]
    pts = a[None, :] + s * (b - a)[None, :]
    idx = np.floor(pts / v).astype(np.int64)
    nx, ny, nz = dims
    if (idx < 0).any() or (idx[:, 0] >= nx).any() or (idx[:, 1] >= ny).any() or (idx[:, 2] >= nz).any():
        return False
    return bool(ok_grid[idx[:, 2], idx[:, 1], idx[:, 0]].all())


def _trajectory(rng, dims, v, occ, k):
    nx, ny, nz = dims
    ext = np.array([nx, ny, nz], dtype=np.float64) * v
    free = ~occ
    lo = np.array([1.0, 1.0, 1.0])
    hi = ext - 1.0
    for _ in range(100000):
        p = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(lo[2], hi[2])])
        if free[tuple(_voxel_of(p, v, dims)[::-1])]:
            break
    pts = [p]
    for _ in range(k - 1):
        cur = pts[-1]
        nxt = cur
        for _try in range(100):
            hd = rng.uniform(0.0, 2.0 * math.pi)
            ln = rng.uniform(0.5, 1.5)
            dz = rng.uniform(-0.3, 0.3)
            cand = cur + np.array([ln * math.cos(hd), ln * math.sin(hd), dz])
            cand = np.clip(cand, lo, hi)
            if _segment_clear(cur, cand, v, dims, free):
                nxt = cand
                break
        pts.append(nxt)
    return np.array(pts)


def _known_mask(dims, v, traj, radius):
    """Voxels whose centre lies within `radius` metres of the polyline `traj`."""
    nx, ny, nz = dims
    known = np.zeros((nz, ny, nx), dtype=bool)
    r2 = radius * radius
    segs = [(traj[i], traj[i + 1]) for i in range(len(traj) - 1)] or [(traj[0], traj[0])]
    for a, b in segs:
        lo = np.minimum(a, b) - radius
        hi = np.maximum(a, b) + radius
        i0 = np.clip(np.floor(lo / v - 0.5).astype(int), 0, [nx, ny, nz])
        i1 = np.clip(np.ceil(hi / v - 0.5).astype(int) + 1, 0, [nx, ny, nz])
        if (i1 <= i0).any():
            continue
        cx = ((np.arange(i0[0], i1[0]) + 0.5) * v).astype(np.float32)
        cy = ((np.arange(i0[1], i1[1]) + 0.5) * v).astype(np.float32)
        cz = ((np.arange(i0[2], i1[2]) + 0.5) * v).astype(np.float32)
        ab = (b - a).astype(np.float32)
        L2 = float(np.dot(ab, ab))
        ax, ay, az = (cx - np.float32(a[0]))[None, None, :], (cy - np.float32(a[1]))[None, :, None], (cz - np.float32(a[2]))[:, None, None]
        if L2 > 0:
            t = (ax * ab[0] + ay * ab[1] + az * ab[2]) / np.float32(L2)
            np.clip(t, 0.0, 1.0, out=t)
            d2 = (ax - t * ab[0]) ** 2 + (ay - t * ab[1]) ** 2 + (az - t * ab[2]) ** 2
        else:
            d2 = ax * ax + ay * ay + az * az
        known[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]] |= d2 <= r2
    return known


def make_map(seed, dims, v, n_boxes, side_lo, side_hi, n_waypoints, known_radius):
    rng_map = np.random.Generator(np.random.PCG64(seed + 0))
    rng_traj = np.random.Generator(np.random.PCG64(seed + 1))
    occ = _gt_boxes(rng_map, dims, v, n_boxes, side_lo, side_hi)
    traj = _trajectory(rng_traj, dims, v, occ, n_waypoints)
    known = _known_mask(dims, v, traj, known_radius)
    states = np.full(occ.shape, UNK, dtype=np.uint8)
    states[known & occ] = OCC
    states[known & ~occ] = FREE
    m = Map(states=states, voxel_m=float(v), origin_m=np.zeros(3, dtype=np.float32), seed=seed)
    return m, traj


# --------------------------------------------------------------------------- trees

def _random_free_root(rng, m: Map):
    fz, fy, fx = np.nonzero(m.states == FREE)
    k = int(rng.integers(0, fx.size))
    off = rng.uniform(0.05, 0.95, size=3)
    return (np.array([fx[k], fy[k], fz[k]], dtype=np.float64) + off) * m.voxel_m


def make_rrt(seed, m: Map, root_m, n_nodes, max_depth, step_m=1.5, max_attempts=10**6):
    """Nearest-parent RRT in known-free space (ids increase, parent < child)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = m.dims
    v = m.voxel_m
    ext = m.extent_m
    freeg = m.states == FREE
    pos = np.zeros((n_nodes, 3), dtype=np.float64)
    par = np.full(n_nodes, -1, dtype=np.int32)
    dep = np.zeros(n_nodes, dtype=np.int32)
    pos[0] = root_m
    n = 1
    attempts = 0
    while n < n_nodes:
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("RRT did not reach %d nodes" % n_nodes)
        x = rng.uniform(0.0, ext)
        ok = dep[:n] < max_depth
        d2 = np.sum((pos[:n] - x) ** 2, axis=1)
        d2 = np.where(ok, d2, np.inf)
        j = int(np.argmin(d2))
        if not np.isfinite(d2[j]):
            raise RuntimeError("no expandable node")
        dist = math.sqrt(d2[j])
        if dist > step_m:
            x = pos[j] + (x - pos[j]) * (step_m / dist)
        if dist < 1e-6:
            continue
        iv = _voxel_of(x, v, dims)
        if not _inside(iv, dims) or not freeg[iv[2], iv[1], iv[0]]:
            continue
        if not _segment_clear(pos[j], x, v, dims, freeg):
            continue
        pos[n] = x
        par[n] = j
        dep[n] = dep[j] + 1
        n += 1
    return Tree(pos_m=(pos + m.origin_m.astype(np.float64)).astype(np.float32), parent=par, seed=seed)


# --------------------------------------------------------------------------- workloads

SENSOR_TINY = dict(n_az=128, n_el=24, fov_h_deg=90.0, fov_v_deg=60.0, range_m=5.0, yaw_bins=36)
SENSOR_STEP = dict(n_az=360, n_el=60, fov_h_deg=90.0, fov_v_deg=60.0, range_m=8.0, yaw_bins=36)
SENSOR_LARGE = dict(n_az=720, n_el=120, fov_h_deg=90.0, fov_v_deg=60.0, range_m=15.0, yaw_bins=72)

WORKLOADS = {
    "tiny": "64x64x32 grid @0.2 m, 12 boxes, one 20-node RRT (depth<=4), 128x24 panorama, 5 m",
    "step": "200x200x60 grid @0.1 m, 40 boxes, one 500-node RRT (depth<=8), 360x60 panorama, 8 m",
    "batch64": "256x256x80 grid @0.1 m, 87 boxes, 64 RRTs of 50..2000 nodes (depth 3..12), 360x60 panorama, 8 m",
    "large": "512x512x128 grid @0.05 m, 150 boxes, 8 RRTs of 3000 nodes (depth<=15), 720x120 panorama, 15 m",
    "serve16": "16 robots with their own maps (128..512 x 128..512 x 64..128 @0.05..0.2 m), Poisson replans at 20 Hz",
}


def make(name: str, n_trees: Optional[int] = None) -> Workload:
    """Build one named workload. `n_trees` (multi-tree workloads) keeps only the first trees."""
    if name == "tiny":
        seed = 1000
        m, traj = make_map(seed, (64, 64, 32), 0.2, 12, 0.4, 2.0, 10, 4.0)
        t = make_rrt(seed + 100, m, traj[-1], 20, 4)
        return Workload(name, m, [t], Sensor(**SENSOR_TINY))
    if name == "step":
        seed = 2000
        m, traj = make_map(seed, (200, 200, 60), 0.1, 40, 0.3, 3.0, 30, 6.0)
        t = make_rrt(seed + 100, m, traj[-1], 500, 8)
        return Workload(name, m, [t], Sensor(**SENSOR_STEP))
    if name == "batch64":
        seed = 3000
        m, _ = make_map(seed, (256, 256, 80), 0.1, 87, 0.3, 3.0, 30, 6.0)
        trees = []
        count = 64 if n_trees is None else n_trees
        for t in range(count):
            rng = np.random.Generator(np.random.PCG64(seed + 100 + t))
            n = int(round(math.exp(rng.uniform(math.log(50), math.log(2000)))))
            depth = int(rng.integers(3, 13))
            root = _random_free_root(rng, m)
            trees.append(make_rrt(seed + 100 + t + 50000, m, root, n, depth))
        return Workload(name, m, trees, Sensor(**SENSOR_STEP))
    if name == "large":
        seed = 4000
        m, traj = make_map(seed, (512, 512, 128), 0.05, 150, 0.2, 4.0, 60, 8.0)
        count = 8 if n_trees is None else n_trees
        trees = [make_rrt(seed + 100 + t, m, traj[-1], 3000, 15) for t in range(count)]
        return Workload(name, m, trees, Sensor(**SENSOR_LARGE))
    raise KeyError(name)


def make_robot(r: int):
    """Robot r of the serving workload: its own map plus the sensor, seeded 5000+1000*(r+1)."""
    seed = 5000 + 1000 * (r + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    nxy = int(rng.choice(np.arange(128, 513, 32)))
    nz = int(rng.choice(np.arange(64, 129, 16)))
    v = float(rng.choice([0.05, 0.1, 0.2]))
    vol = nxy * nxy * nz * v ** 3
    boxes = int(np.clip(round(40 * vol / (20 * 20 * 6)), 12, 150))
    m, traj = make_map(seed, (nxy, nxy, nz), v, boxes, 0.3, 3.0, 30, 6.0)
    return m, traj


def serve_requests(n_requests=1200, n_robots=16, rate_hz=20.0):
    """Poisson arrivals (seed 5002): list of (arrival_s, robot, tree_seed, n_nodes, max_depth)."""
    rng = np.random.Generator(np.random.PCG64(5000 + 2))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        r = int(rng.integers(0, n_robots))
        n = int(round(math.exp(rng.uniform(math.log(100), math.log(3000)))))
        d = int(rng.integers(3, 13))
        out.append((t, r, 5000 + 100 + i, n, d))
    return out


def micro_map(dims, fill=UNK, boxes=(), v=1.0):
    """Hand-built map for unit tests: `boxes` is a list of (lo_idx, hi_idx_exclusive, state)."""
    nx, ny, nz = dims
    st = np.full((nz, ny, nx), fill, dtype=np.uint8)
    for lo, hi, s in boxes:
        st[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = s
    return Map(states=st, voxel_m=float(v), origin_m=np.zeros(3, dtype=np.float32))


def random_micro(seed, dims=(12, 10, 8), n_nodes=6, p_occ=0.08, p_free=0.4, max_depth=3,
                 n_az=16, n_el=6, fov_h=90.0, fov_v=60.0, range_vox=7.0, yaw_bins=8):
    """Tiny random map + tree + sensor for brute-force comparisons."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    u = rng.uniform(size=(nz, ny, nx))
    st = np.full((nz, ny, nx), UNK, dtype=np.uint8)
    st[u < p_free + p_occ] = FREE
    st[u < p_occ] = OCC
    m = Map(states=st, voxel_m=1.0, origin_m=np.zeros(3, dtype=np.float32))
    pos = np.zeros((n_nodes, 3), dtype=np.float32)
    par = np.full(n_nodes, -1, dtype=np.int32)
    dep = np.zeros(n_nodes, dtype=np.int32)
    for i in range(n_nodes):
        pos[i] = rng.uniform([0.5, 0.5, 0.5], [nx - 0.5, ny - 0.5, nz - 0.5])
        if i:
            cand = [j for j in range(i) if dep[j] < max_depth]
            par[i] = int(rng.choice(cand))
            dep[i] = dep[par[i]] + 1
    sen = Sensor(n_az=n_az, n_el=n_el, fov_h_deg=fov_h, fov_v_deg=fov_v, range_m=range_vox,
                 yaw_bins=yaw_bins)
    return m, Tree(pos_m=pos, parent=par), sen
