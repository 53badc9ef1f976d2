"""Pins of the interval-mode oracle (Sec. IV-A pinhole buffers, eq. 5-7 overlap intervals).

Each test checks a part of ``oracle/ivlref.c`` against something it does not
compute itself: the buffer sizes the resolution rule gives for the paper's
parameters, the pinhole geometry (pixel directions project back to pixel
centres through eq. 5), closed-form depths in front of a wall, a dense
double-precision point test of the overlap intervals (projection, clipping,
2D DDA, inverse depth and the map back to t), a node's counts recomposed
from those building blocks with an independent union, and the invariants of
Sec. III-B (the root and blind ancestors do not condition; marginal <=
absolute; a viewpoint repeated at the same yaw sees almost nothing new).
"""
import math

import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _ivl():
    from oracle import ivlref
    return ivlref


def _q(tree, m):
    return ((tree.pos_m - m.origin_m) / np.float32(m.voxel_m)).astype(np.float32)


# ----------------------------------------------------------------- camera (Sec. IV-A, eq. 5)

@pytest.mark.parametrize("sen,v,wh", [(W.SENSOR_TINY, 0.2, (50, 29)), (W.SENSOR_STEP, 0.1, (160, 93)),
                                      (W.SENSOR_LARGE, 0.05, (600, 347))])
def test_resolution_rule(sen, v, wh):
    """W_D = ceil(2 d_max tan(fov_h/2) / v), H_D likewise: one pixel spans one voxel at d_max."""
    s = W.Sensor(**sen)
    Wd, Hd, intr, _, _ = _ivl().camera_tables(s, v)
    assert (Wd, Hd) == wh
    assert Wd == math.ceil(2 * s.range_m * math.tan(math.radians(s.fov_h_deg / 2)) / v - 1e-6)
    assert intr[5] == np.float32(s.range_m) / np.float32(v)
    # explicit sizes override the rule
    assert _ivl().camera_tables(s, v, 32, 24)[:2] == (32, 24)


@pytest.mark.parametrize("wd,hd", [(0, 0), (37, 21)])
def test_pixel_directions_project_to_pixel_centres(wd, hd):
    s = W.Sensor(**W.SENSOR_TINY)
    Wd, Hd, intr, pdir, cs = _ivl().camera_tables(s, 0.2, wd, hd)
    fx, fy, cx, cy = (float(x) for x in intr[:4])
    p = pdir.astype(np.float64)
    assert np.allclose(np.linalg.norm(p, axis=2), 1.0, atol=1e-6) and np.all(p[..., 2] > 0)
    u = fx * p[..., 0] / p[..., 2] + cx
    v = fy * p[..., 1] / p[..., 2] + cy
    assert np.allclose(u, np.arange(Wd)[None, :] + 0.5, atol=2e-3)
    assert np.allclose(v, np.arange(Hd)[:, None] + 0.5, atol=2e-3)
    # the buffer spans the field of view: the left and right buffer edges are fov_h apart
    assert abs(2 * math.degrees(math.atan(cx / fx)) - s.fov_h_deg) < 1e-3
    assert abs(2 * math.degrees(math.atan(cy / fy)) - s.fov_v_deg) < 1e-3


def test_window_yaw_is_the_centre_of_its_columns():
    from oracle import mgref
    for sen in (W.SENSOR_TINY, W.SENSOR_STEP):
        s = W.Sensor(**sen)
        _, _, _, _, cs = _ivl().camera_tables(s, 0.2)
        t = mgref.sensor_tables(s)
        for k in range(s.yaw_bins):
            psi = math.degrees(math.atan2(cs[k, 1], cs[k, 0])) % 360
            cols = (t["c0"][k] + np.arange(s.w_buf)) % s.n_az
            az = (s.az_offset_deg + (cols + 0.5) * 360.0 / s.n_az) % 360
            mid = math.degrees(math.atan2(np.mean(np.sin(np.radians(az))), np.mean(np.cos(np.radians(az))))) % 360
            dev = min(abs(psi - mid), 360 - abs(psi - mid))
            assert dev <= 0.5 * 360.0 / s.n_az + 1e-6, (k, psi, mid)


def test_render_above_a_floor():
    """Occupied floor z < 6 below a camera facing +x: a ray pointing down that reaches the floor
    inside the grid and the range stores z = t * p_z with t = (q_z - 6) / (-d_z); a ray pointing
    up meets nothing and stores the range end."""
    st = np.full((30, 40, 60), W.FREE, np.uint8)
    st[:6, :, :] = W.OCC
    s = W.Sensor(n_az=8, n_el=4, fov_h_deg=90.0, fov_v_deg=60.0, range_m=40.0, yaw_bins=8,
                 az_offset_deg=-45.0)
    cam = _ivl().CameraHandle(s, 1.0, 20, 14)
    _, _, _, pdir, _ = _ivl().camera_tables(s, 1.0, 20, 14)
    q = np.array([5.5, 20.5, 9.5], np.float32)
    D = _ivl().render(st, cam, q, 0)
    p = pdir.astype(np.float64)
    dz = -p[..., 1]                               # world z of the direction: camera y points down
    down = dz < 0
    t_floor = np.where(down, (9.5 - 6.0) / np.where(down, -dz, 1.0), np.inf)
    x_hit = 5.5 + p[..., 2] * t_floor
    y_hit = 20.5 - p[..., 0] * t_floor           # camera x is world -y at yaw 0
    hit = down & (t_floor < 40.0) & (x_hit < 60) & (y_hit >= 0) & (y_hit < 40)
    assert hit.sum() > 50 and (~down).sum() > 50
    assert np.allclose(D[hit], t_floor[hit] * p[hit][:, 2], rtol=1e-5)
    # upward rays meet nothing; leaving the grid counts as reaching the range end
    up = dz > 0
    assert np.allclose(D[up], 40.0 * p[up][:, 2], rtol=1e-6)


def test_merge_is_the_union():
    rng = np.random.Generator(np.random.PCG64(77))
    grid = np.linspace(0, 100, 20001)
    for _ in range(300):
        lists = []
        for _ in range(2):
            k = int(rng.integers(0, 6))
            ends = np.sort(rng.choice(np.arange(0, 100, 0.5), size=2 * k, replace=False)).astype(np.float32)
            lists.append(ends.reshape(-1, 2))
        M = _ivl().merge(lists[0], lists[1])
        assert np.all(M[:, 0] <= M[:, 1]) and np.all(M[1:, 0] > M[:-1, 1])
        want = np.zeros(grid.size, bool)
        for L in lists:
            for lo, hi in L:
                want |= (grid >= lo) & (grid <= hi)
        got = np.zeros(grid.size, bool)
        for lo, hi in M:
            got |= (grid >= lo) & (grid <= hi)
        assert np.array_equal(got, want)
    # nested and touching intervals
    assert np.array_equal(_ivl().merge([[0, 9]], [[0, 5], [9, 12]]), np.array([[0, 12]], np.float32))
    assert np.array_equal(_ivl().merge([[2, 3]], [[0, 9]]), np.array([[0, 9]], np.float32))


def test_render_in_front_of_a_wall():
    """All-free map, occupied half-space x >= X, camera facing +x: every pixel whose ray reaches
    the wall stores z = X - q_x; the others store the range end, Rv * p_z."""
    X = 20
    st = np.full((40, 40, 40), W.FREE, np.uint8)
    st[:, :, X:] = W.OCC
    s = W.Sensor(n_az=8, n_el=4, fov_h_deg=90.0, fov_v_deg=60.0, range_m=30.0, yaw_bins=8,
                 az_offset_deg=-45.0)           # window 0 spans [-45, 45] degrees: yaw 0 (+x)
    cam = _ivl().CameraHandle(s, 1.0, 24, 16)
    _, _, intr, pdir, cs = _ivl().camera_tables(s, 1.0, 24, 16)
    assert cs[0, 0] == 1.0 and cs[0, 1] == 0.0
    q = np.array([12.5, 20.25, 19.75], np.float32)
    D = _ivl().render(st, cam, q, 0)
    p = pdir.astype(np.float64)
    t_wall = (X - 12.5) / p[..., 2]
    y_hit = 20.25 - p[..., 0] * t_wall           # camera x is world -y at yaw 0
    z_hit = 19.75 - p[..., 1] * t_wall           # camera y is world -z
    reach = (t_wall < 30.0) & (y_hit >= 0) & (y_hit < 40) & (z_hit >= 0) & (z_hit < 40)
    assert reach.sum() > 100
    assert np.allclose(D[reach], X - 12.5, rtol=1e-5)
    assert np.allclose(D[~reach], 30.0 * p[~reach][:, 2], rtol=1e-5)


# ----------------------------------------------------------------- intervals (eq. 5-7)

def _frame(c, s, p):
    return np.stack([s * p[..., 0] - c * p[..., 1], -p[..., 2], c * p[..., 0] + s * p[..., 1]], axis=-1)


@pytest.mark.parametrize("seed", range(6))
def test_intervals_match_a_dense_point_test(seed):
    """A point r(t) of the candidate ray lies in an overlap interval iff, computed independently in
    double: znear <= z <= Rv, its projection (eq. 5) falls in the buffer, and z <= D at that pixel.
    Points within a small margin of a pixel edge, of the stored depth or of an interval end are
    skipped (float rounding decides those)."""
    rng = np.random.Generator(np.random.PCG64(900 + seed))
    s = W.Sensor(n_az=16, n_el=4, fov_h_deg=90.0, fov_v_deg=60.0, range_m=12.0, yaw_bins=8)
    wd, hd = int(rng.integers(8, 40)), int(rng.integers(6, 30))
    cam = _ivl().CameraHandle(s, 1.0, wd, hd)
    _, _, intr, _, cs = _ivl().camera_tables(s, 1.0, wd, hd)
    fx, fy, cx, cy, zn, rv = (float(x) for x in intr)
    checked = 0
    for trial in range(40):
        ka = int(rng.integers(0, 8))
        qa = rng.uniform(5, 15, 3).astype(np.float32)
        qn = (qa + rng.normal(0, 3, 3)).astype(np.float32)
        d = rng.normal(0, 1, 3)
        d = (d / np.linalg.norm(d)).astype(np.float32)
        Da = rng.choice([0.0, 2.0, 5.0, 9.0, 30.0], size=(hd, wd)).astype(np.float32)
        Da *= rng.uniform(0.5, 1.5, (hd, wd)).astype(np.float32)
        iv, _ = _ivl().intervals(cam, qn, d, qa, ka, Da)
        if len(iv):
            assert np.all(iv[:, 0] <= iv[:, 1]) and np.all(iv[1:, 0] > iv[:-1, 1])
            assert iv[0, 0] >= 0 and iv[-1, 1] <= rv * (1 + 1e-6)
        c, sn = float(cs[ka, 0]), float(cs[ka, 1])
        t = np.linspace(0, rv, 3001)[1:-1]
        P = _frame(c, sn, (qn.astype(np.float64) - qa)[None, :] + t[:, None] * d.astype(np.float64)[None, :])
        z = P[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = fx * P[:, 0] / z + cx
            v = fy * P[:, 1] / z + cy
        ok = (z >= zn) & (z <= rv) & (u >= 0) & (u < wd) & (v >= 0) & (v < hd)
        iu = np.clip(np.floor(np.nan_to_num(u)), 0, wd - 1).astype(int)
        ivv = np.clip(np.floor(np.nan_to_num(v)), 0, hd - 1).astype(int)
        Dp = Da[ivv, iu].astype(np.float64)
        inside = ok & (z <= Dp)
        member = np.zeros(t.size, bool)
        near_end = np.zeros(t.size, bool)
        for lo, hi in iv.astype(np.float64):
            member |= (t >= lo) & (t <= hi)
            near_end |= (np.abs(t - lo) < 1e-3 * (1 + lo)) | (np.abs(t - hi) < 1e-3 * (1 + hi))
        with np.errstate(invalid="ignore"):
            edge = ((np.abs(u - np.round(u)) < 1e-3) | (np.abs(v - np.round(v)) < 1e-3) |
                    (np.abs(z - Dp) < 1e-4 * (1 + Dp)) | (np.abs(z - zn) < 1e-4) | (np.abs(z - rv) < 1e-3))
        sel = ~(near_end | edge)
        assert np.array_equal(member[sel], inside[sel]), (seed, trial, np.flatnonzero(member[sel] != inside[sel])[:5])
        checked += int(sel.sum())
    assert checked > 50000


def test_intervals_of_a_blind_or_distant_ancestor():
    s = W.Sensor(n_az=16, n_el=4, fov_h_deg=90.0, fov_v_deg=60.0, range_m=12.0, yaw_bins=8)
    cam = _ivl().CameraHandle(s, 1.0, 20, 12)
    qa = np.array([10, 10, 10], np.float32)
    d = np.array([1, 0, 0], np.float32)
    assert len(_ivl().intervals(cam, qa + 1, d, qa, 0, np.zeros((12, 20), np.float32))[0]) == 0
    # a candidate ray entirely behind the ancestor's camera (window 0 looks along +x... or wherever):
    _, _, _, _, cs = _ivl().camera_tables(s, 1.0, 20, 12)
    back = -np.array([cs[3, 0], cs[3, 1], 0], np.float32)
    iv, steps = _ivl().intervals(cam, qa - 3 * np.array([cs[3, 0], cs[3, 1], 0], np.float32), back, qa, 3,
                                 np.full((12, 20), 1e6, np.float32))
    assert len(iv) == 0 and steps == 0


# ----------------------------------------------------------------- composition (Sec. IV-B)

def _node_counts_from_blocks(m, tree, s, o, nd):
    """m_n recomputed for one node from the pinned blocks: intervals of every ancestor (any
    order, union by a plain membership test), the 3D DDA with exit parameters, chord midpoints."""
    from oracle import mgref
    ivl = _ivl()
    t = mgref.sensor_tables(s)
    cam = ivl.CameraHandle(s, m.voxel_m, int(o["wd"]), int(o["hd"]))
    rv = np.float32(s.range_m) / np.float32(m.voxel_m)
    q = _q(tree, m)
    anc = []
    a = int(tree.parent[nd])
    while a >= 0:
        anc.append(a)
        a = int(tree.parent[a])
    ab = np.zeros(s.yaw_bins, np.int64)
    mb = np.zeros(s.yaw_bins, np.int64)
    for r in range(s.n_az * s.n_el):
        c = r // s.n_el
        b = int(t["bins"][c])
        lists = [ivl.intervals(cam, q[nd], t["dir"][r], q[a], int(o["k_db"][a]), o["D"][a])[0] for a in reversed(anc)]
        _, st, te, tx, _ = ivl.trace_ray_exit(m.states, q[nd], t["dir"][r], t["inv"][r], rv)
        for sv, a_, b_ in zip(st, te, tx):
            if sv != W.UNK:
                continue
            ab[b] += 1
            tm = np.float32(0.5) * (np.float32(a_) + np.float32(min(b_, rv)))
            if not any(((L[:, 0] <= tm) & (tm <= L[:, 1])).any() for L in lists if len(L)):
                mb[b] += 1
    return ab, mb


def _window_max(bins, w):
    B = len(bins)
    sums = [sum(bins[(k + i) % B] for i in range(w)) for k in range(B)]
    return max(sums), int(np.argmax(sums))


@pytest.fixture(scope="module")
def micro_eval():
    m, tree, s = W.random_micro(41, dims=(16, 14, 9), n_nodes=10, max_depth=4, range_vox=8.0, p_occ=0.07,
                                p_free=0.45, n_az=24, n_el=5, yaw_bins=12)
    o = _ivl().eval_tree(m, tree, s, wd=20, hd=9, want_bins=True)
    return m, tree, s, o


def test_node_counts_recomposed_from_the_blocks(micro_eval):
    m, tree, s, o = micro_eval
    dep = tree.depth()
    for nd in [int(i) for i in np.flatnonzero(dep >= 1)][:5]:
        ab, mb = _node_counts_from_blocks(m, tree, s, o, nd)
        assert np.array_equal(ab, o["abs_bins"][nd]) and np.array_equal(mb, o["marg_bins"][nd]), nd
        g, k = _window_max(mb, s.window_bins)
        ga, ka = _window_max(ab, s.window_bins)
        assert (g, k) == (o["g_db"][nd], o["k_db"][nd]), nd
        assert (ga, ka) == (o["g_abs"][nd], o["k_abs"][nd]), nd
    # the stored buffer is the render at the chosen window
    cam = _ivl().CameraHandle(s, m.voxel_m, 20, 9)
    q = _q(tree, m)
    for nd in range(tree.n):
        assert np.array_equal(o["D"][nd], _ivl().render(m.states, cam, q[nd], int(o["k_db"][nd])))


def test_root_bound_and_threads(micro_eval):
    m, tree, s, o = micro_eval
    assert o["g_db"][0] == o["g_abs"][0] and o["k_db"][0] == o["k_abs"][0]
    assert np.all(o["g_db"] <= o["g_abs"])
    o8 = _ivl().eval_tree(m, tree, s, wd=20, hd=9, n_threads=8)
    for key in ("g_db", "k_db", "g_abs", "k_abs", "D"):
        assert np.array_equal(o8[key], o[key])


def test_blind_ancestor_does_not_condition():
    """A root inside an occupied voxel stores depth 0 everywhere: its child's marginal gain is its
    absolute gain."""
    st = np.full((12, 16, 16), W.UNK, np.uint8)
    st[6, 8, 8] = W.OCC
    m = W.Map(states=st, voxel_m=1.0, origin_m=np.zeros(3, np.float32))
    tree = W.Tree(pos_m=np.array([[8.5, 8.5, 6.5], [10.2, 7.1, 6.3]], np.float32), parent=np.array([-1, 0], np.int32))
    s = W.Sensor(n_az=24, n_el=5, fov_h_deg=90.0, fov_v_deg=60.0, range_m=6.0, yaw_bins=12)
    o = _ivl().eval_tree(m, tree, s, wd=16, hd=8)
    assert np.all(o["D"][0] == 0)
    assert o["g_db"][1] == o["g_abs"][1] and o["k_db"][1] == o["k_abs"][1]


def test_repeated_viewpoint_sees_little_inside_the_parents_frustum():
    """Child at its parent's position in an all-unknown map: the parent's buffer holds the range end,
    so within the parent's window almost every incidence is covered, and the child's best window is
    at least the best window that avoids the parent's bins."""
    st = np.full((24, 40, 40), W.UNK, np.uint8)
    m = W.Map(states=st, voxel_m=1.0, origin_m=np.zeros(3, np.float32))
    p = np.array([20.5, 20.5, 12.5], np.float32)
    tree = W.Tree(pos_m=np.stack([p, p]), parent=np.array([-1, 0], np.int32))
    s = W.Sensor(n_az=48, n_el=6, fov_h_deg=90.0, fov_v_deg=60.0, range_m=10.0, yaw_bins=12)
    o = _ivl().eval_tree(m, tree, s, want_bins=True)
    from oracle import mgref
    t = mgref.sensor_tables(s)
    w = s.window_bins
    kp = int(o["k_db"][0])
    cam = _ivl().CameraHandle(s, 1.0, int(o["wd"]), int(o["hd"]))
    ab, mb = _node_counts_from_blocks(m, tree, s, o, 1)
    assert np.array_equal(mb, o["marg_bins"][1]) and np.array_equal(ab, o["abs_bins"][1])
    inside = [(kp + i) % s.yaw_bins for i in range(w)]
    assert mb[inside].sum() <= 0.1 * ab[inside].sum()
    outside = [k for k in range(s.yaw_bins) if k not in inside]
    assert np.array_equal(mb[outside], ab[outside])          # rays outside the frustum are never covered
    disjoint = max(sum(ab[(k + i) % s.yaw_bins] for i in range(w)) for k in range(s.yaw_bins)
                   if not set((k + i) % s.yaw_bins for i in range(w)) & set(inside))
    assert o["g_db"][1] >= disjoint
