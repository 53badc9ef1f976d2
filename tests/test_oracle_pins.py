"""Pins of the oracle against what the paper and plain geometry fix.

Each test checks one part of the oracle against something other than itself:
the double-precision slab test over every voxel (ray traversal), closed-form
counts for axis-aligned rays in an unknown map (eq. 1), atan2 angles (pixel
cells of the ancestor test), brute-force window sums (yaw selection), and the
invariants the paper states (Sec. III-B: the root has no conditioning and
marginal <= absolute; eq. 2: exact marginal gains telescope to the size of the
union along a path).
"""
import math

import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from tests import brute

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _mg():
    from oracle import mgref
    return mgref


# ----------------------------------------------------------------- sensor tables

@pytest.mark.parametrize("sen", [W.SENSOR_TINY, W.SENSOR_STEP, W.SENSOR_LARGE])
def test_sensor_tables_geometry(sen):
    s = W.Sensor(**sen)
    t = _mg().sensor_tables(s)
    Wp, H, B = s.n_az, s.n_el, s.yaw_bins
    d = t["dir"].astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    c = np.repeat(np.arange(Wp), H)
    j = np.tile(np.arange(H), Wp)
    az = np.degrees(np.arctan2(d[:, 1], d[:, 0])) % 360.0
    el = np.degrees(np.arcsin(np.clip(d[:, 2], -1, 1)))
    az_ref = (s.az_offset_deg + (c + 0.5) * 360.0 / Wp) % 360.0
    el_ref = -s.fov_v_deg / 2 + (j + 0.5) * s.fov_v_deg / H
    assert np.allclose(np.minimum(abs(az - az_ref), 360 - abs(az - az_ref)), 0, atol=1e-4)
    assert np.allclose(el, el_ref, atol=1e-4)
    nz = d != 0
    assert np.allclose(t["inv"][nz] * t["dir"][nz], 1.0, rtol=1e-6)
    # bins: each column's centre lies in its bin
    lo = t["bins"] * 360.0 / B
    ctr = (np.arange(Wp) + 0.5) * 360.0 / Wp
    assert np.all(ctr >= lo) and np.all(ctr < lo + 360.0 / B)
    # windows: exactly w_buf columns, starting at c0, whose bins are k..k+w-1 (mod B)
    w = s.window_bins
    for k in range(B):
        members = [cc for cc in range(Wp) if (t["bins"][cc] - k) % B < w]
        assert len(members) == s.w_buf
        start = t["c0"][k]
        assert sorted(members) == sorted(((start + i) % Wp) for i in range(s.w_buf))
    # azimuth boundaries and elevation boundary values
    beta = np.radians(s.az_offset_deg + np.arange(Wp) * 360.0 / Wp)
    assert np.allclose(t["bv"][:, 0], np.cos(beta), atol=1e-7)
    assert np.allclose(t["bv"][:, 1], np.sin(beta), atol=1e-7)
    e = np.radians(-s.fov_v_deg / 2 + np.arange(H + 1) * s.fov_v_deg / H)
    assert np.allclose(t["ts"], np.tan(e) * np.abs(np.tan(e)), atol=1e-6)
    assert np.all(np.diff(t["ts"]) > 0)


def test_sensor_rejects_unrepresentable():
    with pytest.raises(ValueError):
        _mg().sensor_tables(W.Sensor(n_az=50, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=5, yaw_bins=36))
    with pytest.raises(ValueError):
        _mg().sensor_tables(W.Sensor(n_az=128, n_el=4, fov_h_deg=200, fov_v_deg=60, range_m=5, yaw_bins=36))


# ----------------------------------------------------------------- DDA traversal

def _random_rays(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    dirs = [v.astype(np.float32)]
    # axis-aligned and diagonal directions exercise the tie rule and zero components
    special = np.array([[1, 0, 0], [0, -1, 0], [0, 0, 1], [1, 1, 0], [-1, 1, 1], [1, -1, -1], [0, 1, 1]],
                       dtype=np.float64)
    special /= np.linalg.norm(special, axis=1, keepdims=True)
    dirs.append(special.astype(np.float32))
    d = np.concatenate(dirs)
    inv = np.where(d != 0, np.float32(1.0) / np.where(d != 0, d, 1).astype(np.float32), 0).astype(np.float32)
    return d, inv


@pytest.mark.parametrize("seed", range(6))
def test_dda_matches_slab_bruteforce(seed):
    """Visit set, order, entry t and first hit vs the fp64 slab test over every voxel."""
    mg = _mg()
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = (13, 11, 9)
    st = rng.choice([W.UNK, W.FREE, W.OCC], p=[0.45, 0.5, 0.05], size=dims[::-1]).astype(np.uint8)
    d, inv = _random_rays(rng, 60)
    checked = 0
    for r in range(d.shape[0]):
        q = rng.uniform([0, 0, 0], dims).astype(np.float32)
        if r % 7 == 0:
            q = np.floor(q).astype(np.float32) + np.float32(0.5)     # voxel centre: ties on diagonals
        rv = float(np.float32(rng.uniform(2.0, 12.0)))
        ids, sts, te, h = mg.trace_ray(st, q, d[r], inv[r], rv)
        must, may, h_ref, h_amb, aux = brute.ray_reference(st, q, d[r], rv)
        got = set(ids.tolist())
        assert must <= got, (seed, r, sorted(must - got))
        assert got <= may, (seed, r, sorted(got - may))
        assert len(got) == len(ids), "a voxel was visited twice"
        assert np.all(np.diff(te) >= 0), "entry parameters must not decrease"
        ent = aux["entry"].reshape(-1)[ids.astype(np.int64)]
        assert np.allclose(te, ent, atol=1e-4, rtol=1e-5)
        flat = st.reshape(-1)
        assert np.array_equal(sts, flat[ids.astype(np.int64)])
        assert not np.any(sts[:-1] == W.OCC), "traversal must stop at the first occupied voxel"
        if not h_amb:
            assert math.isclose(h, h_ref, rel_tol=1e-5, abs_tol=1e-4), (seed, r, h, h_ref)
            checked += 1
    assert checked > 40


def test_dda_start_voxel_and_exit():
    mg = _mg()
    st = np.full((4, 4, 4), W.OCC, np.uint8)
    q = np.array([1.3, 2.2, 0.7], np.float32)
    d = np.array([1, 0, 0], np.float32)
    ids, sts, te, h = mg.trace_ray(st, q, d, d, 10.0)
    assert list(ids) == [1 + 4 * (2 + 4 * 0)] and h == 0.0     # occupied start voxel: depth 0
    st[:] = W.FREE
    ids, sts, te, h = mg.trace_ray(st, q, d, d, 10.0)
    assert len(ids) == 3 and h == np.float32(10.0)                # leaves the grid: depth = range


# ----------------------------------------------------------------- closed forms

@pytest.mark.parametrize("ijk,rv,dims", [((3, 4, 2), 5, (10, 9, 5)), ((0, 8, 4), 3, (9, 9, 9)),
                                         ((6, 1, 1), 20, (7, 12, 3))])
def test_axis_rays_closed_form(ijk, rv, dims):
    """Unknown map, node at a voxel centre, four axis rays: count = voxels up to range or wall."""
    mg = _mg()
    i, j, k = ijk
    nx, ny, nz = dims
    m = W.micro_map(dims, fill=W.UNK)
    sen = W.Sensor(n_az=4, n_el=1, fov_h_deg=90, fov_v_deg=60, range_m=float(rv), yaw_bins=4,
                   az_offset_deg=-45.0)
    tree = W.Tree(pos_m=np.array([[i + 0.5, j + 0.5, k + 0.5]], np.float32), parent=np.array([-1], np.int32))
    o = mg.eval_tree(m, tree, sen, want_bins=True)
    px = min(i + rv, nx - 1) - i + 1
    mx = min(rv, i) + 1
    py = min(j + rv, ny - 1) - j + 1
    my = min(rv, j) + 1
    ref = [px, py, mx, my]                       # columns at 0, 90, 180, 270 degrees
    assert o["abs_bins"][0].tolist() == ref
    assert int(o["g_abs"][0]) == max(ref) and int(o["k_abs"][0]) == ref.index(max(ref))
    assert int(o["g_db"][0]) == max(ref)
    s = mg.node_set(m.states, sen, rv, tree.pos_m[0], int(o["k_db"][0]))
    assert s.size == max(ref)
    # union over the four windows: the start voxel is shared by all four rays
    allv = set()
    for kk in range(4):
        allv |= set(mg.node_set(m.states, sen, rv, tree.pos_m[0], kk).tolist())
    assert len(allv) == sum(ref) - 3


def test_first_hit_half_space_closed_form():
    """Free map with an occupied half-space x >= X: depth = (X - q_x)/d_x before the range."""
    mg = _mg()
    X = 9
    m = W.micro_map((14, 40, 40), fill=W.FREE, boxes=[((X, 0, 0), (14, 40, 40), W.OCC)])
    sen = W.Sensor(n_az=36, n_el=10, fov_h_deg=90, fov_v_deg=60, range_m=7.0, yaw_bins=12)
    t = mg.sensor_tables(sen)
    q = np.array([3.3, 20.4, 19.7], np.float32)
    rv = 7.0
    n = 0
    for r in range(t["dir"].shape[0]):
        d = t["dir"][r].astype(np.float64)
        ids, sts, te, h = mg.trace_ray(m.states, q, t["dir"][r], t["inv"][r], rv)
        if d[0] <= 0:
            assert h == np.float32(rv)
            continue
        tx = (X - float(q[0])) / d[0]
        if abs(tx - rv) < 1e-3:
            continue
        if tx < rv:
            assert math.isclose(h, tx, rel_tol=1e-5), (r, h, tx)
            n += 1
        else:
            assert h == np.float32(rv)
    assert n > 20


# ----------------------------------------------------------------- windows

def test_best_window_bruteforce_and_ties():
    mg = _mg()
    rng = np.random.Generator(np.random.PCG64(7))
    for trial in range(300):
        B = int(rng.integers(3, 80))
        w = int(rng.integers(1, (B + 1) // 2))
        bins = rng.integers(0, 4, size=B).astype(np.uint32)   # small values: many ties
        g, k = mg.best_window(bins, w)
        assert (g, k) == brute.best_window(bins, w)
    assert mg.best_window(np.zeros(36, np.uint32), 9) == (0, 0)


def test_symmetric_four_way_tie_picks_smallest_window():
    mg = _mg()
    n = 9
    m = W.micro_map((n, n, n), fill=W.UNK)
    sen = W.Sensor(n_az=4, n_el=1, fov_h_deg=90, fov_v_deg=60, range_m=3.0, yaw_bins=4, az_offset_deg=-45.0)
    tree = W.Tree(pos_m=np.array([[4.5, 4.5, 4.5]], np.float32), parent=np.array([-1], np.int32))
    o = mg.eval_tree(m, tree, sen, want_bins=True)
    assert o["abs_bins"][0].tolist() == [4, 4, 4, 4]
    assert int(o["k_abs"][0]) == 0 and int(o["k_db"][0]) == 0


# ----------------------------------------------------------------- ancestor test

@pytest.mark.parametrize("sen", [W.SENSOR_TINY, W.SENSOR_STEP, W.SENSOR_LARGE])
def test_obs_matches_atan2_cells(sen):
    mg = _mg()
    s = W.Sensor(**sen)
    h = mg.SensorHandle(s)
    rng = np.random.Generator(np.random.PCG64(11))
    WB, H = s.w_buf, s.n_el
    compared = inside = obs_true = 0
    for trial in range(4000):
        qa = rng.uniform(0, 40, size=3).astype(np.float32)
        c0 = int(rng.integers(0, s.n_az))
        Da = rng.uniform(0.0, 30.0, size=(H, WB)).astype(np.float32)
        ix, iy, iz = (int(x) for x in rng.integers(0, 40, size=3))
        got, row, col = h.obs(qa, c0, Da, ix, iy, iz)
        inn, rrow, rcol, amb = brute.pixel_of(s, qa, c0, ix, iy, iz)
        ref, amb2 = brute.observed(s, qa, c0, Da, ix, iy, iz)
        if amb or amb2:
            continue
        compared += 1
        assert got == ref, (trial, got, ref)
        if inn:
            inside += 1
            assert (row, col) == (rrow, rcol), (trial, row, col, rrow, rcol)
        obs_true += got
    assert compared > 3900 and inside > 100 and obs_true > 20


def test_obs_zero_depth_never_observes():
    mg = _mg()
    s = W.Sensor(**W.SENSOR_TINY)
    h = mg.SensorHandle(s)
    rng = np.random.Generator(np.random.PCG64(3))
    Da = np.zeros((s.n_el, s.w_buf), np.float32)
    for _ in range(500):
        qa = rng.uniform(0, 20, size=3).astype(np.float32)
        x = rng.integers(0, 20, size=3)
        assert not h.obs(qa, int(rng.integers(0, s.n_az)), Da, *x)[0]


# ----------------------------------------------------------------- composition

def _brute_tree(m, tree, sen, mg):
    """Depth-ordered marginal gain from fp64 ray sets and fp64 pixel cells."""
    t = mg.sensor_tables(sen)
    st = m.states
    n = tree.n
    H, Wp, B, wb = sen.n_el, sen.n_az, sen.yaw_bins, sen.w_buf
    rv = float(np.float32(np.float32(sen.range_m) / np.float32(m.voxel_m)))
    q = ((tree.pos_m - m.origin_m) / np.float32(m.voxel_m)).astype(np.float32)
    dep = tree.depth()
    res = dict(g_db=np.zeros(n, np.int64), k_db=np.zeros(n, np.int64), g_abs=np.zeros(n, np.int64),
               k_abs=np.zeros(n, np.int64), D=np.zeros((n, H, wb)), amb=np.zeros(n, bool))
    nz_, ny_, nx_ = st.shape
    for d in range(int(dep.max()) + 1):
        for nd in np.flatnonzero(dep == d):
            anc = []
            a = int(tree.parent[nd])
            while a >= 0:
                anc.append(a)
                a = int(tree.parent[a])
            amb = any(res["amb"][a] for a in anc)
            ab = np.zeros(B, np.int64)
            mb = np.zeros(B, np.int64)
            h = np.zeros((Wp, H))
            for c in range(Wp):
                for j in range(H):
                    r = c * H + j
                    must, may, href, hamb, aux = brute.ray_reference(st, q[nd], t["dir"][r], rv)
                    flat = st.reshape(-1)
                    if {v for v in must if flat[v] == W.UNK} != {v for v in may if flat[v] == W.UNK} or hamb:
                        amb = True
                    h[c, j] = href
                    ent = aux["entry"].reshape(-1)
                    for vid in sorted(must, key=lambda x: ent[x]):
                        ix, iy, iz = vid % nx_, (vid // nx_) % ny_, vid // (nx_ * ny_)
                        if st[iz, iy, ix] != W.UNK:
                            continue
                        ab[t["bins"][c]] += 1
                        seen = False
                        for a in anc:
                            o, oamb = brute.observed(sen, q[a], t["c0"][res["k_db"][a]], res["D"][a], ix, iy, iz)
                            amb |= oamb
                            if o:
                                seen = True
                                break
                        if not seen:
                            mb[t["bins"][c]] += 1
            res["g_abs"][nd], res["k_abs"][nd] = brute.best_window(ab, sen.window_bins)
            res["g_db"][nd], res["k_db"][nd] = brute.best_window(mb, sen.window_bins)
            c0 = t["c0"][res["k_db"][nd]]
            for i in range(wb):
                res["D"][nd][:, i] = h[(c0 + i) % Wp]
            res["amb"][nd] = amb
    return res


@pytest.mark.parametrize("seed", range(4))
def test_tree_composition_bruteforce(seed):
    """Bins, windows, buffers and depth order recomputed from fp64 references."""
    mg = _mg()
    m, tree, sen = W.random_micro(100 + seed, dims=(10, 9, 7), n_nodes=5, n_az=16, n_el=4,
                                  range_vox=6.0, yaw_bins=8)
    o = mg.eval_tree(m, tree, sen)
    b = _brute_tree(m, tree, sen, mg)
    compared = 0
    for nd in range(tree.n):
        if b["amb"][nd]:
            continue
        compared += 1
        assert int(o["g_abs"][nd]) == b["g_abs"][nd]
        assert int(o["k_abs"][nd]) == b["k_abs"][nd]
        assert int(o["g_db"][nd]) == b["g_db"][nd], (seed, nd)
        assert int(o["k_db"][nd]) == b["k_db"][nd]
        assert np.allclose(o["D"][nd], b["D"][nd], rtol=1e-5, atol=1e-4)
    assert compared >= 2


# ----------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def tiny_eval():
    mg = _mg()
    w = W.make("tiny")
    o = mg.eval_tree(w.map, w.trees[0], w.sensor, want_bins=True)
    e = mg.exact(w.map, w.trees[0], w.sensor, o["k_db"], o["D"])
    return w, o, e


def test_root_and_bound_invariants(tiny_eval):
    w, o, e = tiny_eval
    assert o["g_db"][0] == o["g_abs"][0] and o["k_db"][0] == o["k_abs"][0]     # A(root) is empty
    assert np.all(o["g_db"] <= o["g_abs"])                                       # Sec. III-B
    assert np.all(o["marg_bins"] <= o["abs_bins"])
    assert np.all(e["X_set"] <= e["A_set"]) and np.all(e["G_db_set"] <= e["A_set"])
    assert e["X_set"][0] == e["A_set"][0] and e["X_ray"][0] == o["g_db"][0]


def test_exact_union_telescopes(tiny_eval):
    """Eq. (2): summing exact marginal gains along root->n gives the size of the union."""
    mg = _mg()
    w, o, e = tiny_eval
    tree = w.trees[0]
    rv = np.float32(w.sensor.range_m) / np.float32(w.map.voxel_m)
    q = ((tree.pos_m - w.map.origin_m) / np.float32(w.map.voxel_m)).astype(np.float32)
    sets = [set(mg.node_set(w.map.states, w.sensor, rv, q[i], int(o["k_db"][i])).tolist())
            for i in range(tree.n)]
    for nd in range(tree.n):
        path = []
        a = nd
        while a >= 0:
            path.append(a)
            a = int(tree.parent[a])
        union = set().union(*[sets[p] for p in path])
        assert sum(int(e["X_set"][p]) for p in path) == len(union)
        anc_union = set().union(*[sets[p] for p in path[1:]]) if len(path) > 1 else set()
        assert int(e["X_set"][nd]) == len(sets[nd] - anc_union)
        assert int(e["A_set"][nd]) == len(sets[nd])


def test_node_set_matches_bruteforce_rays():
    mg = _mg()
    m, tree, sen = W.random_micro(5, dims=(9, 8, 6), n_nodes=1, n_az=16, n_el=4, range_vox=5.0, yaw_bins=8)
    t = mg.sensor_tables(sen)
    q = tree.pos_m[0]
    for k in range(sen.yaw_bins):
        got = set(mg.node_set(m.states, sen, 5.0, q, k).tolist())
        must, may = set(), set()
        c0 = t["c0"][k]
        for i in range(sen.w_buf):
            c = (c0 + i) % sen.n_az
            for j in range(sen.n_el):
                mu, ma, _, _, _ = brute.ray_reference(m.states, q, t["dir"][c * sen.n_el + j], 5.0)
                flat = m.states.reshape(-1)
                must |= {v for v in mu if flat[v] == W.UNK}
                may |= {v for v in ma if flat[v] == W.UNK}
        assert must <= got <= may


def test_fewer_ancestors_never_lower_counts(tiny_eval):
    """With the ancestors' buffers fixed, conditioning on a subset keeps every bin >= (g_sp case)."""
    mg = _mg()
    w, o, _ = tiny_eval
    tree = w.trees[0]
    t = mg.sensor_tables(w.sensor)
    rv = np.float32(w.sensor.range_m) / np.float32(w.map.voxel_m)
    q = ((tree.pos_m - w.map.origin_m) / np.float32(w.map.voxel_m)).astype(np.float32)
    for nd in [i for i in range(tree.n) if tree.depth()[i] >= 2][:4]:
        anc = []
        a = int(tree.parent[nd])
        while a >= 0:
            anc.append(a)
            a = int(tree.parent[a])
        c0s = [int(t["c0"][o["k_db"][a]]) for a in anc]
        full = mg.eval_node(w.map.states, w.sensor, rv, q[nd], q[anc], c0s, o["D"][anc])
        assert np.array_equal(full[1], o["marg_bins"][nd])
        parent_only = mg.eval_node(w.map.states, w.sensor, rv, q[nd], q[anc[:1]], c0s[:1], o["D"][anc[:1]])
        none = mg.eval_node(w.map.states, w.sensor, rv, q[nd], q[:0], [], o["D"][:0])
        blind = mg.eval_node(w.map.states, w.sensor, rv, q[nd], q[anc], c0s, np.zeros_like(o["D"][anc]))
        assert np.all(parent_only[1] >= full[1])
        assert np.array_equal(none[1], full[0]) and np.array_equal(blind[1], full[0])


def test_relabel_and_threads_invariance(tiny_eval):
    mg = _mg()
    w, o, _ = tiny_eval
    tree = w.trees[0]
    dep = tree.depth()
    rng = np.random.Generator(np.random.PCG64(9))
    order = np.lexsort((rng.permutation(tree.n), dep))          # new id -> old id, sorted by depth
    new_of_old = np.empty(tree.n, np.int64)
    new_of_old[order] = np.arange(tree.n)
    par = np.array([-1 if tree.parent[old] < 0 else new_of_old[tree.parent[old]] for old in order], np.int32)
    t2 = W.Tree(pos_m=tree.pos_m[order], parent=par)
    o2 = mg.eval_tree(w.map, t2, w.sensor, n_threads=3)
    assert np.array_equal(o2["g_db"], o["g_db"][order])
    assert np.array_equal(o2["k_db"], o["k_db"][order])
    assert np.array_equal(o2["D"], o["D"][order])


def test_absolute_mode_equals_unconditioned(tiny_eval):
    mg = _mg()
    w, o, _ = tiny_eval
    a = mg.eval_tree(w.map, w.trees[0], w.sensor, max_anc=0)
    assert np.array_equal(a["g_db"], o["g_abs"]) and np.array_equal(a["k_db"], o["k_abs"])


def test_mask_subset_matches_full(tiny_eval):
    mg = _mg()
    w, o, _ = tiny_eval
    tree = w.trees[0]
    mask = mg.ancestor_closure(tree.parent, [tree.n - 1, tree.n - 5])
    s = mg.eval_tree(w.map, tree, w.sensor, mask=mask)
    sel = mask.astype(bool)
    assert np.array_equal(s["g_db"][sel], o["g_db"][sel])
    assert np.array_equal(s["D"][sel], o["D"][sel])
    bad = mask.copy()
    bad[0] = 0
    with pytest.raises(ValueError):
        mg.eval_tree(w.map, tree, w.sensor, mask=bad)


def test_invalid_trees_rejected():
    mg = _mg()
    m = W.micro_map((8, 8, 8), fill=W.FREE)
    sen = W.Sensor(n_az=16, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=4.0, yaw_bins=8)
    good = np.array([[1, 1, 1], [2, 2, 2]], np.float32)
    for pos, par in [(good, np.array([0, 0], np.int32)),          # root with a parent
                     (good, np.array([-1, 1], np.int32)),         # parent not before child
                     (np.array([[1, 1, 1], [9, 2, 2]], np.float32), np.array([-1, 0], np.int32))]:  # outside
        with pytest.raises(ValueError):
            mg.eval_tree(m, W.Tree(pos_m=pos, parent=par), sen)
    chain = np.tile(np.array([[1.5, 1.5, 1.5]], np.float32), (66, 1))
    with pytest.raises(ValueError):                                 # depth 65 > 64
        mg.eval_tree(m, W.Tree(pos_m=chain, parent=np.arange(-1, 65, dtype=np.int32)), sen)


# ----------------------------------------------------------------- exact-equality conventions

def test_depth_equality_counts_as_observed():
    """Sec. IV-B: a point is previously observed when its depth is <= the stored depth."""
    mg = _mg()
    s = W.Sensor(n_az=8, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=10.0, yaw_bins=8)
    h = mg.SensorHandle(s)
    qa = np.array([0.5, 0.5, 0.5], np.float32)        # voxel centres sit at integer offsets
    Da = np.full((s.n_el, s.w_buf), 5.0, np.float32)
    got, row, col = h.obs(qa, 0, Da, 3, 4, 0)           # r = (3, 4, 0): |r| = 5 exactly
    assert got and row == 2 and col == 1
    Da[:] = np.nextafter(np.float32(5.0), np.float32(0.0))
    assert not h.obs(qa, 0, Da, 3, 4, 0)[0]


def test_pixel_cells_are_half_open():
    """A centre exactly on a row or column boundary belongs to the cell above / to the left."""
    mg = _mg()
    s = W.Sensor(n_az=8, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=10.0, yaw_bins=8)
    h = mg.SensorHandle(s)
    qa = np.array([0.5, 0.5, 0.5], np.float32)
    Da = np.full((s.n_el, s.w_buf), 50.0, np.float32)
    assert h.obs(qa, 0, Da, 3, 0, 0)[:3] == (True, 2, 0)    # azimuth 0 (window edge), elevation 0
    assert h.obs(qa, 0, Da, 2, 2, 0)[:3] == (True, 2, 1)    # on the 45-degree column boundary
    assert h.obs(qa, 0, Da, 0, 3, 0)[0] is False             # 90 degrees: outside [0, 90)


def test_dda_axis_tie_steps_x_first():
    """Exact diagonal from a voxel centre: at a shared corner x steps before y before z."""
    mg = _mg()
    st = np.full((6, 6, 6), W.UNK, np.uint8)
    q = np.array([1.5, 1.5, 1.5], np.float32)
    d = np.array([1, 1, 0], np.float32) / np.float32(np.sqrt(2.0))
    d = d.astype(np.float32)
    inv = (np.float32(1.0) / np.where(d != 0, d, 1)).astype(np.float32) * (d != 0)
    ids, _, te, _ = mg.trace_ray(st, q, d, inv, 3.0)
    xyz = [(int(i) % 6, (int(i) // 6) % 6, int(i) // 36) for i in ids]
    assert xyz[:3] == [(1, 1, 1), (2, 1, 1), (2, 2, 1)]
    assert te[1] == te[2]
    d3 = (np.ones(3, np.float32) / np.float32(np.sqrt(3.0))).astype(np.float32)
    ids, _, _, _ = mg.trace_ray(st, q, d3, (np.float32(1.0) / d3).astype(np.float32), 3.0)
    xyz = [(int(i) % 6, (int(i) // 6) % 6, int(i) // 36) for i in ids]
    assert xyz[:4] == [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)]


@pytest.mark.parametrize("rv", [2.5, 3.0, 0.5, 4.25])
def test_range_cut_is_strict(rv):
    """A voxel is visited only when its entry parameter is below the range (entry t = k - 1/2)."""
    mg = _mg()
    st = np.full((1, 1, 12), W.UNK, np.uint8)
    q = np.array([0.5, 0.5, 0.5], np.float32)
    d = np.array([1, 0, 0], np.float32)
    ids, _, _, h = mg.trace_ray(st, q, d, d, rv)
    assert len(ids) == 1 + sum(1 for k in range(1, 12) if k - 0.5 < rv)
    assert h == np.float32(rv)


# ----------------------------------------------------------------- exact marginal with its own yaw

def test_exact_marginal_argmax_and_consistency():
    """The exact gain with its own yaw choice equals, at every node, the exact per-incidence count
    (X_ray of the pinned exact pass) at its chosen window, and no other window of that node (the
    rest of the tree fixed) counts more; ties go to the smallest window; the root's is its absolute
    gain and no node exceeds its absolute gain."""
    mg = _mg()
    m, tree, s = W.random_micro(55, dims=(14, 12, 8), n_nodes=7, max_depth=3, range_vox=6.0, p_occ=0.06,
                                p_free=0.45, n_az=16, n_el=4, yaw_bins=8)
    e = mg.exact_marginal(m, tree, s)
    o = mg.eval_tree(m, tree, s)
    assert e["g_ex"][0] == o["g_abs"][0] and e["k_ex"][0] == o["k_abs"][0]
    assert np.all(e["g_ex"] <= o["g_abs"])
    x = mg.exact(m, tree, s, e["k_ex"], o["D"])
    assert np.array_equal(x["X_ray"], e["g_ex"])
    for nd in range(tree.n):
        sums = []
        for k in range(s.yaw_bins):
            kk = e["k_ex"].copy()
            kk[nd] = k
            sums.append(int(mg.exact(m, tree, s, kk, o["D"])["X_ray"][nd]))
        assert max(sums) == e["g_ex"][nd] and int(np.argmax(sums)) == e["k_ex"][nd], nd


# ----------------------------------------------------------------- exact quantities (eq. 2)

def _brute_exact(m, tree, sen, mg, k_db, D):
    """X_ray, X_set, A_set and G_db_set of every node from fp64 slab-test ray sets and fp64
    (atan2) pixel cells, at the given windows and ancestor buffers, with Python sets. Returns the
    four arrays and a per-node flag: some decision of the node or of its ancestors lies within
    rounding distance of a boundary."""
    t = mg.sensor_tables(sen)
    st = m.states
    flat = st.reshape(-1)
    nz_, ny_, nx_ = st.shape
    n = tree.n
    H, Wp, wb = sen.n_el, sen.n_az, sen.w_buf
    rv = float(np.float32(np.float32(sen.range_m) / np.float32(m.voxel_m)))
    q = ((tree.pos_m - m.origin_m) / np.float32(m.voxel_m)).astype(np.float32)
    rays, sets, amb = [], [], np.zeros(n, bool)
    for nd in range(n):                      # I_ray(n, c, j) for the window's rays, and I(n)
        c0 = int(t["c0"][int(k_db[nd])])
        per_ray = []
        for i in range(wb):
            c = (c0 + i) % Wp
            for j in range(H):
                must, may, _, _, _ = brute.ray_reference(st, q[nd], t["dir"][c * H + j], rv)
                mu = {v for v in must if flat[v] == W.UNK}
                if mu != {v for v in may if flat[v] == W.UNK}:
                    amb[nd] = True
                per_ray.append(mu)
        rays.append(per_ray)
        sets.append(set().union(*per_ray))
    out = {k: np.zeros(n, np.int64) for k in ("X_ray", "X_set", "A_set", "G_db_set")}
    flag = np.zeros(n, bool)
    for nd in range(n):
        anc = []
        a = int(tree.parent[nd])
        while a >= 0:
            anc.append(a)
            a = int(tree.parent[a])
        flag[nd] = amb[nd] or any(amb[a] for a in anc)
        union = set().union(*[sets[a] for a in anc]) if anc else set()
        out["A_set"][nd] = len(sets[nd])
        out["X_set"][nd] = len(sets[nd] - union)
        out["X_ray"][nd] = sum(len(r - union) for r in rays[nd])
        g = 0
        for vid in sets[nd]:
            ix, iy, iz = vid % nx_, (vid // nx_) % ny_, vid // (nx_ * ny_)
            seen = False
            for a in anc:
                ok, oamb = brute.observed(sen, q[a], int(t["c0"][int(k_db[a])]), D[a], ix, iy, iz)
                flag[nd] |= oamb
                if ok:
                    seen = True
                    break
            g += 0 if seen else 1
        out["G_db_set"][nd] = g
    return out, flag


@pytest.mark.parametrize("seed", range(4))
def test_exact_quantities_bruteforce(seed):
    """Eq. (2) at fixed windows (Sec. V-A protocol): every exact output of the oracle against Python
    sets built from the slab-test references; once at the oracle's own windows and buffers, once at
    seeded random windows with random buffers (so that ancestors observe part of their frustum)."""
    mg = _mg()
    m, tree, sen = W.random_micro(300 + seed, dims=(11, 10, 7), n_nodes=7, max_depth=4, n_az=16, n_el=4,
                                  range_vox=6.0, yaw_bins=8, p_occ=0.05, p_free=0.35)
    o = mg.eval_tree(m, tree, sen)
    rng = np.random.default_rng(seed)
    rv = np.float32(sen.range_m) / np.float32(m.voxel_m)
    cases = [(o["k_db"], o["D"]),
             (rng.integers(0, sen.yaw_bins, tree.n).astype(np.int32),
              (rng.random(o["D"].shape) * rv).astype(np.float32))]
    for k_db, D in cases:
        e = mg.exact(m, tree, sen, k_db, D)
        b, flag = _brute_exact(m, tree, sen, mg, k_db, D)
        cmp = np.flatnonzero(~flag)
        assert cmp.size >= tree.n - 2, (seed, flag)
        for key in ("A_set", "X_set", "X_ray", "G_db_set"):
            assert np.array_equal(e[key][cmp].astype(np.int64), b[key][cmp]), (seed, key, e[key], b[key])
        deep = [nd for nd in cmp if tree.depth()[nd] >= 2]
        assert deep, "the case needs nodes with two or more ancestors"
