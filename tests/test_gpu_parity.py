"""GPU parity: the HIP library against the oracle, element by element.

Bit-exact on gains (uint32 counts), yaw windows and depth buffers (float
bits), because both sides take every decision in IEEE binary32 with the same
operation order. Small workloads are compared in full; the full-size ones in
full where the oracle finishes in seconds, else on ancestor-closed samples of
nodes (a node needs only its ancestors' buffers) plus invariants at every node.
"""
import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from tests.gpu_util import assert_same, gpu_eval_tree, log, threads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_40297_amd import mg as mgmod
    mgmod.lib()          # raises when the HIP library is missing: no fallback
    return mgmod


@pytest.fixture(scope="module")
def orc():
    from oracle import mgref
    if not __import__("os").path.exists(mgref.LIB):
        mgref.build()
    return mgref


def _full_parity(mg, orc, m, tree, sen, label):
    log(f"[parity] {label}: n={tree.n} rays/node={sen.rays}")
    ref = orc.eval_tree(m, tree, sen, n_threads=threads())
    got = gpu_eval_tree(mg, m, tree, sen, depth=True, mode="both")
    assert_same(got, ref, keys=("g_db", "k_db", "D", "g_abs", "k_abs"))
    batched = gpu_eval_tree(mg, m, tree, sen, depth=True, mode="batch")
    assert_same(batched, ref, keys=("g_db", "k_db", "D"))
    return got, ref


# ----------------------------------------------------------------- small cases, full comparison

def test_tiny_full(mg, orc):
    w = W.make("tiny")
    _full_parity(mg, orc, w.map, w.trees[0], w.sensor, "tiny")


@pytest.mark.parametrize("seed", range(6))
def test_random_micro_full(mg, orc, seed):
    sens = [dict(n_az=16, n_el=6, yaw_bins=8), dict(n_az=100, n_el=7, yaw_bins=36),
            dict(n_az=24, n_el=5, yaw_bins=12)]
    s = sens[seed % 3]
    m, tree, sen = W.random_micro(500 + seed, dims=(17, 13, 9), n_nodes=12, max_depth=4, range_vox=9.0,
                                  p_occ=0.06, p_free=0.45, **s)
    _full_parity(mg, orc, m, tree, sen, f"micro{seed}")


def test_axis_rays_closed_form_on_gpu(mg, orc):
    m = W.micro_map((10, 9, 5), fill=W.UNK)
    sen = W.Sensor(n_az=4, n_el=1, fov_h_deg=90, fov_v_deg=60, range_m=5.0, yaw_bins=4, az_offset_deg=-45.0)
    tree = W.Tree(pos_m=np.array([[3.5, 4.5, 2.5], [5.5, 4.5, 2.5]], np.float32), parent=np.array([-1, 0], np.int32))
    got, _ = _full_parity(mg, orc, m, tree, sen, "axis")
    assert int(got["g_abs"][0]) == 6 and int(got["k_abs"][0]) == 0     # +x: voxels 3..8 (6 of them)


def test_single_node_star_and_chain(mg, orc):
    w = W.make("tiny")
    m, sen = w.map, w.sensor
    p = w.trees[0].pos_m
    single = W.Tree(pos_m=p[:1].copy(), parent=np.array([-1], np.int32))
    star = W.Tree(pos_m=p[:9].copy(), parent=np.array([-1] + [0] * 8, np.int32))
    chain_pos = np.repeat(p[:4], 17, axis=0)[:64] + np.float32(0.013) * np.arange(64, dtype=np.float32)[:, None]
    chain_pos = np.clip(chain_pos, 0.05, w.map.extent_m.astype(np.float32) - 0.05)
    chain = W.Tree(pos_m=chain_pos.astype(np.float32), parent=np.arange(-1, 63, dtype=np.int32))  # depth 63
    for tr, lab in ((single, "single"), (star, "star"), (chain, "chain63")):
        _full_parity(mg, orc, m, tr, sen, lab)


def test_boundary_positions(mg, orc):
    """Nodes exactly on voxel faces, edges and centres, and at the grid's corner."""
    m, _, sen = W.random_micro(77, dims=(12, 12, 8), n_nodes=1, n_az=36, n_el=9, yaw_bins=12, range_vox=8.0)
    pos = np.array([[6.0, 6.0, 4.0], [6.5, 6.5, 4.5], [6.0, 5.5, 3.0], [0.0, 0.0, 0.0], [11.99, 11.99, 7.99],
                    [3.25, 7.0, 2.5]], np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 1, 0, 3, 2], np.int32))
    _full_parity(mg, orc, m, tree, sen, "boundary")


def _free_brick_map(seed, dims):
    """A map of whole bricks: about 35 % of its 8x8x8 bricks wholly free, 30 % wholly unknown, the
    others mixing free and unknown voxels, some also occupied ones, so that rays cross many bricks
    that hold one state only."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    st = np.full((nz, ny, nx), W.FREE, np.uint8)
    for bz in range(0, nz, 8):
        for by in range(0, ny, 8):
            for bx in range(0, nx, 8):
                sl = st[bz:bz + 8, by:by + 8, bx:bx + 8]
                u = rng.uniform()
                if u < 0.35:
                    continue
                if u < 0.65:
                    sl[...] = W.UNK
                    continue
                sl[rng.uniform(size=sl.shape) < (0.5 if u < 0.85 else 0.3)] = W.UNK
                if u >= 0.85:
                    sl[rng.uniform(size=sl.shape) < 0.03] = W.OCC
    return W.Map(states=st, voxel_m=1.0, origin_m=np.zeros(3, dtype=np.float32))


@pytest.mark.parametrize("dims", [(40, 32, 24), (37, 29, 21)])
def test_free_bricks_crossed_at_once(mg, orc, dims):
    """Rays through wholly free and wholly unknown bricks (the device traversal crosses a free
    brick, and an unknown one over which the parent's path mask is uniform, in one step) against
    the oracle's voxel-by-voxel DDA: nodes on brick corners, edges and faces, 45-degree rays whose
    boundary parameters tie, horizontal rows (no z motion), and a dense panorama; grids whose
    size is a multiple of the brick and grids whose last bricks reach past the grid."""
    m = _free_brick_map(900 + dims[0], dims)
    pos = np.array([[8.0, 8.0, 8.0], [16.0, 16.0, 8.0], [8.0, 12.5, 12.0], [24.0, 8.0, 16.0], [12.5, 12.5, 12.5],
                    [16.0, 8.0, 4.5], [9.5, 17.0, 8.0], [31.0, 23.0, 15.0], [4.25, 20.75, 19.5], [20.0, 20.0, 10.0]],
                   np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 0, 1, 1, 2, 3, 4, 6, 8], np.int32))
    for sen in (W.Sensor(n_az=8, n_el=3, fov_h_deg=90, fov_v_deg=90, range_m=30.0, yaw_bins=8, az_offset_deg=-22.5),
                W.Sensor(n_az=100, n_el=17, fov_h_deg=90, fov_v_deg=80, range_m=25.0, yaw_bins=20)):
        got, ref = _full_parity(mg, orc, m, tree, sen, f"free bricks {dims} {sen.n_az}x{sen.n_el}")
        assert int(ref["g_abs"].sum()) > 0


def _nested_block_map(seed, dims):
    """A map of nested aligned blocks: each 16x16x16 block wholly free or split into 8x8x8 bricks,
    each brick wholly free, wholly unknown or split into 4x4x4 quarters, each quarter wholly free,
    wholly unknown or split into 2x2x2 blocks, each of those wholly free, wholly unknown or of
    mixed voxels (a few occupied), so that rays cross blocks of every size the traversal crosses
    in one step."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    st = np.full((nz, ny, nx), W.FREE, np.uint8)

    def fill(z, y, x, e):
        sl = st[z:z + e, y:y + e, x:x + e]
        u = rng.uniform()
        if u < 0.3:
            return
        if e == 16 and u >= 0.45:
            u = 0.6                                  # (16-voxel blocks: wholly free, wholly unknown or split)
        if u < 0.55:
            sl[...] = W.UNK
            return
        if e == 2:
            sl[rng.uniform(size=sl.shape) < 0.5] = W.UNK
            sl[rng.uniform(size=sl.shape) < 0.04] = W.OCC
            return
        h = e // 2
        for dz in (0, h):
            for dy in (0, h):
                for dx in (0, h):
                    fill(z + dz, y + dy, x + dx, h)
    for z in range(0, nz, 16):
        for y in range(0, ny, 16):
            for x in range(0, nx, 16):
                fill(z, y, x, 16)
    return W.Map(states=st, voxel_m=1.0, origin_m=np.zeros(3, dtype=np.float32))


@pytest.mark.parametrize("dims", [(40, 32, 24), (37, 29, 21), (48, 48, 34)])
def test_nested_blocks_crossed_at_once(mg, orc, dims):
    """Rays through wholly free blocks of 2x2x2 bricks, bricks, quarter bricks and 2x2x2 blocks and
    wholly unknown bricks and quarter bricks (each crossed in one step on the device) against the oracle's
    voxel-by-voxel DDA: nodes on block corners, edges and faces, 45-degree rays whose boundary
    parameters tie, ranges that end inside blocks; grids whose last blocks reach past the grid."""
    m = _nested_block_map(1200 + dims[0], dims)
    pos = np.array([[8.0, 8.0, 8.0], [16.0, 16.0, 8.0], [12.0, 12.0, 4.0], [24.0, 8.0, 16.0], [10.0, 14.0, 6.0],
                    [16.0, 8.0, 4.5], [9.5, 17.0, 8.0], [30.0, 22.0, 14.0], [4.25, 20.75, 19.5], [20.0, 20.0, 10.0],
                    [6.0, 26.0, 2.0], [18.5, 2.0, 12.0]], np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 0, 1, 1, 2, 3, 4, 6, 8, 9, 10], np.int32))
    for sen in (W.Sensor(n_az=8, n_el=3, fov_h_deg=90, fov_v_deg=90, range_m=30.0, yaw_bins=8, az_offset_deg=-22.5),
                W.Sensor(n_az=100, n_el=17, fov_h_deg=90, fov_v_deg=80, range_m=13.7, yaw_bins=20)):
        got, ref = _full_parity(mg, orc, m, tree, sen, f"nested blocks {dims} {sen.n_az}x{sen.n_el}")
        assert int(ref["g_abs"].sum()) > 0


def test_evaluations_of_one_tree_do_not_see_each_others_masks(mg, orc):
    """A path mask keeps only what can be read (the words of a wholly unknown brick only when its
    code is mixed), so its memory holds what an earlier evaluation of the same tree left there.
    Marginal, single-parent and marginal again on one tree object, each against the oracle, with
    ranges that end inside wholly unknown bricks (a ray whose range ends in such a brick counts
    its last voxels there from the brick's code, not its words, and ends in one step)."""
    import torch
    m = _free_brick_map(955, (40, 32, 24))
    pos = np.array([[8.0, 8.0, 8.0], [16.0, 16.0, 8.0], [8.0, 12.5, 12.0], [24.0, 8.0, 16.0], [12.5, 12.5, 12.5],
                    [16.0, 8.0, 4.5], [9.5, 17.0, 8.0], [31.0, 23.0, 15.0], [4.25, 20.75, 19.5], [20.0, 20.0, 10.0]],
                   np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 0, 1, 1, 2, 3, 4, 6, 8], np.int32))
    for rng in (11.3, 17.7):
        sen = W.Sensor(n_az=72, n_el=13, fov_h_deg=90, fov_v_deg=80, range_m=rng, yaw_bins=24)
        log(f"[parity] alternating evaluations, range {rng}")
        ref = orc.eval_tree(m, tree, sen, n_threads=threads())
        ref1 = orc.eval_tree(m, tree, sen, max_anc=1, n_threads=threads())
        M = mg.Map(m.states, m.voxel_m, m.origin_m)
        T = mg.Tree(M, tree.pos_m, tree.parent, sen)
        try:
            for mode in ("marginal", "single", "marginal", "single"):
                g, y, _ = T.eval_marginal() if mode == "marginal" else T.eval_single_parent()
                torch.cuda.synchronize()
                r = ref if mode == "marginal" else ref1
                assert_same({"g_db": mg.as_u32(g), "k_db": y.cpu().numpy()}, r, keys=("g_db", "k_db"))
        finally:
            T.close()
            M.close()


def test_ranges_that_end_inside_unknown_blocks(mg, orc):
    """A wholly unknown map of 16-voxel blocks (its last blocks reach past the grid): every ray
    ends at the range inside a wholly unknown block, which the device finishes in one step where
    the parent's mask is uniform over the block (or brick, or quarter) and walks voxel by voxel
    where it is mixed. Nodes on block corners, faces and inside; integer ranges that tie the
    boundary parameters of axis-aligned rays (a boundary at exactly the range is not crossed);
    45-degree rays; a finer panorama with a fractional range."""
    m = W.micro_map((48, 40, 36), fill=W.UNK)
    pos = np.array([[16.0, 16.0, 16.0], [24.0, 16.0, 16.0], [16.0, 24.0, 20.0], [32.0, 20.0, 16.0],
                    [8.5, 8.5, 8.5], [20.0, 28.0, 12.0], [30.25, 12.75, 18.5], [40.0, 32.0, 24.0],
                    [16.0, 8.0, 28.0], [24.5, 24.5, 4.5]], np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 0, 1, 1, 2, 3, 6, 5, 2], np.int32))
    for sen in (W.Sensor(n_az=8, n_el=3, fov_h_deg=90, fov_v_deg=90, range_m=12.0, yaw_bins=8, az_offset_deg=-22.5),
                W.Sensor(n_az=8, n_el=3, fov_h_deg=90, fov_v_deg=90, range_m=16.0, yaw_bins=8, az_offset_deg=-22.5),
                W.Sensor(n_az=96, n_el=15, fov_h_deg=90, fov_v_deg=80, range_m=10.5, yaw_bins=24)):
        got, ref = _full_parity(mg, orc, m, tree, sen, f"unknown blocks, range {sen.range_m}")
        assert np.all(ref["g_abs"] > 0)
        assert np.any(ref["g_db"][1:] < ref["g_abs"][1:])   # the parents' masks decide some counts


def test_occupied_everywhere_and_unknown_everywhere(mg, orc):
    sen = W.Sensor(n_az=64, n_el=12, fov_h_deg=90, fov_v_deg=60, range_m=6.0, yaw_bins=16)
    pos = np.array([[4.3, 4.6, 3.2], [5.1, 4.2, 3.7], [3.2, 5.5, 2.9]], np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 1], np.int32))
    occ = W.micro_map((9, 9, 7), fill=W.OCC)
    for p in pos:
        occ.states[int(p[2]), int(p[1]), int(p[0])] = W.FREE
    got, _ = _full_parity(mg, orc, occ, tree, sen, "all-occupied")
    assert np.all(got["g_db"] == 0) and np.all(got["g_abs"] == 0)      # no unknown voxel anywhere
    unk = W.micro_map((9, 9, 7), fill=W.UNK)
    _full_parity(mg, orc, unk, tree, sen, "all-unknown")


def test_widest_panorama_or_clean_refusal(mg, orc):
    """The widest panorama the library accepts (4096 columns): bit-exact if the device's LDS per
    workgroup holds its tables, otherwise MG_E_UNSUPPORTED at upload with nothing launched."""
    w = W.make("tiny")
    sen = W.Sensor(n_az=4096, n_el=2, fov_h_deg=90, fov_v_deg=60, range_m=3.0, yaw_bins=64)
    tree = W.Tree(pos_m=w.trees[0].pos_m[:3].copy(), parent=np.array([-1, 0, 1], np.int32))
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    try:
        T = mg.Tree(M, tree.pos_m, tree.parent, sen)
    except mg.MGError as e:
        log(f"[parity] 4096-column panorama refused: {e}")
        assert e.code == mg.MG_E_UNSUPPORTED
        M.close()
        return
    T.close()
    M.close()
    _full_parity(mg, orc, w.map, tree, sen, "4096 columns")


# ----------------------------------------------------------------- full-size workloads

def test_step_full_parity(mg, orc):
    """The single-planner-step workload (500 nodes, 360x60 rays, 8 m at 0.1 m): every node."""
    w = W.make("step")
    got, ref = _full_parity(mg, orc, w.map, w.trees[0], w.sensor, "step")
    assert np.all(got["g_db"] <= got["g_abs"]) and got["g_db"][0] == got["g_abs"][0]


@pytest.mark.parametrize("case", ["tiny", "micro0", "micro1", "micro2", "step"])
def test_single_parent_full(mg, orc, case):
    """g_sp (parent-only conditioning, the comparison gain of Fig. 4) against the oracle with one
    ancestor, every node; equal to the marginal gain where the parent is the only ancestor."""
    if case == "tiny" or case == "step":
        w = W.make(case)
        m, tree, sen = w.map, w.trees[0], w.sensor
    else:
        k = int(case[-1])
        m, tree, sen = W.random_micro(600 + k, dims=(17, 13, 9), n_nodes=14, max_depth=5, range_vox=9.0,
                                      p_occ=0.06, p_free=0.45, n_az=[16, 100, 24][k], n_el=[6, 7, 5][k],
                                      yaw_bins=[8, 36, 12][k])
    log(f"[parity] single parent {case}: n={tree.n}")
    ref = orc.eval_tree(m, tree, sen, max_anc=1, n_threads=threads())
    got = gpu_eval_tree(mg, m, tree, sen, depth=True, mode="single_parent")
    assert_same(got, ref)
    full = gpu_eval_tree(mg, m, tree, sen, depth=False, mode="marginal")
    dep = tree.depth()
    assert np.array_equal(got["g_db"][dep <= 1], full["g_db"][dep <= 1])
    assert np.all(got["g_db"][dep == 2] >= full["g_db"][dep == 2])


def test_batch64_subset(mg, orc):
    """Four trees of the 64-tree workload: batch call == per-tree calls == oracle (sampled)."""
    import torch
    w = W.make("batch64", n_trees=4)
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    gb, yb, db = mg.eval_batch(trees, depth=True)
    torch.cuda.synchronize()
    off = 0
    for i, (t, T) in enumerate(zip(w.trees, trees)):
        g, y, d = T.eval_marginal(depth=True)
        torch.cuda.synchronize()
        assert torch.equal(g, gb[off:off + t.n]) and torch.equal(y, yb[off:off + t.n])
        assert torch.equal(d, db[off:off + t.n])
        if i < 2:
            dep = t.depth()
            leaves = np.flatnonzero(dep == dep.max())[:3]
            mask = orc.ancestor_closure(t.parent, leaves)
            log(f"[parity] batch64 tree {i}: n={t.n}, sampled {int(mask.sum())} nodes")
            ref = orc.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads())
            sel = np.flatnonzero(mask)
            got = dict(g_db=mg.as_u32(g), k_db=y.cpu().numpy(),
                       D=d.cpu().numpy().reshape(t.n, w.sensor.n_el, w.sensor.w_buf))
            assert_same(got, ref, nodes=sel)
        off += t.n
    for T in trees:
        T.close()
    M.close()


def test_large_sampled(mg, orc):
    """Large map (512x512x128 at 0.05 m, 720x120 rays, 15 m): two leaves' ancestor chains."""
    w = W.make("large", n_trees=1)
    t = w.trees[0]
    got = gpu_eval_tree(mg, w.map, t, w.sensor, depth=True, mode="both")
    assert np.all(got["g_db"] <= got["g_abs"]) and got["g_db"][0] == got["g_abs"][0]
    dep = t.depth()
    leaves = np.flatnonzero(dep == dep.max())[:2]
    mask = orc.ancestor_closure(t.parent, leaves)
    log(f"[parity] large: sampled {int(mask.sum())} nodes")
    ref = orc.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads())
    assert_same(got, ref, nodes=np.flatnonzero(mask))


def test_large_bench_configuration(mg, orc):
    """The large workload as bench.py times it: all 8 trees in one batched call (autotuned launch
    shape, stream groups); two leaves' ancestor chains of two trees against the oracle, and the
    bound G_db <= G_abs with equality at the roots on every node."""
    import torch
    w = W.make("large")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    log(f"[parity] large batched: {len(trees)} trees, {sum(t.n for t in trees)} nodes")
    gb, yb, db = mg.eval_batch(trees, depth=True)
    torch.cuda.synchronize()
    off = 0
    for i, (t, T) in enumerate(zip(w.trees, trees)):
        ga, _ = T.eval_absolute()
        torch.cuda.synchronize()
        g = mg.as_u32(gb[off:off + t.n])
        assert np.all(g <= mg.as_u32(ga)) and g[0] == mg.as_u32(ga)[0], i
        if i in (0, 5):
            dep = t.depth()
            leaves = np.flatnonzero(dep == dep.max())[:2]
            mask = orc.ancestor_closure(t.parent, leaves)
            log(f"[parity] large tree {i}: sampled {int(mask.sum())} nodes")
            ref = orc.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads())
            got = dict(g_db=g, k_db=yb[off:off + t.n].cpu().numpy(),
                       D=db[off:off + t.n].cpu().numpy().reshape(t.n, w.sensor.n_el, w.sensor.w_buf))
            assert_same(got, ref, nodes=np.flatnonzero(mask))
        off += t.n
    for T in trees:
        T.close()
    M.close()


# ----------------------------------------------------------------- modes and determinism

def test_levelsync_and_repeat_are_identical(mg):
    import torch
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    g1, y1, d1 = T.eval_marginal(depth=True)
    g2, y2, d2 = T.eval_marginal(depth=True)
    hg = np.zeros(T.n, np.uint32)
    hy = np.zeros(T.n, np.int32)
    g3, y3, d3 = T.outputs(depth=True)
    mg.mg_eval_marginal_levelsync(T.handle, hg, hy, g3, y3, d3)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(y1, y2) and torch.equal(d1, d2)
    assert torch.equal(g1, g3) and torch.equal(d1, d3)
    assert np.array_equal(hg, mg.as_u32(g1)) and np.array_equal(hy, y1.cpu().numpy())
    T.close()
    M.close()


def test_errors_from_device_api(mg):
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    bad_par = w.trees[0].parent.copy()
    bad_par[3] = 7
    with pytest.raises(mg.MGError) as e:
        mg.Tree(M, w.trees[0].pos_m, bad_par, w.sensor)
    assert e.value.code == mg.MG_E_INVALID
    outside = w.trees[0].pos_m.copy()
    outside[2, 0] = 99.0
    with pytest.raises(mg.MGError):
        mg.Tree(M, outside, w.trees[0].parent, w.sensor)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    with pytest.raises(mg.MGError) as e:
        M.close()                          # a tree still uses the map
    assert e.value.code == mg.MG_E_BUSY
    assert T.footprint_bytes > T.n * w.sensor.rays * 4
    T.close()
    M.close()


def _oracle_chains(orc, jobs):
    """Oracle on several (map, tree, sensor, mask) jobs at once: one host thread per job (the
    library releases the interpreter lock), each job's levels evaluated serially."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        return list(ex.map(lambda j: orc.eval_tree(j[0], j[1], j[2], mask=j[3], n_threads=1), jobs))


def test_batch64_full_call_against_oracle(mg, orc):
    """The 64-tree workload as it is benchmarked: all 64 trees (29 k nodes) in one
    mg_eval_marginal_batch call (autotuned launch shape, stream groups). In every tree the ancestor
    chain of one deepest leaf is compared with the oracle: gains, windows and depth buffers."""
    import torch
    w = W.make("batch64")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    log(f"[parity] batch64 full: {len(trees)} trees, {sum(t.n for t in trees)} nodes in one call")
    gb, yb, db = mg.eval_batch(trees, depth=True)
    torch.cuda.synchronize()
    gb, yb = mg.as_u32(gb), yb.cpu().numpy()
    db = db.cpu().numpy().reshape(-1, w.sensor.n_el, w.sensor.w_buf)
    jobs, offs = [], []
    off = 0
    for t in w.trees:
        dep = t.depth()
        leaf = int(np.flatnonzero(dep == dep.max())[0])
        jobs.append((w.map, t, w.sensor, orc.ancestor_closure(t.parent, [leaf])))
        offs.append(off)
        off += t.n
    log(f"[parity] batch64 full: oracle on {sum(int(j[3].sum()) for j in jobs)} chain nodes")
    refs = _oracle_chains(orc, jobs)
    for i, (t, ref, o) in enumerate(zip(w.trees, refs, offs)):
        got = dict(g_db=gb[o:o + t.n], k_db=yb[o:o + t.n], D=db[o:o + t.n])
        assert_same(got, ref, nodes=np.flatnonzero(jobs[i][3]))
    for T in trees:
        T.close()
    M.close()
