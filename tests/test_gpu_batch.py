"""GPU tests of the multi-tree path (mg_eval_marginal_batch).

The batch must reproduce the per-tree results bit for bit, on one or several
maps, in any tree order, on every call of a cached launch plan.
"""
import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_40297_amd import mg as mgmod
    mgmod.lib()
    return mgmod


def _per_tree(mg, trees):
    import torch
    outs = []
    for T in trees:
        g, y, d = T.eval_marginal(depth=True)
        torch.cuda.synchronize()
        outs.append((g.clone(), y.clone(), d.clone()))
    return outs


def _check_batch(mg, trees, ref, order=None):
    import torch
    order = list(range(len(trees))) if order is None else order
    ts = [trees[i] for i in order]
    g, y, d = mg.eval_batch(ts, depth=True)
    torch.cuda.synchronize()
    off = 0
    for i in order:
        n = trees[i].n
        assert torch.equal(g[off:off + n], ref[i][0]), f"gain of tree {i}"
        assert torch.equal(y[off:off + n], ref[i][1]), f"yaw of tree {i}"
        assert torch.equal(d[off:off + n], ref[i][2]), f"depth of tree {i}"
        off += n


def test_batch_matches_per_tree_and_replays(mg):
    import torch
    w = W.make("batch64", n_trees=6)
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    log(f"[batch] 6 trees, {sum(t.n for t in trees)} nodes")
    ref = _per_tree(mg, trees)
    n = sum(t.n for t in trees)
    g = torch.empty(n, dtype=torch.int32, device="cuda")
    y = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty((n, trees[0].pixels), dtype=torch.float32, device="cuda")
    for rep in range(3):                 # same tree list: the cached plan is reused
        g.fill_(-1)
        mg.mg_eval_marginal_batch([t.handle for t in trees], g, y, d)
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()     # unrelated eager work between calls
        off = 0
        for i, T in enumerate(trees):
            assert torch.equal(g[off:off + T.n], ref[i][0]) and torch.equal(d[off:off + T.n], ref[i][2]), rep
            off += T.n
    _check_batch(mg, trees, ref, order=[5, 2, 0, 4, 1, 3])
    for T in trees:
        T.close()
    M.close()


def test_batch_over_several_maps_and_voxel_sizes(mg):
    """Trees on maps with different voxel sizes (different range in voxels), one sensor geometry."""
    w = W.make("tiny")
    m2, t2, _ = W.random_micro(31, dims=(30, 28, 16), n_nodes=9, max_depth=3, range_vox=1.0)
    sen = w.sensor
    M1 = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    M2 = mg.Map(m2.states, 0.25, (0.0, 0.0, 0.0))       # 5 m range = 20 voxels here, 25 on the tiny map
    trees = [mg.Tree(M1, w.trees[0].pos_m, w.trees[0].parent, sen),
             mg.Tree(M2, (t2.pos_m * np.float32(0.25)).astype(np.float32), t2.parent, sen),
             mg.Tree(M1, w.trees[0].pos_m[:1].copy(), np.array([-1], np.int32), sen)]
    ref = _per_tree(mg, trees)
    _check_batch(mg, trees, ref)
    _check_batch(mg, trees, ref, order=[2, 1, 0])
    for T in trees:
        T.close()
    M1.close()
    M2.close()


def test_batch_of_the_step_tree(mg):
    w = W.make("step")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    ref = _per_tree(mg, [T])
    _check_batch(mg, [T], ref)
    T.close()
    M.close()


def test_batch_rejects_a_tree_listed_twice(mg):
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    a = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    with pytest.raises(mg.MGError) as e:
        mg.eval_batch([a, a])
    assert e.value.code == mg.MG_E_INVALID
    a.close()
    M.close()


def test_batch_rejects_mixed_geometry(mg):
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    other = W.Sensor(n_az=64, n_el=12, fov_h_deg=90, fov_v_deg=60, range_m=5.0, yaw_bins=16)
    a = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    b = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, other)
    with pytest.raises(mg.MGError) as e:
        mg.eval_batch([a, b])
    assert e.value.code == mg.MG_E_INVALID
    a.close()
    b.close()
    M.close()


def test_kernel_timing_counts_trace_launches_and_keeps_results(mg):
    """Timed launches (events carried by the dispatch) give the same results and intervals for every trace
    and mask-builder launch."""
    import torch
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    ref = _per_tree(mg, [T])
    levels = int(w.trees[0].depth().max()) + 1
    mg.mg_timing_read()
    mg.mg_timing_enable(True)
    try:
        for _ in range(2):
            _check_batch(mg, [T], ref)
        ms, busy, n, wg = mg.mg_timing_read()
    finally:
        mg.mg_timing_enable(False)
    sen = w.sensor
    shape, _ = mg.mg_batch_plan_info([T.handle])
    threads = mg.mg_trace_shapes()[shape][0]
    tiles = -(-sen.n_az * sen.n_el // threads)
    # per call: at least one trace launch per level (groups may split levels), and a mask-builder
    # launch for every trace launch whose nodes include one with children (not the deepest level)
    assert n % 2 == 0 and n // 2 >= 2 * levels - 1
    assert wg == 2 * T.n * tiles                # every node traced exactly once per call
    assert ms > 0.0 and 0.0 < busy <= ms * 1.001
    assert mg.mg_timing_read() == (0.0, 0.0, 0, 0)
    _check_batch(mg, [T], ref)                       # timing off again: no intervals recorded
    assert mg.mg_timing_read()[2] == 0
    T.close()
    M.close()


def _subset_trees(mg, n_trees=5):
    w = W.make("batch64", n_trees=n_trees)
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    return M, trees


def test_every_launch_shape_gives_identical_results(mg):
    """Each compiled launch shape of the trace kernel, launched one by one and as a graph."""
    M, trees = _subset_trees(mg)
    ref = _per_tree(mg, trees)
    shapes = mg.mg_trace_shapes()
    log(f"[shapes] {shapes}")
    try:
        for k, (th, bricks) in enumerate(shapes):
            for graph in (False, True):
                mg.mg_batch_config(k, graph)
                log(f"[shapes] shape {k} ({th} rays/WG, {bricks} mask bricks/WG) graph={graph}")
                _check_batch(mg, trees, ref)
                assert mg.mg_batch_plan_info([t.handle for t in trees]) == (k, graph)
    finally:
        mg.mg_batch_config(-1, False)
    for T in trees:
        T.close()
    M.close()


def test_graph_replays_match_eager_launches(mg):
    """The captured plan replayed several times, with unrelated eager work and syncs in between."""
    import torch
    M, trees = _subset_trees(mg, 4)
    ref = _per_tree(mg, trees)
    n = sum(t.n for t in trees)
    g = torch.empty(n, dtype=torch.int32, device="cuda")
    y = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty((n, trees[0].pixels), dtype=torch.float32, device="cuda")
    handles = [t.handle for t in trees]
    try:
        mg.mg_batch_config(0, True)
        for rep in range(4):
            g.fill_(-1)
            y.fill_(-7)
            d.fill_(-1.0)
            mg.mg_eval_marginal_batch(handles, g, y, d)
            torch.cuda.synchronize()
            assert mg.mg_batch_plan_info(handles) == (0, True)
            off = 0
            for i, T in enumerate(trees):
                assert torch.equal(g[off:off + T.n], ref[i][0]), (rep, i)
                assert torch.equal(y[off:off + T.n], ref[i][1]), (rep, i)
                assert torch.equal(d[off:off + T.n], ref[i][2]), (rep, i)
                off += T.n
            x = torch.randn(4096, device="cuda")
            _ = (x * x).sum().item()                     # eager work between replays
    finally:
        mg.mg_batch_config(-1, False)
    for T in trees:
        T.close()
    M.close()


def test_autotune_chooses_a_shape_and_keeps_results(mg):
    M, trees = _subset_trees(mg, 3)
    ref = _per_tree(mg, trees)
    try:
        mg.mg_batch_config(-1, True)
        _check_batch(mg, trees, ref)                     # first call tunes, then replays the graph
        shape, graphed = mg.mg_batch_plan_info([t.handle for t in trees])
        assert 0 <= shape < len(mg.mg_trace_shapes()) and graphed
        _check_batch(mg, trees, ref)
        mg.mg_batch_config(-1, False)                    # tuned shape reused, launches one by one
        _check_batch(mg, trees, ref)
        assert mg.mg_batch_plan_info([t.handle for t in trees]) == (shape, False)
    finally:
        mg.mg_batch_config(-1, False)
    for T in trees:
        T.close()
    M.close()


def test_persistent_launch_equals_per_level_launches(mg):
    """One persistent cooperative launch per call (co-resident workgroups, grid barriers between
    the trace, window and mask phases of every level) gives the per-level launches' gains, windows
    and depth buffers bit for bit: one tree (`step`), and six trees of `batch64` in one call, twice
    in a row; the plan reports the persistent form."""
    import torch
    cases = [("step", None), ("batch64", 6)]
    try:
        mg.mg_batch_barrier_polls(1 << 22)          # each wait ends within about a second
        for name, nt in cases:
            w = W.make(name, n_trees=nt)
            M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
            trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
            mg.mg_batch_config(-1, 0)
            g0, y0, d0 = mg.eval_batch(trees, depth=True)
            torch.cuda.synchronize()
            ref = (mg.as_u32(g0), y0.cpu().numpy(), d0.cpu().numpy())
            mg.mg_batch_config(-1, 2)
            for rep in range(2):
                log(f"[persistent] {name}: {len(trees)} trees, call {rep}")
                g, y, d = mg.eval_batch(trees, depth=True)
                torch.cuda.synchronize()
                assert np.array_equal(mg.as_u32(g), ref[0]), name
                assert np.array_equal(y.cpu().numpy(), ref[1]), name
                assert np.array_equal(d.cpu().numpy().view(np.uint32), ref[2].view(np.uint32)), name
            assert mg.mg_batch_plan_info([t.handle for t in trees])[1] == 2
            mg.mg_batch_config(-1, 0)
            for T in trees:
                T.close()
            M.close()
    finally:
        mg.mg_batch_barrier_polls(1 << 25)
        mg.mg_batch_config(-1, 0)


def test_persistent_barrier_gives_up_when_its_poll_limit_runs_out(mg):
    """With a barrier poll limit of 0 set from the host, the first grid-barrier wait that is not
    already satisfied gives up: every workgroup leaves at its next barrier, the launch ends and
    the call reports MG_E_DEVICE; with the limit restored the next call is correct."""
    import torch
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    try:
        mg.mg_batch_config(-1, 0)
        g0, y0, _ = mg.eval_batch([T])
        torch.cuda.synchronize()
        ref = (mg.as_u32(g0), y0.cpu().numpy())
        mg.mg_batch_config(-1, 2)
        mg.mg_batch_barrier_polls(0)
        log("[persistent] barrier poll limit 0")
        with pytest.raises(mg.MGError) as e:
            mg.eval_batch([T])
        assert e.value.code == mg.MG_E_DEVICE
        mg.mg_batch_barrier_polls(1 << 22)
        g, y, _ = mg.eval_batch([T])
        torch.cuda.synchronize()
        assert np.array_equal(mg.as_u32(g), ref[0]) and np.array_equal(y.cpu().numpy(), ref[1])
    finally:
        mg.mg_batch_barrier_polls(1 << 25)
        mg.mg_batch_config(-1, 0)
        T.close()
        M.close()
