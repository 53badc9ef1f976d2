"""GPU parity of the device path score (mg_score_branches, eq. 3 and eq. 4).

The gains fed to the oracle are the oracle's own; the device scores the gains
the device computed (identical bit for bit, checked again here). Cost is
float64 additions, products and square roots of float32 positions, each
correctly rounded on both sides and taken in the same order, so it must match
bit for bit. The objective also takes exp(), which neither side rounds
correctly: each term may differ by about 2 ulp, and the <= 65 terms of a root
path are summed in the same order, so the relative difference stays below
65 * 2^-52 ~ 1.5e-14; the test allows 1e-13. The best node must be the device
objective's first maximum and, on the oracle's objective, within that
tolerance of the maximum.
"""
import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from oracle import paths
from tests.gpu_util import log, threads

pytestmark = pytest.mark.gpu

RTOL = 1e-13


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_40297_amd import mg as mgmod
    mgmod.lib()
    return mgmod


@pytest.fixture(scope="module")
def orc():
    from oracle import mgref
    if not __import__("os").path.exists(mgref.LIB):
        mgref.build()
    return mgref


def _check_tree(c_gpu, o_gpu, b_gpu, cost, obj, nodes=None):
    sel = np.arange(len(cost)) if nodes is None else np.asarray(nodes)
    assert c_gpu[sel].tobytes() == cost[sel].tobytes(), np.flatnonzero(c_gpu[sel] != cost[sel])[:5]
    assert np.allclose(o_gpu[sel], obj[sel], rtol=RTOL, atol=0), np.max(np.abs(o_gpu[sel] / obj[sel] - 1))
    assert b_gpu == int(np.flatnonzero(o_gpu == o_gpu.max())[0])
    if nodes is None:
        assert obj[b_gpu] >= obj.max() * (1 - RTOL)


def _check_branch(row, parent, best):
    ref = paths.branch(parent, best)
    assert row.shape == (65,)
    assert list(row[:len(ref)]) == ref and bool(np.all(row[len(ref):] == -1))


def test_score_matches_oracle_on_a_mixed_batch(mg, orc):
    """Three maps / voxel sizes and a one-node tree in one batch, three values of lambda."""
    import torch
    w = W.make("tiny")
    sen = w.sensor
    m2, t2, _ = W.random_micro(31, dims=(30, 28, 16), n_nodes=9, max_depth=3, range_vox=1.0)
    m2 = W.Map(states=m2.states, voxel_m=0.25, origin_m=np.zeros(3, np.float32))
    t2 = W.Tree(pos_m=(t2.pos_m * np.float32(0.25)).astype(np.float32), parent=t2.parent)
    m3, t3, _ = W.random_micro(77, dims=(24, 20, 12), n_nodes=14, max_depth=5, range_vox=1.0)
    m3 = W.Map(states=m3.states, voxel_m=0.4, origin_m=np.array([-2.0, 1.0, 0.5], np.float32))
    t3 = W.Tree(pos_m=(t3.pos_m * np.float32(0.4) + m3.origin_m).astype(np.float32), parent=t3.parent)
    t4 = W.Tree(pos_m=w.trees[0].pos_m[:1].copy(), parent=np.array([-1], np.int32))
    cases = [(w.map, w.trees[0]), (m2, t2), (m3, t3), (w.map, t4)]
    maps = {}
    handles = []
    for m, t in cases:
        if id(m) not in maps:
            maps[id(m)] = mg.Map(m.states, m.voxel_m, m.origin_m)
        handles.append(mg.Tree(maps[id(m)], t.pos_m, t.parent, sen))
    g, _, _ = mg.eval_batch(handles)
    torch.cuda.synchronize()
    g_host = mg.as_u32(g)
    refs = []
    off = 0
    for m, t in cases:
        ref = orc.eval_tree(m, t, sen, n_threads=threads())
        assert np.array_equal(g_host[off:off + t.n], ref["g_db"])
        refs.append(ref["g_db"])
        off += t.n
    for lam in (0.5, 0.0, 2.0):
        log(f"[paths] mixed batch, lambda={lam}")
        c, o, b, br = mg.score_batch(handles, g, lam)
        torch.cuda.synchronize()
        c, o, b, br = c.cpu().numpy(), o.cpu().numpy(), b.cpu().numpy(), br.cpu().numpy()
        off = 0
        for k, (m, t) in enumerate(cases):
            cost, obj, _ = paths.score_paths(t.pos_m, t.parent, refs[k], m.voxel_m, lam)
            _check_tree(c[off:off + t.n], o[off:off + t.n], int(b[k]), cost, obj)
            _check_branch(br[k], t.parent, int(b[k]))
            off += t.n
    for T in handles:
        T.close()
    for M in maps.values():
        M.close()


def test_score_of_the_step_tree_on_sampled_branches(mg, orc):
    """500-node planner step: the score of three deepest leaves' root paths against the oracle."""
    import torch
    w = W.make("step")
    t = w.trees[0]
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, t.pos_m, t.parent, w.sensor)
    g, _, _ = mg.eval_batch([T])
    c, o, b, br = mg.score_batch([T], g, 0.5)
    torch.cuda.synchronize()
    _check_branch(br.cpu().numpy()[0], t.parent, int(b.cpu().numpy()[0]))
    dep = t.depth()
    leaves = np.flatnonzero(dep == dep.max())[:3]
    mask = orc.ancestor_closure(t.parent, leaves)
    sel = np.flatnonzero(mask)
    log(f"[paths] step: n={t.n}, sampled {sel.size} nodes")
    ref = orc.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads())
    g_host = mg.as_u32(g)
    assert np.array_equal(g_host[sel], ref["g_db"][sel])
    gains = np.where(mask, ref["g_db"], 0).astype(np.uint32)     # unsampled nodes do not enter sel's scores
    cost, obj, _ = paths.score_paths(t.pos_m, t.parent, gains, w.map.voxel_m, 0.5)
    _check_tree(c.cpu().numpy(), o.cpu().numpy(), int(b.cpu().numpy()[0]), cost, obj, nodes=sel)
    T.close()
    M.close()


def test_score_errors(mg):
    import torch
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    g = torch.zeros(T.n, dtype=torch.int32, device="cuda")
    with pytest.raises(mg.MGError):              # no batch plan for this tree list yet
        mg.score_batch([T], g, 0.5)
    mg.eval_batch([T])
    with pytest.raises(mg.MGError):
        mg.score_batch([T], g, -1.0)
    c, o, b, br = mg.score_batch([T], g, 0.5)    # all-zero gains: every objective 0, best is the root
    torch.cuda.synchronize()
    assert float(o.abs().max()) == 0.0 and int(b[0]) == 0
    assert br[0, 0].item() == 0 and bool((br[0, 1:] == -1).all())
    T.close()
    M.close()


def test_score_of_a_tree_past_the_single_launch_size(mg):
    """A 12,000-node tree (past the single-launch size, so scored by the per-node kernel and the
    argmax kernel) and the 20-node tree in one batch, with seeded gains given to both sides."""
    import torch
    w = W.make("tiny")
    rng = np.random.Generator(np.random.PCG64(31))
    n = 12000
    par = np.concatenate([[-1], rng.integers(0, np.minimum(np.arange(1, n), 200))]).astype(np.int32)
    pos = rng.uniform(0.1, w.map.extent_m.astype(np.float32) - 0.1, (n, 3)).astype(np.float32)
    big = W.Tree(pos_m=pos, parent=par)
    assert big.depth().max() <= 64
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, big.pos_m, big.parent, w.sensor), mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)]
    mg.eval_batch(trees)                               # the plan the score call uses
    gains = rng.integers(0, 20000, n + w.trees[0].n).astype(np.uint32)
    g = torch.from_numpy(gains.view(np.int32)).cuda()
    c, o, b, br = mg.score_batch(trees, g, 0.5)
    torch.cuda.synchronize()
    c, o, b, br = c.cpu().numpy(), o.cpu().numpy(), b.cpu().numpy(), br.cpu().numpy()
    off = 0
    for k, t in enumerate((big, w.trees[0])):
        cost, obj, _ = paths.score_paths(t.pos_m, t.parent, gains[off:off + t.n], w.map.voxel_m, 0.5)
        _check_tree(c[off:off + t.n], o[off:off + t.n], int(b[k]), cost, obj)
        _check_branch(br[k], t.parent, int(b[k]))
        off += t.n
    for T in trees:
        T.close()
    M.close()
