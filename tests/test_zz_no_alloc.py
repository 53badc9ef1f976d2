"""GPU test of the allocation-free batch entry point (mg_eval_marginal_batch_noalloc): through the
C ABI, its gains, windows and depth buffers equal mg_eval_marginal_batch's, on two calls in a row (the
second with a smaller batch), on a batch over two maps with different voxel sizes, and after the
regular entry point ran in between; batches beyond its fixed scratch are refused."""
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


def _outs(mg, trees, fn):
    import torch
    n = sum(t.n for t in trees)
    g = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    y = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    d = torch.full((n, trees[0].pixels), -1.0, dtype=torch.float32, device="cuda")
    fn([t.handle for t in trees], g, y, d)
    torch.cuda.synchronize()
    return g.cpu(), y.cpu(), d.cpu()


def _same(a, b):
    import torch
    assert torch.equal(a[0], b[0]), "gains differ"
    assert torch.equal(a[1], b[1]), "yaw windows differ"
    assert a[2].numpy().tobytes() == b[2].numpy().tobytes(), "depth buffers differ"


def test_noalloc_batch_matches_regular_batch_twice(mg):
    w = W.make("batch64", n_trees=6)
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, w.sensor) for t in w.trees]
    log(f"[noalloc] 6 trees, {sum(t.n for t in trees)} nodes, then 2 trees")
    ref6 = _outs(mg, trees, mg.mg_eval_marginal_batch)
    got6 = _outs(mg, trees, mg.mg_eval_marginal_batch_noalloc)
    _same(got6, ref6)
    small = [trees[3], trees[0]]                  # the second call: a smaller batch, in another order
    ref2 = _outs(mg, small, mg.mg_eval_marginal_batch)
    got2 = _outs(mg, small, mg.mg_eval_marginal_batch_noalloc)
    _same(got2, ref2)
    _same(_outs(mg, trees, mg.mg_eval_marginal_batch_noalloc), ref6)   # and the larger one again
    for T in trees:
        T.close()
    M.close()


def test_noalloc_batch_over_two_maps_and_errors(mg):
    w = W.make("tiny")
    m2, t2, _ = W.random_micro(31, dims=(30, 28, 16), n_nodes=9, max_depth=3, range_vox=1.0)
    sen = w.sensor
    M1 = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    M2 = mg.Map(m2.states, 0.25, (0.0, 0.0, 0.0))
    trees = [mg.Tree(M1, w.trees[0].pos_m, w.trees[0].parent, sen),
             mg.Tree(M2, (t2.pos_m * np.float32(0.25)).astype(np.float32), t2.parent, sen)]
    log("[noalloc] two maps")
    _same(_outs(mg, trees, mg.mg_eval_marginal_batch_noalloc), _outs(mg, trees, mg.mg_eval_marginal_batch))
    with pytest.raises(mg.MGError) as e:
        _outs(mg, [trees[0], trees[0]], mg.mg_eval_marginal_batch_noalloc)
    assert e.value.code == mg.MG_E_INVALID
    # beyond the fixed scratch: 4097 tree handles are refused before anything is read
    import torch
    g = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(mg.MGError) as e:
        mg.mg_eval_marginal_batch_noalloc([trees[0].handle] * 4097, g, g)
    assert e.value.code == mg.MG_E_UNSUPPORTED
    for T in trees:
        T.close()
    M1.close()
    M2.close()


def test_noalloc_batch_refuses_a_batch_beyond_its_scratch(mg):
    """Two star trees of 2^20 nodes need 16 MiB of work lists alone (8 bytes per node), beyond the
    fixed scratch: refused with MG_E_UNSUPPORTED before any device work."""
    import torch
    st = np.full((8, 64, 64), W.FREE, np.uint8)
    M = mg.Map(st, 1.0, (0.0, 0.0, 0.0))
    sen = W.Sensor(n_az=16, n_el=4, fov_h_deg=90.0, fov_v_deg=60.0, range_m=3.0, yaw_bins=8)
    n = 1 << 20                                         # a star: 2^20 nodes, 8 MiB of items, 8 B of masks
    rng = np.random.Generator(np.random.PCG64(3))
    pos = rng.uniform(0.5, 7.5, (n, 3)).astype(np.float32)
    par = np.zeros(n, np.int32)
    par[0] = -1
    T1 = mg.Tree(M, pos, par, sen)
    T2 = mg.Tree(M, pos, par, sen)
    g = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(g)
    log("[noalloc] 2 x 2^20 nodes: 16 MiB of items, beyond the scratch")
    with pytest.raises(mg.MGError) as e:
        mg.mg_eval_marginal_batch_noalloc([T1.handle, T2.handle], g, y)
    assert e.value.code == mg.MG_E_UNSUPPORTED
    T1.close()
    T2.close()
    M.close()
