"""GPU parity of the exact hash-set marginal gain (mg_eval_exact) against the oracle's exact
pass (oracle/mgref.c, sorted voxel sets): X_ray, X_set and A_set at the depth-buffer method's
windows, integer-exact."""
import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from tests.gpu_util import log, threads

pytestmark = pytest.mark.gpu


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


def _check(mg, orc, m, tree, sen, label, mask=None):
    import torch
    M = mg.Map(m.states, m.voxel_m, m.origin_m)
    T = mg.Tree(M, tree.pos_m, tree.parent, sen)
    g, y, d = T.eval_marginal(depth=True)
    xr, xs, a = T.eval_exact(y)
    torch.cuda.synchronize()
    k = y.cpu().numpy()
    D = d.cpu().numpy().reshape(tree.n, sen.n_el, sen.w_buf)
    ref = orc.exact(m, tree, sen, k, D, mask=mask)
    sel = np.arange(tree.n) if mask is None else np.flatnonzero(mask)
    log(f"[exact] {label}: n={tree.n}, compared {sel.size}, X_ray sum {int(ref['X_ray'][sel].sum())}")
    for name, got in (("X_ray", xr), ("X_set", xs), ("A_set", a)):
        assert np.array_equal(mg.as_u32(got)[sel], ref[name][sel]), name
    T.close()
    M.close()
    return ref


def test_exact_tiny(mg, orc):
    w = W.make("tiny")
    ref = _check(mg, orc, w.map, w.trees[0], w.sensor, "tiny")
    assert ref["X_set"][0] == ref["A_set"][0]                  # the root has no ancestors


@pytest.mark.parametrize("seed", range(3))
def test_exact_random_micro(mg, orc, seed):
    sens = [dict(n_az=16, n_el=6, yaw_bins=8), dict(n_az=100, n_el=7, yaw_bins=36),
            dict(n_az=24, n_el=5, yaw_bins=12)]
    m, tree, sen = W.random_micro(800 + seed, dims=(17, 13, 9), n_nodes=12, max_depth=4, range_vox=9.0,
                                  p_occ=0.06, p_free=0.45, **sens[seed])
    _check(mg, orc, m, tree, sen, f"micro{seed}")


@pytest.mark.parametrize("dims", [(40, 32, 24), (37, 29, 21)])
def test_exact_nested_blocks(mg, orc, dims):
    """Maps of nested aligned blocks (free blocks of every size crossed in one step by the device's
    walk, wholly unknown ones walked voxel by voxel; some blocks reach past the grid) against the
    oracle's voxel-by-voxel sets: nodes on block corners, edges and faces, 45-degree rays whose
    boundary parameters tie, an integer range."""
    from tests.test_gpu_parity import _nested_block_map
    m = _nested_block_map(1400 + dims[0], dims)
    pos = np.array([[8.0, 8.0, 8.0], [16.0, 16.0, 8.0], [12.0, 12.0, 4.0], [24.0, 8.0, 16.0], [10.0, 14.0, 6.0],
                    [16.0, 8.0, 4.5], [9.5, 17.0, 8.0], [30.0, 22.0, 14.0], [4.25, 20.75, 19.5], [20.0, 20.0, 10.0]],
                   np.float32)
    tree = W.Tree(pos_m=pos, parent=np.array([-1, 0, 0, 1, 1, 2, 3, 4, 6, 8], np.int32))
    for sen in (W.Sensor(n_az=8, n_el=3, fov_h_deg=90, fov_v_deg=90, range_m=30.0, yaw_bins=8, az_offset_deg=-22.5),
                W.Sensor(n_az=100, n_el=17, fov_h_deg=90, fov_v_deg=80, range_m=13.7, yaw_bins=20)):
        ref = _check(mg, orc, m, tree, sen, f"nested blocks {dims} {sen.n_az}x{sen.n_el}")
        assert int(ref["X_ray"].sum()) > 0


def test_exact_step_sampled(mg, orc):
    w = W.make("step")
    t = w.trees[0]
    dep = t.depth()
    leaves = np.flatnonzero(dep == dep.max())[:3]
    mask = orc.ancestor_closure(t.parent, leaves)
    _check(mg, orc, w.map, t, w.sensor, "step", mask=mask)


def test_exact_rejects_bad_windows(mg):
    import torch
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    T = mg.Tree(M, w.trees[0].pos_m, w.trees[0].parent, w.sensor)
    y = torch.full((T.n,), w.sensor.yaw_bins, dtype=torch.int32, device="cuda")
    with pytest.raises(mg.MGError):
        T.eval_exact(y)
    T.close()
    M.close()


def test_exact_deepest_chain(mg, orc):
    """A 64-node chain: the last node probes 63 ancestors' sets."""
    w = W.make("tiny")
    p = w.trees[0].pos_m
    chain_pos = np.repeat(p[:4], 17, axis=0)[:64] + np.float32(0.013) * np.arange(64, dtype=np.float32)[:, None]
    chain_pos = np.clip(chain_pos, 0.05, w.map.extent_m.astype(np.float32) - 0.05).astype(np.float32)
    chain = W.Tree(pos_m=chain_pos, parent=np.arange(-1, 63, dtype=np.int32))
    _check(mg, orc, w.map, chain, w.sensor, "chain63")


def _check_own_yaw(mg, orc, m, tree, sen, label, mask=None):
    import torch
    M = mg.Map(m.states, m.voxel_m, m.origin_m)
    T = mg.Tree(M, tree.pos_m, tree.parent, sen)
    g, y = T.eval_exact_marginal()
    torch.cuda.synchronize()
    ref = orc.exact_marginal(m, tree, sen, mask=mask)
    sel = np.arange(tree.n) if mask is None else np.flatnonzero(mask)
    log(f"[exact] own yaw {label}: n={tree.n}, compared {sel.size}")
    assert np.array_equal(mg.as_u32(g)[sel], ref["g_ex"][sel])
    assert np.array_equal(y.cpu().numpy()[sel], ref["k_ex"][sel])
    T.close()
    M.close()


@pytest.mark.parametrize("case", ["tiny", "micro0", "micro1", "chain"])
def test_exact_own_yaw(mg, orc, case):
    w = W.make("tiny")
    if case == "tiny":
        m, tree, sen = w.map, w.trees[0], w.sensor
    elif case == "chain":
        p = w.trees[0].pos_m
        cp = np.repeat(p[:4], 17, axis=0)[:64] + np.float32(0.013) * np.arange(64, dtype=np.float32)[:, None]
        cp = np.clip(cp, 0.05, w.map.extent_m.astype(np.float32) - 0.05).astype(np.float32)
        m, tree, sen = w.map, W.Tree(pos_m=cp, parent=np.arange(-1, 63, dtype=np.int32)), w.sensor
    else:
        k = int(case[-1])
        m, tree, sen = W.random_micro(820 + k, dims=(17, 13, 9), n_nodes=12, max_depth=4, range_vox=9.0,
                                      p_occ=0.06, p_free=0.45, n_az=[16, 100][k], n_el=[6, 7][k],
                                      yaw_bins=[8, 36][k])
    _check_own_yaw(mg, orc, m, tree, sen, case)


def test_exact_own_yaw_step_sampled(mg, orc):
    w = W.make("step")
    t = w.trees[0]
    dep = t.depth()
    mask = orc.ancestor_closure(t.parent, np.flatnonzero(dep == dep.max())[:2])
    _check_own_yaw(mg, orc, w.map, t, w.sensor, "step", mask=mask)
