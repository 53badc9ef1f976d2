"""GPU parity of the map conversion and updates (mg_map_create_tsdf, mg_map_update_tsdf,
mg_map_update, mg_map_read) against oracle/maps.py, byte for byte, and of evaluations on
converted and updated maps against evaluations on maps uploaded from the oracle's states."""
import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W
from oracle import maps
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


def _field(seed, dims):
    """TSDF-like field: random distances (metres), weights with unobserved regions, some values
    exactly at the thresholds and some NaNs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    d = rng.normal(0.3, 0.4, (nz, ny, nx)).astype(np.float32)
    w = rng.uniform(0, 3, (nz, ny, nx)).astype(np.float32)
    w[rng.uniform(size=w.shape) < 0.3] = 0.0
    flat_d, flat_w = d.reshape(-1), w.reshape(-1)
    k = flat_d.size
    flat_d[rng.choice(k, k // 50, replace=False)] = np.float32(0.05)      # surface threshold exactly
    flat_w[rng.choice(k, k // 50, replace=False)] = np.float32(1.0)       # minimum weight exactly
    flat_d[rng.choice(k, min(5, k), replace=False)] = np.nan
    flat_w[rng.choice(k, min(5, k), replace=False)] = np.nan
    return d, w


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dims", [(37, 21, 13), (64, 40, 17), (300, 9, 5), (8, 8, 8)])
def test_tsdf_conversion_matches_oracle(mg, dims):
    import torch
    d, w = _field(sum(dims), dims)
    ref = maps.tsdf_states(d, w, 0.05, 1.0)
    M = mg.Map.from_tsdf(_dev(d), _dev(w), 0.1, (0.0, 0.0, 0.0), surface_m=0.05, min_weight=1.0)
    got = M.read()
    torch.cuda.synchronize()
    log(f"[maps] tsdf {dims}: {np.bincount(ref.reshape(-1), minlength=3).tolist()}")
    assert np.array_equal(got.cpu().numpy(), ref)
    M.close()


def test_box_and_voxel_updates_match_oracle(mg):
    import torch
    dims = (45, 30, 22)
    d, w = _field(5, dims)
    ref = maps.tsdf_states(d, w, 0.05, 1.0)
    M = mg.Map.from_tsdf(_dev(d), _dev(w), 0.1, (0.0, 0.0, 0.0), surface_m=0.05, min_weight=1.0)
    for k, (lo, size) in enumerate([((3, 4, 5), (17, 9, 6)), ((0, 0, 0), (45, 30, 22)), ((44, 29, 21), (1, 1, 1)),
                                    ((10, 0, 3), (0, 5, 5))]):
        bd, bw = _field(100 + k, size)
        mg.mg_map_update_tsdf(M.handle, _dev(bd), _dev(bw), lo, -0.1, 0.5)
        ref = maps.apply_box(ref, lo, maps.tsdf_states(bd, bw, -0.1, 0.5))
        assert np.array_equal(M.read().cpu().numpy(), ref), (lo, size)
    rng = np.random.Generator(np.random.PCG64(9))
    nvox = int(np.prod(dims))
    ids = rng.choice(nvox + 50, 4000, replace=False).astype(np.uint32)     # some beyond the grid
    new = rng.integers(0, 4, ids.size).astype(np.uint8)                     # some invalid states
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    mg.mg_map_update(M.handle, _dev(ids.view(np.int32)), _dev(new), rej)
    ref, skipped = maps.apply_updates(ref, ids, new)
    torch.cuda.synchronize()
    assert np.array_equal(M.read().cpu().numpy(), ref)
    assert int(rej.item()) == skipped > 0
    bd, bw = _field(7, (2, 2, 2))
    with pytest.raises(mg.MGError):
        mg.mg_map_update_tsdf(M.handle, _dev(bd), _dev(bw), (44, 0, 0), -0.1, 0.5)   # leaves the grid
    M.close()


def test_evaluation_on_converted_and_updated_maps(mg):
    """A tree evaluated on a TSDF-built map, then after voxel updates, equals the same tree on maps
    uploaded from the oracle's states (gains, windows and depth buffers)."""
    import torch
    w = W.make("tiny")
    st = w.map.states
    rng = np.random.Generator(np.random.PCG64(21))
    # a TSDF whose conversion is exactly the tiny map: occupied -0.1, free 0.3, unknown weight 0
    dist = np.where(st == W.OCC, -0.1, 0.3).astype(np.float32)
    wgt = np.where(st == W.UNK, 0.0, 2.0).astype(np.float32)
    assert np.array_equal(maps.tsdf_states(dist, wgt, 0.0, 1.0), st)
    Mt = mg.Map.from_tsdf(_dev(dist), _dev(wgt), w.map.voxel_m, w.map.origin_m, surface_m=0.0, min_weight=1.0)
    Mu = mg.Map(st, w.map.voxel_m, w.map.origin_m)
    tree = w.trees[0]

    def evaluate(M):
        T = mg.Tree(M, tree.pos_m, tree.parent, w.sensor)
        g, y, d = T.eval_marginal(depth=True)
        torch.cuda.synchronize()
        out = (g.cpu().numpy(), y.cpu().numpy(), d.cpu().numpy())
        T.close()
        return out

    a, b = evaluate(Mt), evaluate(Mu)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    # unknown voxels observed as free or occupied between two replans
    unk = np.flatnonzero(st.reshape(-1) == W.UNK)
    ids = rng.choice(unk, unk.size // 3, replace=False).astype(np.uint32)
    new = rng.choice(np.array([W.FREE, W.OCC], np.uint8), ids.size, p=[0.9, 0.1])
    mg.mg_map_update(Mt.handle, _dev(ids.view(np.int32)), _dev(new))
    st2, _ = maps.apply_updates(st, ids, new)
    M2 = mg.Map(st2, w.map.voxel_m, w.map.origin_m)
    a2, b2 = evaluate(Mt), evaluate(M2)
    assert all(np.array_equal(x, y) for x, y in zip(a2, b2))
    assert a2[0].astype(np.int64).sum() < a[0].astype(np.int64).sum()      # less left unknown
    for M in (Mt, Mu, M2):
        M.close()


# ----------------------------------------------------------------- block marks

def _expected_marks(st):
    """The bytes mg_map_read_marked should return for states st [nz, ny, nx]: every unknown or
    free voxel carries the level of the largest aligned block around it that lies inside the grid
    and holds its state only (1: 16 voxels a side; 2: 8; 3: 4; 4: 2, free only)."""
    nz, ny, nx = st.shape
    level = np.zeros(st.shape, np.uint8)
    for edge, lv, states in ((2, 4, (W.FREE,)), (4, 3, (W.UNK, W.FREE)), (8, 2, (W.UNK, W.FREE)), (16, 1, (W.UNK, W.FREE))):
        bz, by, bx = nz // edge, ny // edge, nx // edge
        if min(bz, by, bx) == 0:
            continue
        blocks = st[:bz * edge, :by * edge, :bx * edge].reshape(bz, edge, by, edge, bx, edge)
        blocks = blocks.transpose(0, 2, 4, 1, 3, 5).reshape(bz, by, bx, -1)
        first = blocks[..., 0]
        uniform = (blocks == first[..., None]).all(-1) & np.isin(first, states)
        full = np.repeat(np.repeat(np.repeat(uniform, edge, 0), edge, 1), edge, 2)
        level[:bz * edge, :by * edge, :bx * edge][full] = lv
    return (st | (level << 2)).astype(np.uint8)


def _nested_states(seed, dims):
    from tests.test_gpu_parity import _nested_block_map
    return _nested_block_map(seed, dims).states


@pytest.mark.parametrize("case", ["nested48", "nested37", "step", "micro"])
def test_block_marks_are_the_largest_uniform_blocks(mg, case):
    """Every unknown and free voxel's mark names the largest aligned uniform block around it (the
    traversal crosses marked blocks in one step, so a missing mark costs time and a wrong one a
    wrong gain): after the map's upload, after listed updates that break and make blocks, after a
    whole-grid TSDF conversion."""
    import torch
    if case == "nested48":
        st = _nested_states(1248, (48, 48, 34))
    elif case == "nested37":
        st = _nested_states(1237, (37, 29, 21))
    elif case == "step":
        st = W.make("step").map.states
    else:
        st = W.random_micro(77, dims=(21, 18, 13), n_nodes=1, range_vox=6.0)[0].states
    st = np.ascontiguousarray(st, dtype=np.uint8)
    log(f"[marks] {case}: {st.shape}")
    M = mg.Map(st, 1.0, (0.0, 0.0, 0.0))
    try:
        got = M.read_marked().cpu().numpy()
        exp = _expected_marks(st)
        assert np.array_equal(got, exp), (case, int((got != exp).sum()))
        # updates: occupied voxels into free and unknown blocks, and a freed region
        rng = np.random.Generator(np.random.PCG64(5))
        nz, ny, nx = st.shape
        ids = rng.choice(st.size, size=min(200, st.size // 20), replace=False).astype(np.uint32)
        new = rng.choice(np.array([W.UNK, W.FREE, W.OCC], np.uint8), size=ids.size)
        z0, y0, x0 = 0, 0, 0
        box = np.arange(st.size, dtype=np.uint32).reshape(st.shape)[z0:z0 + 16, y0:y0 + 16, x0:x0 + 16].ravel()
        ids = np.concatenate([box, ids[~np.isin(ids, box)]])
        new = np.concatenate([np.full(box.size, W.FREE, np.uint8), new[:ids.size - box.size]])
        mg.mg_map_update(M.handle, torch.from_numpy(ids).cuda(), torch.from_numpy(new).cuda())
        st2 = st.copy().reshape(-1)
        st2[ids] = new
        st2 = st2.reshape(st.shape)
        got = M.read_marked().cpu().numpy()
        assert np.array_equal(got, _expected_marks(st2)), (case, "after updates", int((got != _expected_marks(st2)).sum()))
    finally:
        M.close()


def test_block_marks_after_tsdf_conversion(mg):
    """The whole-grid conversion takes the marks in its own pass (and the 16-voxel free blocks in a
    second): on a field of free space with box obstacles and unobserved slabs, the marks equal the
    largest uniform blocks of the converted states."""
    import torch
    nx, ny, nz = 72, 64, 40
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.full((nz, ny, nx), 1.0, np.float32)
    for cx, cy, cz, r in ((20, 20, 10, 5), (50, 40, 25, 7), (10, 50, 30, 3)):
        inside = (np.abs(x - cx) <= r) & (np.abs(y - cy) <= r) & (np.abs(z - cz) <= r)
        d[inside] = -0.5
    w = np.full((nz, ny, nx), 2.0, np.float32)
    w[:, :, 56:] = 0.0                      # an unobserved slab
    w[30:, :20, :] = 0.0
    M = mg.Map.from_tsdf(torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda(), 1.0, (0.0, 0.0, 0.0),
                         surface_m=0.0, min_weight=1.0)
    try:
        st = M.read().cpu().numpy()
        got = M.read_marked().cpu().numpy()
        exp = _expected_marks(st)
        assert (got & 3).tolist() == st.tolist()
        assert np.array_equal(got, exp), int((got != exp).sum())
        assert (exp >> 2 == 1).any() and (exp >> 2 == 2).any() and (exp >> 2 == 3).any()
    finally:
        M.close()
