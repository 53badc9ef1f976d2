"""GPU tests of the serving loop (mg_server_*): continuous batching must not
change any result. Each request's gains and yaw windows are compared with a
plain mg_eval_marginal of the same tree, alone and in a mix, under a small
arena (admission waits for memory), with one request in flight at a time, and
with invalid requests rejected without disturbing the others. Requests failed
through their device status word, and cancelled ones, queued or in flight,
end with their own status while the others complete bit-identically."""
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


@pytest.fixture(scope="module")
def scene(mg):
    """Two maps with different voxel sizes and six trees, one sensor geometry."""
    import torch
    w = W.make("batch64", n_trees=4)
    m2, t2, _ = W.random_micro(41, dims=(40, 36, 20), n_nodes=30, max_depth=5, range_vox=1.0)
    sen = w.sensor
    M1 = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    M2 = mg.Map(m2.states, 0.2, (0.0, 0.0, 0.0))
    reqs = [(M1, t.pos_m, t.parent) for t in w.trees]
    reqs.append((M2, (t2.pos_m * np.float32(0.2)).astype(np.float32), t2.parent))
    reqs.append((M1, w.trees[0].pos_m[:1].copy(), np.array([-1], np.int32)))
    ref = []
    for M, pos, par in reqs:
        T = mg.Tree(M, pos, par, sen)
        g, y, _ = T.eval_marginal()
        torch.cuda.synchronize()
        ref.append((mg.as_u32(g), y.cpu().numpy()))
        T.close()
    log(f"[serve] {len(reqs)} requests, nodes {[len(p) for _, _, p in reqs]}")
    return sen, reqs, ref, (M1, M2)


def _check(res, ref):
    for i, ((g, y), (rg, ry)) in enumerate(zip(res, ref)):
        assert np.array_equal(g, rg), f"gain of request {i}"
        assert np.array_equal(y, ry), f"yaw of request {i}"


def test_alone_and_mixed_are_identical(mg, scene):
    sen, reqs, ref, _ = scene
    S = mg.Server(sen, max_inflight=8, arena_bytes=4 << 30)
    alone = []
    for M, pos, par in reqs:
        t = S.submit(M, pos, par)
        g, y, lat = S.wait(t)
        alone.append((g, y))
    _check(alone, ref)
    tickets = [S.submit(M, pos, par) for M, pos, par in reqs]
    mixed = [S.wait(t)[:2] for t in tickets]
    _check(mixed, ref)
    st = S.stats()
    assert st["completed"] == 2 * len(reqs) and st["in_flight"] == 0 and st["queued"] == 0
    S.close()


def test_small_arena_and_single_slot(mg, scene):
    sen, reqs, ref, _ = scene
    # room for roughly the largest tree only: admission must wait for memory
    biggest = 0
    for M, pos, par in reqs:
        T = mg.Tree(M, pos, par, sen)
        biggest = max(biggest, T.footprint_bytes)
        T.close()
    S = mg.Server(sen, max_inflight=8, arena_bytes=int(biggest * 1.3) + (1 << 20))
    tickets = [S.submit(M, pos, par) for M, pos, par in reqs]
    _check([S.wait(t)[:2] for t in tickets], ref)
    S.close()
    S1 = mg.Server(sen, max_inflight=1, arena_bytes=2 << 30)
    tickets = [S1.submit(M, pos, par) for M, pos, par in reqs]
    got = []
    for t in tickets:
        while True:
            r = S1.poll(t)
            if r is not None:
                got.append(r[:2])
                break
    _check(got, ref)
    S1.close()


def test_bad_requests_do_not_disturb_others(mg, scene):
    sen, reqs, ref, (M1, _) = scene
    S = mg.Server(sen, max_inflight=4, arena_bytes=1 << 30)
    tickets = []
    for i, (M, pos, par) in enumerate(reqs):
        tickets.append(S.submit(M, pos, par))
        if i == 1:
            bad = par.copy()
            bad[-1] = len(bad) + 3                  # parent after the child
            with pytest.raises(mg.MGError) as e:
                S.submit(M, pos, bad)
            assert e.value.code == mg.MG_E_INVALID
            outside = pos.copy()
            outside[0, 0] = -5.0
            with pytest.raises(mg.MGError):
                S.submit(M, outside, par)
    tiny = mg.Server(sen, max_inflight=2, arena_bytes=4096)
    with pytest.raises(mg.MGError) as e:
        tiny.submit(M1, reqs[0][1], reqs[0][2])
    assert e.value.code == mg.MG_E_NOMEM
    tiny.close()
    _check([S.wait(t)[:2] for t in tickets], ref)
    S.close()


def test_map_updates_are_ordered_with_requests(mg):
    """Requests submitted before a map update see the old map, those after it the new one,
    whatever is in flight; each equals a plain evaluation on a map uploaded with that content."""
    import torch
    from oracle import maps
    w = W.make("tiny")
    sen = w.sensor
    st0 = w.map.states
    rng = np.random.Generator(np.random.PCG64(77))
    unk = np.flatnonzero(st0.reshape(-1) == W.UNK)
    ids1 = rng.choice(unk, unk.size // 4, replace=False).astype(np.uint32)
    new1 = rng.choice(np.array([W.FREE, W.OCC], np.uint8), ids1.size, p=[0.85, 0.15])
    st1, _ = maps.apply_updates(st0, ids1, new1)
    ids2 = rng.choice(st0.size, 3000, replace=False).astype(np.uint32)
    new2 = rng.integers(0, 3, ids2.size).astype(np.uint8)
    st2, _ = maps.apply_updates(st1, ids2, new2)
    t0 = w.trees[0]
    trees = [(t0.pos_m, t0.parent), (t0.pos_m[:7].copy(), t0.parent[:7].copy())]

    def plain(states, pos, par):
        M = mg.Map(states, w.map.voxel_m, w.map.origin_m)
        T = mg.Tree(M, pos, par, sen)
        g, y, _ = T.eval_marginal()
        torch.cuda.synchronize()
        out = (mg.as_u32(g), y.cpu().numpy())
        T.close()
        M.close()
        return out

    expect = {k: [plain(s, *tr) for tr in trees] for k, s in ((0, st0), (1, st1), (2, st2))}
    Ms = mg.Map(st0, w.map.voxel_m, w.map.origin_m)
    S = mg.Server(sen, max_inflight=3, arena_bytes=1 << 30)
    plan = [("req", 0), ("req", 1), ("upd", (ids1, new1)), ("req", 0), ("req", 1), ("req", 0),
            ("upd", (ids2, new2)), ("req", 1), ("req", 0)]
    version, tickets = 0, []
    for kind, arg in plan:
        if kind == "upd":
            tickets.append(("upd", S.map_update(Ms, *arg), None))
            version += 1
        else:
            tickets.append(("req", S.submit(Ms, *trees[arg]), (version, arg)))
    for kind, t, info in tickets:
        if kind == "upd":
            S.wait(t)
            continue
        g, y, _ = S.wait(t)
        eg, ey = expect[info[0]][info[1]]
        assert np.array_equal(g, eg) and np.array_equal(y, ey), info
    with pytest.raises(mg.MGError):
        S.map_update(Ms, np.array([st0.size], np.uint32), np.array([1], np.uint8))
    S.close()
    Ms.close()


def test_update_holds_back_only_requests_on_its_map(mg):
    """With the server paused, a request on map A is admitted; an update of A queued next cannot be
    applied while that request is in flight. A request on map B queued behind the update is admitted
    at once (the update does not hold back other maps), a later request on A stays queued behind the
    update. After resuming, the first request on A sees the old map, the later one the updated map,
    and the request on B its own map."""
    import time
    import torch
    from oracle import maps
    w = W.make("tiny")
    sen = w.sensor
    st0 = w.map.states
    rng = np.random.Generator(np.random.PCG64(91))
    unk = np.flatnonzero(st0.reshape(-1) == W.UNK)
    ids = rng.choice(unk, unk.size // 3, replace=False).astype(np.uint32)
    new = rng.choice(np.array([W.FREE, W.OCC], np.uint8), ids.size, p=[0.85, 0.15])
    st1, _ = maps.apply_updates(st0, ids, new)
    stb = st0.copy()
    stb.reshape(-1)[rng.choice(unk, unk.size // 5, replace=False)] = W.FREE
    t0 = w.trees[0]

    def plain(states):
        M = mg.Map(states, w.map.voxel_m, w.map.origin_m)
        T = mg.Tree(M, t0.pos_m, t0.parent, sen)
        g, y, _ = T.eval_marginal()
        torch.cuda.synchronize()
        out = (mg.as_u32(g), y.cpu().numpy())
        T.close()
        M.close()
        return out

    e0, e1, eb = plain(st0), plain(st1), plain(stb)
    MA = mg.Map(st0, w.map.voxel_m, w.map.origin_m)
    MB = mg.Map(stb, w.map.voxel_m, w.map.origin_m)
    S = mg.Server(sen, max_inflight=4, arena_bytes=1 << 30)
    S.pause(True)
    ra1 = S.submit(MA, t0.pos_m, t0.parent)
    upd = S.map_update(MA, ids, new)
    rb = S.submit(MB, t0.pos_m, t0.parent)
    ra2 = S.submit(MA, t0.pos_m, t0.parent)
    for _ in range(2000):                       # admission runs while paused
        st = S.stats()
        if st["in_flight"] == 2:
            break
        time.sleep(0.005)
    assert st["in_flight"] == 2 and st["queued"] == 2 and st["steps"] == 0, st
    S.pause(False)
    for t, e in ((ra1, e0), (rb, eb), (ra2, e1)):
        g, y, _ = S.wait(t)
        assert np.array_equal(g, e[0]) and np.array_equal(y, e[1])
    S.wait(upd)
    S.close()
    MB.close()
    MA.close()


def test_served_robot_maps_against_oracle(mg):
    """The serving workload's own requests (robot maps at 0.05, 0.1 and 0.2 m, trees of 167-1751
    nodes, depth 3-10) submitted together to a 16-slot server; in each request the ancestor chains of
    two deepest leaves are compared with the oracle (gains and windows)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import mgref
    from tests.gpu_util import threads
    reqs = W.serve_requests(64)
    pick = [0, 1, 2, 3, 5, 6]                  # voxel sizes 0.1, 0.05, 0.05, 0.1, 0.2, 0.2
    robots = sorted({reqs[i][1] for i in pick})
    maps = {r: W.make_robot(r) for r in robots}
    assert {maps[reqs[i][1]][0].voxel_m for i in pick} == {0.05, 0.1, 0.2}
    sen = W.Sensor(**W.SENSOR_STEP)
    trees = [W.make_rrt(reqs[i][2], maps[reqs[i][1]][0], maps[reqs[i][1]][1][-1], reqs[i][3], reqs[i][4])
             for i in pick]
    dev = {r: mg.Map(maps[r][0].states, maps[r][0].voxel_m, maps[r][0].origin_m) for r in robots}
    log(f"[serve] oracle parity: {len(pick)} requests, nodes {[t.n for t in trees]}")
    S = mg.Server(sen, max_inflight=16, arena_bytes=16 << 30)
    tickets = [S.submit(dev[reqs[i][1]], t.pos_m, t.parent) for i, t in zip(pick, trees)]
    got = [S.wait(tk)[:2] for tk in tickets]
    S.close()
    jobs = []
    for i, t in zip(pick, trees):
        dep = t.depth()
        leaves = np.flatnonzero(dep == dep.max())[:2]
        jobs.append((maps[reqs[i][1]][0], t, mgref.ancestor_closure(t.parent, leaves)))
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        refs = list(ex.map(lambda j: mgref.eval_tree(j[0], j[1], sen, mask=j[2], n_threads=1), jobs))
    for (g, y), ref, (_, _, mask) in zip(got, refs, jobs):
        sel = np.flatnonzero(mask)
        assert np.array_equal(g[sel].astype(np.int64), ref["g_db"][sel].astype(np.int64))
        assert np.array_equal(y[sel], ref["k_db"][sel])
    for M in dev.values():
        M.close()


def test_map_held_by_pending_requests(mg):
    """A map with queued or in-flight server work refuses to be destroyed (MG_E_BUSY) until that work
    has finished; a ticket retired by one caller is unknown to the next."""
    w = W.make("tiny")
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    S = mg.Server(w.sensor, max_inflight=2, arena_bytes=1 << 30)
    t = w.trees[0]
    tickets = [S.submit(M, t.pos_m, t.parent) for _ in range(3)]
    upd = S.map_update(M, np.array([0], np.uint32), np.array([w.map.states.reshape(-1)[0]], np.uint8))
    with pytest.raises(mg.MGError) as e:
        M.close()
    assert e.value.code == mg.MG_E_BUSY
    for tk in tickets:
        S.wait(tk)
    S.wait(upd)
    with pytest.raises(mg.MGError) as e:
        S.wait(tickets[0])
    assert e.value.code == mg.MG_E_INVALID
    S.close()
    M.close()


def _status(mg, S, t):
    """The request's final status code (0 on success)."""
    try:
        S.wait(t)
        return 0
    except mg.MGError as e:
        return e.code


def test_failed_and_cancelled_requests_leave_the_others_intact(mg, scene):
    """Six requests with two slots, the server paused so that the first two are admitted and
    the rest stay queued: an in-flight request marked failed through its device status word,
    an in-flight one cancelled, a queued one cancelled, a queued one marked failed (marked when
    it is admitted) and two untouched ones. After resuming, the failed and cancelled requests
    report their status with outputs unwritten, and the untouched ones equal the plain path."""
    sen, reqs, ref, _ = scene
    S = mg.Server(sen, max_inflight=2, arena_bytes=4 << 30)
    S.pause(True)
    order = [0, 1, 2, 3, 4, 5]
    tickets = [S.submit(*reqs[i]) for i in order]
    for _ in range(2000):                       # admission runs while paused
        st = S.stats()
        if st["in_flight"] == 2:
            break
        __import__("time").sleep(0.005)
    assert st["in_flight"] == 2 and st["queued"] == 4 and st["steps"] == 0, st
    outs = {t: S._keep[t] for t in tickets}
    S.fail_request(tickets[0], mg.MG_E_DEVICE)  # in flight: device status word
    S.cancel(tickets[1])                        # in flight: dropped at the next step boundary
    S.cancel(tickets[3])                        # queued: dropped at once
    S.fail_request(tickets[4], mg.MG_E_UNSUPPORTED)   # queued: marked when admitted
    log("[serve] failed/cancelled: resuming")
    S.pause(False)
    codes = [_status(mg, S, t) for t in tickets]
    assert codes == [mg.MG_E_DEVICE, mg.MG_E_CANCELLED, 0, mg.MG_E_CANCELLED, mg.MG_E_UNSUPPORTED, 0], codes
    for k in (0, 1, 3, 4):                      # outputs of failed or cancelled requests are not written
        g, y = outs[tickets[k]]
        assert not g.any() and not y.any(), k
    for k in (2, 5):
        g, y = outs[tickets[k]]
        assert np.array_equal(g, ref[order[k]][0]) and np.array_equal(y, ref[order[k]][1]), k
    with pytest.raises(mg.MGError) as ei:       # retired tickets are unknown
        S.cancel(tickets[2])
    assert ei.value.code == mg.MG_E_INVALID
    # the server keeps serving: the same requests again, untouched, are identical
    again = [S.submit(*reqs[i]) for i in order]
    _check([S.wait(t)[:2] for t in again], [ref[i] for i in order])
    st = S.stats()
    assert st["completed"] == 8 and st["in_flight"] == 0 and st["queued"] == 0
    S.close()
