"""Pins of the path-score oracle (eq. 3 traversal cost, eq. 4 exponential objective).

Each test checks the recursion against something it does not compute itself:
closed forms on chains and stars, sums over explicit root paths, the
crossover of two branches as lambda grows, and the tie rule. A dropped term,
a sign flip in the exponent, the parent's cost used in place of the node's,
or a wrong parent index fails one of them.
"""
import math

import numpy as np
import pytest

from oracle import paths


def _chain(k, d):
    pos = np.zeros((k, 3), np.float32)
    pos[:, 0] = np.arange(k, dtype=np.float32) * np.float32(d)
    return pos, np.arange(-1, k - 1, dtype=np.int32)


@pytest.mark.parametrize("lam", [0.0, 0.5, 2.0])
def test_chain_closed_form(lam):
    """Straight chain of equal steps d and equal gain g: c(i) = i d and o(i) is a geometric sum."""
    k, d, g, v = 12, 0.5, 37, 0.25
    pos, par = _chain(k, d)
    cost, obj, best = paths.score_paths(pos, par, np.full(k, g, np.uint32), v, lam)
    assert np.array_equal(cost, np.arange(k) * d)
    r = math.exp(-lam * d)
    for i in range(k):
        ref = g * v ** 3 * ((i + 1) if lam == 0 else (1 - r ** (i + 1)) / (1 - r))
        assert obj[i] == pytest.approx(ref, rel=1e-12)
    assert best == k - 1                  # every step adds a positive term


def test_star_closed_form():
    """Root with children at integer (Pythagorean) offsets: c = |offset| exactly."""
    offs = np.array([[0, 0, 0], [3, 4, 0], [0, 5, 12], [2, 3, 6], [-8, 0, 15]], np.float32)
    root = np.array([10.0, 10.0, 10.0], np.float32)
    pos = offs + root
    par = np.array([-1, 0, 0, 0, 0], np.int32)
    g = np.array([100, 40, 90, 25, 300], np.uint32)
    lam, v = 0.5, 0.1
    cost, obj, best = paths.score_paths(pos, par, g, v, lam)
    assert np.array_equal(cost, [0.0, 5.0, 13.0, 7.0, 17.0])
    vv = float(np.float32(v)) ** 3
    ref = g[0] * vv + g * vv * np.exp(-lam * np.array([0.0, 5.0, 13.0, 7.0, 17.0]))
    ref[0] = g[0] * vv
    assert np.allclose(obj, ref, rtol=1e-13, atol=0)
    assert best == int(np.argmax(ref))


def _random_tree(seed, n=60, max_depth=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    par = np.full(n, -1, np.int32)
    dep = np.zeros(n, np.int32)
    pos = np.zeros((n, 3), np.float32)
    pos[0] = rng.uniform(0, 20, 3)
    for i in range(1, n):
        cand = [j for j in range(i) if dep[j] < max_depth]
        par[i] = rng.choice(cand)
        dep[i] = dep[par[i]] + 1
        pos[i] = pos[par[i]] + rng.normal(0, 1.5, 3).astype(np.float32)
    g = rng.integers(0, 5000, n).astype(np.uint32)
    return pos, par, g


@pytest.mark.parametrize("seed", range(4))
def test_sums_over_explicit_root_paths(seed):
    """c(n) is the length of the polyline root..n; o(n) sums g(m) v^3 exp(-lam c(m)) over that path."""
    pos, par, g = _random_tree(seed)
    v, lam = 0.2, 0.7
    cost, obj, best = paths.score_paths(pos, par, g, v, lam)
    vv = float(np.float32(v)) ** 3
    for n in range(len(par)):
        br = paths.branch(par, n)
        assert br[0] == 0 and br[-1] == n
        assert all(par[b] == a for a, b in zip(br, br[1:]))
        seg = np.diff(pos[br].astype(np.float64), axis=0)
        lens = np.linalg.norm(seg, axis=1)
        cs = np.concatenate([[0.0], np.cumsum(lens)])
        assert cost[n] == pytest.approx(cs[-1], rel=1e-12, abs=1e-12)
        assert obj[n] == pytest.approx(float(np.sum(g[br] * vv * np.exp(-lam * cs))), rel=1e-12)
    # lambda = 0: the objective is the branch's summed gain volume (exact with v a power of two)
    _, obj0, _ = paths.score_paths(pos, par, g, 0.25, 0.0)
    for n in range(len(par)):
        assert obj0[n] == float(np.sum(g[paths.branch(par, n)], dtype=np.int64)) * 0.25 ** 3
    assert best == int(np.flatnonzero(obj == obj.max())[0])


def test_crossover_between_a_near_and_a_far_branch():
    """Two children of the root: the far one wins below lam* = ln(g_far / g_near) / (d_far - d_near)."""
    pos = np.array([[5, 5, 5], [7, 5, 5], [5, 5, 11]], np.float32)       # d_near = 2, d_far = 6
    par = np.array([-1, 0, 0], np.int32)
    g = np.array([0, 100, 1000], np.uint32)
    lam_star = math.log(1000 / 100) / (6 - 2)
    assert paths.score_paths(pos, par, g, 1.0, lam_star * 0.99)[2] == 2
    assert paths.score_paths(pos, par, g, 1.0, lam_star * 1.01)[2] == 1


def test_ties_pick_the_smallest_id():
    """Mirror-image leaves tie; a zero-gain child ties its parent, and the parent (smaller id) wins."""
    pos = np.array([[5, 5, 5], [6, 5, 5], [4, 5, 5]], np.float32)
    par = np.array([-1, 0, 0], np.int32)
    assert paths.score_paths(pos, par, np.array([1, 7, 7], np.uint32), 0.5, 0.5)[2] == 1
    pos = np.array([[5, 5, 5], [6, 5, 5], [7, 5, 5]], np.float32)
    par = np.array([-1, 0, 1], np.int32)
    cost, obj, best = paths.score_paths(pos, par, np.array([1, 7, 0], np.uint32), 0.5, 0.5)
    assert obj[2] == obj[1] and best == 1


@pytest.mark.parametrize("seed", range(3))
def test_invariants(seed):
    """Along every edge: cost grows by the edge length, objective never decreases, and is bounded
    by the undiscounted gain volume of the branch."""
    pos, par, g = _random_tree(100 + seed)
    cost, obj, _ = paths.score_paths(pos, par, g, 0.5, 0.5)
    vv = float(np.float32(0.5)) ** 3
    for n in range(1, len(par)):
        p = par[n]
        assert cost[n] >= cost[p] and obj[n] >= obj[p]
        assert obj[n] <= float(np.sum(g[paths.branch(par, n)], dtype=np.int64)) * vv * (1 + 1e-12)
    assert cost[0] == 0.0 and obj[0] == g[0] * vv
