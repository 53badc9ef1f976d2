"""Oracle of the path score (test infrastructure only; eq. 3 and eq. 4).

For every node n of a tree, parents before children:

    c(root) = 0,   c(n) = c(Pa(n)) + |p_n - p_Pa(n)|          (eq. 3, metres)
    o(root) = g(root),   o(n) = o(Pa(n)) + g(n) exp(-lambda c(n))  (eq. 4)

where g(n) is the node's marginal gain as a volume: its count of unknown-voxel
incidences times the voxel volume v^3 (eq. 2 is a volume). The best branch
ends at the node of largest o (smallest id among equal values); the branch is
that node's root path. All arithmetic in float64 on the float32 positions.
"""
from __future__ import annotations

import math

import numpy as np


def score_paths(pos_m, parent, gain_counts, voxel_m, lam):
    """(cost [n], objective [n], best node) of one tree, by the recursion above."""
    pos = np.asarray(pos_m, dtype=np.float32).astype(np.float64)
    par = np.asarray(parent, dtype=np.int64)
    g = np.asarray(gain_counts, dtype=np.uint32).astype(np.float64)
    v = float(np.float32(voxel_m))
    vox3 = v * v * v
    n = len(par)
    cost = np.zeros(n, np.float64)
    obj = np.zeros(n, np.float64)
    for i in range(n):
        p = par[i]
        if p < 0:
            cost[i] = 0.0
            obj[i] = g[i] * vox3
            continue
        d = pos[i] - pos[p]
        cost[i] = cost[p] + math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        obj[i] = obj[p] + g[i] * vox3 * math.exp(-lam * cost[i])
    best = int(np.argmax(obj))       # first index of the maximum
    return cost, obj, best


def branch(parent, node):
    """Root-to-node path of `node` (node ids)."""
    out = []
    while node >= 0:
        out.append(int(node))
        node = int(parent[node])
    return out[::-1]
