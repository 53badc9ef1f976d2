"""Error of the depth-buffer marginal gain against the exact gain (oracle only).

For each node: G_db (depth-buffer marginal, incidences), X_ray (exact
set-difference marginal of eq. 2 counted per ray incidence, at the same yaw
window, Sec. V-A's fixed-yaw protocol), X_set (eq. 2 as a set), G_abs
(absolute) and g_sp (single-parent conditioning). Reports, per depth, the mean
ratios G_db/X_ray, G_sp/X_ray and G_abs/X_ray (the analogue of Fig. 4b), and
over all nodes the least-squares slope (through the origin) and R^2 of G_db
against X_ray (the statistic form of Sec. V-A). The same statistics are
reported for the interval mode (oracle/ivlref.c: pinhole buffers and overlap
intervals, the paper's own test), against X_ray at the interval mode's own
windows. Test infrastructure: calls only the oracle and the workload
generator.

The exact pass covers every node of tiny and step and seeded node
subsamples (with their ancestor chains) of batch64, large and serve16.

Usage: python oracle/error_report.py [workload ...] > report.json
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import ivlref, mgref  # noqa: E402
from paper_2609_40297_amd import workloads as W  # noqa: E402


def _compare(rows):
    """Statistics over (depth, G_db, X_ray, g_sp, G_abs, G_db_set, X_set) rows of compared nodes."""
    dep, g, x, sp, ab, gs, xs = (np.asarray(c, dtype=np.float64) for c in zip(*rows))
    sel = x > 0
    slope = float(np.sum(g[sel] * x[sel]) / np.sum(x[sel] * x[sel]))
    resid = g[sel] - slope * x[sel]
    r2 = float(1.0 - np.sum(resid ** 2) / np.sum((g[sel] - g[sel].mean()) ** 2))
    per_depth = []
    for d in range(int(dep.max()) + 1):
        m = (dep == d) & sel
        if not m.any():
            continue
        per_depth.append(dict(depth=d, nodes=int(m.sum()),
                              db_over_exact=float(np.mean(g[m] / x[m])),
                              sp_over_exact=float(np.mean(sp[m] / x[m])),
                              abs_over_exact=float(np.mean(ab[m] / x[m])),
                              dbset_over_exactset=float(np.mean(gs[m] / np.maximum(xs[m], 1)))))
    return dict(compared=int(sel.sum()), slope=slope, r2=r2, mean_db_over_exact=float(np.mean(g[sel] / x[sel])),
                overestimate_pct=float(100.0 * (np.sum(g[sel]) / np.sum(x[sel]) - 1.0)), per_depth=per_depth)


def _fit(dep, g, x):
    """Slope through the origin, R^2 and per-depth mean ratio of g against x (nodes with x > 0)."""
    dep, g, x = (np.asarray(c, dtype=np.float64) for c in (dep, g, x))
    sel = x > 0
    slope = float(np.sum(g[sel] * x[sel]) / np.sum(x[sel] * x[sel]))
    resid = g[sel] - slope * x[sel]
    r2 = float(1.0 - np.sum(resid ** 2) / np.sum((g[sel] - g[sel].mean()) ** 2))
    per_depth = [dict(depth=d, nodes=int(((dep == d) & sel).sum()),
                      over_exact=float(np.mean(g[(dep == d) & sel] / x[(dep == d) & sel])))
                 for d in range(int(dep.max()) + 1) if ((dep == d) & sel).any()]
    return dict(compared=int(sel.sum()), slope=slope, r2=r2,
                overestimate_pct=float(100.0 * (np.sum(g[sel]) / np.sum(x[sel]) - 1.0)), per_depth=per_depth)


def _interval_rows(m, t, sensor, mask, n_threads):
    """(depth, G_ivl, X_ray at the interval mode's windows) of the nodes in `mask` or all."""
    ivl = ivlref.eval_tree(m, t, sensor, mask=mask, n_threads=n_threads)
    blind = np.zeros((t.n, sensor.n_el, sensor.w_buf), np.float32)
    ex = mgref.exact(m, t, sensor, ivl["k_db"], blind, mask=mask)
    dep = t.depth()
    idx = np.arange(t.n) if mask is None else np.nonzero(mask)[0]
    return [(dep[i], ivl["g_db"][i], ex["X_ray"][i]) for i in idx], (ivl["wd"], ivl["hd"])


def _tree_rows(m, t, sensor, mask, n_threads):
    """Depth-buffer, single-parent and exact quantities of the nodes in `mask` (ancestor-closed) or all."""
    full = mgref.eval_tree(m, t, sensor, mask=mask, n_threads=n_threads)
    sp = mgref.eval_tree(m, t, sensor, max_anc=1, mask=mask, n_threads=n_threads)
    ex = mgref.exact(m, t, sensor, full["k_db"], full["D"], mask=mask)
    dep = t.depth()
    idx = np.arange(t.n) if mask is None else np.nonzero(mask)[0]
    return [(dep[i], full["g_db"][i], ex["X_ray"][i], sp["g_db"][i], full["g_abs"][i], ex["G_db_set"][i],
             ex["X_set"][i]) for i in idx]


def _sample_mask(t, k, seed):
    """k seeded uniform nodes of tree t and all their ancestors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nodes = rng.choice(t.n, size=min(k, t.n), replace=False)
    return mgref.ancestor_closure(t.parent, [int(i) for i in nodes])


# Exact pass on every node for the small workloads, on seeded node subsamples
# (plus their ancestor chains) for the large ones: (trees used, sampled nodes per tree).
PLANS = {"tiny": (1, None), "step": (1, None), "batch64": (8, 32), "large": (1, 24), "serve16": (6, 16)}


def report(name, n_threads=None):
    n_threads = n_threads or os.cpu_count() or 1
    n_trees, per_tree = PLANS[name]
    rows, irows, evaluated, buf = [], [], 0, None
    if name == "serve16":
        jobs = []
        for _, r, seed, n, d in W.serve_requests(n_trees):
            m, traj = W.make_robot(r)
            jobs.append((m, W.make_rrt(seed, m, traj[-1], n, d), W.Sensor(**W.SENSOR_STEP)))
    else:
        w = W.make(name, n_trees=n_trees)
        jobs = [(w.map, t, w.sensor) for t in w.trees[:n_trees]]
    for j, (m, t, sensor) in enumerate(jobs):
        mask = None if per_tree is None else _sample_mask(t, per_tree, 7000 + j)
        rows += _tree_rows(m, t, sensor, mask, n_threads)
        r, buf = _interval_rows(m, t, sensor, mask, n_threads)
        irows += r
        evaluated += t.n if mask is None else int(mask.sum())
    out = dict(workload=name, trees=len(jobs), nodes_evaluated=evaluated,
               sample="all nodes" if per_tree is None else
               f"{per_tree} seeded nodes per tree (seeds 7000+tree) and their ancestors")
    out.update(_compare(rows))
    out["interval"] = dict(buffer=f"{buf[0]}x{buf[1]}", **_fit(*zip(*irows)))
    return out


if __name__ == "__main__":
    out = [report(n) for n in (sys.argv[1:] or ["tiny", "step", "batch64", "large", "serve16"])]
    print(json.dumps(out, indent=1))
