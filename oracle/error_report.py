"""Error of the depth-buffer marginal gain against the exact gain (oracle only).

For each node: G_db (depth-buffer marginal, incidences), X_ray (exact
set-difference marginal of eq. 2 counted per ray incidence, at the same yaw
window, Sec. V-A's fixed-yaw protocol), X_set (eq. 2 as a set), G_abs
(absolute) and g_sp (single-parent conditioning). Reports, per depth, the mean
ratios G_db/X_ray, G_sp/X_ray and G_abs/X_ray (the analogue of Fig. 4b), and
over all nodes the least-squares slope (through the origin) and R^2 of G_db
against X_ray (the statistic form of Sec. V-A). Test infrastructure: calls
only the oracle and the workload generator.

Usage: python oracle/error_report.py [workload ...] > report.json
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import mgref  # noqa: E402
from paper_2609_40297_amd import workloads as W  # noqa: E402


def report(name, n_threads=None):
    n_threads = n_threads or os.cpu_count() or 1
    w = W.make(name, n_trees=1)
    t = w.trees[0]
    full = mgref.eval_tree(w.map, t, w.sensor, n_threads=n_threads)
    sp = mgref.eval_tree(w.map, t, w.sensor, max_anc=1, n_threads=n_threads)
    ex = mgref.exact(w.map, t, w.sensor, full["k_db"], full["D"])
    dep = t.depth()
    g = full["g_db"].astype(np.float64)
    x = ex["X_ray"].astype(np.float64)
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
                              sp_over_exact=float(np.mean(sp["g_db"][m] / x[m])),
                              abs_over_exact=float(np.mean(full["g_abs"][m] / x[m])),
                              dbset_over_exactset=float(np.mean(ex["G_db_set"][m] / np.maximum(ex["X_set"][m], 1)))))
    return dict(workload=name, nodes=int(t.n), compared=int(sel.sum()), slope=slope, r2=r2,
                mean_db_over_exact=float(np.mean(g[sel] / x[sel])),
                overestimate_pct=float(100.0 * (np.sum(g[sel]) / np.sum(x[sel]) - 1.0)),
                per_depth=per_depth)


if __name__ == "__main__":
    out = [report(n) for n in (sys.argv[1:] or ["tiny", "step"])]
    print(json.dumps(out, indent=1))
