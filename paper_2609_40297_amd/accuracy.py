"""Accuracy study on the device (the comparison of Sec. V-A, Fig. 4, at full scale).

For every node of a workload: the depth-buffer marginal gain (per-voxel
test), the interval-mode gain (the paper's own test), the single-parent gain
and the absolute gain, against the exact marginal gain counted with device
hash sets (mg_eval_exact) at the depth-buffer windows (the interval mode
against the exact gain at its own windows); and how often the depth-buffer
method picks the window the exact planner gain picks (mg_eval_exact_marginal,
its own yaw choice on its own sets). Reports, as the CPU error report
does, the least-squares slope through the origin, R^2 and the over/under
estimate of each conditioned gain against the exact one, and per depth the
mean ratios. Uses only the HIP library and the seeded workload generator.

Usage: python -m paper_2609_40297_amd.accuracy [workload[:trees] ...]
"""
from __future__ import annotations

import json
import sys

import numpy as np


def _fit(dep, g, x):
    dep, g, x = (np.asarray(c, dtype=np.float64) for c in (dep, g, x))
    sel = x > 0
    slope = float(np.sum(g[sel] * x[sel]) / np.sum(x[sel] * x[sel]))
    resid = g[sel] - slope * x[sel]
    r2 = float(1.0 - np.sum(resid ** 2) / np.sum((g[sel] - g[sel].mean()) ** 2))
    return dict(compared=int(sel.sum()), slope=slope, r2=r2,
                overestimate_pct=float(100.0 * (np.sum(g[sel]) / np.sum(x[sel]) - 1.0)))


def _per_depth(dep, x, **gains):
    dep = np.asarray(dep)
    x = np.asarray(x, np.float64)
    rows = []
    for d in range(int(dep.max()) + 1):
        m = (dep == d) & (x > 0)
        if m.any():
            rows.append(dict(depth=d, nodes=int(m.sum()),
                             **{k: float(np.mean(np.asarray(v, np.float64)[m] / x[m])) for k, v in gains.items()}))
    return rows


def study(name: str, n_trees=None) -> dict:
    import torch
    from paper_2609_40297_amd import mg, workloads as W
    w = W.make(name, n_trees=n_trees)
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    cols = {k: [] for k in ("dep", "g_db", "x_db", "g_iv", "x_iv", "g_sp", "g_abs", "k_db", "g_ex", "k_ex")}
    for t in w.trees:
        T = mg.Tree(M, t.pos_m, t.parent, w.sensor)
        g_db, k_db, _ = T.eval_marginal()
        x_db = T.eval_exact(k_db)[0]
        g_iv, k_iv, _ = T.eval_interval()
        x_iv = T.eval_exact(k_iv)[0]
        g_sp = T.eval_single_parent()[0]
        g_abs = T.eval_absolute()[0]
        g_ex, k_ex = T.eval_exact_marginal()
        torch.cuda.synchronize()
        cols["dep"].append(t.depth())
        for k, v in (("g_db", g_db), ("x_db", x_db), ("g_iv", g_iv), ("x_iv", x_iv), ("g_sp", g_sp),
                     ("g_abs", g_abs), ("g_ex", g_ex)):
            cols[k].append(mg.as_u32(v))
        cols["k_db"].append(k_db.cpu().numpy())
        cols["k_ex"].append(k_ex.cpu().numpy())
        T.close()
    M.close()
    c = {k: np.concatenate(v) for k, v in cols.items()}
    return dict(workload=name, trees=len(w.trees), nodes=int(c["dep"].size),
                depth_buffer=_fit(c["dep"], c["g_db"], c["x_db"]),
                interval=_fit(c["dep"], c["g_iv"], c["x_iv"]),
                # against the exact planner gain with its own yaw choice: same window chosen, and the gain
                same_window=float(np.mean(c["k_db"] == c["k_ex"])),
                depth_buffer_vs_own_yaw_exact=_fit(c["dep"], c["g_db"], c["g_ex"]),
                per_depth=_per_depth(c["dep"], c["x_db"], db=c["g_db"], sp=c["g_sp"], abs=c["g_abs"]),
                interval_per_depth=_per_depth(c["dep"], c["x_iv"], interval=c["g_iv"]))


if __name__ == "__main__":
    out = []
    for arg in sys.argv[1:] or ["step", "batch64"]:
        name, _, nt = arg.partition(":")
        out.append(study(name, int(nt) if nt else None))
        print(json.dumps(out[-1]), flush=True)
