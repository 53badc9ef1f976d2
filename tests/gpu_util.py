"""Helpers for GPU tests: run the HIP library on a workload and the oracle beside it."""
from __future__ import annotations

import os
import sys

import numpy as np


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gpu_eval_tree(mgmod, m, tree, sensor, depth=True, mode="marginal"):
    """Upload one map + tree, evaluate, return numpy outputs (uint32 gains)."""
    import torch
    M = mgmod.Map(m.states, m.voxel_m, m.origin_m)
    T = mgmod.Tree(M, tree.pos_m, tree.parent, sensor)
    out = {}
    if mode in ("marginal", "both"):
        g, y, d = T.eval_marginal(depth=depth)
        torch.cuda.synchronize()
        out["g_db"] = mgmod.as_u32(g)
        out["k_db"] = y.cpu().numpy()
        if depth:
            out["D"] = d.cpu().numpy().reshape(tree.n, sensor.n_el, sensor.w_buf)
    if mode == "batch":                     # the multi-tree path on this one tree (autotuned, stream groups)
        g, y, d = mgmod.eval_batch([T], depth=depth)
        torch.cuda.synchronize()
        out["g_db"] = mgmod.as_u32(g)
        out["k_db"] = y.cpu().numpy()
        if depth:
            out["D"] = d.cpu().numpy().reshape(tree.n, sensor.n_el, sensor.w_buf)
    if mode == "single_parent":             # g_sp: parent-only conditioning
        g, y, d = T.eval_single_parent(depth=depth)
        torch.cuda.synchronize()
        out["g_db"] = mgmod.as_u32(g)
        out["k_db"] = y.cpu().numpy()
        if depth:
            out["D"] = d.cpu().numpy().reshape(tree.n, sensor.n_el, sensor.w_buf)
    if mode in ("absolute", "both"):
        g, y = T.eval_absolute()
        torch.cuda.synchronize()
        out["g_abs"] = mgmod.as_u32(g)
        out["k_abs"] = y.cpu().numpy()
    T.close()
    M.close()
    return out


def assert_same(gpu, ref, nodes=None, keys=("g_db", "k_db", "D")):
    sel = slice(None) if nodes is None else np.asarray(nodes)
    for k in keys:
        if k not in gpu or k not in ref:
            continue
        a, b = gpu[k][sel], ref[k][sel]
        if a.dtype.kind == "f":
            assert a.tobytes() == b.tobytes(), (k, _first_diff(a, b))
        else:
            assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), (k, _first_diff(a, b))


def _first_diff(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1) if np.asarray(a).ndim > 1 else np.asarray(a)[:, None]
    b = np.asarray(b).reshape(a.shape)
    bad = np.nonzero((a != b).any(axis=1))[0]
    if bad.size == 0:
        return "equal"
    i = bad[0]
    j = np.nonzero(a[i] != b[i])[0][:5]
    return f"{bad.size} rows differ; first row {i} at {j.tolist()}: {a[i][j].tolist()} vs {b[i][j].tolist()}"
