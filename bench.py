#!/usr/bin/env python3
"""Benchmark: marginal-gain rays/s and replan p50/p99 latency, batched vs plain, one MI355X.

One step = one replanning request: every node of the workload's tree(s) is
evaluated (depth-buffer marginal gain, yaw window, depth buffer) and the gains
and yaw windows are copied back to host memory. Inputs (map and trees) are
resident on the GPU before the timed region starts.

Workloads (seeded, synthetic): `large` (default, the headline: 8 trees of 3000
nodes on a 512x512x128 grid at 0.05 m, 720x120 rays, 15 m), `step`, `batch64`,
`tiny`, and `serve16` (its own serving line). With the default headline the
line also carries `step` and `batch64` as extra keys, and the next-row paths
(single-parent gain, interval mode, exact hash sets, path score, map
conversion) timed on `step`.

Modes
  plain    paper-style (Sec. IV-C): tree after tree, one launch group per depth
           level, stream synchronised and gains/yaws copied to the host after
           every level.
  batched  the whole request in one call (mg_eval_marginal_batch), one copy
           of the results at the end; per depth level a trace, a window and a
           mask-builder launch on three stream groups.
  graph    the same call with the plan's launches recorded once into a HIP
           graph and replayed (mg_batch_config(-1, 1)).
  persistent  the same call configured as one cooperative launch per step
           (co-resident workgroups, grid barriers between the phases).
`value` is the batched mode's rays/s; the other modes are reported beside it.

Prints ONE JSON line (rank 0, N = 1). Extra fields: latency percentiles,
the roofline of the marginal-gain kernels (trace and path-mask builder) and
the oracle's CPU rate on a bounded sample (the oracle is used only in that leg).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def score_bench(mg, trees, gain, n_total, depth_sum, reps=200):
    """Device path score (eq. 3, eq. 4, best branch) of the evaluated batch: HIP events around
    `reps` back-to-back mg_score_branches calls on the current stream."""
    import torch
    dev = gain.device
    cost = torch.empty(n_total, dtype=torch.float64, device=dev)
    obj = torch.empty(n_total, dtype=torch.float64, device=dev)
    best = torch.empty(len(trees), dtype=torch.int32, device=dev)
    branch = torch.empty((len(trees), mg.MG_BRANCH_LEN), dtype=torch.int32, device=dev)
    handles = [t.handle for t in trees]
    for _ in range(5):
        mg.mg_score_branches(handles, gain, 0.5, cost, obj, best, branch)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        mg.mg_score_branches(handles, gain, 0.5, cost, obj, best, branch)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    # algorithmic bytes: per node its gain (4 B), position (16 B), parent link (4 B) and cost + objective
    # (16 B) once, each ancestor id of its root path (4 B) once; per tree the branch row (65 x 4 B)
    alg = n_total * 40 + depth_sum * 4 + len(trees) * (mg.MG_BRANCH_LEN * 4 + 4)
    gbs = alg / (us * 1e-6) / 1e9
    return {"us_per_call": us, "nodes_per_s": n_total / (us * 1e-6),
            "launches_per_call": 1 if max(t.n for t in trees) <= 8192 else 2,
            "lambda": 0.5, "algorithmic_bytes_per_call": alg,
            "roofline": {"bound": "latency", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": None},
            "d2h_bytes_replaced": n_total * 8, "d2h_bytes_after": len(trees) * (mg.MG_BRANCH_LEN * 4 + 4)}


def map_bench(mg, dims=(512, 512, 128), voxel_m=0.05, reps=20, n_updates=1 << 20):
    """Map conversion and deltas on the grid of the large configuration: a whole-grid TSDF update
    (reads 8 B, writes the bricked byte per voxel) and listed voxel updates, timed with HIP events
    over `reps` calls on the current stream; inputs resident on the device, seeded."""
    import torch
    nx, ny, nz = dims
    g = torch.Generator(device="cuda")
    g.manual_seed(1234)
    dist = torch.randn((nz, ny, nx), generator=g, device="cuda") * 0.4 + 0.3
    wgt = torch.rand((nz, ny, nx), generator=g, device="cuda") * 3.0
    M = mg.Map.from_tsdf(dist, wgt, voxel_m, (0.0, 0.0, 0.0), surface_m=0.05, min_weight=1.0)
    ids = torch.randint(0, nx * ny * nz, (n_updates,), generator=g, device="cuda", dtype=torch.int32)
    new = torch.randint(0, 3, (n_updates,), generator=g, device="cuda", dtype=torch.uint8)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {"grid": f"{nx}x{ny}x{nz}", "voxels": nx * ny * nz}
    for name, fn in (("tsdf_update", lambda: mg.mg_map_update_tsdf(M.handle, dist, wgt, (0, 0, 0), 0.05, 1.0)),
                     ("voxel_updates", lambda: mg.mg_map_update(M.handle, ids, new))):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_us"] = e0.elapsed_time(e1) * 1e3 / reps
    M.close()
    nb = [((n + 7) // 8) for n in dims]
    alg = 8 * nx * ny * nz + nb[0] * nb[1] * nb[2] * 512       # TSDF in, bricks holding grid voxels out
    gbs = alg / (out["tsdf_update_us"] * 1e-6) / 1e9
    out["tsdf_voxels_per_s"] = nx * ny * nz / (out["tsdf_update_us"] * 1e-6)
    out["tsdf_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": gbs / HBM_PEAK_GBS,
                            "traffic": summary_traffic(TSDF_TRAFFIC_SUMMARY, TSDF_SOURCES) if dims == (512, 512, 128)
                            else None, "algorithmic_bytes": alg}
    out["voxel_updates_per_s"] = n_updates / (out["voxel_updates_us"] * 1e-6)
    return out


def score_oracle(w):
    """The path-score oracle over every tree of the workload, on gains of 1 per node (its cost does
    not depend on the values)."""
    from oracle import paths
    t0 = time.perf_counter()
    for t in w.trees:
        paths.score_paths(t.pos_m, t.parent, np.ones(t.n, np.uint32), w.map.voxel_m, 0.5)
    dt = time.perf_counter() - t0
    n = sum(t.n for t in w.trees)
    return {"us_per_call": dt * 1e6, "nodes_per_s": n / dt, "cores": 1, "kind": "oracle",
            "sample": f"all {len(w.trees)} trees, {n} nodes, one thread"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["tiny", "step", "batch64", "large", "serve16"])
    ap.add_argument("--extras", default=None,
                    help="comma-separated extra workloads timed in the same line (default: step,batch64 with "
                         "the large headline, none otherwise; 'none' skips them)")
    ap.add_argument("--requests", type=int, default=64, help="serve16: number of replanning requests")
    ap.add_argument("--trees", type=int, default=None, help="keep only the first trees of a multi-tree workload")
    ap.add_argument("--modes", default="plain,batched,graph,persistent",
                    help="plain, batched (per-level launches), graph (those launches replayed from a HIP graph), "
                         "persistent (one cooperative launch per step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sp-steps", type=int, default=5, help="timed single-parent (g_sp) passes; 0 skips")
    ap.add_argument("--ivl-steps", type=int, default=3, help="timed interval-mode passes; 0 skips")
    ap.add_argument("--exact-steps", type=int, default=3, help="timed exact hash-set passes; 0 skips")
    ap.add_argument("--map-bench-only", action="store_true",
                    help="only run the map conversion / update timing (3 calls each) and exit")
    ap.add_argument("--no-map-bench", dest="map_bench", action="store_false",
                    help="skip the map conversion / update timing")
    ap.add_argument("--cpu-sample-rays", type=float, default=None,
                    help="oracle sample, rays per host thread (default: 1.5e6, 0.5e6 on large)")
    ap.add_argument("--profile-summary", default=None, metavar="CSV",
                    help="print per-step figures of the last --steps batched calls from a rocprofv3 "
                         "kernel-trace or counter-collection CSV of a bench run, and exit (no GPU)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this size (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def work_counts(name, rays_total=None):
    """Per-workload oracle work counts (visits V, unknown visits U, ancestor tests T). An entry that
    counted only the first trees of a multi-tree workload (trees_counted < trees) is scaled to
    `rays_total` by its per-ray rates and says so in "counted"."""
    p = os.path.join(ROOT, "tests", "golden", "work_counts.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        wc = json.load(f).get(name)
    if wc is None or not wc.get("rays"):
        return None
    done, trees = wc.get("trees_counted"), wc.get("trees")
    if done is None or done == trees or rays_total is None:
        return dict(wc, counted="all trees, exact")
    f = rays_total / wc["rays"]
    out = {k: (wc[k] * f if k in ("visits", "unk_visits", "anc_tests") else wc[k]) for k in wc}
    out["rays"] = rays_total
    out["counted"] = (f"first {done} of {trees} trees exactly ({wc['rays']} rays); the rest at their per-ray "
                      f"rates")
    return out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_trace_multi_large_traffic.md")
# the trace kernel and the scheduler that decides how its launches are cut
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2609_40297_amd", "csrc", f)
                  for f in ("mg_kernels.hip", "mg_batch.hip", "mg_internal.h")]


def kernel_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summary_traffic(path, sources, key="hbm_bytes_per_launch"):
    """HBM bytes per launch from a committed counter summary, or None.

    The summary records the SHA-256 of the sources it was taken with; when they
    have changed since, the figure no longer applies."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for ln in f:
            if ln.startswith("- ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash(sources) or key not in vals:
        return None
    return float(vals[key])


def measured_traffic(workload):
    """HBM bytes per step of the trace and mask-builder dispatches of the large workload (committed counter
    summary), or None."""
    return summary_traffic(TRAFFIC_SUMMARY, KERNEL_SOURCES, "hbm_bytes_per_step") if workload == "large" else None


TSDF_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_tsdf_grid_512x512x128_traffic.md")
TSDF_SOURCES = [os.path.join(ROOT, "paper_2609_40297_amd", "csrc", "mg_map.hip")]


PATH_KERNELS = ("k_trace_multi", "k_mask_build_multi", "k_finish_multi")


def _short(name):
    return next((k for k in PATH_KERNELS + ("k_batch_zero",) if k in name), name.split("(")[0])


def _union_ns(iv):
    tot, end = 0, None
    for a, b in sorted(iv):
        if end is None or a > end:
            tot += b - a
            end = b
        elif b > end:
            tot += b - end
            end = b
    return tot


def profile_summary(path, steps):
    """Per-step figures of the last `steps` mg_eval_marginal_batch calls in a rocprofv3 CSV (kernel
    trace, or counter collection): each call starts with its k_batch_zero dispatch. For a trace:
    dispatches, summed and average durations per path kernel, the union of the trace and mask-builder
    intervals (what bench.py's roofline divides by) and the call's span. For counters: each
    counter summed over each path kernel's dispatches, per call."""
    import csv
    with open(path) as f:
        rows = list(csv.DictReader(f))
    counters = "Counter_Name" in rows[0]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    starts = [i for i, r in enumerate(rows) if "k_batch_zero" in r["Kernel_Name"]]
    if len(starts) < steps:
        raise SystemExit(f"{path}: {len(starts)} batched calls, fewer than {steps}")
    first = starts[len(starts) - steps:]
    calls = [rows[a:b] for a, b in zip(first, first[1:] + [len(rows)])]
    out = [f"Last {steps} batched calls of `{os.path.basename(path)}` (each starts at its k_batch_zero)", ""]
    if counters:
        names = sorted({r["Counter_Name"] for r in rows})
        tot = {}
        for c in calls:
            for r in c:
                k = (_short(r["Kernel_Name"]), r["Counter_Name"])
                tot[k] = tot.get(k, 0.0) + float(r["Counter_Value"])
        out += ["| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
        for kn in PATH_KERNELS:
            out.append(f"| {kn} | " + " | ".join(f"{tot.get((kn, n), 0.0) / steps:.6g}" for n in names) + " |")
        out += ["", "(per call: counter values summed over the kernel's dispatches, averaged over the calls)"]
        return "\n".join(out)
    out += ["| call | dispatches | " + " | ".join(f"{k} ms (n)" for k in PATH_KERNELS) +
            " | union trace+builder ms | span ms |", "|---" * (len(PATH_KERNELS) + 4) + "|"]
    agg = {k: [0, 0] for k in PATH_KERNELS}
    un_sum = span_sum = 0
    for i, c in enumerate(calls):
        per = {k: [0, 0] for k in PATH_KERNELS}
        iv = []
        for r in c:
            k = _short(r["Kernel_Name"])
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if k in per:
                per[k][0] += b - a
                per[k][1] += 1
            if k in ("k_trace_multi", "k_mask_build_multi"):
                iv.append((a, b))
        un = _union_ns(iv)
        span = max(int(r["End_Timestamp"]) for r in c) - min(int(r["Start_Timestamp"]) for r in c)
        un_sum += un
        span_sum += span
        for k in PATH_KERNELS:
            agg[k][0] += per[k][0]
            agg[k][1] += per[k][1]
        out.append(f"| {i} | {len(c)} | " + " | ".join(f"{per[k][0] / 1e6:.3f} ({per[k][1]})" for k in PATH_KERNELS)
                   + f" | {un / 1e6:.3f} | {span / 1e6:.3f} |")
    out += ["", "Per call (mean over the calls):", ""]
    for k in PATH_KERNELS:
        n = agg[k][1]
        out.append(f"- {k}: {n / steps:.1f} dispatches, {agg[k][0] / steps / 1e6:.3f} ms summed, "
                   f"{(agg[k][0] / n / 1e3) if n else 0:.1f} us average")
    out.append(f"- union of k_trace_multi and k_mask_build_multi intervals: {un_sum / steps / 1e6:.3f} ms")
    out.append(f"- call span (first dispatch start to last dispatch end): {span_sum / steps / 1e6:.3f} ms")
    return "\n".join(out)


def copy_probe(mib):
    """A plain copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 3}), flush=True)


def cpu_threads():
    """Host threads for the oracle leg: the cores this process may use, at most 16 (one GPU's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    """The host CPU's model name and logical CPU count (as the OS reports them)."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    name = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count() or 1


def cpu_baseline(w, target_rays_per_thread):
    """The oracle as it stands, with its threaded driver (the nodes of one depth level in parallel), on
    a seeded uniform sample of nodes of tree 0 and their ancestors (the whole tree if the target
    exceeds it). The driver starts min(threads, level width) threads per level: `cores` is the most it
    started and `threads_mean` the node-weighted mean over the sample's levels."""
    from oracle import mgref
    threads = cpu_threads()
    target_rays = target_rays_per_thread * threads
    t = w.trees[0]
    dep = t.depth()
    order = np.random.Generator(np.random.PCG64(12345)).permutation(t.n)
    picked = []
    mask = np.zeros(t.n, np.uint8)
    for nd in order:
        picked.append(int(nd))
        mask = mgref.ancestor_closure(t.parent, picked)
        if mask.sum() * w.sensor.rays >= target_rays:
            break
    t0 = time.perf_counter()
    mgref.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads)
    dt = time.perf_counter() - t0
    nodes = int(mask.sum())
    rays = nodes * w.sensor.rays
    widths = np.bincount(dep[mask.astype(bool)])
    widths = widths[widths > 0]
    used = np.minimum(widths, threads)
    what = "all nodes of tree 0" if mask.all() else f"{len(picked)} uniformly drawn nodes of tree 0 and their ancestors"
    model, nproc = cpu_model()
    return {"value": rays / dt, "unit": "rays/s", "cores": int(used.max()), "kind": "oracle",
            "threads_mean": float((used * widths).sum() / widths.sum()),
            "sample": f"{nodes} nodes ({what}; level widths {widths.tolist()}), {rays} rays, {dt:.1f} s, "
                      f"up to {threads} threads",
            "cpu_model": model, "nproc": nproc}


def next_row_oracles(w, threads):
    """The oracles of the next-row paths, each on a bounded sample, for context beside the device
    figures: the interval mode and the exact sets on the three deepest leaves of tree 0 and their
    ancestors (the exact pass at the depth-buffer windows of the same nodes), the TSDF conversion
    on a 512x512x128 grid; and the depth-buffer oracle itself on one thread over the same nodes."""
    from oracle import ivlref, maps, mgref
    t = w.trees[0]
    dep = t.depth()
    leaves = [int(i) for i in np.flatnonzero(dep == dep.max())[:3]]
    mask = mgref.ancestor_closure(t.parent, leaves)
    nodes = int(mask.sum())
    out = {}
    t0 = time.perf_counter()
    ivlref.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=threads)
    dt = time.perf_counter() - t0
    out["interval"] = {"value": nodes * w.sensor.rays / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
                       "sample": f"{nodes} nodes (3 deepest leaves of tree 0 and their ancestors), {dt:.2f} s"}
    t0 = time.perf_counter()
    ref = mgref.eval_tree(w.map, t, w.sensor, mask=mask, n_threads=1)
    dt = time.perf_counter() - t0
    out["serial"] = {"value": nodes * w.sensor.rays / dt, "unit": "rays/s", "cores": 1, "kind": "oracle",
                     "sample": f"the same {nodes} nodes, depth-buffer marginal gain on one thread, {dt:.2f} s"}
    t0 = time.perf_counter()
    mgref.exact(w.map, t, w.sensor, ref["k_db"], ref["D"], mask=mask)
    dt = time.perf_counter() - t0
    out["exact"] = {"value": nodes * w.sensor.n_el * w.sensor.w_buf / dt, "unit": "window rays/s", "cores": 1,
                    "kind": "oracle", "sample": f"the same {nodes} nodes, sorted voxel sets, {dt:.2f} s"}
    rng = np.random.Generator(np.random.PCG64(5))
    d = rng.normal(0.3, 0.4, (128, 512, 512)).astype(np.float32)
    wt = rng.uniform(0, 3, d.shape).astype(np.float32)
    t0 = time.perf_counter()
    maps.tsdf_states(d, wt, 0.05, 1.0)
    dt = time.perf_counter() - t0
    out["tsdf"] = {"value": d.size / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
                   "sample": f"512x512x128 grid, {dt:.2f} s"}
    return out


def serve_bench(args):
    """16 robots, Poisson replanning requests at 20 Hz (seeded), replayed in real time.

    plain-FIFO: one request at a time in arrival order, paper-style per-level
    synchronisation; served: the continuous-batching server (16 slots). Latency
    is arrival to results in host memory. Saturated throughput: all requests
    submitted at once.
    """
    import torch
    from paper_2609_40297_amd import mg, workloads as W

    torch.cuda.set_device(0)
    mg.lib()
    reqs = W.serve_requests(args.requests)
    robots = sorted({r for _, r, _, _, _ in reqs})
    log(f"[bench] serve16: generating {len(robots)} robot maps and {len(reqs)} request trees")
    maps, trajs = {}, {}
    for r in robots:
        maps[r], trajs[r] = W.make_robot(r)
    sen = W.Sensor(**W.SENSOR_STEP)
    trees = [W.make_rrt(seed, maps[r], trajs[r][-1], n, d) for _, r, seed, n, d in reqs]
    arrivals = np.array([a for a, _, _, _, _ in reqs]) - reqs[0][0]
    rays = [t.n * sen.rays for t in trees]
    dev_maps = {r: mg.Map(maps[r].states, maps[r].voxel_m, maps[r].origin_m) for r in robots}
    robot_of = [r for _, r, _, _, _ in reqs]
    log(f"[bench] {sum(t.n for t in trees)} nodes, {sum(rays)} rays")

    # plain FIFO, real-time arrivals
    def plain_one(i):
        T = mg.Tree(dev_maps[robot_of[i]], trees[i].pos_m, trees[i].parent, sen)
        hg = np.zeros(T.n, np.uint32)
        hy = np.zeros(T.n, np.int32)
        mg.mg_eval_marginal_levelsync(T.handle, hg, hy, None, None, None)
        T.close()
        return hg, hy

    for i in range(min(2, len(trees))):
        plain_one(i)
    torch.cuda.synchronize()
    lat_plain, res_plain = [], []
    t0 = time.perf_counter()
    for i in range(len(trees)):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        res_plain.append(plain_one(i))
        lat_plain.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
    # served, real-time arrivals
    S = mg.Server(sen, max_inflight=16, arena_bytes=16 << 30)
    for i in range(min(2, len(trees))):
        S.wait(S.submit(dev_maps[robot_of[i]], trees[i].pos_m, trees[i].parent))
    tickets = []
    t0 = time.perf_counter()
    for i in range(len(trees)):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        tickets.append(S.submit(dev_maps[robot_of[i]], trees[i].pos_m, trees[i].parent))
    served = [S.wait(t) for t in tickets]
    lat_served = [x[2] / 1e3 for x in served]
    for (g, y, _), (pg, py) in zip(served, res_plain):
        assert np.array_equal(g, pg) and np.array_equal(y, py), "served and plain results differ"
    # saturated throughput: everything submitted at once
    t0 = time.perf_counter()
    tickets = [S.submit(dev_maps[robot_of[i]], trees[i].pos_m, trees[i].parent) for i in range(len(trees))]
    for t in tickets:
        S.wait(t)
    sat_served = time.perf_counter() - t0
    # served with map updates between replans: after each request, 10k voxels of its robot's map change
    # (queued with the requests, so later requests of that robot see them)
    rng = np.random.Generator(np.random.PCG64(4242))
    upd = []
    for i in range(len(trees)):
        st = maps[robot_of[i]].states
        ids = rng.choice(st.size, 10000, replace=False).astype(np.uint32)
        upd.append((ids, rng.integers(0, 3, ids.size).astype(np.uint8)))
    tickets, utickets = [], []
    t0 = time.perf_counter()
    for i in range(len(trees)):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        tickets.append(S.submit(dev_maps[robot_of[i]], trees[i].pos_m, trees[i].parent))
        utickets.append(S.map_update(dev_maps[robot_of[i]], *upd[i]))
    with_upd = [S.wait(t)[2] / 1e3 for t in tickets]
    for t in utickets:
        S.wait(t)
    S.close()
    t0 = time.perf_counter()
    for i in range(len(trees)):
        plain_one(i)
    sat_plain = time.perf_counter() - t0
    total_rays = float(sum(rays))
    res = {
        "plain": {"p50_ms": float(np.percentile(lat_plain, 50)), "p99_ms": float(np.percentile(lat_plain, 99)),
                  "saturated_rays_per_s": total_rays / sat_plain},
        "served": {"p50_ms": float(np.percentile(lat_served, 50)), "p99_ms": float(np.percentile(lat_served, 99)),
                   "saturated_rays_per_s": total_rays / sat_served},
        "served_with_map_updates": {"p50_ms": float(np.percentile(with_upd, 50)),
                                    "p99_ms": float(np.percentile(with_upd, 99)),
                                    "updates": len(utickets), "voxels_per_update": 10000},
    }
    log(f"[bench] serve16: {res}")
    line = {
        "metric": "marginal-gain rays/s + replan p50/p99 ms, batched vs plain, 1xMI355X",
        "value": res["served"]["saturated_rays_per_s"],
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": len(trees),
        "warmup": 2,
        "ms_per_step": sat_served * 1e3 / len(trees),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serve16: {W.WORKLOADS['serve16']}", "requests": len(trees),
                   "nodes": int(sum(t.n for t in trees)), "rays": int(total_rays), "mode": "served",
                   "offered_rate_hz": 20.0},
        "p50_ms": res["served"]["p50_ms"],
        "p99_ms": res["served"]["p99_ms"],
        "modes": res,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    for m in dev_maps.values():
        m.close()


def roofline_of(wc, trace, steps, n_total, yaw_bins, ms_per_step, traffic):
    """Roofline of the marginal-gain kernels (trace + path-mask builder) from the oracle's work counts
    and the live launch intervals, or None when either is missing."""
    if wc is None or not trace or not trace["launches"]:
        return None
    # algorithmic bytes of the path, per step: 1 B per voxel visit (grid gather), 4 B per ancestor depth
    # read (ancestor tests, parent first, to the first that observes), 4 B per ray (first-hit write),
    # 2 x B x 4 B of bin counts per node
    alg_step = wc["visits"] * 1 + wc["anc_tests"] * 4 + wc["rays"] * 4 + n_total * 2 * yaw_bins * 4
    busy = trace["busy_ms"] / steps                 # union of the trace and builder launch intervals
    summed = trace["total_ms"] / steps              # their summed durations (groups overlap on their streams)
    achieved = alg_step / (busy * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per step of the trace and mask-builder dispatches (rocprofv3 FETCH_SIZE + "
                            "WRITE_SIZE, each scaled by what it reads for a plain device copy)",
            "kernels": ["k_trace_multi", "k_mask_build_multi"],
            "algorithmic_bytes_per_step": alg_step, "work_counts": wc.get("counted"),
            "busy_ms_per_step": busy, "summed_launch_ms_per_step": summed,
            "launches_per_step": trace["launches"] / steps,
            "achieved_over_summed_launches": alg_step / (summed * 1e-3) / 1e9,
            "achieved_over_whole_step": alg_step / (ms_per_step * 1e-3) / 1e9,
            "timing": "HIP events recorded by each trace and mask-builder dispatch over the timed steps; "
                      "achieved = algorithmic bytes per step / union of those launch intervals per step"}


def measure(mg, W, name, steps, warmup, modes, n_trees=None):
    """Times one workload: plain (tree after tree, per-level sync) and batched (one call) steps.
    Returns a dict with the results and the objects the next-row legs reuse."""
    import torch
    log(f"[bench] generating workload {name}")
    w = W.make(name, n_trees=n_trees)
    sen = w.sensor
    n_total = sum(t.n for t in w.trees)
    rays_per_step = n_total * sen.rays
    log(f"[bench] {name}: {len(w.trees)} trees, {n_total} nodes, {rays_per_step} rays per step")
    stream = torch.cuda.current_stream()
    M = mg.Map(w.map.states, w.map.voxel_m, w.map.origin_m)
    trees = [mg.Tree(M, t.pos_m, t.parent, sen) for t in w.trees]
    dev = torch.device("cuda", 0)
    g_all = torch.empty(n_total, dtype=torch.int32, device=dev)
    y_all = torch.empty(n_total, dtype=torch.int32, device=dev)
    host_g = torch.empty(n_total, dtype=torch.int32).pin_memory()
    host_y = torch.empty(n_total, dtype=torch.int32).pin_memory()
    per_tree_host = [(np.zeros(t.n, np.uint32), np.zeros(t.n, np.int32)) for t in trees]
    handles = [t.handle for t in trees]

    def step_plain():
        for T, (hg, hy) in zip(trees, per_tree_host):
            mg.mg_eval_marginal_levelsync(T.handle, hg, hy, None, None, None)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kernel_ms = []

    def step_batched():
        ev0.record(stream)
        mg.mg_eval_marginal_batch(handles, g_all, y_all, None)
        ev1.record(stream)
        host_g.copy_(g_all, non_blocking=True)
        host_y.copy_(y_all, non_blocking=True)
        stream.synchronize()
        kernel_ms.append(ev0.elapsed_time(ev1))

    results = {}
    trace = None
    saved = None
    for mode in modes:
        fn = {"plain": step_plain, "batched": step_batched, "graph": step_batched, "persistent": step_batched}[mode]
        if mode in ("graph", "persistent"):
            # the same call, its plan's launches replayed from a HIP graph, or one cooperative launch
            if "batched" in results:
                saved = (host_g.numpy().copy(), host_y.numpy().copy())
            mg.mg_batch_config(-1, 1 if mode == "graph" else 2)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        kernel_ms.clear()
        lat = []
        if mode == "batched":     # trace and builder launches timed by events their own dispatches record
            mg.mg_timing_read()
            mg.mg_timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            fn()
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        if mode == "batched":
            t_ms, t_busy, t_n, t_wg = mg.mg_timing_read()
            mg.mg_timing_enable(False)
            trace = dict(total_ms=t_ms, busy_ms=t_busy, launches=t_n, workgroups=t_wg)
        results[mode] = dict(rays_per_s=rays_per_step * steps / total, ms_per_step=total * 1e3 / steps,
                             p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                             kernel_ms=float(np.mean(kernel_ms)) if kernel_ms else None)
        log(f"[bench] {name} {mode}: {results[mode]}")
        if mode in ("graph", "persistent"):
            if saved is not None:
                assert np.array_equal(saved[0], host_g.numpy()), f"batched and {mode} differ"
                assert np.array_equal(saved[1], host_y.numpy()), f"batched and {mode} differ"
            mg.mg_batch_config(-1, 0)
            if "batched" in results:
                step_batched()              # the default plan again (its shape is cached)
    # parity of the two modes on this workload (identical results required)
    if "plain" in results and "batched" in results:
        off = 0
        for (hg, hy), t in zip(per_tree_host, trees):
            assert np.array_equal(hg, host_g.numpy()[off:off + t.n].view(np.uint32)), "plain and batched differ"
            assert np.array_equal(hy, host_y.numpy()[off:off + t.n]), "plain and batched differ"
            off += t.n
    main_mode = "batched" if "batched" in results else "plain"
    shape_idx, graphed = mg.mg_batch_plan_info(handles) if "batched" in results else (0, False)
    shape = mg.mg_trace_shapes()[shape_idx]
    wc = work_counts(name if n_trees is None else f"{name}:{n_trees}", rays_per_step)
    roof = roofline_of(wc, trace, steps, n_total, sen.yaw_bins, results[main_mode]["ms_per_step"],
                       measured_traffic(name))
    return dict(w=w, M=M, trees=trees, g_all=g_all, y_all=y_all, n_total=n_total, rays_per_step=rays_per_step,
                results=results, main_mode=main_mode, roof=roof, trace=trace,
                launch_shape={"rays_per_workgroup": shape[0], "mask_bricks_per_workgroup": shape[1],
                              "chosen_by": "autotune", "graph": graphed})


def close(m):
    for T in m["trees"]:
        T.close()
    m["M"].close()


def next_rows(mg, m, args):
    """The next-row paths on one measured workload: single-parent gain, interval mode, exact hash sets."""
    import torch
    w, trees, n_total, rays_per_step = m["w"], m["trees"], m["n_total"], m["rays_per_step"]
    sen = w.sensor
    dev = m["g_all"].device
    out = {}
    if args.sp_steps > 0:
        # single-parent gain g_sp (the comparison gain of Fig. 4) on the same trees, per-tree path
        g_sp = torch.empty(max(t.n for t in trees), dtype=torch.int32, device=dev)
        y_sp = torch.empty_like(g_sp)
        for T in trees:
            mg.mg_eval_single_parent(T.handle, g_sp, y_sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.sp_steps):
            for T in trees:
                mg.mg_eval_single_parent(T.handle, g_sp, y_sp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.sp_steps
        out["single_parent"] = {"rays_per_s": rays_per_step / dt, "ms_per_step": dt * 1e3, "steps": args.sp_steps,
                                "path": "mg_eval_single_parent, tree after tree"}
        log(f"[bench] single parent: {out['single_parent']}")
    if args.ivl_steps > 0:
        # interval mode (the paper's pinhole buffers and overlap intervals), per-tree level path
        wd, hd, _, _, _ = mg.interval_tables(sen, w.map.voxel_m)
        g_iv = torch.empty(max(t.n for t in trees), dtype=torch.int32, device=dev)
        y_iv = torch.empty_like(g_iv)
        for T in trees:                        # first call allocates the buffers
            mg.mg_eval_interval(T.handle, wd, hd, g_iv, y_iv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.ivl_steps):
            for T in trees:
                mg.mg_eval_interval(T.handle, wd, hd, g_iv, y_iv)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.ivl_steps
        ivl = {"rays_per_s": rays_per_step / dt, "ms_per_step": dt * 1e3, "steps": args.ivl_steps,
               "buffer": f"{wd}x{hd}", "path": "mg_eval_interval, tree after tree"}
        wci = work_counts(w.name + "/interval")
        if wci is not None:
            # algorithmic bytes: 1 B per voxel visit, 4 B per pixel walked in an ancestor buffer, 4 B per
            # rendered pixel, 2 x B x 4 B of bins per node; divided by the whole call's time
            alg = wci["visits"] + 4 * wci["pixel_steps"] + 4 * wci["nodes"] * wci["wd"] * wci["hd"] + \
                n_total * 2 * sen.yaw_bins * 4
            ivl["algorithmic_bytes_per_step"] = alg
            ivl["achieved_GBps_whole_call"] = alg / dt / 1e9
            ivl["pixel_steps_per_ray"] = wci["pixel_steps"] / wci["rays"]
        out["interval"] = ivl
        log(f"[bench] interval: {ivl}")
    if args.exact_steps > 0 and "batched" in m["results"]:
        # exact marginal gain with device hash sets at the depth-buffer windows just computed
        # (the exact comparison of Sec. V-A), per tree: X_ray, X_set, A_set
        y_all = m["y_all"]
        batched_ms = m["results"]["batched"]["ms_per_step"]
        xr = torch.empty(max(t.n for t in trees), dtype=torch.int32, device=dev)
        xs, xa = torch.empty_like(xr), torch.empty_like(xr)
        ys = []
        off = 0
        for T in trees:
            ys.append(y_all[off:off + T.n])
            off += T.n
        for T, yk in zip(trees, ys):
            mg.mg_eval_exact(T.handle, yk, xr, xs, xa)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.exact_steps):
            for T, yk in zip(trees, ys):
                mg.mg_eval_exact(T.handle, yk, xr, xs, xa)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.exact_steps
        exact = {"ms_per_step": dt * 1e3, "window_rays_per_s": n_total * sen.n_el * sen.w_buf / dt,
                 "steps": args.exact_steps, "over_depth_buffer": dt * 1e3 / batched_ms,
                 "path": "mg_eval_exact per tree (hash sets of the window rays' unknown voxels; X_ray, X_set, A_set)"}
        # the exact planner gain with its own yaw choice (depth order, hash sets), the device
        # counterpart of the paper's exact CPU implementation
        ge, ye = torch.empty_like(xr), torch.empty_like(xr)
        for T in trees:
            mg.mg_eval_exact_marginal(T.handle, ge, ye)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.exact_steps):
            for T in trees:
                mg.mg_eval_exact_marginal(T.handle, ge, ye)
        torch.cuda.synchronize()
        dt2 = (time.perf_counter() - t0) / args.exact_steps
        exact["own_yaw"] = {"ms_per_step": dt2 * 1e3, "rays_per_s": rays_per_step / dt2,
                            "over_depth_buffer": dt2 * 1e3 / batched_ms,
                            "path": "mg_eval_exact_marginal per tree"}
        out["exact"] = exact
        log(f"[bench] exact: {exact}")
    if "batched" in m["results"]:
        # the path score runs on the evaluated batch (it needs its plan), after the exact leg
        # rewrote nothing it reads (gains are passed in)
        out["path_score"] = score_bench(mg, trees, m["g_all"], n_total,
                                        int(sum(t.depth().sum() for t in w.trees)))
        log(f"[bench] path score: {out['path_score']}")
    return out


def summary_of(m):
    """The compact record of an extra workload."""
    r = {"workload": f"{m['w'].name}: {W_DESC(m['w'].name)}", "trees": len(m["trees"]), "nodes": m["n_total"],
         "rays_per_step": m["rays_per_step"], "modes": m["results"], "roofline": m["roof"],
         "launch_shape": m["launch_shape"]}
    if "batched" in m["results"]:
        r["rays_per_s"] = m["results"]["batched"]["rays_per_s"]
        r["ms_per_step"] = m["results"]["batched"]["ms_per_step"]
    return r


def W_DESC(name):
    from paper_2609_40297_amd import workloads as W
    return W.WORKLOADS[name]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; use --gpus 1"}))
        log("bench.py: only --gpus 1 is supported (the library runs on one GPU)")
        sys.exit(2)
    if args.profile_summary:
        print(profile_summary(args.profile_summary, args.steps))
        return
    if args.copy_probe_mib:
        return copy_probe(args.copy_probe_mib)
    if args.map_bench_only:
        import torch
        from paper_2609_40297_amd import mg
        torch.cuda.set_device(0)
        print(json.dumps({"maps": map_bench(mg, reps=3)}), flush=True)
        return
    if args.workload == "serve16":
        return serve_bench(args)
    import torch
    from paper_2609_40297_amd import mg, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mg.lib()
    modes = args.modes.split(",")
    extras = args.extras
    if extras is None:
        extras = "step,batch64" if args.workload == "large" and args.trees is None else "none"
    extras = [] if extras == "none" else [e for e in extras.split(",") if e and e != args.workload]

    head = measure(mg, W, args.workload, args.steps, args.warmup, modes, n_trees=args.trees)
    R = head["results"][head["main_mode"]]
    rows = {}
    if not extras:
        rows = next_rows(mg, head, args)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on the host threads, bounded sample)")
        per_thread = args.cpu_sample_rays or (0.3e6 if args.workload == "large" else 1.5e6)
        cpu = cpu_baseline(head["w"], per_thread)
        log(f"[bench] cpu: {cpu}")
    line_extras = {}
    head_summary = {"workload": f"{args.workload}: {W.WORKLOADS[args.workload]}", "trees": len(head["trees"]),
                    "nodes": head["n_total"], "rays_per_step": head["rays_per_step"], "mode": head["main_mode"],
                    "launch_shape": head["launch_shape"]}
    close(head)
    for name in extras:
        ex = measure(mg, W, name, max(3, args.steps) if name != "step" else 20, max(1, args.warmup), modes)
        line_extras[name] = summary_of(ex)
        if name == "step":
            rows = next_rows(mg, ex, args)
            if cpu is not None:
                rows_cpu = {"path_score": score_oracle(ex["w"])}
                rows_cpu.update(next_row_oracles(ex["w"], cpu_threads()))
                line_extras[name]["cpu_baseline_next_rows"] = rows_cpu
        close(ex)
    mapb = map_bench(mg) if args.map_bench else None
    if mapb:
        log(f"[bench] maps: {mapb}")

    line = {
        "metric": "marginal-gain rays/s + replan p50/p99 ms, batched vs plain, 1xMI355X",
        "value": R["rays_per_s"],
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head_summary,
        "p50_ms": R["p50_ms"],
        "p99_ms": R["p99_ms"],
        "modes": head["results"],
        "roofline": head["roof"],
        "cpu_baseline": cpu,
        "extras": line_extras,
        "next_rows_on": "step" if "step" in line_extras else args.workload,
        "single_parent": rows.get("single_parent"),
        "interval": rows.get("interval"),
        "exact": rows.get("exact"),
        "path_score": rows.get("path_score"),
        "maps": mapb,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
