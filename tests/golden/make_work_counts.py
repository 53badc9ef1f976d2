"""Writes work_counts.json: per-workload work of the method, counted by the oracle.

visits V (voxels visited by the DDA), unk_visits U (unknown ones), anc_tests T
(ancestor tests, parent first, stopping at the first that observes), rays R.
These are the numerators of the roofline figures (algorithmic bytes per ray:
V/R grid gathers of 1 byte, T/R depth reads of 4 bytes, one 4-byte first-hit
write). Entries named "<workload>/interval" hold the interval mode's work:
V, U, pixel_steps (pixels walked by the 2D DDAs, one 4-byte depth read
each), merged intervals, and the buffer size. Calls only the oracle and the
workload generator.

Multi-tree workloads are counted tree by tree and the file is rewritten after
each tree, with "trees_counted" out of "trees": an interrupted run resumes at
the next tree, and a partial entry holds exact counts of the first trees.

Usage: python tests/golden/make_work_counts.py [workload[/interval] ...]
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ivlref, mgref  # noqa: E402
from paper_2609_40297_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "work_counts.json")
KEYS = ("visits", "unk_visits", "anc_tests")
IKEYS = ("visits", "unk_visits", "pixel_steps", "intervals")


def count(name, prev, save, n_trees=None):
    w = W.make(name, n_trees=n_trees)
    tot = dict(visits=0, unk_visits=0, anc_tests=0, rays=0, nodes=0, trees_counted=0)
    if prev and prev.get("trees", 1) == len(w.trees) and "trees_counted" in prev:
        tot.update({k: prev[k] for k in tot})
    for i, t in enumerate(w.trees):
        if i < tot["trees_counted"]:
            continue
        o = mgref.eval_tree(w.map, t, w.sensor, n_threads=os.cpu_count() or 1)
        for k in KEYS:
            tot[k] += int(o["counters"][k])
        tot["rays"] += t.n * w.sensor.rays
        tot["nodes"] += t.n
        tot["trees_counted"] = i + 1
        save(dict(tot, trees=len(w.trees)))
    return dict(tot, trees=len(w.trees))


def count_interval(name, prev, save, n_trees=None):
    w = W.make(name, n_trees=n_trees)
    tot = dict(visits=0, unk_visits=0, pixel_steps=0, intervals=0, max_merged=0, rays=0, nodes=0)
    for t in w.trees:
        o = ivlref.eval_tree(w.map, t, w.sensor, n_threads=os.cpu_count() or 1)
        for k in IKEYS:
            tot[k] += int(o["counters"][k])
        tot["max_merged"] = max(tot["max_merged"], int(o["counters"]["max_merged"]))
        tot["rays"] += t.n * w.sensor.rays
        tot["nodes"] += t.n
        tot["wd"], tot["hd"] = int(o["wd"]), int(o["hd"])
    return tot


if __name__ == "__main__":
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}

    def write():
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)

    for arg in sys.argv[1:] or ["tiny", "step"]:
        base, _, mode = arg.partition("/")
        name, _, nt = base.partition(":")

        def save(entry, arg=arg):
            data[arg] = entry
            print(arg, entry, flush=True)
            write()

        fn = count_interval if mode == "interval" else count
        data[arg] = fn(name, data.get(arg), save, int(nt) if nt else None)
        print(arg, data[arg], flush=True)
        write()
