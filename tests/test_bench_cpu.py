"""Host-side parts of bench.py (no GPU): the one-GPU refusal, the oracle work counts that define
the roofline numerator, and the rule that a committed traffic summary applies only to the kernel
sources it was measured with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_large_work_counts_give_the_documented_algorithmic_bytes():
    wc = bench.work_counts("large", 8 * 3000 * 720 * 120)
    assert wc["counted"] == "all trees, exact" and wc["nodes"] == 24000 and wc["rays"] == 2073600000
    per_step = wc["visits"] + 4 * wc["anc_tests"] + 4 * wc["rays"] + 2 * 72 * 4 * wc["nodes"]
    assert per_step == pytest.approx(757.57e9, rel=1e-4)


def test_step_work_counts_give_the_documented_algorithmic_bytes():
    wc = bench.work_counts("step")
    assert wc["nodes"] == 500 and wc["rays"] == 500 * 360 * 60
    assert 0 < wc["unk_visits"] < wc["visits"]
    # 1 B per voxel visit, 4 B per ancestor test, 4 B per first hit written, 2 B x 4 B of bins per node
    per_step = wc["visits"] + 4 * wc["anc_tests"] + 4 * wc["rays"] + 2 * 36 * 4 * wc["nodes"]
    assert per_step == pytest.approx(4.342e9, rel=1e-3)


def test_traffic_summary_applies_only_to_its_sources(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("// version 1\n")
    summary = tmp_path / "traffic.md"
    summary.write_text("# traffic\n\n- hbm_bytes_per_launch: 12345\n"
                       f"- kernel_source_sha256: `{bench.kernel_source_hash([str(src)])}`\n")
    assert bench.summary_traffic(str(summary), [str(src)]) == 12345.0
    src.write_text("// version 2\n")
    assert bench.summary_traffic(str(summary), [str(src)]) is None
    assert bench.summary_traffic(str(tmp_path / "missing.md"), [str(src)]) is None



def test_roofline_uses_the_union_of_launch_intervals():
    wc = {"visits": 1000, "anc_tests": 100, "rays": 10, "counted": "all trees, exact"}
    trace = {"launches": 6, "busy_ms": 2.0, "total_ms": 3.0}
    r = bench.roofline_of(wc, trace, steps=2, n_total=2, yaw_bins=4, ms_per_step=5.0, traffic=None)
    alg = 1000 + 4 * 100 + 4 * 10 + 2 * 2 * 4 * 4
    assert r["algorithmic_bytes_per_step"] == alg
    assert r["busy_ms_per_step"] == 1.0 and r["summed_launch_ms_per_step"] == 1.5
    assert r["achieved"] == pytest.approx(alg / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["achieved_over_whole_step"] == pytest.approx(alg / 5e-3 / 1e9)
    assert bench.roofline_of(None, trace, 2, 2, 4, 5.0, None) is None


def test_partial_work_counts_are_scaled_by_rays(tmp_path, monkeypatch):
    d = tmp_path / "tests" / "golden"
    d.mkdir(parents=True)
    (d / "work_counts.json").write_text(json.dumps({
        "w": {"visits": 300, "unk_visits": 30, "anc_tests": 60, "rays": 100, "nodes": 2, "trees": 4,
              "trees_counted": 1},
        "v": {"visits": 7, "unk_visits": 1, "anc_tests": 2, "rays": 5, "nodes": 1, "trees": 1,
              "trees_counted": 1}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    w = bench.work_counts("w", 400)
    assert (w["visits"], w["unk_visits"], w["anc_tests"], w["rays"]) == (1200, 120, 240, 400)
    assert "first 1 of 4 trees" in w["counted"]
    v = bench.work_counts("v", 5)
    assert v["visits"] == 7 and v["counted"] == "all trees, exact"
    assert bench.work_counts("missing", 5) is None
