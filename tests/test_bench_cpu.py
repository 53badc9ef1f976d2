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

