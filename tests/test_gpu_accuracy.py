"""The device accuracy study (paper_2609_40297_amd/accuracy.py) against the oracle's error report
on the same workload: every gain and exact count is integer, so the statistics must agree to
rounding."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_40297_amd import mg as mgmod
    mgmod.lib()
    return mgmod


def test_study_matches_oracle_report(mg):
    from oracle import error_report
    from paper_2609_40297_amd import accuracy
    dev = accuracy.study("tiny")
    ref = error_report.report("tiny", n_threads=8)
    assert dev["nodes"] == ref["nodes_evaluated"] == 20
    for k in ("slope", "r2", "overestimate_pct"):
        assert dev["depth_buffer"][k] == pytest.approx(ref[k], rel=1e-12, abs=1e-12), k
        assert dev["interval"][k] == pytest.approx(ref["interval"][k], rel=1e-12, abs=1e-12), k
    for a, b in zip(dev["per_depth"], ref["per_depth"]):
        assert a["depth"] == b["depth"] and a["nodes"] == b["nodes"]
        assert a["db"] == pytest.approx(b["db_over_exact"], rel=1e-12)
        assert a["sp"] == pytest.approx(b["sp_over_exact"], rel=1e-12)
        assert a["abs"] == pytest.approx(b["abs_over_exact"], rel=1e-12)
    for a, b in zip(dev["interval_per_depth"], ref["interval"]["per_depth"]):
        assert a["interval"] == pytest.approx(b["over_exact"], rel=1e-12)
