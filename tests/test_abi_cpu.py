"""Host-side checks of the HIP library that need no GPU.

The library must load, export every entry point its header declares, validate
its inputs on the host (returning an error before any device work), and build
exactly the sensor tables the oracle builds (same double-precision recipe,
written independently on each side).
"""
import os
import re

import numpy as np
import pytest

from paper_2609_40297_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mglib():
    from paper_2609_40297_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        from paper_2609_40297_amd import build
        build.build()
    return mg


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|int32_t|int64_t|const char\*)\s+(mg_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol(mglib):
    declared = _declared()
    assert "mg_eval_marginal" in declared and "mg_map_create" in declared
    L = mglib.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(mglib.EXPORTS)


def test_library_exports_via_nm(mglib):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", mglib.LIB_PATH], capture_output=True, text=True).stdout
    syms = set(re.findall(r"\bT (mg_\w+)", out))
    assert _declared() <= syms


@pytest.mark.parametrize("sen", [W.SENSOR_TINY, W.SENSOR_STEP, W.SENSOR_LARGE,
                                 dict(n_az=4, n_el=1, fov_h_deg=90, fov_v_deg=60, range_m=3.0, yaw_bins=4,
                                      az_offset_deg=-45.0),
                                 dict(n_az=100, n_el=7, fov_h_deg=90, fov_v_deg=50, range_m=3.0, yaw_bins=36,
                                      az_offset_deg=12.5)])
def test_sensor_tables_equal_oracle_bitwise(mglib, oracle_lib, sen):
    s = W.Sensor(**sen)
    a = mglib.mg_sensor_tables(s)
    b = oracle_lib.sensor_tables(s)
    for k in ("dir", "inv", "bv", "ts", "bins", "c0"):
        assert a[k].tobytes() == b[k].tobytes(), k


@pytest.mark.parametrize("sen,v,wd,hd", [(W.SENSOR_TINY, 0.2, 0, 0), (W.SENSOR_STEP, 0.1, 0, 0),
                                         (W.SENSOR_LARGE, 0.05, 0, 0), (W.SENSOR_STEP, 0.1, 37, 21),
                                         (dict(n_az=100, n_el=7, fov_h_deg=90, fov_v_deg=50, range_m=3.0,
                                               yaw_bins=36, az_offset_deg=12.5), 0.25, 0, 0)])
def test_interval_camera_equals_oracle_bitwise(mglib, oracle_lib, sen, v, wd, hd):
    from oracle import ivlref
    s = W.Sensor(**sen)
    a = mglib.interval_tables(s, v, wd, hd)
    b = ivlref.camera_tables(s, v, wd, hd)
    assert a[:2] == b[:2]
    for x, y in zip(a[2:], b[2:]):
        assert x.tobytes() == y.tobytes()


def test_host_validation_errors(mglib):
    mg = mglib
    st = np.zeros((4, 4, 4), np.uint8)
    with pytest.raises(mg.MGError) as e:
        mg.mg_map_create(np.full((4, 4, 4), 3, np.uint8), 0.1, (0, 0, 0), stream=0)
    assert e.value.code == mg.MG_E_INVALID
    with pytest.raises(mg.MGError) as e:
        mg.mg_map_create(st, -1.0, (0, 0, 0), stream=0)
    assert e.value.code == mg.MG_E_INVALID
    with pytest.raises(mg.MGError) as e:
        mg.mg_sensor_tables(W.Sensor(n_az=50, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=5, yaw_bins=36))
    assert e.value.code == mg.MG_E_INVALID
    with pytest.raises(mg.MGError) as e:
        mg.mg_sensor_tables(W.Sensor(n_az=8192, n_el=4, fov_h_deg=90, fov_v_deg=60, range_m=5, yaw_bins=36))
    assert e.value.code == mg.MG_E_UNSUPPORTED
    import ctypes as C
    assert mg.lib().mg_tree_nodes(None) == -1
    assert mg.lib().mg_map_destroy(None) == mg.MG_E_INVALID
    assert mg.lib().mg_eval_marginal(None, None, None, None, None) == mg.MG_E_INVALID
    assert b"NULL" in mg.lib().mg_last_error()


def test_oracle_and_library_share_no_code():
    """Neither side includes, imports or links the other."""
    csrc = os.path.join(ROOT, "paper_2609_40297_amd", "csrc")
    for fn in os.listdir(csrc):
        txt = open(os.path.join(csrc, fn)).read()
        assert "mgref" not in txt and "oracle" not in txt.lower(), fn
    for fn in ("mg.py", "build.py", "__init__.py"):
        txt = open(os.path.join(ROOT, "paper_2609_40297_amd", fn)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, fn
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".c", ".h", ".py")):
            txt = open(os.path.join(ROOT, "oracle", fn)).read()
            assert "paper_2609_40297_amd.mg" not in txt and "mg.h" not in txt.replace("mgref.h", ""), fn


def test_launch_shape_table_and_config_validation():
    """Host-only: the compiled launch shapes and argument checks of mg_batch_config."""
    from paper_2609_40297_amd import mg
    shapes = mg.mg_trace_shapes()
    assert len(shapes) >= 2
    for th, bricks in shapes:      # rays per trace workgroup, bricks per mask-builder workgroup
        # (a builder chunk holds whole blocks of 2x2x2 bricks, at most 1024 bricks)
        assert th % 64 == 0 and 64 <= th <= 1024 and 16 <= bricks <= 1024 and bricks % 8 == 0
    for bad in [(-2, 0), (len(shapes), 0), (0, 3), (0, -1)]:
        with pytest.raises(mg.MGError) as e:
            mg._check(mg.lib().mg_batch_config(*bad))
        assert e.value.code == mg.MG_E_INVALID
    for bad in (-1, 1 << 31):
        with pytest.raises(mg.MGError) as e:
            mg.mg_batch_barrier_polls(bad)
        assert e.value.code == mg.MG_E_INVALID
