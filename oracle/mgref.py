"""ctypes wrapper of the oracle library ``libmgref.so`` (test infrastructure only).

``build()`` compiles ``mgref.c`` and ``ivlref.c`` (the interval mode) with gcc (-O2 -ffp-contract=off, no fast-math)
into this directory. The wrapper takes numpy arrays and workload objects and
returns numpy arrays; it does no arithmetic of its own.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "mgref.c"), os.path.join(HERE, "ivlref.c")]
# MGREF_LIB selects another build of the same sources (the sanitizer build of the tests)
LIB = os.environ.get("MGREF_LIB") or os.path.join(HERE, "libmgref.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fno-unsafe-math-optimizations", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter"]
# host-only AddressSanitizer + UndefinedBehaviorSanitizer build (any report aborts the process)
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True, out: Optional[str] = None, sanitize: bool = False) -> str:
    out = out or LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *(SANITIZE if sanitize else []), *SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class SensorParams(C.Structure):
    _fields_ = [("n_az", C.c_int32), ("n_el", C.c_int32), ("fov_h_deg", C.c_float),
                ("fov_v_deg", C.c_float), ("range_m", C.c_float), ("yaw_bins", C.c_int32),
                ("az_offset_deg", C.c_float)]


class Counters(C.Structure):
    _fields_ = [("visits", C.c_uint64), ("unk_visits", C.c_uint64), ("anc_tests", C.c_uint64)]


class _Sensor(C.Structure):
    _fields_ = [("p", SensorParams), ("win_bins", C.c_int32), ("w_buf", C.c_int32),
                ("dir", C.POINTER(C.c_float)), ("inv", C.POINTER(C.c_float)),
                ("bvx", C.POINTER(C.c_float)), ("bvy", C.POINTER(C.c_float)),
                ("ts", C.POINTER(C.c_float)), ("bin_of_col", C.POINTER(C.c_int32)),
                ("c0_of_win", C.POINTER(C.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.mgref_sensor_tables.argtypes = [C.POINTER(SensorParams), P, P, P, P, P, P]
        L.mgref_sensor_tables.restype = C.c_int
        L.mgref_sensor_init.argtypes = [C.POINTER(SensorParams), C.POINTER(_Sensor)]
        L.mgref_sensor_init.restype = C.c_int
        L.mgref_sensor_free.argtypes = [C.POINTER(_Sensor)]
        L.mgref_trace_ray.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_float,
                                      C.c_int32, P, P, P, P]
        L.mgref_trace_ray.restype = C.c_int
        L.mgref_obs.argtypes = [C.POINTER(_Sensor), P, C.c_int32, P, C.c_int32, C.c_int32, C.c_int32,
                                P, P]
        L.mgref_obs.restype = C.c_int
        L.mgref_eval_node.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(SensorParams),
                                      C.c_float, P, C.c_int32, P, P, P, P, P, P, C.POINTER(Counters)]
        L.mgref_eval_node.restype = C.c_int
        L.mgref_node_set.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(SensorParams),
                                     C.c_float, P, C.c_int32, C.c_int64, P]
        L.mgref_node_set.restype = C.c_int64
        L.mgref_best_window.argtypes = [P, C.c_int32, C.c_int32, P]
        L.mgref_best_window.restype = C.c_uint32
        L.mgref_eval_tree.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_int32,
                                      C.POINTER(SensorParams), C.c_int32, P, P, P, P, P, P, P, P,
                                      C.POINTER(Counters), C.c_int32]
        L.mgref_eval_tree.restype = C.c_int
        L.mgref_exact.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_int32,
                                  C.POINTER(SensorParams), P, P, P, P, P, P, P]
        L.mgref_exact.restype = C.c_int
        L.mgref_exact_marginal.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_int32,
                                           C.POINTER(SensorParams), P, P, P]
        L.mgref_exact_marginal.restype = C.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def sensor_params(sensor) -> SensorParams:
    return SensorParams(int(sensor.n_az), int(sensor.n_el), float(sensor.fov_h_deg),
                        float(sensor.fov_v_deg), float(sensor.range_m), int(sensor.yaw_bins),
                        float(getattr(sensor, "az_offset_deg", 0.0)))


def sensor_tables(sensor):
    sp = sensor_params(sensor)
    W, H, B = sp.n_az, sp.n_el, sp.yaw_bins
    out = dict(dir=np.zeros((W * H, 3), np.float32), inv=np.zeros((W * H, 3), np.float32),
               bv=np.zeros((W, 2), np.float32), ts=np.zeros(H + 1, np.float32),
               bins=np.zeros(W, np.int32), c0=np.zeros(B, np.int32))
    rc = lib().mgref_sensor_tables(C.byref(sp), _p(out["dir"]), _p(out["inv"]), _p(out["bv"]),
                                   _p(out["ts"]), _p(out["bins"]), _p(out["c0"]))
    if rc != 0:
        raise ValueError("sensor not representable")
    return out


class SensorHandle:
    """Oracle sensor tables kept alive for repeated ``obs`` calls."""

    def __init__(self, sensor):
        self.sp = sensor_params(sensor)
        self.s = _Sensor()
        if lib().mgref_sensor_init(C.byref(self.sp), C.byref(self.s)) != 0:
            raise ValueError("sensor not representable")
        self.w_buf = self.s.w_buf
        self.win_bins = self.s.win_bins

    def obs(self, qa, c0a, Da, ix, iy, iz):
        qa = np.ascontiguousarray(qa, dtype=np.float32)
        Da = np.ascontiguousarray(Da, dtype=np.float32)
        row = C.c_int32()
        col = C.c_int32()
        r = lib().mgref_obs(C.byref(self.s), _p(qa), int(c0a), _p(Da), int(ix), int(iy), int(iz),
                            C.byref(row), C.byref(col))
        return bool(r), row.value, col.value

    def __del__(self):
        try:
            lib().mgref_sensor_free(C.byref(self.s))
        except Exception:
            pass


def trace_ray(states, q, d, inv, rv, cap=4096):
    st3 = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st3.shape
    q = np.ascontiguousarray(q, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    inv = np.ascontiguousarray(inv, dtype=np.float32)
    ids = np.zeros(cap, np.uint32)
    st = np.zeros(cap, np.uint8)
    te = np.zeros(cap, np.float32)
    h = np.zeros(1, np.float32)
    n = lib().mgref_trace_ray(_p(st3), nx, ny, nz, _p(q), _p(d), _p(inv), float(np.float32(rv)), cap,
                              _p(ids), _p(st), _p(te), _p(h))
    if n < 0:
        raise RuntimeError("trace buffer too small")
    return ids[:n].copy(), st[:n].copy(), te[:n].copy(), float(h[0])


def eval_node(states, sensor, rv, q, anc_q, anc_c0, anc_D):
    """One node against explicitly given ancestors (nearest first)."""
    sp = sensor_params(sensor)
    st = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st.shape
    q = np.ascontiguousarray(q, dtype=np.float32)
    na = len(anc_c0)
    aq = np.ascontiguousarray(np.asarray(anc_q, dtype=np.float32).reshape(na, 3))
    ac0 = np.ascontiguousarray(np.asarray(anc_c0, dtype=np.int32).reshape(na))
    aD = np.ascontiguousarray(np.asarray(anc_D, dtype=np.float32))
    ab = np.zeros(sp.yaw_bins, np.uint32)
    mb = np.zeros(sp.yaw_bins, np.uint32)
    h = np.zeros(sp.n_az * sp.n_el, np.float32)
    cnt = Counters()
    rc = lib().mgref_eval_node(_p(st), nx, ny, nz, C.byref(sp), float(np.float32(rv)), _p(q), na,
                               _p(aq), _p(ac0), _p(aD), _p(ab), _p(mb), _p(h), C.byref(cnt))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return ab, mb, h


def node_set(states, sensor, rv, q, k, cap=1 << 22):
    sp = sensor_params(sensor)
    st = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st.shape
    q = np.ascontiguousarray(q, dtype=np.float32)
    out = np.zeros(cap, np.uint32)
    n = lib().mgref_node_set(_p(st), nx, ny, nz, C.byref(sp), float(np.float32(rv)), _p(q), int(k),
                             int(cap), _p(out))
    if n < 0:
        raise RuntimeError("node_set failed")
    return out[:n].copy()


def best_window(bins, w):
    bins = np.ascontiguousarray(bins, dtype=np.uint32)
    k = C.c_int32()
    g = lib().mgref_best_window(_p(bins), int(bins.shape[0]), int(w), C.byref(k))
    return int(g), k.value


def eval_tree(m, tree, sensor, max_anc=-1, mask=None, n_threads=1, want_bins=False):
    """Depth-ordered evaluation of one tree. Returns a dict of numpy arrays."""
    sp = sensor_params(sensor)
    st = np.ascontiguousarray(m.states, dtype=np.uint8)
    nz, ny, nx = st.shape
    n = tree.n
    H, B = sp.n_el, sp.yaw_bins
    handle = SensorHandle(sensor)
    WB = handle.w_buf
    out = dict(g_abs=np.zeros(n, np.uint32), k_abs=np.full(n, -1, np.int32),
               g_db=np.zeros(n, np.uint32), k_db=np.full(n, -1, np.int32),
               D=np.zeros((n, H, WB), np.float32))
    if want_bins:
        out["abs_bins"] = np.zeros((n, B), np.uint32)
        out["marg_bins"] = np.zeros((n, B), np.uint32)
    cnt = Counters()
    origin = np.ascontiguousarray(m.origin_m, dtype=np.float32)
    pos = np.ascontiguousarray(tree.pos_m, dtype=np.float32)
    par = np.ascontiguousarray(tree.parent, dtype=np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().mgref_eval_tree(_p(st), nx, ny, nz, float(m.voxel_m), _p(origin), _p(pos), _p(par), n,
                               C.byref(sp), int(max_anc), _p(mk), _p(out["g_abs"]), _p(out["k_abs"]),
                               _p(out["g_db"]), _p(out["k_db"]), _p(out["D"]),
                               _p(out.get("abs_bins")), _p(out.get("marg_bins")), C.byref(cnt),
                               int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    out["counters"] = dict(visits=cnt.visits, unk_visits=cnt.unk_visits, anc_tests=cnt.anc_tests)
    return out


def exact(m, tree, sensor, k_db, D, mask=None):
    sp = sensor_params(sensor)
    st = np.ascontiguousarray(m.states, dtype=np.uint8)
    nz, ny, nx = st.shape
    n = tree.n
    out = dict(A_set=np.zeros(n, np.uint32), X_set=np.zeros(n, np.uint32),
               X_ray=np.zeros(n, np.uint32), G_db_set=np.zeros(n, np.uint32))
    origin = np.ascontiguousarray(m.origin_m, dtype=np.float32)
    pos = np.ascontiguousarray(tree.pos_m, dtype=np.float32)
    par = np.ascontiguousarray(tree.parent, dtype=np.int32)
    kd = np.ascontiguousarray(k_db, dtype=np.int32)
    Dd = np.ascontiguousarray(D, dtype=np.float32)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().mgref_exact(_p(st), nx, ny, nz, float(m.voxel_m), _p(origin), _p(pos), _p(par), n,
                           C.byref(sp), _p(kd), _p(Dd), _p(mk), _p(out["A_set"]), _p(out["X_set"]),
                           _p(out["X_ray"]), _p(out["G_db_set"]))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return out


def ancestor_closure(parent, nodes):
    """Mask of the given nodes plus all their ancestors."""
    parent = np.asarray(parent)
    mask = np.zeros(parent.shape[0], np.uint8)
    for i in nodes:
        i = int(i)
        while i >= 0 and not mask[i]:
            mask[i] = 1
            i = int(parent[i])
    return mask


def exact_marginal(m, tree, sensor, mask=None):
    """Exact marginal gain with its own yaw choice: dict(g_ex, k_ex)."""
    sp = sensor_params(sensor)
    st = np.ascontiguousarray(m.states, dtype=np.uint8)
    nz, ny, nx = st.shape
    n = tree.n
    out = dict(g_ex=np.zeros(n, np.uint32), k_ex=np.full(n, -1, np.int32))
    origin = np.ascontiguousarray(m.origin_m, dtype=np.float32)
    pos = np.ascontiguousarray(tree.pos_m, dtype=np.float32)
    par = np.ascontiguousarray(tree.parent, dtype=np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().mgref_exact_marginal(_p(st), nx, ny, nz, float(m.voxel_m), _p(origin), _p(pos), _p(par), n,
                                    C.byref(sp), _p(mk), _p(out["g_ex"]), _p(out["k_ex"]))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return out
