"""ctypes wrapper of the interval-mode oracle (``ivlref.c`` in ``libmgref.so``; test infrastructure only).

Same conventions as ``mgref.py``: numpy arrays and workload objects in, numpy
arrays out, no arithmetic of its own.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from oracle import mgref
from oracle.mgref import SensorParams, _p, sensor_params


class Counters(C.Structure):
    _fields_ = [("visits", C.c_uint64), ("unk_visits", C.c_uint64), ("pixel_steps", C.c_uint64),
                ("intervals", C.c_uint64), ("max_merged", C.c_uint64)]


class Camera(C.Structure):
    _fields_ = [("wd", C.c_int32), ("hd", C.c_int32), ("B", C.c_int32), ("w", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("znear", C.c_float), ("rv", C.c_float),
                ("pdir", C.POINTER(C.c_float)), ("cs", C.POINTER(C.c_float))]


_ready = False


def lib():
    global _ready
    L = mgref.lib()
    if not _ready:
        P = C.c_void_p
        I32 = C.c_int32
        L.ivlref_camera_init.argtypes = [C.POINTER(SensorParams), C.c_float, I32, I32, C.POINTER(Camera)]
        L.ivlref_camera_init.restype = C.c_int
        L.ivlref_camera_free.argtypes = [C.POINTER(Camera)]
        L.ivlref_camera_tables.argtypes = [C.POINTER(SensorParams), C.c_float, I32, I32, P, P, P, P]
        L.ivlref_camera_tables.restype = C.c_int
        L.ivlref_render.argtypes = [P, I32, I32, I32, C.POINTER(Camera), P, I32, P]
        L.ivlref_render.restype = C.c_int
        L.ivlref_intervals.argtypes = [C.POINTER(Camera), P, P, P, I32, P, P, I32, C.POINTER(C.c_uint64)]
        L.ivlref_intervals.restype = I32
        L.ivlref_eval_tree.argtypes = [P, I32, I32, I32, C.c_float, P, P, P, I32, C.POINTER(SensorParams),
                                       I32, I32, P, P, P, P, P, P, P, P, C.POINTER(Counters), I32]
        L.ivlref_eval_tree.restype = C.c_int
        L.ivlref_merge.argtypes = [P, I32, P, I32, P]
        L.ivlref_merge.restype = I32
        L.mgref_trace_ray_exit.argtypes = [P, I32, I32, I32, P, P, P, C.c_float, I32, P, P, P, P, P]
        L.mgref_trace_ray_exit.restype = C.c_int
        _ready = True
    return L


def camera_tables(sensor, voxel_m, wd=0, hd=0):
    """(wd, hd, intrinsics [fx, fy, cx, cy, znear, rv], pixel directions [hd, wd, 3], yaw cos/sin [B, 2])."""
    sp = sensor_params(sensor)
    wh = np.zeros(2, np.int32)
    if lib().ivlref_camera_tables(C.byref(sp), float(voxel_m), int(wd), int(hd), _p(wh), None, None, None) != 0:
        raise ValueError("oracle rejected the camera")
    W, H = int(wh[0]), int(wh[1])
    intr = np.zeros(6, np.float32)
    pdir = np.zeros((H, W, 3), np.float32)
    cs = np.zeros((sp.yaw_bins, 2), np.float32)
    lib().ivlref_camera_tables(C.byref(sp), float(voxel_m), int(wd), int(hd), _p(wh), _p(intr), _p(pdir), _p(cs))
    return W, H, intr, pdir, cs


class CameraHandle:
    def __init__(self, sensor, voxel_m, wd=0, hd=0):
        self.sp = sensor_params(sensor)
        self.cam = Camera()
        if lib().ivlref_camera_init(C.byref(self.sp), float(voxel_m), int(wd), int(hd), C.byref(self.cam)) != 0:
            raise ValueError("oracle rejected the camera")

    def __del__(self):
        try:
            lib().ivlref_camera_free(C.byref(self.cam))
        except Exception:
            pass


def render(states, cam: CameraHandle, q, k):
    st = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st.shape
    D = np.zeros((cam.cam.hd, cam.cam.wd), np.float32)
    qq = np.ascontiguousarray(q, dtype=np.float32)
    if lib().ivlref_render(_p(st), nx, ny, nz, C.byref(cam.cam), _p(qq), int(k), _p(D)) != 0:
        raise ValueError("oracle render failed")
    return D


def intervals(cam: CameraHandle, qn, d, qa, ka, Da, cap=4096):
    """Overlap intervals [m, 2] of one ancestor on one candidate ray (0 <= t <= Rv), and the pixels visited."""
    out = np.zeros((cap, 2), np.float32)
    steps = C.c_uint64(0)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    Dd = f(Da)
    n = lib().ivlref_intervals(C.byref(cam.cam), _p(f(qn)), _p(f(d)), _p(f(qa)), int(ka), _p(Dd), _p(out), cap,
                               C.byref(steps))
    if n > cap:
        raise ValueError("interval cap too small")
    return out[:n].copy(), int(steps.value)


def merge(M, S):
    """Union of two sorted lists of disjoint intervals ([m, 2] and [ns, 2] float32)."""
    M = np.ascontiguousarray(M, dtype=np.float32).reshape(-1, 2)
    S = np.ascontiguousarray(S, dtype=np.float32).reshape(-1, 2)
    out = np.zeros((len(M) + len(S), 2), np.float32)
    n = lib().ivlref_merge(_p(M), len(M), _p(S), len(S), _p(out))
    return out[:n].copy()


def trace_ray_exit(states, q, d, inv, rv, cap=4096):
    st3 = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st3.shape
    ids = np.zeros(cap, np.uint32)
    st = np.zeros(cap, np.uint8)
    te = np.zeros(cap, np.float32)
    tx = np.zeros(cap, np.float32)
    h = C.c_float(0)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    n = lib().mgref_trace_ray_exit(_p(st3), nx, ny, nz, _p(f(q)), _p(f(d)), _p(f(inv)), float(np.float32(rv)), cap,
                                   _p(ids), _p(st), _p(te), _p(tx), C.byref(h))
    if n < 0:
        raise ValueError("cap too small")
    return ids[:n], st[:n], te[:n], tx[:n], h.value


def eval_tree(m, tree, sensor, wd=0, hd=0, mask=None, n_threads=1, want_bins=False):
    """Depth-ordered interval-mode evaluation of one tree. Returns a dict of numpy arrays."""
    sp = sensor_params(sensor)
    W, H, _, _, _ = camera_tables(sensor, m.voxel_m, wd, hd)
    st = np.ascontiguousarray(m.states, dtype=np.uint8)
    nz, ny, nx = st.shape
    n = tree.n
    out = dict(g_abs=np.zeros(n, np.uint32), k_abs=np.full(n, -1, np.int32),
               g_db=np.zeros(n, np.uint32), k_db=np.full(n, -1, np.int32),
               D=np.zeros((n, H, W), np.float32))
    if want_bins:
        out["abs_bins"] = np.zeros((n, sp.yaw_bins), np.uint32)
        out["marg_bins"] = np.zeros((n, sp.yaw_bins), np.uint32)
    cnt = Counters()
    origin = np.ascontiguousarray(m.origin_m, dtype=np.float32)
    pos = np.ascontiguousarray(tree.pos_m, dtype=np.float32)
    par = np.ascontiguousarray(tree.parent, dtype=np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().ivlref_eval_tree(_p(st), nx, ny, nz, float(m.voxel_m), _p(origin), _p(pos), _p(par), n, C.byref(sp),
                                int(W), int(H), _p(mk), _p(out["g_abs"]), _p(out["k_abs"]), _p(out["g_db"]),
                                _p(out["k_db"]), _p(out["D"]), _p(out.get("abs_bins")), _p(out.get("marg_bins")),
                                C.byref(cnt), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    out["counters"] = dict(visits=cnt.visits, unk_visits=cnt.unk_visits, pixel_steps=cnt.pixel_steps,
                           intervals=cnt.intervals, max_merged=cnt.max_merged)
    out["wd"], out["hd"] = W, H
    return out
