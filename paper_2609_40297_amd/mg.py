"""Python binding of the C ABI in ``include/mg.h`` (argument marshalling only).

Every step of the gain evaluation runs in the HIP library ``libmg.so``; this
module converts numpy arrays and torch tensors to pointers and raises on error
codes. Importing it loads the library and fails loudly when it is missing:
there is no fallback implementation.

Device outputs are torch tensors on the current device; the HIP stream passed
to the library is ``torch.cuda.current_stream()`` unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

MG_OK, MG_E_INVALID, MG_E_NOMEM, MG_E_DEVICE, MG_E_BUSY, MG_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
_NAMES = {-1: "MG_E_INVALID", -2: "MG_E_NOMEM", -3: "MG_E_DEVICE", -4: "MG_E_BUSY", -5: "MG_E_UNSUPPORTED",
          -6: "MG_E_CANCELLED"}
MG_E_INVALID, MG_E_NOMEM, MG_E_DEVICE, MG_E_BUSY, MG_E_UNSUPPORTED, MG_E_CANCELLED = -1, -2, -3, -4, -5, -6

# Every entry point declared in include/mg.h.
EXPORTS = ("mg_map_create", "mg_map_destroy", "mg_tree_upload", "mg_tree_destroy", "mg_tree_nodes",
           "mg_tree_buffer_pixels", "mg_tree_footprint_bytes", "mg_eval_marginal", "mg_eval_marginal_levelsync",
           "mg_eval_marginal_batch", "mg_eval_absolute", "mg_eval_single_parent", "mg_sensor_tables", "mg_last_error",
           "mg_server_create", "mg_server_submit", "mg_server_poll", "mg_server_wait", "mg_server_stats",
           "mg_server_destroy", "mg_timing_enable", "mg_timing_read", "mg_batch_config", "mg_trace_shapes",
           "mg_batch_plan_info", "mg_score_branches", "mg_eval_interval", "mg_interval_tables",
           "mg_interval_config", "mg_map_create_tsdf", "mg_map_update_tsdf", "mg_map_update", "mg_map_read",
           "mg_eval_exact", "mg_server_map_update", "mg_eval_exact_marginal", "mg_eval_marginal_batch_noalloc",
           "mg_server_cancel", "mg_server_fail_request", "mg_server_pause", "mg_batch_barrier_polls",
           "mg_map_read_marked")


class MGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class mg_sensor(C.Structure):
    _fields_ = [("n_az", C.c_int32), ("n_el", C.c_int32), ("fov_h_deg", C.c_float), ("fov_v_deg", C.c_float),
                ("range_m", C.c_float), ("yaw_bins", C.c_int32), ("az_offset_deg", C.c_float)]


class mg_server_config(C.Structure):
    _fields_ = [("sensor", mg_sensor), ("max_inflight", C.c_int32), ("arena_bytes", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.mg_map_create.argtypes = [P, I32, I32, I32, C.c_float, P, P, C.POINTER(P)]
        L.mg_map_destroy.argtypes = [P]
        L.mg_tree_upload.argtypes = [P, P, P, I32, C.POINTER(mg_sensor), P, C.POINTER(P)]
        L.mg_tree_destroy.argtypes = [P]
        L.mg_tree_nodes.argtypes = [P]
        L.mg_tree_nodes.restype = I32
        L.mg_tree_buffer_pixels.argtypes = [P]
        L.mg_tree_buffer_pixels.restype = I32
        L.mg_tree_footprint_bytes.argtypes = [P]
        L.mg_tree_footprint_bytes.restype = I64
        L.mg_eval_marginal.argtypes = [P, P, P, P, P]
        L.mg_eval_single_parent.argtypes = [P, P, P, P, P]
        L.mg_eval_interval.argtypes = [P, P, I32, I32, P, P, P]
        L.mg_map_create_tsdf.argtypes = [P, P, I32, I32, I32, C.c_float, P, C.c_float, C.c_float, P, C.POINTER(P)]
        L.mg_map_update_tsdf.argtypes = [P, P, P, P, P, P, C.c_float, C.c_float]
        L.mg_map_update.argtypes = [P, P, P, P, I32, P]
        L.mg_map_read.argtypes = [P, P, P]
        L.mg_map_read_marked.argtypes = [P, P, P]
        L.mg_eval_exact.argtypes = [P, P, P, P, P, P]
        L.mg_eval_exact_marginal.argtypes = [P, P, P, P]
        L.mg_interval_config.argtypes = [I32]
        L.mg_interval_tables.argtypes = [C.POINTER(mg_sensor), C.c_float, I32, I32, P, P, P, P]
        L.mg_eval_marginal_levelsync.argtypes = [P, P, P, P, P, P, P]
        L.mg_eval_marginal_batch.argtypes = [P, I32, P, P, P, P]
        L.mg_eval_marginal_batch_noalloc.argtypes = [P, I32, P, P, P, P]
        L.mg_eval_marginal_batch_noalloc.restype = C.c_int
        L.mg_eval_absolute.argtypes = [P, P, P, P]
        L.mg_sensor_tables.argtypes = [C.POINTER(mg_sensor), P, P, P, P, P, P]
        L.mg_server_create.argtypes = [C.POINTER(mg_server_config), C.POINTER(P)]
        L.mg_server_submit.argtypes = [P, P, P, P, I32, P, P, C.POINTER(I64)]
        L.mg_server_map_update.argtypes = [P, P, P, P, I32, C.POINTER(I64)]
        L.mg_server_poll.argtypes = [P, I64, C.POINTER(I32), C.POINTER(C.c_double)]
        L.mg_server_wait.argtypes = [P, I64, C.POINTER(C.c_double)]
        L.mg_server_cancel.argtypes = [P, I64]
        L.mg_server_fail_request.argtypes = [P, I64, I32]
        L.mg_server_pause.argtypes = [P, I32]
        L.mg_batch_barrier_polls.argtypes = [I64]
        L.mg_server_stats.argtypes = [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(C.c_double), C.POINTER(I32),
                                      C.POINTER(I32)]
        L.mg_server_destroy.argtypes = [P]
        L.mg_batch_config.argtypes = [I32, I32]
        L.mg_trace_shapes.argtypes = [C.POINTER(I32), P, P, I32]
        L.mg_batch_plan_info.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I32)]
        L.mg_score_branches.argtypes = [P, I32, P, P, C.c_double, P, P, P, P]
        L.mg_timing_enable.argtypes = [I32]
        L.mg_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(I64), C.POINTER(I64)]
        L.mg_last_error.argtypes = []
        L.mg_last_error.restype = C.c_char_p
        for name in ("mg_map_create", "mg_map_destroy", "mg_tree_upload", "mg_tree_destroy", "mg_eval_marginal",
                     "mg_eval_marginal_levelsync", "mg_eval_marginal_batch", "mg_eval_absolute",
                     "mg_eval_single_parent", "mg_eval_interval", "mg_interval_tables",
                     "mg_sensor_tables", "mg_server_create", "mg_server_submit", "mg_server_poll",
                     "mg_server_wait", "mg_server_stats", "mg_server_destroy", "mg_timing_enable",
                     "mg_timing_read", "mg_batch_config", "mg_trace_shapes", "mg_batch_plan_info",
                     "mg_score_branches", "mg_server_cancel", "mg_server_fail_request", "mg_server_pause", "mg_batch_barrier_polls"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != MG_OK:
        raise MGError(rc, lib().mg_last_error().decode())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_sensor(s) -> mg_sensor:
    return mg_sensor(int(s.n_az), int(s.n_el), float(s.fov_h_deg), float(s.fov_v_deg), float(s.range_m),
                     int(s.yaw_bins), float(getattr(s, "az_offset_deg", 0.0)))


# ----------------------------------------------------------------- raw entry points (same names)

def mg_map_create(states: np.ndarray, voxel_m: float, origin_m, stream=None) -> int:
    st = np.ascontiguousarray(states, dtype=np.uint8)
    nz, ny, nx = st.shape
    org = np.ascontiguousarray(origin_m, dtype=np.float32)
    out = C.c_void_p()
    _check(lib().mg_map_create(_np_ptr(st), nx, ny, nz, float(voxel_m), _np_ptr(org), _stream(stream),
                               C.byref(out)))
    return out.value


def mg_map_destroy(handle: int):
    _check(lib().mg_map_destroy(C.c_void_p(handle)))


def mg_tree_upload(map_handle: int, pos_m: np.ndarray, parent: np.ndarray, sensor, stream=None) -> int:
    pos = np.ascontiguousarray(pos_m, dtype=np.float32)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    sp = make_sensor(sensor)
    out = C.c_void_p()
    _check(lib().mg_tree_upload(C.c_void_p(map_handle), _np_ptr(pos), _np_ptr(par), int(par.shape[0]),
                                C.byref(sp), _stream(stream), C.byref(out)))
    return out.value


def mg_tree_destroy(handle: int):
    _check(lib().mg_tree_destroy(C.c_void_p(handle)))


def mg_tree_footprint_bytes(handle: int) -> int:
    return int(lib().mg_tree_footprint_bytes(C.c_void_p(handle)))


def mg_eval_marginal(tree: int, gain, yaw_bin, depth=None, stream=None):
    _check(lib().mg_eval_marginal(C.c_void_p(tree), _stream(stream), _dev_ptr(gain), _dev_ptr(yaw_bin),
                                  _dev_ptr(depth)))


def mg_eval_interval(tree: int, wd: int, hd: int, gain, yaw_bin, depth=None, stream=None):
    _check(lib().mg_eval_interval(C.c_void_p(tree), _stream(stream), int(wd), int(hd), _dev_ptr(gain),
                                  _dev_ptr(yaw_bin), _dev_ptr(depth)))


def mg_interval_config(cap: int = -1):
    _check(lib().mg_interval_config(int(cap)))


def interval_tables(sensor, voxel_m, wd=0, hd=0):
    """Host tables of the interval-mode camera: (wd, hd, intr[6], pdir[hd, wd, 3], cs[B, 2])."""
    s = make_sensor(sensor)
    wh = np.zeros(2, np.int32)
    _check(lib().mg_interval_tables(C.byref(s), float(voxel_m), int(wd), int(hd), _np_ptr(wh), None, None, None))
    W, H = int(wh[0]), int(wh[1])
    intr = np.zeros(6, np.float32)
    pdir = np.zeros((H, W, 3), np.float32)
    cs = np.zeros((s.yaw_bins, 2), np.float32)
    _check(lib().mg_interval_tables(C.byref(s), float(voxel_m), int(wd), int(hd), _np_ptr(wh), _np_ptr(intr),
                                    _np_ptr(pdir), _np_ptr(cs)))
    return W, H, intr, pdir, cs


def mg_eval_exact(tree: int, yaw_bin, x_ray, x_set=None, a_set=None, stream=None):
    _check(lib().mg_eval_exact(C.c_void_p(tree), _stream(stream), _dev_ptr(yaw_bin), _dev_ptr(x_ray), _dev_ptr(x_set),
                               _dev_ptr(a_set)))


def mg_eval_exact_marginal(tree: int, gain, yaw_bin, stream=None):
    _check(lib().mg_eval_exact_marginal(C.c_void_p(tree), _stream(stream), _dev_ptr(gain), _dev_ptr(yaw_bin)))


def mg_eval_single_parent(tree: int, gain, yaw_bin, depth=None, stream=None):
    _check(lib().mg_eval_single_parent(C.c_void_p(tree), _stream(stream), _dev_ptr(gain), _dev_ptr(yaw_bin),
                                       _dev_ptr(depth)))


def mg_eval_marginal_levelsync(tree: int, host_gain: np.ndarray, host_yaw: np.ndarray, gain=None, yaw_bin=None,
                               depth=None, stream=None):
    assert host_gain.dtype == np.uint32 and host_yaw.dtype == np.int32
    assert host_gain.flags.c_contiguous and host_yaw.flags.c_contiguous
    _check(lib().mg_eval_marginal_levelsync(C.c_void_p(tree), _stream(stream), _dev_ptr(gain), _dev_ptr(yaw_bin),
                                            _dev_ptr(depth), _np_ptr(host_gain), _np_ptr(host_yaw)))


def mg_eval_marginal_batch(trees: Sequence[int], gain, yaw_bin, depth=None, stream=None):
    arr = (C.c_void_p * len(trees))(*trees)
    _check(lib().mg_eval_marginal_batch(C.cast(arr, C.c_void_p), len(trees), _stream(stream), _dev_ptr(gain),
                                        _dev_ptr(yaw_bin), _dev_ptr(depth)))


def mg_eval_marginal_batch_noalloc(trees: Sequence[int], gain, yaw_bin, depth=None, stream=None):
    arr = (C.c_void_p * len(trees))(*trees)
    _check(lib().mg_eval_marginal_batch_noalloc(C.cast(arr, C.c_void_p), len(trees), _stream(stream),
                                                _dev_ptr(gain), _dev_ptr(yaw_bin), _dev_ptr(depth)))


def mg_eval_absolute(tree: int, gain, yaw_bin, stream=None):
    _check(lib().mg_eval_absolute(C.c_void_p(tree), _stream(stream), _dev_ptr(gain), _dev_ptr(yaw_bin)))


MG_BRANCH_LEN = 65


def mg_score_branches(trees: Sequence[int], gain, lam: float, cost, objective, best, branch=None, stream=None):
    arr = (C.c_void_p * len(trees))(*trees)
    _check(lib().mg_score_branches(C.cast(arr, C.c_void_p), len(trees), _stream(stream), _dev_ptr(gain), float(lam),
                                   _dev_ptr(cost), _dev_ptr(objective), _dev_ptr(best), _dev_ptr(branch)))


def score_batch(trees, gain, lam=0.5, stream=None):
    """Device path score of a batch already evaluated: (cost, objective, best, branch) tensors."""
    import torch
    n = sum(t.n for t in trees)
    dev = gain.device
    cost = torch.empty(n, dtype=torch.float64, device=dev)
    obj = torch.empty(n, dtype=torch.float64, device=dev)
    best = torch.empty(len(trees), dtype=torch.int32, device=dev)
    branch = torch.empty((len(trees), MG_BRANCH_LEN), dtype=torch.int32, device=dev)
    mg_score_branches([t.handle for t in trees], gain, lam, cost, obj, best, branch, stream)
    return cost, obj, best, branch


def mg_batch_config(shape: int = -1, launch: int = 0):
    """launch: 0 launches one by one on stream groups, 1 graph replay, 2 one persistent cooperative launch."""
    _check(lib().mg_batch_config(int(shape), int(launch)))


def mg_batch_barrier_polls(polls: int):
    """Polls of one grid-barrier wait of the persistent launch before it gives up."""
    _check(lib().mg_batch_barrier_polls(int(polls)))


def mg_trace_shapes():
    """[(rays per trace workgroup, bricks per mask-builder workgroup), ...] of the compiled launch shapes."""
    n = C.c_int32()
    _check(lib().mg_trace_shapes(C.byref(n), None, None, 0))
    th = np.zeros(n.value, np.int32)
    q = np.zeros(n.value, np.int32)
    _check(lib().mg_trace_shapes(C.byref(n), _np_ptr(th), _np_ptr(q), n.value))
    return list(zip(th.tolist(), q.tolist()))


def mg_batch_plan_info(trees: Sequence[int]):
    """(shape index, launch form: 0 one by one, 1 graph, 2 persistent) of the cached plan of this tree list."""
    arr = (C.c_void_p * len(trees))(*trees)
    sh, gr = C.c_int32(), C.c_int32()
    _check(lib().mg_batch_plan_info(C.cast(arr, C.c_void_p), len(trees), C.byref(sh), C.byref(gr)))
    return sh.value, int(gr.value)


def mg_timing_enable(on: bool):
    _check(lib().mg_timing_enable(1 if on else 0))


def mg_timing_read():
    """(summed trace-kernel ms, ms during which one ran, timed launches, workgroups) since the last read."""
    ms, busy, n, wg = C.c_double(), C.c_double(), C.c_int64(), C.c_int64()
    _check(lib().mg_timing_read(C.byref(ms), C.byref(busy), C.byref(n), C.byref(wg)))
    return ms.value, busy.value, n.value, wg.value


def mg_sensor_tables(sensor):
    sp = make_sensor(sensor)
    W, H, B = sp.n_az, sp.n_el, sp.yaw_bins
    out = dict(dir=np.zeros((W * H, 3), np.float32), inv=np.zeros((W * H, 3), np.float32),
               bv=np.zeros((W, 2), np.float32), ts=np.zeros(H + 1, np.float32), bins=np.zeros(W, np.int32),
               c0=np.zeros(B, np.int32))
    _check(lib().mg_sensor_tables(C.byref(sp), _np_ptr(out["dir"]), _np_ptr(out["inv"]), _np_ptr(out["bv"]),
                                  _np_ptr(out["ts"]), _np_ptr(out["bins"]), _np_ptr(out["c0"])))
    return out


# ----------------------------------------------------------------- owning wrappers

def mg_map_create_tsdf(distance, weight, voxel_m, origin_m, surface_m, min_weight, stream=None) -> int:
    """distance, weight: device float32 tensors [nz, ny, nx]."""
    nz, ny, nx = (int(v) for v in distance.shape)
    org = np.ascontiguousarray(origin_m, dtype=np.float32)
    out = C.c_void_p()
    _check(lib().mg_map_create_tsdf(_dev_ptr(distance), _dev_ptr(weight), nx, ny, nz, float(voxel_m), _np_ptr(org),
                                    float(surface_m), float(min_weight), _stream(stream), C.byref(out)))
    return out.value


def mg_map_update_tsdf(m: int, distance, weight, lo, surface_m, min_weight, stream=None):
    """distance, weight: device float32 tensors [sz, sy, sx] for the box starting at lo = (x, y, z)."""
    sz, sy, sx = (int(v) for v in distance.shape)
    lo_a = np.ascontiguousarray(lo, dtype=np.int32)
    size_a = np.array([sx, sy, sz], np.int32)
    _check(lib().mg_map_update_tsdf(C.c_void_p(m), _stream(stream), _dev_ptr(distance), _dev_ptr(weight),
                                    _np_ptr(lo_a), _np_ptr(size_a), float(surface_m), float(min_weight)))


def mg_map_update(m: int, voxel_ids, states, rejected=None, stream=None):
    """voxel_ids: device int32/uint32 tensor, states: device uint8 tensor, rejected: device int32 [1] or None."""
    _check(lib().mg_map_update(C.c_void_p(m), _stream(stream), _dev_ptr(voxel_ids), _dev_ptr(states),
                               int(voxel_ids.numel()), _dev_ptr(rejected)))


def mg_map_read(m: int, states, stream=None):
    _check(lib().mg_map_read(C.c_void_p(m), _stream(stream), _dev_ptr(states)))


def mg_map_read_marked(m: int, out, stream=None):
    _check(lib().mg_map_read_marked(C.c_void_p(m), _stream(stream), _dev_ptr(out)))


class Map:
    """Device-resident occupancy grid (wraps mg_map_create / mg_map_destroy)."""

    def __init__(self, states: np.ndarray, voxel_m: float, origin_m=(0.0, 0.0, 0.0), stream=None, handle=None):
        self.handle = handle if handle is not None else mg_map_create(states, voxel_m, origin_m, stream)
        self.shape = tuple(np.asarray(states).shape)
        self.voxel_m = float(np.float32(voxel_m))

    @classmethod
    def from_tsdf(cls, distance, weight, voxel_m, origin_m=(0.0, 0.0, 0.0), surface_m=0.0, min_weight=1e-3,
                  stream=None):
        """Map converted on the device from a TSDF (device float32 tensors [nz, ny, nx])."""
        h = mg_map_create_tsdf(distance, weight, voxel_m, origin_m, surface_m, min_weight, stream)
        return cls(np.empty(tuple(distance.shape), np.uint8), voxel_m, origin_m, handle=h)

    def read(self, stream=None):
        """Device uint8 tensor [nz, ny, nx] with the map's states."""
        import torch
        out = torch.empty(self.shape, dtype=torch.uint8, device="cuda")
        mg_map_read(self.handle, out, stream)
        return out

    def read_marked(self, stream=None):
        """Device uint8 tensor [nz, ny, nx]: each voxel's byte with its block mark (mg_map_read_marked)."""
        import torch
        out = torch.empty(self.shape, dtype=torch.uint8, device="cuda")
        mg_map_read_marked(self.handle, out, stream)
        return out

    def close(self):
        if self.handle:
            mg_map_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Device-resident candidate tree (wraps mg_tree_upload / mg_tree_destroy)."""

    def __init__(self, m: Map, pos_m: np.ndarray, parent: np.ndarray, sensor, stream=None):
        self.map = m
        self.sensor = sensor
        self.handle = mg_tree_upload(m.handle, pos_m, parent, sensor, stream)
        self.n = int(np.asarray(parent).shape[0])
        self.pixels = int(lib().mg_tree_buffer_pixels(C.c_void_p(self.handle)))

    @property
    def footprint_bytes(self) -> int:
        return mg_tree_footprint_bytes(self.handle)

    def outputs(self, depth=False, device=None):
        import torch
        dev = device or torch.device("cuda", torch.cuda.current_device())
        g = torch.empty(self.n, dtype=torch.int32, device=dev)      # uint32 bits
        y = torch.empty(self.n, dtype=torch.int32, device=dev)
        d = torch.empty((self.n, self.pixels), dtype=torch.float32, device=dev) if depth else None
        return g, y, d

    def eval_marginal(self, depth=False, stream=None):
        g, y, d = self.outputs(depth)
        mg_eval_marginal(self.handle, g, y, d, stream)
        return g, y, d

    def eval_exact(self, yaw_bin, stream=None):
        """Exact marginal gain with hash sets at the windows yaw_bin (device int32 [n]): (x_ray, x_set, a_set)."""
        import torch
        xr = torch.empty(self.n, dtype=torch.int32, device=yaw_bin.device)
        xs = torch.empty_like(xr)
        a = torch.empty_like(xr)
        mg_eval_exact(self.handle, yaw_bin, xr, xs, a, stream)
        return xr, xs, a

    def eval_exact_marginal(self, stream=None):
        """Exact marginal gain with its own yaw choice (hash sets): (gain, yaw)."""
        g, y, _ = self.outputs(False)
        mg_eval_exact_marginal(self.handle, g, y, stream)
        return g, y

    def eval_interval(self, wd=0, hd=0, depth=False, stream=None):
        """Interval mode (the paper's pinhole buffers and overlap intervals): (gain, yaw, depth or None)."""
        import torch
        W, H, _, _, _ = interval_tables(self.sensor, self.map.voxel_m, wd, hd)
        g, y, _ = self.outputs(False)
        d = torch.empty((self.n, H, W), dtype=torch.float32, device=g.device) if depth else None
        mg_eval_interval(self.handle, W, H, g, y, d, stream)
        return g, y, d

    def eval_single_parent(self, depth=False, stream=None):
        g, y, d = self.outputs(depth)
        mg_eval_single_parent(self.handle, g, y, d, stream)
        return g, y, d

    def eval_absolute(self, stream=None):
        g, y, _ = self.outputs(False)
        mg_eval_absolute(self.handle, g, y, stream)
        return g, y

    def close(self):
        if self.handle:
            mg_tree_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_batch(trees: Sequence[Tree], depth=False, stream=None):
    import torch
    n = sum(t.n for t in trees)
    dev = torch.device("cuda", torch.cuda.current_device())
    g = torch.empty(n, dtype=torch.int32, device=dev)
    y = torch.empty(n, dtype=torch.int32, device=dev)
    d = torch.empty((n, trees[0].pixels), dtype=torch.float32, device=dev) if depth else None
    mg_eval_marginal_batch([t.handle for t in trees], g, y, d, stream)
    return g, y, d


def as_u32(t) -> np.ndarray:
    """Host copy of an int32 tensor holding uint32 gains."""
    return t.cpu().numpy().view(np.uint32)


class Server:
    """Continuous-batching request server (wraps the mg_server_* calls)."""

    def __init__(self, sensor, max_inflight=16, arena_bytes=8 << 30):
        cfg = mg_server_config(make_sensor(sensor), int(max_inflight), int(arena_bytes))
        out = C.c_void_p()
        _check(lib().mg_server_create(C.byref(cfg), C.byref(out)))
        self.handle = out.value
        self._keep = {}

    def submit(self, m: Map, pos_m, parent) -> int:
        pos = np.ascontiguousarray(pos_m, dtype=np.float32)
        par = np.ascontiguousarray(parent, dtype=np.int32)
        n = int(par.shape[0])
        g = np.zeros(n, np.uint32)
        y = np.zeros(n, np.int32)
        t = C.c_int64()
        _check(lib().mg_server_submit(C.c_void_p(self.handle), C.c_void_p(m.handle), _np_ptr(pos), _np_ptr(par), n,
                                      _np_ptr(g), _np_ptr(y), C.byref(t)))
        self._keep[t.value] = (g, y)
        return t.value

    def map_update(self, m: Map, voxel_ids, states) -> int:
        """Queues new states for listed voxels of map m (applied after the requests submitted before it)."""
        ids = np.ascontiguousarray(voxel_ids, dtype=np.uint32)
        st = np.ascontiguousarray(states, dtype=np.uint8)
        t = C.c_int64()
        _check(lib().mg_server_map_update(C.c_void_p(self.handle), C.c_void_p(m.handle), _np_ptr(ids), _np_ptr(st),
                                          int(ids.size), C.byref(t)))
        self._keep[t.value] = (None, None)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (gain, yaw, latency_us)."""
        st = C.c_int32()
        lat = C.c_double()
        _check(lib().mg_server_poll(C.c_void_p(self.handle), C.c_int64(ticket), C.byref(st), C.byref(lat)))
        if st.value == 0:
            return None
        g, y = self._keep.pop(ticket, (None, None))
        if st.value < 0:
            raise MGError(st.value, "request failed")
        return g, y, lat.value

    def wait(self, ticket: int):
        lat = C.c_double()
        rc = lib().mg_server_wait(C.c_void_p(self.handle), C.c_int64(ticket), C.byref(lat))
        g, y = self._keep.pop(ticket, (None, None))    # (an unknown ticket fails in _check)
        _check(rc)
        return g, y, lat.value

    def cancel(self, ticket: int):
        """Cancels a queued or in-flight request (it then reports MG_E_CANCELLED)."""
        _check(lib().mg_server_cancel(C.c_void_p(self.handle), C.c_int64(ticket)))

    def fail_request(self, ticket: int, code: int = MG_E_DEVICE):
        """Marks a request failed with `code` through its device status word."""
        _check(lib().mg_server_fail_request(C.c_void_p(self.handle), C.c_int64(ticket), int(code)))

    def pause(self, paused: bool):
        """Stops (True) or resumes (False) the steps; requests are still admitted while paused."""
        _check(lib().mg_server_pause(C.c_void_p(self.handle), 1 if paused else 0))

    def stats(self):
        steps, done, q, f = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        rays = C.c_double()
        _check(lib().mg_server_stats(C.c_void_p(self.handle), C.byref(steps), C.byref(done), C.byref(rays),
                                     C.byref(f), C.byref(q)))
        return dict(steps=steps.value, completed=done.value, rays=rays.value, in_flight=f.value, queued=q.value)

    def close(self):
        if self.handle:
            _check(lib().mg_server_destroy(C.c_void_p(self.handle)))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
