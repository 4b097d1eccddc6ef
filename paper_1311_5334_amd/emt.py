"""Python binding of the C ABI in ``include/emt.h`` (argument marshalling only).

Every computation runs in the HIP kernels of ``libemt.so``; this module only
converts arguments and results. It raises at load time if the library has not
been built, so there is no silent fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemt.so")

EMT_ABI_VERSION = 2
EMT_OK, EMT_EINVAL, EMT_ERANGE, EMT_ENOMEM, EMT_EDEVICE, EMT_EOVERFLOW = 0, -1, -2, -3, -4, -5
EMT_F_STATS, EMT_F_FP64_FIT_ALWAYS, EMT_F_DEVICE_PTRS, EMT_F_CANDIDATES = 0x1, 0x2, 0x4, 0x8
STAGES = ("stage", "bin", "seed", "count", "members", "merge", "fit", "out")
EMT_N_STAGES = len(STAGES)
EXPORTS = ("emt_default_config", "emt_validate", "emt_create", "emt_track_views",
           "emt_last_stats", "emt_destroy", "emt_strerror", "emt_server_create",
           "emt_server_submit", "emt_server_poll", "emt_server_get_stats",
           "emt_server_destroy", "emt_find_grains", "emt_filter_stack",
           "emt_view_candidates", "emt_server_create2", "emt_measure_peaks",
           "emt_find_grains_noalloc")
# the paper's view (300 x 250 x 50 um) at 1280 x 1024 x 40 pixels: pitches
# in 0.01 um units as exact fractions
PAPER_PITCH_NUM, PAPER_PITCH_DEN = (375, 3125, 125), (16, 128, 1)


class EmtConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("seed_dist", C.c_int32),
                ("tol_radius", C.c_int32), ("min_grains", C.c_int32),
                ("cell", C.c_int32 * 3), ("device", C.c_int32),
                ("flags", C.c_uint32), ("hbm_budget", C.c_uint64), ("stream", C.c_void_p),
                ("cyl_ext", C.c_int32), ("thr_slope", C.c_int32 * 2), ("thr_max", C.c_int32)]


class EmtViewIn(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n_grains", C.c_uint32), ("reserved", C.c_uint32),
                ("view_id", C.c_uint64)]


class EmtTrack(C.Structure):
    _fields_ = [("seed", C.c_uint32 * 2), ("grain_offset", C.c_uint32),
                ("n_grains", C.c_uint32), ("axis", C.c_uint32), ("fit_fp64", C.c_uint32),
                ("degenerate", C.c_uint32), ("slope", C.c_float * 2), ("dir", C.c_float * 3),
                ("centroid", C.c_float * 3), ("t_begin", C.c_float), ("t_end", C.c_float)]


class EmtViewStats(C.Structure):
    _fields_ = [("n_seeds", C.c_uint64), ("n_candidates", C.c_uint32),
                ("n_tracks", C.c_uint32)]


class EmtViewOut(C.Structure):
    _fields_ = [("view_id", C.c_uint64), ("n_tracks", C.c_uint32),
                ("n_track_grains", C.c_uint32), ("tracks", C.POINTER(EmtTrack)),
                ("grains", C.POINTER(C.c_uint32)), ("stats", EmtViewStats)]


class EmtCallStats(C.Structure):
    _fields_ = [("n_seeds", C.c_uint64), ("n_tests", C.c_uint64), ("n_hits", C.c_uint64),
                ("n_candidates", C.c_uint32), ("n_tracks", C.c_uint32),
                ("merge_rounds", C.c_uint32), ("n_fp64_fits", C.c_uint32),
                ("retries", C.c_uint32), ("n_views", C.c_uint32),
                ("ms", C.c_float * EMT_N_STAGES), ("ms_total", C.c_float)]


class EmtStackGeom(C.Structure):
    _fields_ = [("nx", C.c_uint32), ("ny", C.c_uint32), ("nz", C.c_uint32),
                ("threshold", C.c_uint32), ("pitch_num", C.c_uint32 * 3),
                ("pitch_den", C.c_uint32 * 3)]


class EmtServed(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("view_id", C.c_uint64), ("status", C.c_int32),
                ("n_tracks", C.c_uint32), ("n_track_grains", C.c_uint32),
                ("batch_views", C.c_uint32), ("tracks", C.POINTER(EmtTrack)),
                ("grains", C.POINTER(C.c_uint32)), ("stats", EmtViewStats),
                ("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double),
                ("t_done_ms", C.c_double)]


class EmtServerLimits(C.Structure):
    _fields_ = [("n_pipes", C.c_uint32), ("max_batch_views", C.c_uint32),
                ("max_batch_grains", C.c_uint64)]


class EmtServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("batches", C.c_uint64),
                ("max_batch_views_seen", C.c_uint32), ("n_pipes", C.c_uint32),
                ("busy_ms", C.c_double), ("overlap_ms", C.c_double),
                ("elapsed_ms", C.c_double)]


class EmtPeaks(C.Structure):
    _fields_ = [("int_lane_ops", C.c_double), ("fp32_lane_ops", C.c_double),
                ("lds_bytes", C.c_double), ("hbm_copy_bytes", C.c_double),
                ("compute_units", C.c_uint32), ("clock_khz", C.c_uint32)]


TRACK_DTYPE = np.dtype([("seed", "<u4", (2,)), ("grain_offset", "<u4"), ("n_grains", "<u4"),
                        ("axis", "<u4"), ("fit_fp64", "<u4"), ("degenerate", "<u4"),
                        ("slope", "<f4", (2,)), ("dir", "<f4", (3,)),
                        ("centroid", "<f4", (3,)), ("t_begin", "<f4"), ("t_end", "<f4")])
assert TRACK_DTYPE.itemsize == C.sizeof(EmtTrack)


class EmtError(RuntimeError):
    def __init__(self, rc: int, what: str = ""):
        self.rc = rc
        msg = emt_strerror(rc) if _lib is not None else str(rc)
        super().__init__(f"{what}: {msg} ({rc})" if what else f"{msg} ({rc})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libemt.so; fail loudly if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1311_5334_amd.build`")
    lib = C.CDLL(path)
    lib.emt_default_config.argtypes = [C.POINTER(EmtConfig)]
    lib.emt_default_config.restype = None
    lib.emt_validate.argtypes = [C.POINTER(EmtConfig), C.POINTER(EmtViewIn), C.c_uint32]
    lib.emt_validate.restype = C.c_int
    lib.emt_create.argtypes = [C.POINTER(EmtConfig), C.POINTER(C.c_void_p)]
    lib.emt_create.restype = C.c_int
    lib.emt_track_views.argtypes = [C.c_void_p, C.POINTER(EmtViewIn), C.c_uint32,
                                    C.POINTER(EmtViewOut)]
    lib.emt_track_views.restype = C.c_int
    lib.emt_view_candidates.argtypes = [C.c_void_p, C.c_uint32,
                                        C.POINTER(C.POINTER(C.c_uint32)),
                                        C.POINTER(C.c_uint32)]
    lib.emt_view_candidates.restype = C.c_int
    lib.emt_last_stats.argtypes = [C.c_void_p, C.POINTER(EmtCallStats)]
    lib.emt_last_stats.restype = C.c_int
    lib.emt_destroy.argtypes = [C.c_void_p]
    lib.emt_destroy.restype = None
    lib.emt_strerror.argtypes = [C.c_int]
    lib.emt_strerror.restype = C.c_char_p
    lib.emt_server_create.argtypes = [C.POINTER(EmtConfig), C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_void_p)]
    lib.emt_server_create.restype = C.c_int
    lib.emt_server_create2.argtypes = [C.POINTER(EmtConfig), C.POINTER(EmtServerLimits),
                                       C.POINTER(C.c_void_p)]
    lib.emt_server_create2.restype = C.c_int
    lib.emt_server_submit.argtypes = [C.c_void_p, C.POINTER(EmtViewIn), C.POINTER(C.c_uint64)]
    lib.emt_server_submit.restype = C.c_int
    lib.emt_server_poll.argtypes = [C.c_void_p, C.POINTER(EmtServed), C.c_uint32,
                                    C.POINTER(C.c_uint32), C.c_int32]
    lib.emt_server_poll.restype = C.c_int
    lib.emt_server_get_stats.argtypes = [C.c_void_p, C.POINTER(EmtServerStats)]
    lib.emt_server_get_stats.restype = C.c_int
    lib.emt_server_destroy.argtypes = [C.c_void_p]
    lib.emt_server_destroy.restype = None
    lib.emt_find_grains.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(EmtStackGeom), C.c_void_p,
                                    C.c_uint32, C.POINTER(C.c_uint32)]
    lib.emt_find_grains.restype = C.c_int
    lib.emt_filter_stack.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(EmtStackGeom), C.c_void_p,
                                     C.c_void_p, C.c_void_p]
    lib.emt_filter_stack.restype = C.c_int
    lib.emt_find_grains_noalloc.argtypes = lib.emt_find_grains.argtypes
    lib.emt_find_grains_noalloc.restype = C.c_int
    lib.emt_measure_peaks.argtypes = [C.c_int32, C.POINTER(EmtPeaks)]
    lib.emt_measure_peaks.restype = C.c_int
    _lib = lib
    return lib


def emt_measure_peaks(device: int = 0) -> dict:
    """Measured int32 and FP32 lane-operation rates, LDS read bandwidth and
    HBM copy bandwidth of one device (emt_measure_peaks)."""
    pk = EmtPeaks()
    rc = load().emt_measure_peaks(device, C.byref(pk))
    if rc != 0:
        raise EmtError(rc, "emt_measure_peaks")
    return {f: getattr(pk, f) for f, _ in EmtPeaks._fields_}


def emt_strerror(rc: int) -> str:
    return load().emt_strerror(rc).decode()


def emt_default_config(**overrides) -> EmtConfig:
    cfg = EmtConfig()
    load().emt_default_config(C.byref(cfg))
    for k, v in overrides.items():
        if k == "cell":
            cfg.cell = (C.c_int32 * 3)(*v)
        elif k == "thr_slope":
            cfg.thr_slope = (C.c_int32 * 2)(*v)
        else:
            setattr(cfg, k, v)
    return cfg


def _view_ins(views, device_ptrs: bool):
    """Marshal views: numpy (N,3) int32 arrays, or CUDA tensors when the
    context reads device pointers. Returns (array, keepalive)."""
    arr = (EmtViewIn * max(1, len(views)))()
    keep = []
    for i, v in enumerate(views):
        if device_ptrs:
            t = v
            if not (t.is_cuda and t.dtype.__str__() == "torch.int32" and t.is_contiguous()):
                raise TypeError("device views must be contiguous int32 CUDA tensors")
            n = int(t.shape[0]) if t.numel() else 0
            ptr = t.data_ptr() if n else None
            keep.append(t)
        else:
            a = np.ascontiguousarray(np.asarray(v, dtype=np.int32).reshape(-1, 3))
            n = int(a.shape[0])
            ptr = a.ctypes.data if n else None
            keep.append(a)
        arr[i].xyz = ptr
        arr[i].n_grains = n
        arr[i].view_id = i
    return arr, keep


def emt_validate(cfg: EmtConfig, views=()) -> int:
    arr, _keep = _view_ins(list(views), bool(cfg.flags & EMT_F_DEVICE_PTRS))
    return load().emt_validate(C.byref(cfg), arr if len(views) else None, len(views))


def emt_create(cfg: EmtConfig):
    h = C.c_void_p()
    rc = load().emt_create(C.byref(cfg), C.byref(h))
    if rc != EMT_OK:
        raise EmtError(rc, "emt_create")
    return h


def _result(nt: int, ng: int, tracks_p, grains_p):
    if nt:
        raw = np.ctypeslib.as_array(C.cast(tracks_p, C.POINTER(C.c_uint8)),
                                    shape=(nt * TRACK_DTYPE.itemsize,))
        tracks = raw.view(TRACK_DTYPE).copy()
    else:
        tracks = np.zeros(0, TRACK_DTYPE)
    grains = np.ctypeslib.as_array(grains_p, shape=(ng,)).copy() if ng else np.zeros(0, np.uint32)
    return tracks, grains


def emt_track_views(ctx, views, device_ptrs: bool = False):
    """Track a list of views; returns one dict per view with ``tracks`` (a
    numpy array of TRACK_DTYPE), ``grains`` (uint32 input indices) and
    ``stats``. Results are copied out of the context."""
    lib = load()
    views = list(views)
    arr, _keep = _view_ins(views, device_ptrs)
    out = (EmtViewOut * max(1, len(views)))()
    rc = lib.emt_track_views(ctx, arr, len(views), out)
    if rc != EMT_OK:
        raise EmtError(rc, "emt_track_views")
    res = []
    for i in range(len(views)):
        o = out[i]
        tracks, grains = _result(o.n_tracks, o.n_track_grains, o.tracks, o.grains)
        res.append({"view_id": int(o.view_id), "tracks": tracks, "grains": grains,
                    "n_seeds": int(o.stats.n_seeds),
                    "n_candidates": int(o.stats.n_candidates)})
    return res


def stack_geom(shape_zyx, threshold: int, pitch_num=PAPER_PITCH_NUM,
               pitch_den=PAPER_PITCH_DEN) -> EmtStackGeom:
    g = EmtStackGeom()
    g.nz, g.ny, g.nx = (int(v) for v in shape_zyx)
    g.threshold = threshold
    g.pitch_num = (C.c_uint32 * 3)(*pitch_num)
    g.pitch_den = (C.c_uint32 * 3)(*pitch_den)
    return g


def emt_find_grains(ctx, stack, threshold: int, device_ptrs: bool = False, max_out=None,
                    pitch_num=PAPER_PITCH_NUM, pitch_den=PAPER_PITCH_DEN, out=None):
    """Grains of a (nz, ny, nx) uint8 stack: a numpy array, or a contiguous
    uint8 CUDA tensor when the context reads device pointers. Returns an
    (n, 3) int32 array (host) or the first n rows of ``out`` / a new int32
    CUDA tensor (device)."""
    lib = load()
    g = stack_geom(stack.shape, threshold, pitch_num, pitch_den)
    n = C.c_uint32()
    if device_ptrs:
        import torch
        if not (stack.is_cuda and stack.dtype == torch.uint8 and stack.is_contiguous()):
            raise TypeError("device stacks must be contiguous uint8 CUDA tensors")
        cap = max_out if max_out is not None else max(1024, stack.numel() // 64)
        if out is None:
            out = torch.empty((cap, 3), dtype=torch.int32, device=stack.device)
        if not (out.is_cuda and out.dtype == torch.int32 and out.is_contiguous()
                and out.dim() == 2 and out.shape[1] == 3):
            raise TypeError("out must be a contiguous (n, 3) int32 CUDA tensor")
        cap = min(cap, out.shape[0])
        rc = lib.emt_find_grains(ctx, stack.data_ptr(), C.byref(g), out.data_ptr(), cap,
                                 C.byref(n))
        if rc == EMT_EOVERFLOW and max_out is None:
            out = torch.empty((n.value, 3), dtype=torch.int32, device=stack.device)
            rc = lib.emt_find_grains(ctx, stack.data_ptr(), C.byref(g), out.data_ptr(),
                                     n.value, C.byref(n))
        if rc != EMT_OK:
            raise EmtError(rc, "emt_find_grains")
        return out[:n.value]
    a = np.ascontiguousarray(np.asarray(stack, dtype=np.uint8))
    cap = max_out if max_out is not None else max(1024, a.size // 64)
    buf = np.zeros((max(cap, 1), 3), np.int32)
    rc = lib.emt_find_grains(ctx, a.ctypes.data, C.byref(g), buf.ctypes.data, cap, C.byref(n))
    if rc == EMT_EOVERFLOW and max_out is None:
        buf = np.zeros((n.value, 3), np.int32)
        rc = lib.emt_find_grains(ctx, a.ctypes.data, C.byref(g), buf.ctypes.data, n.value,
                                 C.byref(n))
    if rc != EMT_OK:
        raise EmtError(rc, "emt_find_grains")
    return buf[:n.value].copy()


def emt_filter_stack(ctx, raw, gain, thr, device_ptrs: bool = False, out=None):
    """Filter a (nz, ny, nx) uint8 stack with (ny, nx) uint16 gains (1/256
    units) and (ny, nx) uint8 thresholds: numpy arrays, or contiguous CUDA
    tensors when the context reads device pointers. Returns the filtered
    stack (numpy, or ``out`` / a new CUDA tensor)."""
    lib = load()
    nz, ny, nx = (int(v) for v in raw.shape)
    g = stack_geom(raw.shape, 0)
    if tuple(gain.shape) != (ny, nx) or tuple(thr.shape) != (ny, nx):
        raise ValueError("gain and thr must be (ny, nx) maps")
    if device_ptrs:
        import torch
        for t, size in ((raw, 1), (gain, 2), (thr, 1)):
            if not (t.is_cuda and t.is_contiguous() and t.element_size() == size):
                raise TypeError("device stacks and maps must be contiguous CUDA tensors "
                                "(8-bit stack and thresholds, 16-bit gains)")
        if out is None:
            out = torch.empty_like(raw)
        if not (out.is_cuda and out.is_contiguous() and out.element_size() == 1
                and out.numel() == raw.numel()):
            raise TypeError("out must be a contiguous 8-bit CUDA tensor of the stack's size")
        rc = lib.emt_filter_stack(ctx, raw.data_ptr(), C.byref(g), gain.data_ptr(),
                                  thr.data_ptr(), out.data_ptr())
        if rc != EMT_OK:
            raise EmtError(rc, "emt_filter_stack")
        return out
    a = np.ascontiguousarray(np.asarray(raw, dtype=np.uint8))
    gm = np.ascontiguousarray(np.asarray(gain, dtype=np.uint16))
    tm = np.ascontiguousarray(np.asarray(thr, dtype=np.uint8))
    res = np.empty_like(a) if out is None else out
    if not (isinstance(res, np.ndarray) and res.dtype == np.uint8 and res.size == a.size
            and res.flags.c_contiguous and res.flags.writeable):
        raise TypeError("out must be a writable contiguous uint8 array of the stack's size")
    rc = lib.emt_filter_stack(ctx, a.ctypes.data, C.byref(g), gm.ctypes.data, tm.ctypes.data,
                              res.ctypes.data)
    if rc != EMT_OK:
        raise EmtError(rc, "emt_filter_stack")
    return res


def emt_view_candidates(ctx, view: int) -> np.ndarray:
    """Candidates (i, j, n) of one view of the last call, as a (K, 3) uint32
    array in the device's list order (the context needs EMT_F_CANDIDATES)."""
    p = C.POINTER(C.c_uint32)()
    n = C.c_uint32()
    rc = load().emt_view_candidates(ctx, view, C.byref(p), C.byref(n))
    if rc != EMT_OK:
        raise EmtError(rc, "emt_view_candidates")
    if n.value == 0:
        return np.zeros((0, 3), np.uint32)
    return np.ctypeslib.as_array(p, shape=(3 * n.value,)).reshape(-1, 3).copy()


def emt_last_stats(ctx) -> dict:
    st = EmtCallStats()
    rc = load().emt_last_stats(ctx, C.byref(st))
    if rc != EMT_OK:
        raise EmtError(rc, "emt_last_stats")
    d = {k: getattr(st, k) for k, _ in EmtCallStats._fields_ if k != "ms"}
    d["ms"] = {name: float(st.ms[i]) for i, name in enumerate(STAGES)}
    return d


def emt_destroy(ctx) -> None:
    if ctx is not None:
        load().emt_destroy(ctx)


class Tracker:
    """A context plus convenience: ``Tracker(**cfg)(views) -> results``."""

    def __init__(self, **cfg):
        self.device_ptrs = bool(cfg.get("flags", 0) & EMT_F_DEVICE_PTRS)
        self.cfg = emt_default_config(**cfg)
        self.ctx = emt_create(self.cfg)

    def __call__(self, views):
        return emt_track_views(self.ctx, views, self.device_ptrs)

    def stats(self) -> dict:
        return emt_last_stats(self.ctx)

    def candidates(self, view: int = 0) -> np.ndarray:
        return emt_view_candidates(self.ctx, view)

    def find_grains(self, stack, threshold: int, **kw):
        return emt_find_grains(self.ctx, stack, threshold, self.device_ptrs, **kw)

    def filter_stack(self, raw, gain, thr, **kw):
        return emt_filter_stack(self.ctx, raw, gain, thr, self.device_ptrs, **kw)

    def close(self):
        if self.ctx is not None:
            emt_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The served form: ``submit`` views as they arrive, ``poll`` finished
    ones. Wraps emt_server_* (argument marshalling only)."""

    def __init__(self, n_pipes: int = 2, max_batch_views: int = 64, max_batch_grains: int = 0,
                 **cfg):
        self.cfg = emt_default_config(**cfg)
        h = C.c_void_p()
        lim = EmtServerLimits(n_pipes, max_batch_views, max_batch_grains)
        rc = load().emt_server_create2(C.byref(self.cfg), C.byref(lim), C.byref(h))
        if rc != EMT_OK:
            raise EmtError(rc, "emt_server_create")
        self.h = h
        self._buf = (EmtServed * 256)()

    def submit(self, xyz, view_id: int = 0) -> int:
        a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
        v = EmtViewIn()
        v.xyz = a.ctypes.data if len(a) else None
        v.n_grains = len(a)
        v.view_id = view_id
        t = C.c_uint64()
        rc = load().emt_server_submit(self.h, C.byref(v), C.byref(t))
        if rc != EMT_OK:
            raise EmtError(rc, "emt_server_submit")
        return int(t.value)

    def poll(self, wait_ms: int = 0, max_out: int = 256) -> list:
        """Finished views as dicts (tracks and grains copied out)."""
        max_out = min(max_out, len(self._buf))
        n = C.c_uint32()
        rc = load().emt_server_poll(self.h, self._buf, max_out, C.byref(n), wait_ms)
        res = []
        for i in range(n.value):
            o = self._buf[i]
            tracks, grains = _result(o.n_tracks, o.n_track_grains, o.tracks, o.grains)
            res.append({"ticket": int(o.ticket), "view_id": int(o.view_id),
                        "status": int(o.status), "batch_views": int(o.batch_views),
                        "tracks": tracks, "grains": grains,
                        "n_seeds": int(o.stats.n_seeds),
                        "n_candidates": int(o.stats.n_candidates),
                        "t_submit_ms": o.t_submit_ms, "t_admit_ms": o.t_admit_ms,
                        "t_done_ms": o.t_done_ms})
        if rc != EMT_OK:
            raise EmtError(rc, "emt_server_poll")
        return res

    def stats(self) -> dict:
        st = EmtServerStats()
        rc = load().emt_server_get_stats(self.h, C.byref(st))
        if rc != EMT_OK:
            raise EmtError(rc, "emt_server_get_stats")
        return {k: getattr(st, k) for k, _ in EmtServerStats._fields_}

    def close(self):
        if getattr(self, "h", None) is not None:
            load().emt_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
