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

EMT_ABI_VERSION = 1
EMT_OK, EMT_EINVAL, EMT_ERANGE, EMT_ENOMEM, EMT_EDEVICE, EMT_EOVERFLOW = 0, -1, -2, -3, -4, -5
EMT_F_STATS, EMT_F_FP64_FIT_ALWAYS, EMT_F_DEVICE_PTRS = 0x1, 0x2, 0x4
STAGES = ("stage", "bin", "seed", "count", "members", "merge", "fit", "out")
EMT_N_STAGES = len(STAGES)
EXPORTS = ("emt_default_config", "emt_validate", "emt_create", "emt_track_views",
           "emt_last_stats", "emt_destroy", "emt_strerror")


class EmtConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("seed_dist", C.c_int32),
                ("tol_radius", C.c_int32), ("min_grains", C.c_int32),
                ("cell", C.c_int32 * 3), ("device", C.c_int32),
                ("flags", C.c_uint32), ("hbm_budget", C.c_uint64), ("stream", C.c_void_p)]


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
    lib.emt_last_stats.argtypes = [C.c_void_p, C.POINTER(EmtCallStats)]
    lib.emt_last_stats.restype = C.c_int
    lib.emt_destroy.argtypes = [C.c_void_p]
    lib.emt_destroy.restype = None
    lib.emt_strerror.argtypes = [C.c_int]
    lib.emt_strerror.restype = C.c_char_p
    _lib = lib
    return lib


def emt_strerror(rc: int) -> str:
    return load().emt_strerror(rc).decode()


def emt_default_config(**overrides) -> EmtConfig:
    cfg = EmtConfig()
    load().emt_default_config(C.byref(cfg))
    for k, v in overrides.items():
        if k == "cell":
            cfg.cell = (C.c_int32 * 3)(*v)
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
        nt, ng = o.n_tracks, o.n_track_grains
        if nt:
            raw = np.ctypeslib.as_array(C.cast(o.tracks, C.POINTER(C.c_uint8)),
                                        shape=(nt * TRACK_DTYPE.itemsize,))
            tracks = raw.view(TRACK_DTYPE).copy()
        else:
            tracks = np.zeros(0, TRACK_DTYPE)
        grains = (np.ctypeslib.as_array(o.grains, shape=(ng,)).copy() if ng
                  else np.zeros(0, np.uint32))
        res.append({"view_id": int(o.view_id), "tracks": tracks, "grains": grains,
                    "n_seeds": int(o.stats.n_seeds),
                    "n_candidates": int(o.stats.n_candidates)})
    return res


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
