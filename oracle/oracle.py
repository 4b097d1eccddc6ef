"""ctypes loader for the CPU oracle (``emt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark. The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emt_oracle.c")
LIB = os.path.join(HERE, "libemt_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "emt_oracle.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("seed_dist", C.c_int64), ("tol_radius", C.c_int64),
                ("min_grains", C.c_int32), ("scan_all", C.c_int32),
                ("cell", C.c_int32 * 3), ("thr_num", C.c_int32), ("thr_den", C.c_int32),
                ("thr_max", C.c_int32), ("cyl_ext", C.c_int64)]


class _Cand(C.Structure):
    _fields_ = [("i", C.c_uint32), ("j", C.c_uint32), ("n", C.c_uint32)]


class _Track(C.Structure):
    _fields_ = [("i", C.c_uint32), ("j", C.c_uint32),
                ("grain_offset", C.c_uint32), ("n_grains", C.c_uint32),
                ("axis", C.c_uint32), ("fit_fp64", C.c_uint32),
                ("degenerate", C.c_uint32),
                ("slope", C.c_double * 2), ("dir", C.c_double * 3),
                ("centroid", C.c_double * 3),
                ("t_begin", C.c_double), ("t_end", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("n_seeds", C.c_uint64), ("n_tests", C.c_uint64),
                ("n_cand", C.c_uint32), ("cand", C.POINTER(_Cand)),
                ("n_tracks", C.c_uint32), ("tracks", C.POINTER(_Track)),
                ("n_track_grains", C.c_uint32), ("grains", C.POINTER(C.c_uint32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.emto_track_view.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(_Params),
                                         C.POINTER(_Result)]
        _lib.emto_track_view.restype = C.c_int
        _lib.emto_free.argtypes = [C.POINTER(_Result)]
        _lib.emto_count_seed.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32,
                                         C.c_uint32, C.c_int64]
        _lib.emto_count_seed.restype = C.c_uint32
    return _lib


@dataclass
class OracleResult:
    n_seeds: int
    n_tests: int
    cand: np.ndarray          # (K, 3) uint32: i, j, n in priority order
    tracks: list              # dicts in acceptance order
    grains: np.ndarray        # uint32, concatenated per-track grain lists

    def track_grains(self, t: int) -> np.ndarray:
        tr = self.tracks[t]
        return self.grains[tr["grain_offset"]:tr["grain_offset"] + tr["n_grains"]]


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__(f"oracle error {rc}")
        self.rc = rc


def track_view(xyz, R: int = 2500, r: int = 50, n_min: int = 8,
               scan_all: bool = False, cell=(750, 750, 170), cyl_ext: int = -1,
               thr_slope=(0, 1), thr_max: int = 0) -> OracleResult:
    """Track one view. Acceptance variants: cyl_ext >= 0 counts only grains
    projecting at most cyl_ext units beyond a seed grain (finite cylinder);
    thr_slope = (num, den) raises the grain-count threshold to
    n_min + ceil(num/den tan(theta)) of the seed, capped at thr_max if set."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    p = _Params(R, r, n_min, 1 if scan_all else 0, (C.c_int32 * 3)(*cell),
                int(thr_slope[0]), int(thr_slope[1]), int(thr_max), int(cyl_ext))
    res = _Result()
    rc = lib.emto_track_view(a.ctypes.data if a.size else None, a.shape[0],
                             C.byref(p), C.byref(res))
    if rc != 0:
        raise OracleError(rc)
    try:
        k = res.n_cand
        cand = np.zeros((k, 3), np.uint32)
        if k:
            buf = np.ctypeslib.as_array(C.cast(res.cand, C.POINTER(C.c_uint32)),
                                        shape=(k * 3,))
            cand[:] = buf.reshape(k, 3)
        tracks = []
        for t in range(res.n_tracks):
            T = res.tracks[t]
            tracks.append({
                "i": T.i, "j": T.j, "grain_offset": T.grain_offset,
                "n_grains": T.n_grains, "axis": T.axis, "fit_fp64": T.fit_fp64,
                "degenerate": T.degenerate, "slope": (T.slope[0], T.slope[1]),
                "dir": (T.dir[0], T.dir[1], T.dir[2]),
                "centroid": (T.centroid[0], T.centroid[1], T.centroid[2]),
                "t_begin": T.t_begin, "t_end": T.t_end})
        ng = res.n_track_grains
        grains = np.zeros(ng, np.uint32)
        if ng:
            grains[:] = np.ctypeslib.as_array(res.grains, shape=(ng,))
        return OracleResult(int(res.n_seeds), int(res.n_tests), cand, tracks, grains)
    finally:
        lib.emto_free(C.byref(res))


def count_seed(xyz, i: int, j: int, r: int = 50) -> int:
    lib = _load()
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    return int(lib.emto_count_seed(a.ctypes.data, a.shape[0], i, j, r))
