"""Host-only checks of the C ABI: the library loads without a GPU, exports
every function the header declares, agrees with the header on struct layout,
and rejects bad configurations and views before touching a device."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emt.h")


@pytest.fixture(scope="module")
def emt():
    from paper_1311_5334_amd import emt as m
    m.load()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(emt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(emt):
    names = declared_functions()
    assert set(names) == set(emt.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", emt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (emt_[a-z0-9_]+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(emt.load(), n)


def test_struct_layout_matches_header(emt):
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "emt.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(emt_config) S(emt_view_in) S(emt_track) S(emt_view_stats) S(emt_view_out) S(emt_call_stats)
  S(emt_served) S(emt_server_stats) S(emt_stack_geom) S(emt_server_limits) S(emt_peaks)
  O(emt_peaks, hbm_copy_bytes) O(emt_peaks, clock_khz)
  O(emt_server_limits, max_batch_grains)
  O(emt_stack_geom, threshold) O(emt_stack_geom, pitch_den)
  O(emt_config, hbm_budget) O(emt_config, stream) O(emt_config, cyl_ext)
  O(emt_config, thr_slope) O(emt_config, thr_max) O(emt_track, slope) O(emt_track, t_end)
  O(emt_view_out, tracks) O(emt_view_out, stats) O(emt_call_stats, ms) O(emt_call_stats, ms_total)
  O(emt_served, tracks) O(emt_served, stats) O(emt_served, t_done_ms)
  O(emt_server_stats, busy_ms) O(emt_server_stats, elapsed_ms)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in lines if line)
    exp = {
        "emt_config": C.sizeof(emt.EmtConfig), "emt_view_in": C.sizeof(emt.EmtViewIn),
        "emt_track": C.sizeof(emt.EmtTrack), "emt_view_stats": C.sizeof(emt.EmtViewStats),
        "emt_view_out": C.sizeof(emt.EmtViewOut), "emt_call_stats": C.sizeof(emt.EmtCallStats),
        "emt_config.hbm_budget": emt.EmtConfig.hbm_budget.offset,
        "emt_config.stream": emt.EmtConfig.stream.offset,
        "emt_config.cyl_ext": emt.EmtConfig.cyl_ext.offset,
        "emt_config.thr_slope": emt.EmtConfig.thr_slope.offset,
        "emt_config.thr_max": emt.EmtConfig.thr_max.offset,
        "emt_track.slope": emt.EmtTrack.slope.offset,
        "emt_track.t_end": emt.EmtTrack.t_end.offset,
        "emt_view_out.tracks": emt.EmtViewOut.tracks.offset,
        "emt_view_out.stats": emt.EmtViewOut.stats.offset,
        "emt_call_stats.ms": emt.EmtCallStats.ms.offset,
        "emt_call_stats.ms_total": emt.EmtCallStats.ms_total.offset,
        "emt_served": C.sizeof(emt.EmtServed), "emt_server_stats": C.sizeof(emt.EmtServerStats),
        "emt_stack_geom": C.sizeof(emt.EmtStackGeom),
        "emt_server_limits": C.sizeof(emt.EmtServerLimits),
        "emt_peaks": C.sizeof(emt.EmtPeaks),
        "emt_peaks.hbm_copy_bytes": emt.EmtPeaks.hbm_copy_bytes.offset,
        "emt_peaks.clock_khz": emt.EmtPeaks.clock_khz.offset,
        "emt_server_limits.max_batch_grains": emt.EmtServerLimits.max_batch_grains.offset,
        "emt_stack_geom.threshold": emt.EmtStackGeom.threshold.offset,
        "emt_stack_geom.pitch_den": emt.EmtStackGeom.pitch_den.offset,
        "emt_served.tracks": emt.EmtServed.tracks.offset,
        "emt_served.stats": emt.EmtServed.stats.offset,
        "emt_served.t_done_ms": emt.EmtServed.t_done_ms.offset,
        "emt_server_stats.busy_ms": emt.EmtServerStats.busy_ms.offset,
        "emt_server_stats.elapsed_ms": emt.EmtServerStats.elapsed_ms.offset,
    }
    for k, v in exp.items():
        assert int(got[k]) == v, (k, got[k], v)
    assert emt.TRACK_DTYPE.itemsize == C.sizeof(emt.EmtTrack)


def test_defaults_and_strerror(emt):
    cfg = emt.emt_default_config()
    assert cfg.abi_version == emt.EMT_ABI_VERSION
    assert (cfg.seed_dist, cfg.tol_radius, cfg.min_grains) == (2500, 50, 8)
    assert (cfg.cyl_ext, tuple(cfg.thr_slope), cfg.thr_max) == (-1, (0, 1), 0)
    for rc in (0, -1, -2, -3, -4, -5):
        assert emt.emt_strerror(rc)
    assert emt.emt_strerror(12345) == "unknown error"


@pytest.mark.parametrize("field,value,rc", [
    ("abi_version", 7, -1), ("flags", 0x100, -1), ("cell", (-5, 0, 0), -1), ("device", -1, -1),
    ("seed_dist", 0, -2), ("seed_dist", 4097, -2), ("tol_radius", -1, -2),
    ("tol_radius", 2500, -2), ("min_grains", 1, -2), ("min_grains", 1 << 20, -2),
    ("cell", (0, 0, (1 << 18) + 1), -2), ("cyl_ext", -2, -2), ("cyl_ext", (1 << 18) + 1, -2),
    ("thr_slope", (-1, 1), -2), ("thr_slope", (1025, 1), -2), ("thr_slope", (1, 0), -2),
    ("thr_slope", (1, 1025), -2), ("thr_max", -1, -2), ("thr_max", 7, -2),
    ("thr_max", 1 << 20, -2),
])
def test_validate_rejects_bad_config(emt, field, value, rc):
    cfg = emt.emt_default_config(**{field: value})
    assert emt.emt_validate(cfg) == rc


@pytest.mark.parametrize("field,value", [
    ("cyl_ext", 0), ("cyl_ext", 1 << 18), ("thr_slope", (1024, 1024)), ("thr_slope", (0, 1)),
    ("thr_max", 8), ("thr_max", (1 << 20) - 1)])
def test_validate_accepts_variant_limits(emt, field, value):
    assert emt.emt_validate(emt.emt_default_config(**{field: value})) == 0


def test_validate_views(emt):
    cfg = emt.emt_default_config()
    ok = np.array([[0, 0, 0], [100, 200, 300]], np.int32)
    assert emt.emt_validate(cfg, [ok, np.zeros((0, 3), np.int32)]) == 0
    wide = np.array([[0, 0, 0], [(1 << 18) + 1, 0, 0]], np.int32)
    assert emt.emt_validate(cfg, [ok, wide]) == -2
    edge = np.array([[0, 0, 0], [0, 0, 1 << 18]], np.int32)
    assert emt.emt_validate(cfg, [edge]) == 0
    neg = np.array([[-(1 << 17), 0, 0], [(1 << 17) + 1, 0, 0]], np.int32)
    assert emt.emt_validate(cfg, [neg]) == -2


def test_validate_null_and_count(emt):
    lib = emt.load()
    cfg = emt.emt_default_config()
    assert lib.emt_validate(None, None, 0) == -1
    assert lib.emt_validate(C.byref(cfg), None, 1) == -1
    v = (emt.EmtViewIn * 1)()
    v[0].xyz = None
    v[0].n_grains = 5
    assert lib.emt_validate(C.byref(cfg), v, 1) == -1
    v[0].n_grains = 1 << 20
    v[0].xyz = 8  # never read: the count is rejected first
    assert lib.emt_validate(C.byref(cfg), v, 1) == -2


def test_create_and_track_reject_null_without_device(emt):
    lib = emt.load()
    assert lib.emt_create(None, None) == -1
    h = C.c_void_p()
    bad = emt.emt_default_config(abi_version=3)
    assert lib.emt_create(C.byref(bad), C.byref(h)) == -1
    assert h.value is None
    assert lib.emt_track_views(None, None, 0, None) == -1
    assert lib.emt_last_stats(None, None) == -1
    lib.emt_destroy(None)


def test_server_rejects_bad_arguments_without_device(emt):
    lib = emt.load()
    cfg = emt.emt_default_config()
    h = C.c_void_p()
    assert lib.emt_server_create(None, 2, 8, C.byref(h)) == -1
    assert lib.emt_server_create(C.byref(cfg), 2, 8, None) == -1
    assert lib.emt_server_create(C.byref(cfg), 0, 8, C.byref(h)) == -1
    assert lib.emt_server_create(C.byref(cfg), 9, 8, C.byref(h)) == -1
    assert lib.emt_server_create(C.byref(cfg), 2, 0, C.byref(h)) == -1
    dev = emt.emt_default_config(flags=emt.EMT_F_DEVICE_PTRS)
    assert lib.emt_server_create(C.byref(dev), 2, 8, C.byref(h)) == -1
    bad = emt.emt_default_config(seed_dist=0)
    assert lib.emt_server_create(C.byref(bad), 2, 8, C.byref(h)) == -2
    assert h.value is None
    n = C.c_uint32()
    assert lib.emt_server_submit(None, None, None) == -1
    assert lib.emt_server_poll(None, None, 0, C.byref(n), 0) == -1
    assert lib.emt_server_get_stats(None, None) == -1
    lib.emt_server_destroy(None)


def test_find_grains_rejects_null_without_device(emt):
    lib = emt.load()
    n = C.c_uint32(7)
    g = emt.stack_geom((4, 8, 16), 60)
    assert lib.emt_find_grains(None, None, C.byref(g), None, 0, C.byref(n)) == -1
    assert lib.emt_find_grains(None, None, None, None, 0, None) == -1


def test_filter_stack_rejects_null_without_device(emt):
    lib = emt.load()
    g = emt.stack_geom((4, 8, 16), 0)
    assert lib.emt_filter_stack(None, None, C.byref(g), None, None, None) == -1
    assert lib.emt_filter_stack(None, None, None, None, None, None) == -1


def test_filter_binding_rejects_a_wrong_output_buffer(emt):
    """The binding refuses an output array the library would write past."""
    raw = np.zeros((2, 3, 8), np.uint8)
    gain = np.zeros((3, 8), np.uint16)
    thr = np.zeros((3, 8), np.uint8)
    for bad in (np.zeros(10, np.uint8), np.zeros((2, 3, 8), np.int32),
                np.zeros((2, 3, 16), np.uint8)[:, :, ::2]):
        with pytest.raises(TypeError):
            emt.emt_filter_stack(None, raw, gain, thr, out=bad)
    with pytest.raises(ValueError):
        emt.emt_filter_stack(None, raw, np.zeros((3, 4), np.uint16), thr)
