"""Comparison of GPU library results with the CPU oracle.

Bars (see the arithmetic in the fit): track lists -- seeds, order, grain
lists and grain order, fit axis and the FP64 flag -- must be identical;
slopes as angles atan(s) and the direction vector within 1e-5 rad; centroid
within 4 FP32 ulps of its magnitude plus 1e-5 um; the extent along the
direction within 1e-3 um (FP32 dot products of coordinates up to ~3.5 mm).
"""
from __future__ import annotations

import math

import numpy as np

ANGLE_TOL = 1e-5


def _angle(u, v) -> float:
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    c = float(np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v)))
    return math.acos(max(-1.0, min(1.0, c)))


def assert_view_parity(xyz, got: dict, ref, check_fit: bool = True) -> None:
    tr = got["tracks"]
    assert got["n_seeds"] == ref.n_seeds, (got["n_seeds"], ref.n_seeds)
    assert got["n_candidates"] == len(ref.cand), (got["n_candidates"], len(ref.cand))
    assert len(tr) == len(ref.tracks), (len(tr), len(ref.tracks))
    for k, rt in enumerate(ref.tracks):
        g = tr[k]
        assert (int(g["seed"][0]), int(g["seed"][1])) == (rt["i"], rt["j"]), k
        assert int(g["n_grains"]) == rt["n_grains"], k
        off = int(g["grain_offset"])
        mine = got["grains"][off:off + int(g["n_grains"])]
        assert np.array_equal(mine, ref.track_grains(k)), k
        if not check_fit:
            continue
        assert int(g["axis"]) == rt["axis"], k
        assert int(g["fit_fp64"]) == rt["fit_fp64"], k
        assert int(g["degenerate"]) == rt["degenerate"], k
        for s in range(2):
            d = abs(math.atan(float(g["slope"][s])) - math.atan(rt["slope"][s]))
            assert d <= ANGLE_TOL, (k, s, d)
        assert _angle(g["dir"], rt["dir"]) <= ANGLE_TOL, k
        c_ref = np.asarray(rt["centroid"])
        tol = 4 * np.spacing(np.abs(c_ref).astype(np.float32)).astype(np.float64) + 1e-5
        assert np.all(np.abs(g["centroid"] - c_ref) <= tol), (k, g["centroid"], c_ref)
        assert abs(float(g["t_begin"]) - rt["t_begin"]) <= 1e-3, k
        assert abs(float(g["t_end"]) - rt["t_end"]) <= 1e-3, k


def assert_candidates_equal(got_ijn, ref) -> None:
    """Candidate lists element by element: the device's list (any order)
    sorted into the priority order (n descending, then i, j) must equal the
    oracle's (i, j, n) list exactly."""
    g = np.asarray(got_ijn, np.int64).reshape(-1, 3)
    order = np.lexsort((g[:, 1], g[:, 0], -g[:, 2]))
    g = g[order]
    r = np.asarray(ref.cand, np.int64).reshape(-1, 3)
    assert g.shape == r.shape, (g.shape, r.shape)
    bad = np.nonzero(np.any(g != r, axis=1))[0]
    assert len(bad) == 0, (bad[:5], g[bad[:5]], r[bad[:5]])
