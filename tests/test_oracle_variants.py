"""Pins of the oracle's acceptance variants: the finite cylinder around a
seed (instead of the infinite line of the tracking paragraph of Sec. 2) and
the grain-count threshold rising with the track angle (Sec. 3, the cut of
Fig. 8c), against closed forms on lattice tracks, an independent brute
force on tiny views, and exact containment relations."""
import numpy as np
import pytest

import brute
from paper_1311_5334_amd import synth

R, RT = 2500, 50


def lattice(step, n, origin=(20000, 20000, 20000)):
    return (np.asarray(origin, np.int64)[None, :] +
            np.arange(n, dtype=np.int64)[:, None] * np.asarray(step, np.int64)[None, :]
            ).astype(np.int32)


def cand_count(res, i, j):
    for ci, cj, n in res.cand.tolist():
        if (ci, cj) == (i, j):
            return n
    return 0


@pytest.mark.parametrize("step,ext,expect", [
    ((100, 0, 0), 200, 6),     # -2 .. +3 steps: both ends exactly on the boundary
    ((100, 0, 0), 199, 4),     # -1 .. +2 steps
    ((100, 0, 0), 0, 2),       # the seed grains only
    ((300, 400, 0), 500, 4),   # |d| = 500: one step beyond each seed grain
    ((300, 400, 0), 499, 2),
    ((100, 100, 0), 141, 2),   # |d| = 141.42..: 141 does not reach the next grain
    ((100, 100, 0), 142, 4),
    ((0, 0, 120), 240, 6),
])
def test_finite_cylinder_on_a_lattice(oracle_mod, step, ext, expect):
    xyz = lattice(step, 21)
    res = oracle_mod.track_view(xyz, n_min=2, cyl_ext=ext)
    # seed of the adjacent grains 10 and 11 (input order follows the lattice)
    assert cand_count(res, 10, 11) == expect
    # the infinite line holds all 21
    assert cand_count(oracle_mod.track_view(xyz, n_min=2), 10, 11) == 21


def test_finite_cylinder_extremes(oracle_mod):
    v = synth.make_c1(0)
    inf = oracle_mod.track_view(v.xyz)
    huge = oracle_mod.track_view(v.xyz, cyl_ext=1 << 18)
    assert np.array_equal(inf.cand, huge.cand)
    assert [t["i"] for t in inf.tracks] == [t["i"] for t in huge.tracks]
    # a longer cylinder only adds grains: every candidate of the shorter one
    # is a candidate of the longer one with at least as many grains
    a = {(i, j): n for i, j, n in oracle_mod.track_view(v.xyz, cyl_ext=500).cand.tolist()}
    b = {(i, j): n for i, j, n in oracle_mod.track_view(v.xyz, cyl_ext=2000).cand.tolist()}
    assert a and all(k in b and b[k] >= n for k, n in a.items())


@pytest.mark.parametrize("step,slope,cap,n_min,need", [
    ((0, 0, 100), (5, 1), 0, 6, 6),        # vertical: tan 0, the threshold stays n_min
    ((100, 0, 100), (3, 1), 0, 6, 9),      # tan 1
    ((100, 100, 100), (1, 1), 0, 6, 8),    # tan sqrt 2 = 1.414.. -> +2
    ((100, 100, 100), (7, 5), 0, 6, 8),    # 1.4 * 1.414.. = 1.98 -> +2
    ((100, 100, 100), (3, 2), 0, 6, 9),    # 1.5 * 1.414.. = 2.12 -> +3
    ((300, 0, 100), (1, 3), 0, 6, 7),      # exactly 1 -> +1
    ((100, 0, 100), (1024, 1), 12, 6, 12), # capped
])
def test_angle_threshold_on_lattice_tracks(oracle_mod, step, slope, cap, n_min, need):
    for n in (need - 1, need):
        xyz = lattice(step, n)
        res = oracle_mod.track_view(xyz, n_min=n_min, thr_slope=slope, thr_max=cap)
        assert len(res.tracks) == (1 if n == need else 0), (n, need)


def test_horizontal_seed_needs_the_cap(oracle_mod):
    xyz = lattice((100, 0, 0), 20)
    assert len(oracle_mod.track_view(xyz, n_min=6, thr_slope=(1, 1)).tracks) == 0
    assert len(oracle_mod.track_view(xyz, n_min=6, thr_slope=(1, 1), thr_max=20).tracks) == 1
    assert len(oracle_mod.track_view(xyz, n_min=6, thr_slope=(1, 1), thr_max=21).tracks) == 0


def test_threshold_slope_only_removes_candidates(oracle_mod):
    v = synth.make_c1(1)
    base = {(i, j) for i, j, _ in oracle_mod.track_view(v.xyz).cand.tolist()}
    steep = {(i, j) for i, j, _ in
             oracle_mod.track_view(v.xyz, thr_slope=(2, 1)).cand.tolist()}
    assert steep < base


SETTINGS = [dict(ext=0), dict(ext=300), dict(ext=1500), dict(slope=(1, 1)),
            dict(slope=(5, 2), cap=9), dict(ext=700, slope=(3, 4), cap=12)]


@pytest.mark.parametrize("seed", range(24))
def test_variants_match_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    if seed % 2:
        v = synth.make_tiny_tracks(3000 + seed, n_tracks=int(rng.integers(2, 6)),
                                   n_fog=int(rng.integers(20, 100)), side_um=30.0,
                                   density=float(rng.uniform(0.6, 1.5)))
        xyz, n_min = v.xyz, 6
    else:
        xyz = (rng.integers(0, 6, size=(int(rng.integers(30, 120)), 3)) * 300).astype(np.int32)
        n_min = 4
    st = SETTINGS[seed % len(SETTINGS)]
    ext, slope, cap = st.get("ext", -1), st.get("slope", (0, 1)), st.get("cap", 0)
    ns, cand, tr = brute.track(xyz, R, RT, n_min, ext=ext, slope=slope, cap=cap)
    for scan_all in (False, True):
        res = oracle_mod.track_view(xyz, n_min=n_min, scan_all=scan_all, cyl_ext=ext,
                                    thr_slope=slope, thr_max=cap)
        assert res.n_seeds == ns
        assert np.array_equal(res.cand.astype(np.int64), cand)
        assert [(t["i"], t["j"], res.track_grains(k).tolist())
                for k, t in enumerate(res.tracks)] == tr
