"""Pins of the CPU oracle against facts fixed by the paper and by geometry.

The oracle is the bar for the GPU library, so it is checked here against
things other than itself: an independent brute force on tiny views, exact
integer boundary cases, lattice tracks with closed-form answers, exact
invariances, exact rational slopes, and the statistics of planted tracks and
of pure fog. Tracking paragraph of paper Sec. 2 throughout.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
from paper_1311_5334_amd import synth

R, RT, NMIN = 2500, 50, 8
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def signed_perms():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), np.int64)
            for row, (col, s) in enumerate(zip(perm, signs)):
                M[row, col] = s
            yield M


def tracks_of(res):
    return [(t["i"], t["j"], res.track_grains(k).tolist())
            for k, t in enumerate(res.tracks)]


def assert_same_as_brute(oracle_mod, xyz, r=RT, n_min=NMIN, R_=R):
    ns, cand, tr = brute.track(xyz, R_, r, n_min)
    for scan_all in (False, True):
        for cell in ((750, 750, 170), (137, 211, 59)):
            res = oracle_mod.track_view(xyz, R=R_, r=r, n_min=n_min,
                                        scan_all=scan_all, cell=cell)
            assert res.n_seeds == ns
            assert np.array_equal(res.cand.astype(np.int64), cand)
            assert tracks_of(res) == tr


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(120))
def test_tiny_views_match_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        v = synth.make_tiny_tracks(1000 + seed, n_tracks=int(rng.integers(2, 6)),
                                   n_fog=int(rng.integers(20, 120)), side_um=30.0,
                                   density=float(rng.uniform(0.6, 1.5)))
    elif kind == 1:
        v = synth.make_box_view(2000 + seed, int(rng.integers(20, 200)), (15.0, 15.0, 15.0))
    else:
        # coarse lattice points: many exact collinearities and count ties
        pts = rng.integers(0, 6, size=(int(rng.integers(30, 150)), 3)) * 300
        v = synth.View(pts.astype(np.int32), np.full(len(pts), -1, np.int32), (18, 18))
    n_min = 4 if kind == 1 else (5 if kind == 2 else NMIN)
    assert_same_as_brute(oracle_mod, v.xyz, n_min=n_min)


@pytest.mark.parametrize("index", [0, 1])
def test_config1_views_match_brute_force(oracle_mod, index):
    v = synth.make_c1(index)
    assert_same_as_brute.__wrapped__ if False else None
    ns, cand, tr = brute.track(v.xyz, R, RT, NMIN)
    res = oracle_mod.track_view(v.xyz)
    assert res.n_seeds == ns
    assert np.array_equal(res.cand.astype(np.int64), cand)
    assert tracks_of(res) == tr


def test_cell_walk_equals_scan_all_on_config1(oracle_mod):
    for index in range(2, 6):
        v = synth.make_c1(index)
        a = oracle_mod.track_view(v.xyz)
        b = oracle_mod.track_view(v.xyz, scan_all=True)
        assert np.array_equal(a.cand, b.cand)
        assert tracks_of(a) == tracks_of(b)
        assert a.n_tests < b.n_tests


def test_dense_crop_of_config5_matches_brute_force(oracle_mod):
    v = synth.make_c5(0)
    x = v.xyz
    lo = np.array([15000, 15000, 0])
    keep = np.all((x >= lo) & (x < lo + np.array([2500, 2500, 5000])), axis=1)
    crop = x[keep]
    assert 100 < len(crop) < 800
    ns, cand, tr = brute.track(crop, R, RT, 4)
    res = oracle_mod.track_view(crop, n_min=4)
    assert res.n_seeds == ns
    assert np.array_equal(res.cand.astype(np.int64), cand)
    assert tracks_of(res) == tr


# ------------------------------------------------------- integer boundaries

def _boundary_cases():
    with open(os.path.join(GOLDEN, "boundary_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _boundary_cases(), ids=lambda c: c["name"])
def test_integer_boundaries_all_signed_axis_permutations(oracle_mod, case):
    base = np.array([100000, 100000, 100000], np.int64)
    for M in signed_perms():
        pts = [base + M @ np.array(p, np.int64) for p in case["points"]]
        xyz = np.array(pts, np.int64).astype(np.int32)
        if case["kind"] == "seed":
            res = oracle_mod.track_view(xyz, n_min=2)
            assert res.n_seeds == case["expect_seeds"]
        else:
            assert oracle_mod.count_seed(xyz, 0, 1, RT) == case["expect_count"]


# ------------------------------------------------------------ closed forms

def lattice(g0, delta, L):
    return np.array([np.asarray(g0) + m * np.asarray(delta) for m in range(L)], np.int64)


@pytest.mark.parametrize("delta", [(300, 0, 0), (0, 0, 170), (211, -97, 33),
                                   (-50, 400, -400), (120, 120, 120), (7, 0, -1000)])
def test_lattice_track_closed_form(oracle_mod, delta):
    L = 12
    g = lattice((20000, 30000, 2500), delta, L)
    perm = np.random.default_rng(7).permutation(L)
    xyz = g[perm].astype(np.int32)
    res = oracle_mod.track_view(xyz)
    assert len(res.tracks) == 1
    t = res.tracks[0]
    assert sorted(res.track_grains(0).tolist()) == list(range(L))
    # every seed sees the whole lattice: all candidates count L
    assert np.all(res.cand[:, 2] == L)
    d = np.array(delta, np.int64)
    a = int(np.argmax(np.abs(d)))  # spread along m is proportional to delta_m^2
    assert t["axis"] == a
    b, c = [m for m in range(3) if m != a]
    assert t["slope"][0] == pytest.approx(d[b] / d[a], abs=1e-15)
    assert t["slope"][1] == pytest.approx(d[c] / d[a], abs=1e-15)
    u = d / np.linalg.norm(d)
    if u[2] < 0 or (u[2] == 0 and (u[1] < 0 or (u[1] == 0 and u[0] < 0))):
        u = -u
    assert np.allclose(t["dir"], u, atol=1e-15)
    # grains ordered along the seed direction
    gi, gj = g[perm[t["i"]]], g[perm[t["j"]]]
    proj = [(g[perm[k]] - gi) @ (gj - gi) for k in res.track_grains(0)]
    assert proj == sorted(proj)


@pytest.mark.parametrize("L,expect", [(NMIN - 1, 0), (NMIN, 1), (NMIN + 5, 1)])
def test_threshold_on_collinear_grains(oracle_mod, L, expect):
    xyz = lattice((5000, 5000, 5000), (400, 300, 100), L).astype(np.int32)
    assert len(oracle_mod.track_view(xyz).tracks) == expect


def test_shared_grain_goes_to_higher_priority_track(oracle_mod):
    shared = np.array([40000, 40000, 2500])
    A = lattice(shared - 5 * np.array([400, 0, 0]), (400, 0, 0), 14)  # 14 grains
    B = lattice(shared - 4 * np.array([0, 350, 100]), (0, 350, 100), 11)  # 11 grains
    B = np.array([b for b in B if not np.array_equal(b, shared)])
    xyz = np.concatenate([B, A]).astype(np.int32)  # B first in input order
    res = oracle_mod.track_view(xyz)
    assert len(res.tracks) == 2
    k_shared = int(np.nonzero(np.all(xyz == shared, axis=1))[0][0])
    first, second = res.track_grains(0).tolist(), res.track_grains(1).tolist()
    assert len(first) == 14 and k_shared in first
    assert len(second) == 10 and k_shared not in second


def test_reassociation_threshold_drops_a_duplicate(oracle_mod):
    # a second line sharing all but NMIN-1 of its grains with a longer track
    A = lattice((10000, 10000, 1000), (300, 0, 0), 16)
    extra = lattice((10000 + 300 * 16, 10000, 1000), (300, 0, 0), NMIN - 1)
    xyz = np.concatenate([A, extra]).astype(np.int32)
    res = oracle_mod.track_view(xyz)
    assert len(res.tracks) == 1 and res.tracks[0]["n_grains"] == 16 + NMIN - 1


@pytest.mark.parametrize("pts", [[], [[1, 2, 3]], [[0, 0, 0], [100, 0, 0]],
                                 [[5, 5, 5]] * 20])
def test_degenerate_inputs(oracle_mod, pts):
    xyz = np.array(pts, np.int64).reshape(-1, 3).astype(np.int32)
    res = oracle_mod.track_view(xyz)
    assert len(res.tracks) == 0
    if len(pts) == 20:
        assert res.n_seeds == 0  # coincident grains define no line


# -------------------------------------------------------------- invariants

def test_translation_invariance(oracle_mod):
    v = synth.make_c1(3)
    a = oracle_mod.track_view(v.xyz)
    b = oracle_mod.track_view(v.xyz + np.array([-7001, 12345, -333], np.int32))
    assert np.array_equal(a.cand, b.cand)
    assert tracks_of(a) == tracks_of(b)
    for ta, tb in zip(a.tracks, b.tracks):
        assert ta["dir"] == pytest.approx(tb["dir"], abs=1e-12)


def test_signed_axis_permutation_invariance(oracle_mod):
    v = synth.make_c1(4)
    a = oracle_mod.track_view(v.xyz)
    for M in signed_perms():
        xyz = (v.xyz.astype(np.int64) @ M.T).astype(np.int32)
        b = oracle_mod.track_view(xyz)
        assert np.array_equal(a.cand, b.cand)
        assert tracks_of(a) == tracks_of(b)
        for ta, tb in zip(a.tracks, b.tracks):
            da = M @ np.array(ta["dir"])
            assert min(np.abs(da - tb["dir"]).max(), np.abs(da + tb["dir"]).max()) < 1e-12


def test_far_grain_changes_nothing(oracle_mod):
    v = synth.make_c1(5)
    a = oracle_mod.track_view(v.xyz)
    g = v.xyz.astype(np.int64)
    far = np.array([g[:, 0].max() + 2 * R + 5, g[:, 1].min() - 3 * R, 2500])
    # confirm it is off every seed line (distance > r) before relying on it
    for i, j, _ in a.cand:
        d = g[j] - g[i]
        c = np.cross(far - g[i], d)
        assert int(c @ c) > RT * RT * int(d @ d)
    b = oracle_mod.track_view(np.concatenate([v.xyz, far[None].astype(np.int32)]))
    assert np.array_equal(a.cand, b.cand)
    assert tracks_of(a) == tracks_of(b)


def test_monotone_in_radius_and_threshold(oracle_mod):
    v = synth.make_c1(6)
    base = {(i, j) for i, j, _ in oracle_mod.track_view(v.xyz).cand}
    wider = {(i, j) for i, j, _ in oracle_mod.track_view(v.xyz, r=70).cand}
    lower = {(i, j) for i, j, _ in oracle_mod.track_view(v.xyz, n_min=6).cand}
    assert base <= wider and base <= lower
    assert len(wider) > len(base) and len(lower) > len(base)


# --------------------------------------------------------------------- fit

def _exact_slopes(xyz, grains, i):
    g = np.asarray(xyz, np.int64)[grains]
    w = g - np.asarray(xyz, np.int64)[i]
    n = len(g)
    S1 = [int(x) for x in w.sum(axis=0)]
    Q = [[n * int((w[:, u] * w[:, v]).sum()) - S1[u] * S1[v] for v in range(3)]
         for u in range(3)]
    a = max(range(3), key=lambda m: (Q[m][m], -m))
    b, c = [m for m in range(3) if m != a]
    return a, Fraction(Q[a][b], Q[a][a]), Fraction(Q[a][c], Q[a][a]), Q, n


def test_fit_slopes_match_exact_rationals(oracle_mod):
    for idx in (0, 7):
        v = synth.make_c1(idx)
        res = oracle_mod.track_view(v.xyz)
        assert res.tracks
        for k, t in enumerate(res.tracks):
            gr = res.track_grains(k)
            a, sb, sc, Q, n = _exact_slopes(v.xyz, gr, t["i"])
            assert t["axis"] == a
            tol = 4 * n * 2.0 ** -52 + 1e-15
            assert abs(t["slope"][0] - float(sb)) <= tol
            assert abs(t["slope"][1] - float(sc)) <= tol
            assert abs(np.linalg.norm(t["dir"]) - 1.0) < 1e-14
            dz, dy = t["dir"][2], t["dir"][1]
            assert dz > 0 or (dz == 0 and dy >= 0)
            assert t["fit_fp64"] == int(a == 2 or Q[a][a] < 250000 * n * n)
            # centroid is the mean of the associated grains (um)
            assert np.allclose(t["centroid"], v.xyz[gr].mean(axis=0) / 100.0, atol=1e-9)
            proj = (v.xyz[gr] / 100.0 - np.array(t["centroid"])) @ np.array(t["dir"])
            assert t["t_begin"] == pytest.approx(proj.min(), abs=1e-9)
            assert t["t_end"] == pytest.approx(proj.max(), abs=1e-9)


def test_eight_grains_with_their_partner_are_an_ordinary_track(oracle_mod):
    # 8 copies of one grain plus a seed partner: the partner gives the track
    # a spread, so it is fitted as usual (not degenerate)
    pts = [[20000, 20000, 2000]] * NMIN + [[20300, 20400, 2000]]
    res = oracle_mod.track_view(np.array(pts, np.int32))
    assert len(res.tracks) == 1
    t = res.tracks[0]
    assert t["n_grains"] == NMIN + 1 and t["degenerate"] == 0


def _canonical(v):
    v = np.asarray(v, np.float64)
    if v[2] != 0:
        s = v[2] < 0
    elif v[1] != 0:
        s = v[1] < 0
    else:
        s = v[0] < 0
    return -v if s else v


@pytest.mark.parametrize("q_offset,delta", [((1000, 0, 0), (0, 300, 100)),
                                            ((0, -900, 300), (250, 0, 0)),
                                            ((0, 0, -1200), (170, -170, 0)),
                                            ((-700, 700, 0), (0, 0, 170))])
def test_fit_of_all_coincident_members_is_degenerate(oracle_mod, q_offset, delta):
    # 8 copies at P and a lattice line through a partner Q: the line's seeds
    # (11 grains) outrank every seed through P (the copies, the partner and
    # at most a few line grains), take their grains first, and leave the best
    # seed through P with the 8 coincident copies only
    xyz = synth.make_degenerate_view(q_offset=q_offset, delta=delta)
    assert_same_as_brute(oracle_mod, xyz)
    res = oracle_mod.track_view(xyz)
    assert len(res.tracks) == 2
    line = set(range(NMIN, len(xyz)))
    assert set(res.track_grains(0).tolist()) == line
    assert res.tracks[0]["degenerate"] == 0
    t = res.tracks[1]
    assert t["degenerate"] == 1
    assert res.track_grains(1).tolist() == list(range(NMIN))
    i, j = t["i"], t["j"]
    assert i < NMIN <= j  # a copy of P and a grain of the line
    d = xyz[j].astype(np.int64) - xyz[i].astype(np.int64)
    a = int(np.argmax(np.abs(d)))  # ties to the lowest axis
    b, c = [u for u in range(3) if u != a]
    assert t["axis"] == a
    # slopes are the seed's own ratios, correctly rounded
    assert t["slope"][0] == float(Fraction(int(d[b]), int(d[a])))
    assert t["slope"][1] == float(Fraction(int(d[c]), int(d[a])))
    want = _canonical(d / np.linalg.norm(d))
    assert np.allclose(t["dir"], want, rtol=0, atol=1e-15)
    # no spread: FP64 by the 5 um rule, extent zero, centroid at P
    assert t["fit_fp64"] == 1
    assert t["t_begin"] == 0.0 and t["t_end"] == 0.0
    assert np.allclose(t["centroid"], xyz[0] / 100.0, rtol=0, atol=1e-12)


# --------------------------------------------------------- statistics (MC)

def _recovered(view, res, min_frac=0.7):
    truth = view.truth
    n_tracks = int(truth.max()) + 1 if (truth >= 0).any() else 0
    found, eligible, splits = 0, 0, 0
    out_sets = [set(res.track_grains(k).tolist()) for k in range(len(res.tracks))]
    for tid in range(n_tracks):
        mine = set(np.nonzero(truth == tid)[0].tolist())
        if len(mine) < 2 * NMIN:
            continue
        eligible += 1
        hits = 0
        for s in out_sets:
            inter = len(s & mine)
            if inter >= min_frac * len(mine) and inter * 2 > len(s):
                hits = 1
            if inter * 2 > len(s) and inter >= NMIN:
                splits += 1
        found += hits
    return found, eligible, splits


def test_planted_tracks_are_recovered_config1(oracle_mod):
    found = eligible = 0
    for idx in range(10):
        v = synth.make_c1(idx)
        f, e, _ = _recovered(v, oracle_mod.track_view(v.xyz))
        found += f
        eligible += e
    assert eligible > 100
    assert found / eligible >= 0.95


def test_fog_only_candidates_follow_poisson_expectation(oracle_mod):
    """Pure fog, density rho: a seed of line length L inside the box holds its
    two grains plus Poisson(rho * pi r^2 * L) others (ends of the box aside),
    so E[#candidates] = sum over seeds P(Pois >= n_min - 2)."""
    from scipy.spatial import cKDTree
    from scipy.stats import poisson
    rng = np.random.default_rng(11)
    side = np.array([60.0, 60.0, 50.0])
    rho = 0.01
    n = rng.poisson(rho * side.prod())
    pts_um = rng.uniform(0, 1, (n, 3)) * side
    xyz = synth.to_units(pts_um).reshape(-1, 3)
    nmin = 5
    res = oracle_mod.track_view(xyz, n_min=nmin)
    pairs = cKDTree(xyz.astype(np.float64)).query_pairs(R - 1e-6, output_type="ndarray")
    g = xyz.astype(np.float64)
    d = g[pairs[:, 1]] - g[pairs[:, 0]]
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    box = side * 100.0
    t_lo = np.full(len(u), -np.inf)
    t_hi = np.full(len(u), np.inf)
    p = g[pairs[:, 0]]
    for m in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            a = (0.0 - p[:, m]) / u[:, m]
            b = (box[m] - p[:, m]) / u[:, m]
        lo = np.where(u[:, m] != 0, np.minimum(a, b), -np.inf)
        hi = np.where(u[:, m] != 0, np.maximum(a, b), np.inf)
        t_lo = np.maximum(t_lo, lo)
        t_hi = np.minimum(t_hi, hi)
    L_um = np.clip(t_hi - t_lo, 0, None) / 100.0
    lam = rho * math.pi * (RT / 100.0) ** 2 * L_um
    expect = poisson.sf(nmin - 3, lam).sum()
    assert res.n_seeds == len(pairs)
    got = len(res.cand)
    assert expect > 200
    assert abs(got - expect) < 5 * math.sqrt(3 * expect), (got, expect)
