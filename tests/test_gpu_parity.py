"""GPU library vs CPU oracle, through the C ABI, on seeded synthetic views.

Track lists (seed pairs, order, grain lists, grain order) must be identical;
fitted quantities within the tolerances stated in tests/parity.py.
"""
import os
import sys

import numpy as np
import pytest

from paper_1311_5334_amd import synth
from parity import assert_view_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def emt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1311_5334_amd import emt as m
    m.load()
    return m


@pytest.fixture(scope="module")
def tracker(emt):
    t = emt.Tracker(device=0, flags=emt.EMT_F_STATS)
    yield t
    t.close()


def run1(tracker, xyz):
    return tracker([xyz])[0]


@pytest.mark.parametrize("index", range(6))
def test_config1_views(tracker, oracle_mod, index):
    v = synth.make_c1(index)
    _say(f"c1 view {index}: {v.n} grains")
    assert_view_parity(v.xyz, run1(tracker, v.xyz), oracle_mod.track_view(v.xyz))


@pytest.mark.parametrize("seed", range(40))
def test_tiny_dense_views(emt, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        v = synth.make_tiny_tracks(1000 + seed, int(rng.integers(2, 6)),
                                   int(rng.integers(20, 120)), 30.0,
                                   float(rng.uniform(0.6, 1.5)))
        n_min = 8
    elif kind == 1:
        v = synth.make_box_view(2000 + seed, int(rng.integers(20, 200)), (15.0, 15.0, 15.0))
        n_min = 4
    else:
        pts = rng.integers(0, 6, size=(int(rng.integers(30, 150)), 3)) * 300
        v = synth.View(pts.astype(np.int32), np.full(len(pts), -1, np.int32), (18, 18))
        n_min = 5
    with emt.Tracker(device=0, min_grains=n_min) as t:
        got = run1(t, v.xyz)
    assert_view_parity(v.xyz, got, oracle_mod.track_view(v.xyz, n_min=n_min))


@pytest.mark.parametrize("index", range(2))
def test_config2_full_views(tracker, oracle_mod, index):
    v = synth.make_c2(index)
    _say(f"c2 view {index}: {v.n} grains")
    got = run1(tracker, v.xyz)
    st = tracker.stats()
    assert st["retries"] == 0 or index == 0
    assert_view_parity(v.xyz, got, oracle_mod.track_view(v.xyz))


def test_edge_cases(emt, oracle_mod):
    cases = [
        np.zeros((0, 3), np.int32),
        np.array([[5, 6, 7]], np.int32),
        np.array([[0, 0, 0], [100, 0, 0]], np.int32),
        np.array([[5, 5, 5]] * 20, np.int32),
        np.array([[20000 + 300 * m, 30000 - 200 * m, 100 * m] for m in range(12)], np.int32),
        np.array([[-(1 << 17), 0, 0], [(1 << 17) - 1, 0, 0], [0, 5, 5]], np.int32),
    ]
    with emt.Tracker(device=0) as t:
        for xyz in cases:
            assert_view_parity(xyz, run1(t, xyz), oracle_mod.track_view(xyz))
        # all of them in one batch
        res = t(cases)
        for xyz, got in zip(cases, res):
            assert_view_parity(xyz, got, oracle_mod.track_view(xyz))


def test_span_limit_is_an_error(emt):
    wide = np.array([[0, 0, 0], [(1 << 18) + 1, 0, 0]], np.int32)
    with emt.Tracker(device=0) as t:
        with pytest.raises(emt.EmtError) as e:
            t([wide])
        assert e.value.rc == emt.EMT_ERANGE


def test_span_limit_device_pointers(emt):
    import torch
    wide = torch.tensor([[0, 0, 0], [(1 << 18) + 1, 0, 0]], dtype=torch.int32, device="cuda:0")
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as t:
        with pytest.raises(emt.EmtError) as e:
            t([wide])
        assert e.value.rc == emt.EMT_ERANGE


def test_boundary_cases_counted_exactly(emt, oracle_mod):
    import json
    from test_oracle import signed_perms
    here = os.path.dirname(os.path.abspath(__file__))
    cases = json.load(open(os.path.join(here, "golden", "boundary_cases.json")))["cases"]
    base = np.array([100000, 100000, 100000], np.int64)
    with emt.Tracker(device=0, min_grains=2) as t2, emt.Tracker(device=0, min_grains=3) as t3:
        for case in cases:
            for M in signed_perms():
                xyz = np.array([base + M @ np.array(p, np.int64) for p in case["points"]],
                               np.int64).astype(np.int32)
                if case["kind"] == "seed":
                    got = run1(t2, xyz)
                    assert got["n_seeds"] == case["expect_seeds"], case["name"]
                else:
                    got = run1(t3, xyz)
                    ref = oracle_mod.track_view(xyz, n_min=3)
                    assert_view_parity(xyz, got, ref)
                    has = any(int(tr["seed"][0]) == 0 and int(tr["seed"][1]) == 1
                              for tr in got["tracks"])
                    if case["expect_count"] == 3:
                        assert got["n_candidates"] >= 1
                    else:
                        assert not has


def test_device_pointers_match_host(emt, tracker):
    import torch
    v = synth.make_c1(9)
    host = run1(tracker, v.xyz)
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as t:
        dev = t([torch.from_numpy(v.xyz).to("cuda:0")])[0]
    assert host["tracks"].tobytes() == dev["tracks"].tobytes()
    assert np.array_equal(host["grains"], dev["grains"])


def test_repeat_is_byte_identical(tracker):
    v = synth.make_c1(11)
    first = run1(tracker, v.xyz)
    for _ in range(5):
        again = run1(tracker, v.xyz)
        assert again["tracks"].tobytes() == first["tracks"].tobytes()
        assert np.array_equal(again["grains"], first["grains"])


def test_batch_equals_views_alone(tracker, oracle_mod):
    views = [synth.make_c1(i).xyz for i in range(12, 16)] + [synth.make_c4(i).xyz for i in range(3)]
    views = [x for x in views if len(x) < 8000] + [np.zeros((0, 3), np.int32)]
    alone = [run1(tracker, x) for x in views]
    batch = tracker(views)
    for a, b in zip(alone, batch):
        assert a["tracks"].tobytes() == b["tracks"].tobytes()
        assert np.array_equal(a["grains"], b["grains"])
    for x, b in zip(views[:4], batch[:4]):
        assert_view_parity(x, b, oracle_mod.track_view(x))


def test_overflow_retry_gives_same_result(emt, tracker, monkeypatch):
    v = synth.make_c1(17)
    ref = run1(tracker, v.xyz)
    monkeypatch.setenv("EMT_INITIAL_CAPS", "tiny")
    with emt.Tracker(device=0) as t:
        got = run1(t, v.xyz)
        assert t.stats()["retries"] >= 1
    assert got["tracks"].tobytes() == ref["tracks"].tobytes()
    assert np.array_equal(got["grains"], ref["grains"])


def test_cell_geometry_never_changes_results(emt, oracle_mod):
    v = synth.make_c1(18)
    ref = oracle_mod.track_view(v.xyz)
    for cell in ((150, 150, 170), (500, 500, 500), (1200, 1200, 300), (3000, 3000, 5000),
                 (97, 97, 61), (750, 750, 170), (100, 900, 400)):
        with emt.Tracker(device=0, cell=cell) as t:
            assert_view_parity(v.xyz, run1(t, v.xyz), ref)


def test_axis_permutations_on_gpu(tracker, oracle_mod):
    from test_oracle import signed_perms
    v = synth.make_c1(19)
    ref = oracle_mod.track_view(v.xyz)
    for M in list(signed_perms())[::5]:
        xyz = (v.xyz.astype(np.int64) @ M.T).astype(np.int32)
        got = run1(tracker, xyz)
        assert len(got["tracks"]) == len(ref.tracks)
        for k in range(len(ref.tracks)):
            g = got["tracks"][k]
            off = int(g["grain_offset"])
            assert np.array_equal(got["grains"][off:off + int(g["n_grains"])],
                                  ref.track_grains(k))


def test_fp64_always_flag(emt, oracle_mod):
    v = synth.make_c1(20)
    ref = oracle_mod.track_view(v.xyz)
    with emt.Tracker(device=0, flags=emt.EMT_F_FP64_FIT_ALWAYS) as t:
        got = run1(t, v.xyz)
    assert np.all(got["tracks"]["fit_fp64"] == 1)
    for k, rt in enumerate(ref.tracks):
        for s in range(2):
            assert abs(np.arctan(got["tracks"][k]["slope"][s]) - np.arctan(rt["slope"][s])) < 1e-6


def test_graph_replays_match_eager_launches(emt, monkeypatch):
    """One captured launch sequence serves every batch in its capacity bucket;
    each replay must equal the eager launches, with unrelated device work and
    synchronisations in between."""
    import torch
    views = [synth.make_c1(i).xyz for i in range(21, 27)]
    monkeypatch.setenv("EMT_NO_GRAPH", "1")
    eager = emt.Tracker(device=0)
    monkeypatch.delenv("EMT_NO_GRAPH")
    graph = emt.Tracker(device=0)
    try:
        junk = torch.zeros(1 << 20, device="cuda:0")
        for rep in range(3):
            for x in views:
                a = eager([x])[0]
                junk.add_(1.0)
                torch.cuda.synchronize()
                b = graph([x])[0]
                assert a["tracks"].tobytes() == b["tracks"].tobytes(), rep
                assert np.array_equal(a["grains"], b["grains"])
                assert a["n_seeds"] == b["n_seeds"] and a["n_candidates"] == b["n_candidates"]
        # a batch of several views replays its own captured sequence
        for rep in range(2):
            ra = eager(views)
            rb = graph(views)
            for a, b in zip(ra, rb):
                assert a["tracks"].tobytes() == b["tracks"].tobytes()
                assert np.array_equal(a["grains"], b["grains"])
    finally:
        eager.close()
        graph.close()


def _check_track_properties(xyz, got, R=2500, r=50, n_min=8):
    """Exact checks that hold at any size: every grain of a track lies within
    r of its seed line, tracks share no grain, each keeps n_min grains, and
    the grain order follows the seed direction."""
    g = np.asarray(xyz, np.int64)
    seen = np.zeros(len(g), bool)
    for t in got["tracks"]:
        i, j = int(t["seed"][0]), int(t["seed"][1])
        d = g[j] - g[i]
        D = int(d @ d)
        assert 0 < D < R * R and i < j
        off, n = int(t["grain_offset"]), int(t["n_grains"])
        ks = got["grains"][off:off + n].astype(np.int64)
        assert n >= n_min
        c = np.cross(g[ks] - g[i], d)
        assert np.all((c * c).sum(axis=1) <= r * r * D)
        assert not seen[ks].any()
        seen[ks] = True
        tk = (g[ks] - g[i]) @ d
        assert np.all((np.diff(tk) > 0) | ((np.diff(tk) == 0) & (np.diff(ks) > 0)))


def _pair_count(xyz, R=2500):
    from scipy.spatial import cKDTree
    pts = np.asarray(xyz, np.float64)
    pairs = cKDTree(pts).query_pairs(R + 0.5, output_type="ndarray")
    g = np.asarray(xyz, np.int64)
    d = g[pairs[:, 1]] - g[pairs[:, 0]]
    D = (d * d).sum(axis=1)
    return int(((D > 0) & (D < R * R)).sum())


def test_config3_batch_of_64_uneven_views(emt, oracle_mod):
    import torch
    views = [synth.make_c3(i) for i in range(64)]
    _say(f"c3 batch: {sum(v.n for v in views)} grains, sizes {min(v.n for v in views)}..{max(v.n for v in views)}")
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as t:
        devs = [torch.from_numpy(v.xyz).to("cuda:0") for v in views]
        batch = t(devs)
        alone = [t([x])[0] for x in devs]
    for a, b in zip(alone, batch):
        assert a["tracks"].tobytes() == b["tracks"].tobytes()
        assert np.array_equal(a["grains"], b["grains"])
        assert a["n_seeds"] == b["n_seeds"] and a["n_candidates"] == b["n_candidates"]
    small = sorted(range(64), key=lambda k: views[k].n)[:4]
    for k in small:
        _say(f"c3 view {k}: {views[k].n} grains vs oracle")
        assert_view_parity(views[k].xyz, batch[k], oracle_mod.track_view(views[k].xyz))


def test_config5_group_properties_and_alone_equals_batch(emt):
    views = [synth.make_c5(i) for i in range(4)]
    with emt.Tracker(device=0) as t:
        batch = t([v.xyz for v in views])
        for v, b in zip(views, batch):
            a = t([v.xyz])[0]
            assert a["tracks"].tobytes() == b["tracks"].tobytes()
            assert np.array_equal(a["grains"], b["grains"])
            assert b["n_seeds"] == _pair_count(v.xyz)
            _check_track_properties(v.xyz, b)
            assert len(b["tracks"]) > 1000


def test_config5_batch_of_32_equals_views_alone(emt):
    """The benchmark's call: 32 dense c5 views, over 8 M candidates, so the
    counting kernel takes its items in per-XCD grabs both when counting the
    seeds and when listing the candidates' members. Views tracked alone
    (fewer items, fixed chunks) must give byte-identical tracks and grains
    and the same candidates (i, j, n)."""
    views = [synth.make_c5(i).xyz for i in range(32)]
    picks = (0, 13, 31)

    def rows(c):
        return c[np.lexsort((c[:, 1], c[:, 0], c[:, 2]))]

    with emt.Tracker(device=0, flags=emt.EMT_F_STATS | emt.EMT_F_CANDIDATES) as t:
        batch = t(views)
        st = t.stats()
        _say(f"c5 x32: {st['n_seeds']} seeds, {st['n_candidates']} candidates")
        assert st["n_candidates"] > 8_000_000
        cand_b = {k: rows(t.candidates(k)) for k in picks}
        for k in picks:
            a = t([views[k]])[0]
            b = batch[k]
            assert len(b["tracks"]) > 1000
            assert a["tracks"].tobytes() == b["tracks"].tobytes()
            assert np.array_equal(a["grains"], b["grains"])
            assert np.array_equal(rows(t.candidates(0)), cand_b[k])


def test_config5_dense_crop_matches_oracle(emt, oracle_mod):
    v = synth.make_c5(5)
    x = v.xyz
    lo = np.array([10000, 10000, -1000])
    keep = np.all((x >= lo) & (x < lo + np.array([12000, 12000, 7000])), axis=1)
    crop = x[keep]
    _say(f"c5 crop: {len(crop)} grains")
    with emt.Tracker(device=0) as t:
        got = t([crop])[0]
    assert_view_parity(crop, got, oracle_mod.track_view(crop))


def test_config4_mixed_sizes_match_oracle(emt, oracle_mod):
    with emt.Tracker(device=0) as t:
        for i in range(6):
            v = synth.make_c4(i)
            if v.n > 15000:
                continue
            _say(f"c4 view {i}: {v.n} grains")
            assert_view_parity(v.xyz, t([v.xyz])[0], oracle_mod.track_view(v.xyz))


def test_auto_cells_match_fixed_cells(emt):
    """Per-view cells picked by density never change a result."""
    views = [synth.make_c3(i).xyz for i in range(6)] + [synth.make_c1(3).xyz]
    with emt.Tracker(device=0) as auto, emt.Tracker(device=0, cell=(250, 750, 500)) as fixed, \
            emt.Tracker(device=0, cell=(400, 0, 0)) as partial:
        a, b, c = auto(views), fixed(views), partial(views)
    for x, y, z in zip(a, b, c):
        assert x["tracks"].tobytes() == y["tracks"].tobytes() == z["tracks"].tobytes()
        assert np.array_equal(x["grains"], y["grains"]) and np.array_equal(x["grains"], z["grains"])


def test_merge_rounds_adapt_without_changing_results(emt):
    """A context sizes its grid-wide merge rounds from the previous call; a
    dense batch after a sparse call leaves many rounds to the tail kernel,
    and must still give the results of a fresh context."""
    dense = [synth.make_c5(i).xyz for i in (1, 2)]
    with emt.Tracker(device=0) as fresh:
        ref = fresh(dense)
        ref_rounds = fresh.stats()["merge_rounds"]
    with emt.Tracker(device=0, flags=emt.EMT_F_STATS) as t:
        t([synth.make_c1(0).xyz])
        assert t.stats()["merge_rounds"] <= 6
        got = t(dense)  # six grid-wide rounds, the rest in the tail kernel
        tail_rounds = t.stats()["merge_rounds"]
        again = t(dense)
    # rounds depend on timing (a candidate may see a grain taken in its own
    # round or only in the next), the outcome does not
    _say(f"dense pair: {ref_rounds} merge rounds fresh, {tail_rounds} after a sparse call")
    assert ref_rounds > 8 and tail_rounds > 8
    for a, b, c in zip(ref, got, again):
        assert a["tracks"].tobytes() == b["tracks"].tobytes() == c["tracks"].tobytes()
        assert np.array_equal(a["grains"], b["grains"]) and np.array_equal(a["grains"], c["grains"])


def test_stats_time_every_stage(emt):
    """With EMT_F_STATS every stage of a full view reports a positive device
    time (the counting kernel's roofline in the benchmark rests on it)."""
    from paper_1311_5334_amd import synth
    v = synth.make_c2(0)
    with emt.Tracker(device=0, flags=emt.EMT_F_STATS) as tr:
        tr([v.xyz])
        tr([v.xyz])
        st = tr.stats()
    assert all(ms > 0 for ms in st["ms"].values()), st["ms"]
    assert st["n_tests"] > 0 and st["n_seeds"] > 0


@pytest.mark.parametrize("q_offset,delta", [((1000, 0, 0), (0, 300, 100)),
                                            ((0, -900, 300), (250, 0, 0)),
                                            ((0, 0, -1200), (170, -170, 0)),
                                            ((-700, 700, 0), (0, 0, 170))])
def test_degenerate_fit_matches_oracle(tracker, oracle_mod, q_offset, delta):
    """A track left with coincident grains only takes the seed direction
    (the fit's degenerate branch), alone and inside a batch."""
    xyz = synth.make_degenerate_view(q_offset=q_offset, delta=delta)
    ref = oracle_mod.track_view(xyz)
    assert [t["degenerate"] for t in ref.tracks] == [0, 1]
    got = run1(tracker, xyz)
    assert_view_parity(xyz, got, ref)
    assert int(got["tracks"][1]["degenerate"]) == 1
    other = synth.make_c1(2).xyz
    batch = tracker([other, xyz, xyz[::-1].copy()])
    assert_view_parity(xyz, batch[1], ref)
    assert_view_parity(xyz[::-1].copy(), batch[2], oracle_mod.track_view(xyz[::-1].copy()))


def test_seed_total_above_2_32_is_an_overflow(emt):
    """96,000 grains in a 14 um cube: every pair is a seed, 4.6e9 in all,
    more than a uint32 scan holds. The call must fail with EMT_EOVERFLOW
    (the wrapped total would otherwise look like a small, fitting one), and
    the context must stay usable."""
    rng = np.random.default_rng(20250)
    n = 96000
    xyz = (rng.integers(0, 1400, size=(n, 3)) + 50000).astype(np.int32)
    assert n * (n - 1) // 2 > (1 << 32) + (1 << 28)
    _say(f"dense cube: {n} grains, {n * (n - 1) // 2} pairs")
    with emt.Tracker(device=0) as t:
        with pytest.raises(emt.EmtError) as e:
            t([xyz])
        assert e.value.rc == emt.EMT_EOVERFLOW
        small = synth.make_c1(3).xyz
        again = t([small])[0]
    with emt.Tracker(device=0) as t2:
        ref = t2([small])[0]
    assert again["tracks"].tobytes() == ref["tracks"].tobytes()


def _with_candidates(emt, xyz, **cfg):
    with emt.Tracker(device=0, flags=emt.EMT_F_CANDIDATES, **cfg) as t:
        got = t([xyz])[0]
        cands = t.candidates(0)
    return got, cands


@pytest.mark.parametrize("which", ["c1-0", "c1-1", "c2-0", "c5-crop"])
def test_candidate_lists_match_oracle(emt, oracle_mod, which):
    """Every candidate (i, j, n), i.e. the count n(s) of every seed that
    reaches the threshold, element by element against the oracle."""
    from parity import assert_candidates_equal
    if which.startswith("c1"):
        xyz = synth.make_c1(int(which[-1])).xyz
    elif which == "c2-0":
        xyz = synth.make_c2(0).xyz
    else:
        x = synth.make_c5(5).xyz
        lo = np.array([10000, 10000, -1000])
        xyz = x[np.all((x >= lo) & (x < lo + np.array([12000, 12000, 7000])), axis=1)]
    _say(f"candidates {which}: {len(xyz)} grains")
    ref = oracle_mod.track_view(xyz)
    got, cands = _with_candidates(emt, xyz)
    assert got["n_candidates"] == len(cands)
    assert_candidates_equal(cands, ref)
    assert_view_parity(xyz, got, ref)


def test_candidate_lists_in_a_batch(emt, oracle_mod):
    from parity import assert_candidates_equal
    views = [synth.make_c1(i).xyz for i in (4, 5, 6)] + [np.zeros((0, 3), np.int32)]
    with emt.Tracker(device=0, flags=emt.EMT_F_CANDIDATES, min_grains=6) as t:
        t(views)
        for k, x in enumerate(views):
            assert_candidates_equal(t.candidates(k), oracle_mod.track_view(x, n_min=6))
        with pytest.raises(emt.EmtError):
            t.candidates(len(views))
    with emt.Tracker(device=0) as t:
        t(views[:1])
        with pytest.raises(emt.EmtError):
            t.candidates(0)
