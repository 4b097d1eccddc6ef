"""The served form through the C ABI: views submitted one by one while
others are on the device come back identical to the same views tracked
alone, and the admission rule (HBM budget, batch size) holds."""
import sys
import time

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


def _c4_views(count, max_grains):
    out, i = [], 0
    while len(out) < count:
        v = synth.make_c4(i)
        if v.n <= max_grains:
            out.append(v)
        i += 1
    return out


def _collect(srv, n, timeout_s=120.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < n:
        assert time.time() < t_end, f"only {len(got)} of {n} views came back"
        for r in srv.poll(wait_ms=200):
            got[r["view_id"]] = r
    return got


def _same(a, b):
    assert a["tracks"].tobytes() == b["tracks"].tobytes()
    assert np.array_equal(a["grains"], b["grains"])


def test_served_alone_equals_mix(emt, oracle_mod):
    views = _c4_views(20, 30000)
    _say("served views: " + " ".join(str(v.n) for v in views))
    with emt.Tracker(device=0) as t:
        alone = [t([v.xyz])[0] for v in views]
    rng = np.random.default_rng(7)
    with emt.Server(n_pipes=2, max_batch_views=6, device=0) as srv:
        tickets = []
        # a trickle (views mostly find a free pipeline), then a burst (views
        # queue behind the two busy pipelines and are batched)
        for k, v in enumerate(views):
            tickets.append(srv.submit(v.xyz, view_id=k))
            if k < 6:
                time.sleep(float(rng.uniform(0.0, 0.004)))
        got = _collect(srv, len(views))
        st = srv.stats()
    assert tickets == sorted(tickets) and len(set(tickets)) == len(tickets)
    for k in range(len(views)):
        r = got[k]
        assert r["status"] == 0, (k, r["status"])
        _same(r, alone[k])
        assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]
        assert 1 <= r["batch_views"] <= 6
    assert st["submitted"] == st["completed"] == len(views)
    assert st["batches"] < len(views)  # the burst was batched
    assert st["max_batch_views_seen"] > 1
    # the smallest two against the oracle too
    for k in np.argsort([v.n for v in views])[:2]:
        assert_view_parity(views[k].xyz, got[int(k)], oracle_mod.track_view(views[k].xyz))


def test_served_one_pipe_and_burst(emt):
    views = _c4_views(12, 12000)
    with emt.Tracker(device=0) as t:
        alone = [t([v.xyz])[0] for v in views]
    with emt.Server(n_pipes=1, max_batch_views=64, device=0) as srv:
        for k, v in enumerate(views):
            srv.submit(v.xyz, view_id=k)
        got = _collect(srv, len(views))
        st = srv.stats()
    for k in range(len(views)):
        _same(got[k], alone[k])
    assert st["overlap_ms"] == 0.0  # one pipeline never overlaps itself
    assert st["batches"] <= len(views)


def test_served_budget_rejects_oversized_view(emt):
    small = synth.make_c1(0)
    big = synth.make_c2(0)
    with emt.Tracker(device=0) as t:
        ref = t([small.xyz])[0]
    # 160 MB over two pipelines: a c1 view fits a pipeline's share, a full
    # c2 view's seed buffers do not
    with emt.Server(n_pipes=2, max_batch_views=8, device=0, hbm_budget=160 << 20) as srv:
        srv.submit(big.xyz, view_id=1)
        srv.submit(small.xyz, view_id=2)
        srv.submit(np.zeros((0, 3), np.int32), view_id=3)
        got = _collect(srv, 3)
    assert got[1]["status"] == -3 and len(got[1]["tracks"]) == 0
    assert got[2]["status"] == 0
    _same(got[2], ref)
    assert got[3]["status"] == 0 and len(got[3]["tracks"]) == 0


def test_served_submit_checks_span(emt):
    wide = np.array([[0, 0, 0], [(1 << 18) + 5, 0, 0]], np.int32)
    with emt.Server(n_pipes=2, max_batch_views=4, device=0) as srv:
        with pytest.raises(emt.EmtError) as e:
            srv.submit(wide, view_id=0)
        assert e.value.rc == -2
        srv.submit(synth.make_c1(1).xyz, view_id=5)
        got = _collect(srv, 1)
    assert got[5]["status"] == 0


def test_served_variant_matches_batched(emt):
    """A server built with acceptance variants (n_min 6, a 5 um finite
    cylinder, an angle-dependent threshold) gives every view the bytes the
    batched call with the same configuration gives it."""
    from paper_1311_5334_amd import synth
    cfg = dict(min_grains=6, cyl_ext=500, thr_slope=(1, 2), thr_max=16)
    views = [synth.make_c4(i) for i in range(8)]
    with emt.Tracker(device=0, **cfg) as tr:
        ref = tr([v.xyz for v in views])
    got = {}
    with emt.Server(n_pipes=2, max_batch_views=4, device=0, **cfg) as srv:
        for i, v in enumerate(views):
            srv.submit(v.xyz, view_id=i)
        while len(got) < len(views):
            for r in srv.poll(wait_ms=200):
                got[r["view_id"]] = r
    for i, r in enumerate(ref):
        assert got[i]["status"] == 0
        assert got[i]["tracks"].tobytes() == r["tracks"].tobytes()
        assert np.array_equal(got[i]["grains"], r["grains"])
