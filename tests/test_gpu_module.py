"""The module workload on the GPU (paper, Sec. 3): every view of a small
module tracked in one batched call matches the oracle view by view, and the
efficiency and fake-rate method gives the same counts on both track sets;
on a full module the tracking efficiency is high and the fake rate low."""
import sys

import numpy as np
import pytest

from paper_1311_5334_amd import module
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


def _oracle_results(refs):
    dt = np.dtype([("dir", "<f8", (3,)), ("centroid", "<f8", (3,)), ("n_grains", "<u4")])
    out = []
    for ref in refs:
        rec = np.array([(t["dir"], t["centroid"], t["n_grains"]) for t in ref.tracks], dt)
        out.append({"tracks": rec})
    return out


def test_small_module_matches_oracle(emt):
    from oracle import oracle
    m = module.make_module(1, nx_views=3, ny_views=2, fog_per_1000_um3=1.0,
                           cosmics_per_mm2=300)
    _say(f"small module: {len(m.views)} views, {sum(len(v.xyz) for v in m.views)} grains")
    with emt.Tracker(device=0) as tr:
        got = tr([v.xyz for v in m.views])
    refs = [oracle.track_view(v.xyz) for v in m.views]
    for v, g, r in zip(m.views, got, refs):
        assert_view_parity(v.xyz, g, r)
    kw = dict(margin=10.0, displace=300.0)
    e_gpu = module.measure_efficiency(m, module.layer_tracks(m, got), **kw)
    e_ref = module.measure_efficiency(m, module.layer_tracks(m, _oracle_results(refs)), **kw)
    assert e_gpu.selected.sum() > 30 and e_gpu.fake_selected.sum() > 10
    for f in ("selected", "found", "fake_selected", "fake_found"):
        assert np.array_equal(getattr(e_gpu, f), getattr(e_ref, f)), f


def test_full_module_efficiency(emt):
    m = module.make_module(0)
    _say(f"module: {len(m.views)} views, {sum(len(v.xyz) for v in m.views)} grains")
    res = []
    with emt.Tracker(device=0) as tr:
        for k in range(0, len(m.views), 64):
            res += tr([v.xyz for v in m.views[k:k + 64]])
    eff = module.measure_efficiency(m, module.layer_tracks(m, res))
    _say(f"module: efficiency {eff.efficiency:.4f} of {eff.selected.sum()}, "
         f"fake rate {eff.fake_rate:.4f} of {eff.fake_selected.sum()}")
    assert eff.selected.sum() > 300
    assert eff.efficiency > 0.95
    assert eff.fake_rate < 0.05
