"""The module workload and the efficiency / fake-rate method (paper, Sec. 3;
Fig. 8, 9) on the host: module geometry and cosmic-ray angles, and the
method's matching pinned with exact track lists made from the generated
lines (every crossing found, none found, displaced data)."""
import numpy as np
import pytest

from paper_1311_5334_amd import module, synth


def test_cosmic_zenith_distribution():
    rng = np.random.default_rng(1)
    u = module.cosmic_directions(rng, 200000, 2.5)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)
    c = u[:, 2]
    c_min = 1.0 / np.sqrt(1.0 + 2.5 ** 2)
    assert c.min() >= c_min - 1e-12
    # p(c) ~ c^3 on [c_min, 1]: E[c] = 4/5 (1 - c_min^5) / (1 - c_min^4)
    expect = 0.8 * (1 - c_min ** 5) / (1 - c_min ** 4)
    assert abs(c.mean() - expect) < 4 * c.std() / np.sqrt(len(c))


def test_module_views_tile_the_layers():
    m = module.make_module(3, nx_views=3, ny_views=2, fog_per_1000_um3=0.5)
    assert len(m.views) == 4 * 3 * 2
    for v in m.views:
        z0, z1 = module.LAYERS_Z[v.layer]
        assert v.origin_um[2] == z0
        assert v.xyz.dtype == np.int32
        if len(v.xyz):
            assert v.xyz.min() >= 0
            assert v.xyz[:, 0].max() <= 100 * module.VIEW_XY[0]
            assert v.xyz[:, 1].max() <= 100 * module.VIEW_XY[1]
            assert v.xyz[:, 2].max() <= 100 * (z1 - z0)


def _perfect_results(m, drop_layer=None, shift=None):
    """Tracking results that hold exactly the cosmic lines: one track per
    line and view crossed in that layer (the chord inside the view)."""
    res = []
    for v in m.views:
        z0, z1 = module.LAYERS_Z[v.layer]
        rec = []
        if v.layer != drop_layer:
            for p, u in zip(m.lines_p, m.lines_u):
                a = p + (z0 / u[2]) * u
                b = p + (z1 / u[2]) * u
                # clip the chord to the view's x, y range
                t0, t1 = 0.0, 1.0
                for ax in (0, 1):
                    lo = v.origin_um[ax]
                    hi = lo + module.VIEW_XY[ax]
                    da = b[ax] - a[ax]
                    if abs(da) < 1e-12:
                        if not lo <= a[ax] < hi:
                            t0, t1 = 1.0, 0.0
                        continue
                    ta, tb = (lo - a[ax]) / da, (hi - a[ax]) / da
                    t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
                if t1 - t0 < 0.2:
                    continue
                c = a + 0.5 * (t0 + t1) * (b - a) - v.origin_um
                if shift is not None and v.layer == 2:
                    c = c + shift
                r = np.zeros((), synth_track_dtype())
                r["dir"] = u
                r["centroid"] = c
                r["n_grains"] = 20
                rec.append(r)
        res.append({"tracks": np.array(rec, synth_track_dtype())})
    return res


def synth_track_dtype():
    return np.dtype([("dir", "<f4", (3,)), ("centroid", "<f4", (3,)), ("n_grains", "<u4")])


@pytest.fixture(scope="module")
def sparse_module():
    return module.make_module(5, nx_views=6, ny_views=6, cosmics_per_mm2=80,
                              fog_per_1000_um3=0.0, electrons_per_view=0)


def test_every_crossing_found_with_exact_tracks(sparse_module):
    m = sparse_module
    eff = module.measure_efficiency(m, module.layer_tracks(m, _perfect_results(m)))
    assert eff.selected.sum() > 100
    assert eff.efficiency == 1.0
    assert eff.fake_rate < 0.02
    rows = eff.table()
    assert sum(r["selected"] for r in rows) == eff.selected.sum()
    assert all(r["lo68"] <= (r["eff"] or 0) <= r["hi68"] for r in rows if r["selected"])


def test_missing_layer_two_gives_zero_and_displacement_finds_nothing_true(sparse_module):
    m = sparse_module
    eff = module.measure_efficiency(m, module.layer_tracks(m, _perfect_results(m, drop_layer=2)))
    assert eff.selected.sum() > 100 and eff.found.sum() == 0
    # layer 2 really displaced by 1 mm: the displaced search finds the true
    # tracks, the undisplaced one finds none
    res = _perfect_results(m, shift=np.array([1000.0, 0.0, 0.0]))
    eff2 = module.measure_efficiency(m, module.layer_tracks(m, res))
    assert eff2.fake_selected.sum() > 50
    assert eff2.fake_found.sum() == eff2.fake_selected.sum()
    assert eff2.found.sum() < 0.05 * eff2.selected.sum()


def test_reference_selection_needs_layers_0_1_and_3(sparse_module):
    m = sparse_module
    for drop in (0, 1, 3):
        eff = module.measure_efficiency(m, module.layer_tracks(m, _perfect_results(m, drop)))
        assert eff.selected.sum() == 0


def test_oracle_tracks_are_efficient_on_a_small_module():
    """The oracle's own tracks of a small module (fog, electrons, views cut
    by their edges) find nearly every reference line in layer 2."""
    from oracle import oracle
    m = module.make_module(1, nx_views=2, ny_views=2, fog_per_1000_um3=1.0,
                           cosmics_per_mm2=300)
    dt = np.dtype([("dir", "<f8", (3,)), ("centroid", "<f8", (3,)), ("n_grains", "<u4")])
    res = []
    for v in m.views:
        ref = oracle.track_view(v.xyz)
        res.append({"tracks": np.array([(t["dir"], t["centroid"], t["n_grains"])
                                        for t in ref.tracks], dt)})
    eff = module.measure_efficiency(m, module.layer_tracks(m, res), margin=10.0)
    assert eff.selected.sum() > 20
    assert eff.efficiency >= 0.95


def test_empty_module_has_empty_views_and_no_references():
    m = module.make_module(9, nx_views=2, ny_views=2, cosmics_per_mm2=0.0,
                           fog_per_1000_um3=0.0, electrons_per_view=0)
    assert all(len(v.xyz) == 0 and v.xyz.shape == (0, 3) for v in m.views)
    res = [{"tracks": np.zeros(0, synth_track_dtype())} for _ in m.views]
    eff = module.measure_efficiency(m, module.layer_tracks(m, res))
    assert eff.selected.sum() == 0 and eff.efficiency == 0.0 and eff.fake_rate == 0.0
