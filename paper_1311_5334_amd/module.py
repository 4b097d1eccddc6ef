"""A synthetic emulsion module and the paper's efficiency and fake-rate
method (Sec. 3; Fig. 8, Fig. 9): a second workload for the unchanged
tracking path.

Module (Sec. 3): a detector is a 200 um plastic base with a 50 um emulsion
layer on each side; two detectors are stacked, giving four sensitive layers
at z = 0-50, 250-300, 300-350 and 550-600 um (the detectors are taken to
touch, and to be perfectly aligned). It is exposed to cosmic rays: straight
lines through the whole module, crossing a horizontal plane with a cos^3
distribution of the zenith angle (a cos^2 flux per solid angle, seen
through the plane) up to a maximum tan(theta). A MIP leaves 42 grains per
100 um of emulsion (Sec. 3). Low-energy electrons add short random tracks,
and fog fills every layer. Each layer is scanned in views of 300 x 250 um
(Sec. 2) tiling the module; every view is tracked on its own, in its own
coordinates (0.01 um units from the view's corner), so a track crossing a
view edge is cut in two as on the microscope.

Method (Sec. 3, Fig. 9 left): tracks found in layers 0, 1 and 3 that line
up are joined into one reference line; its prediction in layer 2 is
searched for among layer 2's tracks; the fraction found is the efficiency,
per bin of the zenith angle. The fake rate is the same search with the data
of layer 2 displaced by 1 mm. The matching tolerances are readings (the
paper gives none).

This module generates inputs and evaluates tracks; it holds no step of the
tracking itself, which runs in the library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import synth

LAYERS_Z = ((0.0, 50.0), (250.0, 300.0), (300.0, 350.0), (550.0, 600.0))
VIEW_XY = (300.0, 250.0)
MIP_GRAINS_PER_UM = 0.42
SEED_MODULE = 7


@dataclass
class ModuleView:
    layer: int
    ix: int
    iy: int
    origin_um: np.ndarray          # (x0, y0, z0) of the view's corner in module coordinates
    xyz: np.ndarray                # (n, 3) int32, 0.01 um units from origin


@dataclass
class Module:
    nx_views: int
    ny_views: int
    views: list = field(default_factory=list)
    lines_p: np.ndarray = None     # cosmic lines: point at z = 0, um
    lines_u: np.ndarray = None     # unit directions, u_z > 0
    seed: int = 0

    @property
    def area_um(self):
        return self.nx_views * VIEW_XY[0], self.ny_views * VIEW_XY[1]


def cosmic_directions(rng: np.random.Generator, n: int, max_tan: float) -> np.ndarray:
    """Unit directions (u_z > 0) with density in c = cos(theta) proportional
    to c^3 on [c_min, 1] (cos^2 flux per solid angle, seen through a
    horizontal plane), phi uniform; tan(theta) <= max_tan."""
    c_min = 1.0 / np.sqrt(1.0 + max_tan * max_tan)
    u = rng.uniform(0.0, 1.0, n)
    c = (c_min ** 4 + u * (1.0 - c_min ** 4)) ** 0.25
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.stack([s * np.cos(phi), s * np.sin(phi), c], axis=1)


def make_module(seed: int = 0, nx_views: int = 8, ny_views: int = 8,
                cosmics_per_mm2: float = 150.0, fog_per_1000_um3: float = 3.0,
                electrons_per_view: float = 2.0, max_tan: float = 2.5) -> Module:
    """Grains of every view of every layer of a seeded module."""
    rng = np.random.default_rng(synth.view_seed(SEED_MODULE, seed))
    w, h = nx_views * VIEW_XY[0], ny_views * VIEW_XY[1]
    # lines start anywhere a track at max_tan can still reach the module
    reach = max_tan * LAYERS_Z[-1][1]
    lo = np.array([-reach, -reach]), np.array([w + reach, h + reach])
    n_lines = rng.poisson(cosmics_per_mm2 * (lo[1] - lo[0]).prod() / 1e6)
    p_mid = rng.uniform(lo[0], lo[1], (n_lines, 2))
    u = cosmic_directions(rng, n_lines, max_tan)
    z_mid = 0.5 * LAYERS_Z[-1][1]
    p0 = np.concatenate([p_mid - (z_mid / u[:, 2])[:, None] * u[:, :2],
                         np.zeros((n_lines, 1))], axis=1)        # point at z = 0
    mod = Module(nx_views, ny_views, [], p0, u, seed)
    for layer, (z0, z1) in enumerate(LAYERS_Z):
        pts = []
        for p, d in zip(p0, u):
            a = p + (z0 / d[2]) * d
            b = p + (z1 / d[2]) * d
            pts.append(synth._grains_on_segment(rng, a, b, MIP_GRAINS_PER_UM))
        n_views = nx_views * ny_views
        vol = VIEW_XY[0] * VIEW_XY[1] * (z1 - z0)
        for iy in range(ny_views):
            for ix in range(nx_views):
                o = np.array([ix * VIEW_XY[0], iy * VIEW_XY[1], z0])
                fog = o + rng.uniform(0, 1, (rng.poisson(fog_per_1000_um3 * 1e-3 * vol), 3)) * \
                    np.array([VIEW_XY[0], VIEW_XY[1], z1 - z0])
                el = []
                for _ in range(rng.poisson(electrons_per_view)):
                    start = o + rng.uniform(0, 1, 3) * np.array([VIEW_XY[0], VIEW_XY[1], z1 - z0])
                    dirn = synth.isotropic(rng, 1)[0]
                    end = start + rng.uniform(5.0, 40.0) * dirn
                    g = synth._grains_on_segment(rng, start, end, 0.8)
                    el.append(g[(g[:, 2] >= z0) & (g[:, 2] < z1)])
                pts.append(fog)
                pts.extend(el)
                mod.views.append(ModuleView(layer, ix, iy, o, None))
        nonempty = [q for q in pts if len(q)]
        allp = np.concatenate(nonempty, axis=0) if nonempty else np.zeros((0, 3))
        allp = allp[(allp[:, 2] >= z0) & (allp[:, 2] < z1)]
        vx = np.floor(allp[:, 0] / VIEW_XY[0]).astype(np.int64)
        vy = np.floor(allp[:, 1] / VIEW_XY[1]).astype(np.int64)
        inside = (vx >= 0) & (vx < nx_views) & (vy >= 0) & (vy < ny_views)
        allp, vx, vy = allp[inside], vx[inside], vy[inside]
        for v in mod.views[layer * n_views:(layer + 1) * n_views]:
            sel = (vx == v.ix) & (vy == v.iy)
            xyz = synth.to_units(allp[sel] - v.origin_um)
            v.xyz = xyz[rng.permutation(len(xyz))]
    return mod


# ------------------------------------------------------------ evaluation

@dataclass
class LayerTracks:
    pos: np.ndarray      # (K, 2) x, y at the layer's mid-plane, module um
    slope: np.ndarray    # (K, 2) dx/dz, dy/dz
    n: np.ndarray        # (K,) grains


def layer_tracks(module: Module, results, min_uz: float = 0.2) -> list:
    """Per layer, the tracks of all its views in module coordinates.
    results[i] is the tracking result (dict with a 'tracks' record array)
    of module.views[i]. Tracks steeper than the plane (u_z < min_uz) are
    left out: they cannot be followed across layers."""
    out = []
    for layer, (z0, z1) in enumerate(LAYERS_Z):
        zm = 0.5 * (z0 + z1)
        P, S, N = [], [], []
        for v, r in zip(module.views, results):
            if v.layer != layer:
                continue
            t = r["tracks"]
            if len(t) == 0:
                continue
            d = t["dir"].astype(np.float64)
            c = t["centroid"].astype(np.float64) + v.origin_um[None, :]
            ok = d[:, 2] >= min_uz
            d, c = d[ok], c[ok]
            k = (zm - c[:, 2]) / d[:, 2]
            P.append(c[:, :2] + k[:, None] * d[:, :2])
            S.append(d[:, :2] / d[:, 2:3])
            N.append(t["n_grains"][ok])
        out.append(LayerTracks(np.concatenate(P) if P else np.zeros((0, 2)),
                               np.concatenate(S) if S else np.zeros((0, 2)),
                               np.concatenate(N) if N else np.zeros(0, np.uint32)))
    return out


def _nearest(lt: LayerTracks, pos, slope, pos_tol, slope_tol):
    """Index of the track of lt closest in position to (pos, slope) within
    the tolerances, or -1."""
    if len(lt.pos) == 0:
        return -1
    dp = np.hypot(*(lt.pos - pos).T)
    ds = np.hypot(*(lt.slope - slope).T)
    ok = (dp <= pos_tol) & (ds <= slope_tol)
    if not ok.any():
        return -1
    i = np.flatnonzero(ok)
    return int(i[np.argmin(dp[i])])


@dataclass
class Efficiency:
    tan_edges: np.ndarray
    selected: np.ndarray         # reference lines per tan(theta) bin
    found: np.ndarray            # of them with a layer-2 track
    fake_selected: np.ndarray    # references whose displaced prediction is scanned
    fake_found: np.ndarray       # of them with a layer-2 track at the displaced place

    @property
    def efficiency(self) -> float:
        return float(self.found.sum() / max(1, self.selected.sum()))

    @property
    def fake_rate(self) -> float:
        return float(self.fake_found.sum() / max(1, self.fake_selected.sum()))

    def bounds(self, k, n, cl=0.68):
        """Shortest interval holding `cl` of the posterior of a binomial
        efficiency k/n with a flat prior on [0, 1], Beta(k + 1, n - k + 1)
        (as the paper's error bars: Bayesian 68 % bounds, constant prior)."""
        from scipy.optimize import minimize_scalar
        from scipy.stats import beta
        a, b = k + 1, n - k + 1
        if k == n:
            return float((1.0 - cl) ** (1.0 / a)), 1.0
        if k == 0:
            return 0.0, float(1.0 - (1.0 - cl) ** (1.0 / b))
        width = lambda lo: beta.ppf(lo + cl, a, b) - beta.ppf(lo, a, b)
        lo = minimize_scalar(width, bounds=(0.0, 1.0 - cl), method="bounded").x
        return float(beta.ppf(lo, a, b)), float(beta.ppf(lo + cl, a, b))

    def table(self):
        rows = []
        for b in range(len(self.selected)):
            n, k = int(self.selected[b]), int(self.found[b])
            lo, hi = self.bounds(k, n) if n else (0.0, 1.0)
            rows.append({"tan_lo": float(self.tan_edges[b]), "tan_hi": float(self.tan_edges[b + 1]),
                         "selected": n, "found": k, "eff": k / n if n else None,
                         "lo68": lo, "hi68": hi})
        return rows


def measure_efficiency(module: Module, lts: list, pos_tol: float = 10.0,
                       slope_tol: float = 0.1, margin: float = 25.0, displace: float = 1000.0,
                       tan_edges=(0.0, 0.5, 1.0, 1.5, 2.0, 2.5)) -> Efficiency:
    """The paper's method on the per-layer tracks: references from layers
    0, 1, 3; a layer-2 track within pos_tol um and slope_tol of the
    reference's prediction counts as found. References whose prediction
    lies within `margin` um of a view edge, or outside the module, are not
    used. Fakes: the same search at the prediction moved by `displace` um
    in x."""
    zm = [0.5 * (a + b) for a, b in LAYERS_Z]
    w, h = module.area_um
    edges = np.asarray(tan_edges, np.float64)
    nb = len(edges) - 1
    sel, fnd = np.zeros(nb, np.int64), np.zeros(nb, np.int64)
    fsel, ffnd = np.zeros(nb, np.int64), np.zeros(nb, np.int64)

    def fiducial(p):
        if not (0.0 <= p[0] < w and 0.0 <= p[1] < h):
            return False
        fx = p[0] - VIEW_XY[0] * np.floor(p[0] / VIEW_XY[0])
        fy = p[1] - VIEW_XY[1] * np.floor(p[1] / VIEW_XY[1])
        return (margin <= fx <= VIEW_XY[0] - margin) and (margin <= fy <= VIEW_XY[1] - margin)

    l0, l1, l2, l3 = lts
    for i in range(len(l0.pos)):
        p0, s0 = l0.pos[i], l0.slope[i]
        j = _nearest(l1, p0 + (zm[1] - zm[0]) * s0, s0, pos_tol, slope_tol)
        if j < 0:
            continue
        s01 = (l1.pos[j] - p0) / (zm[1] - zm[0])
        k = _nearest(l3, l1.pos[j] + (zm[3] - zm[1]) * s01, s01, pos_tol, slope_tol)
        if k < 0:
            continue
        # the reference line: least squares through the three positions
        z = np.array([zm[0], zm[1], zm[3]])
        P = np.stack([p0, l1.pos[j], l3.pos[k]])
        A = np.stack([np.ones(3), z - z.mean()], axis=1)
        coef, *_ = np.linalg.lstsq(A, P, rcond=None)
        slope = coef[1]
        pred = coef[0] + (zm[2] - z.mean()) * slope
        tan = float(np.hypot(*slope))
        b = int(np.searchsorted(edges, tan, side="right")) - 1
        if b < 0 or b >= nb:
            continue
        if fiducial(pred):
            sel[b] += 1
            fnd[b] += _nearest(l2, pred, slope, pos_tol, slope_tol) >= 0
        moved = pred + np.array([displace, 0.0])
        if fiducial(moved):
            fsel[b] += 1
            ffnd[b] += _nearest(l2, moved, slope, pos_tol, slope_tol) >= 0
    return Efficiency(edges, sel, fnd, fsel, ffnd)
