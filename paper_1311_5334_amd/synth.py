"""Seeded synthetic emulsion views.

The paper measures on real microscope scans of exposed emulsion (Sec. 3); those
data are not available, so every input here is drawn from a seeded model with
the workload shapes of the five standard configurations:

* ``c1`` -- 100x100x50 um layer, 20 through-going tracks at 0.3 grains/um,
  fog 1 grain per 1000 um^3 (CPU-sized, one view).
* ``c2`` -- 350x350x50 um, 300 tracks (20 % stopping, range U(5, 50) um),
  fog 3/1000 um^3 (one full view).
* ``c3`` -- uneven views for batching: grain count log-uniform in [2k, 40k],
  50-500 tracks and fog U(1, 5)/1000 um^3, square side solved from the count.
* ``c4`` -- served stream mix: 100^2, 200^2 or 350^2 um^2, fog U(1, 10)/1000,
  track density of c2, 20 % stopping.
* ``c5`` -- dense stars: 10 vertices with 3-8 prongs each (0.3-1.0 grains/um,
  range 3-200 um), 200 through-going tracks, fog 10/1000 um^3.

Geometry: the emulsion layer is 50 um thick (Sec. 2, the view definition),
directions are isotropic over the full solid angle (4 pi acceptance, Table 1),
grains sit Poisson-distributed along each trajectory, each with a Gaussian
position smear of 0.2 um per axis, and coordinates are stored as int32 fixed
point in 0.01 um units (rounded half away from zero).

This module holds only the input model. It computes nothing of the tracking
method itself and is shared by the oracle tests, the GPU tests and the bench.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UNITS_PER_UM = 100          # fixed point: 1 unit = 0.01 um
THICKNESS_UM = 50.0         # emulsion layer thickness
SMEAR_UM = 0.2              # per-axis Gaussian smear of a track grain
SEED_BASE = 0x13115334


@dataclass
class View:
    """One synthetic microscope view.

    ``xyz`` is an (N, 3) int32 array in 0.01 um units; ``truth`` is an (N,)
    int32 array holding the index of the trajectory a grain belongs to, or -1
    for fog. ``tracks`` lists the generated trajectories (entry point and exit
    point in um, grain density) for efficiency studies.
    """

    xyz: np.ndarray
    truth: np.ndarray
    size_um: tuple
    tracks: list = field(default_factory=list)
    config: str = ""
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def area_mm2(self) -> float:
        return self.size_um[0] * self.size_um[1] * 1e-6


def view_seed(config: int, index: int) -> int:
    return SEED_BASE + 1000 * config + index


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def to_units(um: np.ndarray) -> np.ndarray:
    """Round micrometres to int32 0.01 um units, half away from zero."""
    v = np.asarray(um, dtype=np.float64) * UNITS_PER_UM
    return (np.sign(v) * np.floor(np.abs(v) + 0.5)).astype(np.int32)


def isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: u_z ~ U(-1, 1), phi ~ U(0, 2 pi)."""
    uz = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - uz * uz))
    return np.stack([s * np.cos(phi), s * np.sin(phi), uz], axis=1)


def _box_exit(p: np.ndarray, u: np.ndarray, box: np.ndarray):
    """Parameters t_lo <= 0 <= t_hi where p + t u leaves the box [0, box]."""
    t_lo, t_hi = -np.inf, np.inf
    for m in range(3):
        if u[m] != 0.0:
            a = (0.0 - p[m]) / u[m]
            b = (box[m] - p[m]) / u[m]
            t_lo = max(t_lo, min(a, b))
            t_hi = min(t_hi, max(a, b))
    return t_lo, t_hi


def _grains_on_segment(rng, a, b, density, smear=True):
    length = float(np.linalg.norm(b - a))
    k = rng.poisson(density * length) if length > 0 else 0
    t = rng.uniform(0.0, 1.0, k)
    pts = a[None, :] + t[:, None] * (b - a)[None, :]
    if smear and k:
        pts = pts + rng.normal(0.0, SMEAR_UM, size=pts.shape)
    return pts


def through_going(rng, box):
    p = rng.uniform(0.0, 1.0, 3) * box
    u = isotropic(rng, 1)[0]
    t_lo, t_hi = _box_exit(p, u, box)
    return p + t_lo * u, p + t_hi * u


def stopping(rng, box, r_lo, r_hi, start=None, u=None):
    p = rng.uniform(0.0, 1.0, 3) * box if start is None else start
    if u is None:
        u = isotropic(rng, 1)[0]
    rng_len = rng.uniform(r_lo, r_hi)
    _, t_hi = _box_exit(p, u, box)
    return p, p + min(rng_len, t_hi) * u


def _assemble(rng, box, segments, fog_density, config, seed):
    parts, labels, tracks = [], [], []
    for tid, (a, b, dens) in enumerate(segments):
        pts = _grains_on_segment(rng, a, b, dens)
        parts.append(pts)
        labels.append(np.full(len(pts), tid, np.int32))
        tracks.append({"a": a.tolist(), "b": b.tolist(), "density": dens})
    vol = float(box[0] * box[1] * box[2])
    nf = rng.poisson(fog_density * vol)
    parts.append(rng.uniform(0.0, 1.0, (nf, 3)) * box)
    labels.append(np.full(nf, -1, np.int32))
    pts = np.concatenate(parts) if parts else np.zeros((0, 3))
    lab = np.concatenate(labels) if labels else np.zeros(0, np.int32)
    perm = rng.permutation(len(pts))
    xyz = to_units(pts[perm]).reshape(-1, 3)
    return View(np.ascontiguousarray(xyz, dtype=np.int32), lab[perm],
                (float(box[0]), float(box[1])), tracks, config, seed)


def make_c1(index: int = 0) -> View:
    seed = view_seed(1, index)
    rng = _rng(seed)
    box = np.array([100.0, 100.0, THICKNESS_UM])
    segs = [(*through_going(rng, box), 0.3) for _ in range(20)]
    return _assemble(rng, box, segs, 1e-3, "c1", seed)


def _tracks_mixed(rng, box, n_tracks, stop_frac=0.2, r_lo=5.0, r_hi=50.0):
    n_stop = int(round(stop_frac * n_tracks))
    segs = []
    for t in range(n_tracks):
        if t < n_stop:
            segs.append((*stopping(rng, box, r_lo, r_hi), 0.3))
        else:
            segs.append((*through_going(rng, box), 0.3))
    return segs


def make_c2(index: int = 0) -> View:
    seed = view_seed(2, index)
    rng = _rng(seed)
    box = np.array([350.0, 350.0, THICKNESS_UM])
    segs = _tracks_mixed(rng, box, 300)
    return _assemble(rng, box, segs, 3e-3, "c2", seed)


_CHORD_TABLE = None


def _chord_table():
    """Mean length of a through-going chord (uniform point, isotropic
    direction) in an L x L x 50 um box, for 48 log-spaced L in [20, 2000] um;
    fixed-seed, vectorised Monte Carlo with 4000 chords per L."""
    global _CHORD_TABLE
    if _CHORD_TABLE is None:
        rng = _rng(0x5EED)
        sides = np.exp(np.linspace(np.log(20.0), np.log(2000.0), 48))
        means = []
        for L in sides:
            box = np.array([L, L, THICKNESS_UM])
            p = rng.uniform(0.0, 1.0, (4000, 3)) * box
            u = isotropic(rng, 4000)
            with np.errstate(divide="ignore", invalid="ignore"):
                a = (0.0 - p) / u
                b = (box - p) / u
            lo = np.where(u != 0, np.minimum(a, b), -np.inf).max(axis=1)
            hi = np.where(u != 0, np.maximum(a, b), np.inf).min(axis=1)
            means.append(float(np.mean(hi - lo)))
        _CHORD_TABLE = (np.log(sides), np.array(means))
    return _CHORD_TABLE


def mean_chord_um(side: float) -> float:
    xs, ys = _chord_table()
    return float(np.interp(np.log(side), xs, ys))


def _solve_side(n_target, n_tracks, fog):
    """Side L (um) with fog*L^2*50 + 0.3*T*E[chord(L)] = N* (bisection)."""
    lo, hi = 20.0, 2000.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        v = fog * mid * mid * THICKNESS_UM + 0.3 * n_tracks * mean_chord_um(mid)
        if v < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def make_c3(index: int = 0) -> View:
    seed = view_seed(3, index)
    rng = _rng(seed)
    n_star = math.exp(rng.uniform(math.log(2000.0), math.log(40000.0)))
    fog = rng.uniform(1.0, 5.0) * 1e-3
    for _ in range(200):
        n_tracks = int(rng.integers(50, 501))
        side = _solve_side(n_star, n_tracks, fog)
        track_grains = 0.3 * n_tracks * mean_chord_um(side)
        if track_grains <= 0.6 * n_star and 60.0 <= side <= 700.0:
            break
    box = np.array([side, side, THICKNESS_UM])
    segs = [(*through_going(rng, box), 0.3) for _ in range(n_tracks)]
    return _assemble(rng, box, segs, fog, "c3", seed)


def make_c4(index: int = 0) -> View:
    seed = view_seed(4, index)
    rng = _rng(seed)
    side = float(rng.choice([100.0, 200.0, 350.0]))
    fog = rng.uniform(1.0, 10.0) * 1e-3
    n_tracks = int(round(2449.0 * side * side * 1e-6))
    box = np.array([side, side, THICKNESS_UM])
    segs = _tracks_mixed(rng, box, n_tracks)
    return _assemble(rng, box, segs, fog, "c4", seed)


def make_c5(index: int = 0) -> View:
    seed = view_seed(5, index)
    rng = _rng(seed)
    box = np.array([350.0, 350.0, THICKNESS_UM])
    segs = []
    for _ in range(10):
        vtx = rng.uniform(0.0, 1.0, 3) * box
        for _p in range(int(rng.integers(3, 9))):
            dens = rng.uniform(0.3, 1.0)
            a, b = stopping(rng, box, 3.0, 200.0, start=vtx)
            segs.append((a, b, dens))
    segs += [(*through_going(rng, box), 0.3) for _ in range(200)]
    return _assemble(rng, box, segs, 10e-3, "c5", seed)


def make_density_view(seed: int, per_1000_um3: float, side_um: float = 200.0) -> View:
    """A c4-like view (2449 tracks/mm^2, 20 % stopping) whose fog is chosen so
    that the whole view holds about per_1000_um3 grains per 1000 um^3; the
    cell autotuner sweeps these. Track grains alone may exceed the target at
    low densities; then there is no fog."""
    rng = _rng(seed)
    box = np.array([side_um, side_um, THICKNESS_UM])
    n_tracks = int(round(2449.0 * side_um * side_um * 1e-6))
    segs = _tracks_mixed(rng, box, n_tracks)
    track_grains = sum(0.3 * float(np.linalg.norm(np.asarray(b) - np.asarray(a)))
                       for a, b, _d in segs)
    vol = float(box.prod())
    fog = max(0.0, per_1000_um3 * 1e-3 * vol - track_grains) / vol
    return _assemble(rng, box, segs, fog, "density", seed)


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5}


def make_view(config: str, index: int = 0) -> View:
    return MAKERS[config](index)


def make_box_view(seed: int, n: int, side_um, smear: bool = False) -> View:
    """Uniform random grains in a box (tiny dense cases for brute force)."""
    rng = _rng(seed)
    box = np.asarray(side_um, dtype=np.float64)
    pts = rng.uniform(0.0, 1.0, (n, 3)) * box
    if smear:
        pts = pts + rng.normal(0.0, SMEAR_UM, size=pts.shape)
    return View(to_units(pts).reshape(-1, 3), np.full(n, -1, np.int32),
                (float(box[0]), float(box[1])), [], "box", seed)


def make_tiny_tracks(seed: int, n_tracks: int, n_fog: int, side_um: float,
                     density: float = 1.0) -> View:
    """A small dense view with a few tracks and fog, so that seeds, shared
    grains and ties in the grain count all occur."""
    rng = _rng(seed)
    box = np.array([side_um, side_um, min(side_um, THICKNESS_UM)])
    segs = [(*through_going(rng, box), density) for _ in range(n_tracks)]
    vol = float(box.prod())
    parts, labels = [], []
    for tid, (a, b, dens) in enumerate(segs):
        pts = _grains_on_segment(rng, a, b, dens)
        parts.append(pts)
        labels.append(np.full(len(pts), tid, np.int32))
    parts.append(rng.uniform(0.0, 1.0, (n_fog, 3)) * box)
    labels.append(np.full(n_fog, -1, np.int32))
    pts = np.concatenate(parts)
    lab = np.concatenate(labels)
    perm = rng.permutation(len(pts))
    _ = vol
    return View(to_units(pts[perm]).reshape(-1, 3), lab[perm],
                (float(box[0]), float(box[1])), [], "tiny", seed)


def make_degenerate_view(p=(20000, 20000, 2000), q_offset=(1000, 0, 0),
                         delta=(0, 300, 100), n_copies: int = 8, n_line: int = 11,
                         shift: int = 0) -> np.ndarray:
    """Units, int32: n_copies grains at one point P (indices 0 .. n_copies-1),
    then n_line grains on a lattice line through Q = P + q_offset with step
    delta, which does not pass near P. The line's seeds outrank every seed
    through P, so it takes Q and its neighbours first; a seed through P is
    then left with the coincident copies only, which have no spread to fit.
    shift moves the line along itself by that many steps."""
    P = np.asarray(p, np.int64)
    Q = P + np.asarray(q_offset, np.int64)
    D = np.asarray(delta, np.int64)
    half = n_line // 2
    line = [Q + (m + shift) * D for m in range(-half, n_line - half)]
    return np.concatenate([np.repeat(P[None, :], n_copies, axis=0),
                           np.array(line, np.int64)]).astype(np.int32)


def make_c4_fixed(index: int, side_um: float, fog_per_1000_um3: float) -> View:
    """A served-mix view of a given size and fog (e.g. the largest and
    foggiest, 350 x 350 um at 10 per 1000 um^3), otherwise as make_c4."""
    seed = view_seed(4, 100000 + index)
    rng = _rng(seed)
    n_tracks = int(round(2449.0 * side_um * side_um * 1e-6))
    box = np.array([side_um, side_um, THICKNESS_UM])
    segs = _tracks_mixed(rng, box, n_tracks)
    return _assemble(rng, box, segs, fog_per_1000_um3 * 1e-3, "c4", seed)


SPAN_MAX = 1 << 18


def make_far_line_view(d, n_far: int = 9, offsets=((0, 0, 70), (0, 70, 0), (70, 0, 0),
                                                   (0, 52, 50), (50, 0, 52), (45, 55, 0),
                                                   (0, 0, 95), (60, -60, 0), (-40, 0, 41))):
    """Units, int32: a seed pair a few units apart (g0, g0 + d) and, near the
    far end of the largest span a view may have (2^18 units per axis),
    n_far grains exactly on the line g0 + m d and grains displaced from it by
    the given offsets, some within and some beyond 0.5 um of the line. The
    pair's line must be followed across the whole view to count them."""
    d = np.asarray(d, np.int64)
    base = np.where(d >= 0, 1000, SPAN_MAX - 1000).astype(np.int64)
    nz = np.abs(d) > 0
    M = int(np.min((SPAN_MAX - 2400) // np.abs(d[nz])))
    pts = [base, base + d]
    steps = [M - 53 * k for k in range(n_far)]
    pts += [base + m * d for m in steps]
    for k, off in enumerate(offsets):
        pts.append(base + (M - 29 * k - 11) * d + np.asarray(off, np.int64))
    xyz = np.array(pts, np.int64)
    assert xyz.min() >= 0 and xyz.max() < SPAN_MAX
    return xyz.astype(np.int32)
