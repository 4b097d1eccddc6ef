"""Seeded synthetic tomographic stacks: what the grain recognition reads.

A view is digitised as nz frames of ny x nx pixels (paper, Sec. 2: 1280 x
1024 pixels and 40 frames for a 300 x 250 x 50 um view). After the
filtering step (gain tuning, threshold, inversion) a grain is a bright spot
a few pixels wide and a few frames deep on a dark background. This module
renders such filtered stacks: every grain of a seeded view (tracks and fog,
as in the tracking workloads) becomes a 3D Gaussian spot, on a background
with uniform integer noise, clipped to 8 bits. It holds no step of the
recognition itself.

It also models the raw camera images the filtering step starts from: the
same scene seen in bright field (grains dark on a bright background)
through a camera whose pixels differ in gain, column by column and pixel by
pixel, together with the per-pixel gain corrections and pedestals a
calibration would give. It holds no step of the filtering itself.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import synth

# the paper's view and digitisation (Sec. 2)
VIEW_UM = (300.0, 250.0, 50.0)
DIMS = (1280, 1024, 40)            # nx, ny, nz
# pixel pitch in 0.01 um units as exact fractions: 30000/1280, 25000/1024, 5000/40
PITCH_NUM = (375, 3125, 125)
PITCH_DEN = (16, 128, 1)


@dataclass
class Stack:
    img: np.ndarray        # (nz, ny, nx) uint8, x fastest
    truth_um: np.ndarray   # (G, 3) float64 grain centres rendered, um
    threshold: int
    seed: int

    @property
    def shape(self):
        nz, ny, nx = self.img.shape
        return nx, ny, nz


def pitch_um(axis: int) -> float:
    return PITCH_NUM[axis] / PITCH_DEN[axis] / 100.0


def render(rng: np.random.Generator, centres_um: np.ndarray, dims=DIMS, amp=(110, 200),
           sigma_um=(0.25, 0.25, 0.8), background=12, noise=16) -> np.ndarray:
    """Filtered stack with a Gaussian spot per centre (peak amplitude drawn
    uniformly in amp), on background + uniform integer noise in [0, noise)."""
    nx, ny, nz = dims
    img = (background + rng.integers(0, noise, size=(nz, ny, nx), dtype=np.int16))
    img = img.astype(np.float32)
    if len(centres_um):
        pc = np.stack([centres_um[:, m] / pitch_um(m) for m in range(3)], axis=1)  # pixels
        sig = np.array([sigma_um[m] / pitch_um(m) for m in range(3)])
        half = np.ceil(3.0 * sig).astype(int)
        a = rng.uniform(amp[0], amp[1], len(pc)).astype(np.float32)
        offs = np.stack(np.meshgrid(np.arange(-half[0], half[0] + 1),
                                    np.arange(-half[1], half[1] + 1),
                                    np.arange(-half[2], half[2] + 1), indexing="ij"),
                        axis=-1).reshape(-1, 3)
        base = np.floor(pc).astype(int)
        for chunk in range(0, len(pc), 4096):
            b = base[chunk:chunk + 4096, None, :] + offs[None, :, :]           # (C, P, 3)
            d = (b - pc[chunk:chunk + 4096, None, :]) / sig  # pixel k is centred at k pitches
            w = a[chunk:chunk + 4096, None] * np.exp(-0.5 * (d * d).sum(-1))
            ok = np.all((b >= 0) & (b < np.array([nx, ny, nz])), axis=-1)
            np.add.at(img, (b[..., 2][ok], b[..., 1][ok], b[..., 0][ok]), w[ok].astype(np.float32))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def make_stack(index: int = 0, fog_per_1000_um3: float = 1.0, n_tracks: int = 60,
               dims=DIMS, threshold: int = 60) -> Stack:
    """A seeded filtered stack of the paper's view: tracks (20 % stopping)
    and fog grains as in the tracking workloads, rendered as spots."""
    seed = synth.view_seed(6, index)
    rng = np.random.default_rng(seed)
    box = np.array(VIEW_UM)
    segs = synth._tracks_mixed(rng, box, n_tracks)
    v = synth._assemble(rng, box, segs, fog_per_1000_um3 * 1e-3, "stack", seed)
    centres = v.xyz.astype(np.float64) / 100.0
    keep = np.all((centres >= 0) & (centres < box), axis=1)
    centres = centres[keep]
    return Stack(render(rng, centres, dims), centres, threshold, seed)


def make_small_stack(seed: int, dims=(64, 48, 12), n_grains: int = 20, threshold: int = 60,
                     **kw) -> Stack:
    """A small stack with n_grains spots at uniform positions (tests)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    ext = np.array([nx * pitch_um(0), ny * pitch_um(1), nz * pitch_um(2)])
    centres = rng.uniform(0.0, 1.0, (n_grains, 3)) * ext
    return Stack(render(rng, centres, dims, **kw), centres, threshold, seed)


@dataclass
class RawStack:
    raw: np.ndarray        # (nz, ny, nx) uint8 camera pulse heights, grains dark
    gain: np.ndarray       # (ny, nx) uint16 gain corrections, 1/256 units
    thr: np.ndarray        # (ny, nx) uint8 pedestals
    scene: np.ndarray      # (nz, ny, nx) uint8 bright-spot scene the raw image shows
    truth_um: np.ndarray
    seed: int


def camera(rng: np.random.Generator, scene: np.ndarray, bright: int = 235,
           col_sigma: float = 0.04, pix_sigma: float = 0.01, pedestal: int = 30):
    """Bright-field raw stack of a bright-spot scene: light = bright - scene,
    seen through per-pixel camera responses c(x, y) = (1 + column term) (1 +
    pixel term); the calibration's gain correction is 256 / c and its
    pedestal `pedestal` plus a small per-pixel spread."""
    nz, ny, nx = scene.shape
    col = 1.0 + rng.normal(0.0, col_sigma, nx)
    pix = 1.0 + rng.normal(0.0, pix_sigma, (ny, nx))
    c = np.clip(col[None, :] * pix, 0.7, 1.3)
    light = np.clip(bright - scene.astype(np.float64), 0, 255)
    raw = np.clip(np.rint(light * c[None, :, :]), 0, 255).astype(np.uint8)
    gain = np.rint(256.0 / c).astype(np.uint16)
    thr = (pedestal + rng.integers(0, 4, (ny, nx))).astype(np.uint8)
    return raw, gain, thr


def make_raw_stack(index: int = 0, fog_per_1000_um3: float = 1.0, n_tracks: int = 60,
                   dims=DIMS) -> RawStack:
    """The raw camera stack of make_stack's scene, with its calibration."""
    st = make_stack(index, fog_per_1000_um3, n_tracks, dims)
    rng = np.random.default_rng(st.seed + 77)
    raw, gain, thr = camera(rng, st.img)
    return RawStack(raw, gain, thr, st.img, st.truth_um, st.seed)


def make_small_raw_stack(seed: int, dims=(64, 48, 12), n_grains: int = 20, **kw) -> RawStack:
    st = make_small_stack(seed, dims, n_grains)
    rng = np.random.default_rng(seed + 77)
    raw, gain, thr = camera(rng, st.img, **kw)
    return RawStack(raw, gain, thr, st.img, st.truth_um, seed)
