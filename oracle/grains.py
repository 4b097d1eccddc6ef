"""CPU oracle of the 3D grain recognition (paper, Sec. 2, the grain
recognition paragraph and Fig. 3c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark. The product library never imports it.

On a filtered stack (frames z, rows y, columns x; 8-bit pulse heights):

* a pixel whose pulse height is above the threshold is compared with its
  3 x 3 x 3 neighbours (those inside the stack); it defines a grain if none
  of them is higher. Reading: a neighbour of equal height outranks it only
  if that neighbour comes first in frame, row, column order, so a flat top
  of equal pixels gives one grain, at its first pixel;
* the grain's coordinates are the pulse-height-weighted centre of mass of
  that 3 x 3 x 3 block (the pixels inside the stack, every pulse height as
  its weight). Reading: pixel k of an axis is centred at k pitches; the
  pitch of each axis is an exact fraction num/den of 0.01 um, and the
  coordinate is rounded to the nearest 0.01 um, halves up, from the exact
  integer sums.

Grains come out in frame, row, column order of their defining pixel.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def find_grains(img: np.ndarray, threshold: int, pitch_num=(375, 3125, 125),
                pitch_den=(16, 128, 1)):
    """Grains of a (nz, ny, nx) uint8 stack.

    Returns (xyz, pix): xyz (G, 3) int32 in 0.01 um units (x, y, z), and
    pix (G, 3) int64 of the defining pixels (z, y, x)."""
    img = np.asarray(img)
    assert img.ndim == 3 and img.dtype == np.uint8
    nz, ny, nx = img.shape
    v = img.astype(np.int64)
    cand = np.argwhere(v > threshold)          # row-major: frame, row, column order
    if len(cand) == 0:
        return np.zeros((0, 3), np.int32), np.zeros((0, 3), np.int64)
    z, y, x = cand[:, 0], cand[:, 1], cand[:, 2]
    v0 = v[z, y, x]
    lin0 = (z * ny + y) * nx + x
    is_grain = np.ones(len(cand), bool)
    for dz, dy, dx in OFFSETS:
        if dz == dy == dx == 0:
            continue
        z2, y2, x2 = z + dz, y + dy, x + dx
        inside = (z2 >= 0) & (z2 < nz) & (y2 >= 0) & (y2 < ny) & (x2 >= 0) & (x2 < nx)
        zc, yc, xc = np.clip(z2, 0, nz - 1), np.clip(y2, 0, ny - 1), np.clip(x2, 0, nx - 1)
        w = v[zc, yc, xc]
        lin2 = (zc * ny + yc) * nx + xc
        outranks = inside & ((w > v0) | ((w == v0) & (lin2 < lin0)))
        is_grain &= ~outranks
    g = cand[is_grain]
    z, y, x = g[:, 0], g[:, 1], g[:, 2]
    sw = np.zeros(len(g), np.int64)
    s = [np.zeros(len(g), np.int64) for _ in range(3)]   # sums of weight * x, y, z
    for dz, dy, dx in OFFSETS:
        z2, y2, x2 = z + dz, y + dy, x + dx
        inside = (z2 >= 0) & (z2 < nz) & (y2 >= 0) & (y2 < ny) & (x2 >= 0) & (x2 < nx)
        zc, yc, xc = np.clip(z2, 0, nz - 1), np.clip(y2, 0, ny - 1), np.clip(x2, 0, nx - 1)
        w = np.where(inside, v[zc, yc, xc], 0)
        sw += w
        s[0] += w * xc
        s[1] += w * yc
        s[2] += w * zc
    out = np.zeros((len(g), 3), np.int64)
    for m in range(3):
        # nearest integer to s[m] * num / (sw * den), halves up: all terms >= 0
        num = 2 * s[m] * pitch_num[m] + sw * pitch_den[m]
        den = 2 * sw * pitch_den[m]
        out[:, m] = num // den
    return out.astype(np.int32), g
