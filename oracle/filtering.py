"""CPU oracle of the image filtering (paper, Sec. 2, the image processing
paragraph; Fig. 3a and 3b; Table 2, first row).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark. The product library never imports it.

The camera's pixels differ in gain (the vertical stripes of a raw image), so
every camera pixel (x, y) gets its own gain correction and its own
threshold, the same in every frame of a stack, and the image is inverted so
that grains, dark in the bright-field picture, become bright spots on a dark
background. The paper names the three operations and no formula; the
reading taken here, on 8-bit pulse heights:

* gain tuning: t = min(255, nearest integer of raw * gain / 256, halves
  up), with the gain an unsigned 16-bit number in units of 1/256
  (256 = unchanged);
* inversion: u = 255 - t;
* threshold: out = u - thr if u > thr, else 0: the per-pixel threshold is
  a pedestal removed from every pixel, so the background becomes 0 and a
  grain keeps the part of its pulse height above it.

Output: a stack of the same shape, what the grain recognition reads.
"""
from __future__ import annotations

import numpy as np


def filter_stack(raw: np.ndarray, gain: np.ndarray, thr: np.ndarray) -> np.ndarray:
    """Filter a (nz, ny, nx) uint8 stack with (ny, nx) uint16 gains (1/256
    units) and (ny, nx) uint8 thresholds."""
    raw = np.asarray(raw)
    assert raw.ndim == 3 and raw.dtype == np.uint8
    assert gain.shape == raw.shape[1:] and gain.dtype == np.uint16
    assert thr.shape == raw.shape[1:] and thr.dtype == np.uint8
    r = raw.astype(np.int64)
    g = gain.astype(np.int64)[None, :, :]
    t = thr.astype(np.int64)[None, :, :]
    tuned = np.minimum(255, (r * g + 128) // 256)     # nearest integer of r*g/256, halves up
    inv = 255 - tuned
    out = np.where(inv > t, inv - t, 0)
    return out.astype(np.uint8)
