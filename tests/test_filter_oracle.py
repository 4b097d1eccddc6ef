"""Pins of the image-filtering oracle (paper, Sec. 2, image processing;
Fig. 3a, 3b): closed forms, the rounding and clamping of the gain tuning,
the strict threshold, an independent brute force with exact fractions, the
per-pixel maps applying to every frame, and recovery of the scene behind a
modelled camera."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.filtering import filter_stack
from paper_1311_5334_amd import synth_stack


def _maps(ny, nx, gain=256, thr=0):
    return (np.full((ny, nx), gain, np.uint16), np.full((ny, nx), thr, np.uint8))


def test_unit_gain_and_zero_threshold_is_inversion():
    raw = np.arange(256, dtype=np.uint8).reshape(1, 16, 16)
    g, t = _maps(16, 16)
    assert np.array_equal(filter_stack(raw, g, t), 255 - raw)


@pytest.mark.parametrize("raw,gain,expect", [
    (1, 128, 254),     # 0.5 rounds up to 1
    (3, 128, 253),     # 1.5 -> 2
    (1, 127, 255),     # 0.496 -> 0
    (100, 256, 155),
    (100, 512, 55),    # 200
    (200, 512, 0),     # 400 clamps at 255
    (255, 65535, 0),
    (0, 65535, 255),
    (10, 300, 243),    # 11.72 -> 12
])
def test_gain_rounding_and_clamp(raw, gain, expect):
    img = np.full((1, 1, 4), raw, np.uint8)
    g, t = _maps(1, 4, gain=gain)
    assert filter_stack(img, g, t).tolist() == [[[expect] * 4]]


def test_threshold_is_a_strict_pedestal():
    img = np.array([[[155, 154, 153, 0]]], np.uint8)        # inverted: 100, 101, 102, 255
    g, t = _maps(1, 4, thr=100)
    assert filter_stack(img, g, t).tolist() == [[[0, 1, 2, 155]]]
    t[:] = 255
    assert filter_stack(img, g, t).max() == 0


def _brute(raw, gain, thr):
    nz, ny, nx = raw.shape
    out = np.zeros_like(raw)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f = Fraction(int(raw[z, y, x]) * int(gain[y, x]), 256) + Fraction(1, 2)
                tuned = min(255, f.numerator // f.denominator)
                inv = 255 - tuned
                out[z, y, x] = inv - int(thr[y, x]) if inv > int(thr[y, x]) else 0
    return out


@pytest.mark.parametrize("seed", range(4))
def test_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    raw = rng.integers(0, 256, (3, 5, 8)).astype(np.uint8)
    gain = rng.integers(0, 1024 if seed % 2 else 65536, (5, 8)).astype(np.uint16)
    thr = rng.integers(0, 256, (5, 8)).astype(np.uint8)
    assert np.array_equal(filter_stack(raw, gain, thr), _brute(raw, gain, thr))


def test_maps_are_per_pixel_and_shared_by_frames():
    rng = np.random.default_rng(9)
    raw = rng.integers(0, 256, (6, 7, 12)).astype(np.uint8)
    gain = rng.integers(100, 400, (7, 12)).astype(np.uint16)
    thr = rng.integers(0, 40, (7, 12)).astype(np.uint8)
    whole = filter_stack(raw, gain, thr)
    for z in range(6):
        assert np.array_equal(whole[z:z + 1], filter_stack(raw[z:z + 1], gain, thr))
    # a pixel's result depends on its own maps only
    g2 = gain.copy()
    g2[3, 5] += 50
    diff = filter_stack(raw, g2, thr) != whole
    assert not diff[:, np.arange(7) != 3].any() and not diff[:, :, np.arange(12) != 5].any()


def test_recovers_the_scene_behind_the_camera():
    """The calibration of a modelled camera undoes its stripes: the filtered
    image is the bright-spot scene less the pedestal, to within the
    rounding of the camera (one count per step)."""
    rs = synth_stack.make_small_raw_stack(3, (96, 64, 10), n_grains=30)
    out = filter_stack(rs.raw, rs.gain, rs.thr).astype(np.int64)
    expect = rs.scene.astype(np.int64) + (255 - 235) - rs.thr.astype(np.int64)[None]
    ok = expect > 3                         # away from the clipping at 0
    err = np.abs(out - expect)[ok]
    assert err.max() <= 3 and err.mean() < 0.7
    # without the gain correction the column stripes stay
    g1 = np.full_like(rs.gain, 256)
    raw_err = np.abs(filter_stack(rs.raw, g1, rs.thr).astype(np.int64) - expect)[ok]
    assert raw_err.max() > 5
