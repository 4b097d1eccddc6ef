"""Pins of the grain-recognition oracle (paper, Sec. 2): hand-worked
examples, the threshold and tie rules, rounding, a brute-force reference
on small random stacks, and recovery of rendered spots at known places."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.grains import find_grains
from paper_1311_5334_amd import synth_stack

P_NUM, P_DEN = (375, 3125, 125), (16, 128, 1)


def _empty(nz=5, ny=6, nx=9):
    return np.zeros((nz, ny, nx), np.uint8)


def test_single_voxel_sits_at_its_pixel():
    img = _empty()
    img[2, 3, 5] = 90
    xyz, pix = find_grains(img, 60)
    assert pix.tolist() == [[2, 3, 5]]
    # 5 * 375/16 = 117.1875 -> 117; 3 * 3125/128 = 73.24 -> 73; 2 * 125 = 250
    assert xyz.tolist() == [[117, 73, 250]]


def test_worked_centre_of_mass():
    img = _empty()
    img[2, 3, 5] = 200
    img[2, 3, 6] = 100
    xyz, pix = find_grains(img, 60)
    assert pix.tolist() == [[2, 3, 5]]           # 6 is outranked by 5
    # x = (200*5 + 100*6) / 300 = 16/3 px; * 375/16 units = 125 exactly
    assert xyz.tolist() == [[125, 73, 250]]


def test_equal_neighbours_first_pixel_wins_and_halves_round_up():
    img = _empty()
    img[1, 2, 4] = img[1, 2, 5] = 150
    xyz, pix = find_grains(img, 60)
    assert pix.tolist() == [[1, 2, 4]]
    # x = 4.5 px * 375/16 = 105.47 -> 105
    assert xyz[0, 0] == 105
    xyz1, _ = find_grains(img, 60, pitch_num=(1, 1, 1), pitch_den=(1, 1, 1))
    assert xyz1.tolist() == [[5, 2, 1]]            # 4.5 rounds up


def test_threshold_is_strict():
    img = _empty()
    img[2, 2, 2] = 60
    assert len(find_grains(img, 60)[0]) == 0
    img[2, 2, 2] = 61
    assert len(find_grains(img, 60)[0]) == 1


def test_flat_run_gives_one_grain_at_its_start():
    img = _empty(nx=12)
    img[3, 1, 2:7] = 150
    xyz, pix = find_grains(img, 60)
    assert pix.tolist() == [[3, 1, 2]]
    # centre of mass of the block around x=2: pixels 1..3 -> (0 + 2 + 3)*150 / 300 = 2.5 px
    assert xyz[0, 0] == (2 * 5 * 375 + 2 * 16) // (2 * 2 * 16)


def test_corner_uses_pixels_inside_only():
    img = _empty()
    img[0, 0, 0] = 100
    img[0, 0, 1] = 50
    img[1, 1, 1] = 50
    xyz, pix = find_grains(img, 40)
    assert pix.tolist() == [[0, 0, 0]]
    sw = 200
    assert xyz[0, 0] == (2 * 100 * 375 + sw * 16) // (2 * sw * 16)          # x: (50+50)/200 px
    assert xyz[0, 2] == (2 * 50 * 125 + sw * 1) // (2 * sw * 1)            # z: 50/200 frames


def _brute(img, threshold, num=P_NUM, den=P_DEN):
    nz, ny, nx = img.shape
    out = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                v = int(img[z, y, x])
                if v <= threshold:
                    continue
                best = True
                sw = 0
                sums = [0, 0, 0]
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            zz, yy, xx = z + dz, y + dy, x + dx
                            if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
                                continue
                            w = int(img[zz, yy, xx])
                            sw += w
                            sums[0] += w * xx
                            sums[1] += w * yy
                            sums[2] += w * zz
                            if (dz, dy, dx) == (0, 0, 0):
                                continue
                            earlier = (zz, yy, xx) < (z, y, x)
                            if w > v or (w == v and earlier):
                                best = False
                if best:
                    c = []
                    for m in range(3):
                        f = Fraction(sums[m] * num[m], sw * den[m]) + Fraction(1, 2)
                        c.append(f.numerator // f.denominator)
                    out.append((c, [z, y, x]))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_matches_brute_force_on_random_stacks(seed):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(6, 7, 9)).astype(np.uint8)
    if seed % 2:
        img = (img // 64 * 64).astype(np.uint8)    # many exact ties
    xyz, pix = find_grains(img, 100)
    ref = _brute(img, 100)
    assert pix.tolist() == [r[1] for r in ref]
    assert xyz.tolist() == [r[0] for r in ref]


@pytest.mark.parametrize("seed", range(4))
def test_no_two_grains_are_neighbours(seed):
    """Two grains are never in each other's 3 x 3 x 3 block (one of them
    would outrank the other): in particular two pixels next to each other in
    a row are never both grains, so a run of 2k pixels holds at most k."""
    rng = np.random.default_rng(50 + seed)
    img = rng.integers(0, 256, size=(7, 11, 16)).astype(np.uint8)
    if seed % 2:
        img = (img // 128 * 128 + 1).astype(np.uint8)   # two levels: ties everywhere
    _, pix = find_grains(img, 0)
    assert len(pix) > 0
    d = np.abs(pix[:, None, :] - pix[None, :, :]).max(axis=2)
    np.fill_diagonal(d, 2)
    assert d.min() >= 2


def test_recovers_isolated_rendered_spots():
    rng = np.random.default_rng(11)
    dims = (96, 80, 16)
    ext = np.array([dims[m] * synth_stack.pitch_um(m) for m in range(3)])
    # a grid of spots far apart, away from the edges
    g = np.stack(np.meshgrid(np.linspace(0.15, 0.85, 4), np.linspace(0.15, 0.85, 4),
                             [0.5], indexing="ij"), -1).reshape(-1, 3)
    centres = g * ext + rng.uniform(-0.3, 0.3, g.shape)
    img = synth_stack.render(rng, centres, dims, amp=(180, 200), noise=1)
    xyz, _ = find_grains(img, 60)
    got = xyz / 100.0
    assert len(got) == len(centres)
    for c in centres:
        d = np.abs(got - c).max(axis=1)
        k = int(np.argmin(d))
        # a 3-pixel window biases the centre of mass towards the peak pixel:
        # within a quarter pixel across, half a frame in depth
        assert abs(got[k, 0] - c[0]) < 0.25 * synth_stack.pitch_um(0) + 0.01
        assert abs(got[k, 1] - c[1]) < 0.25 * synth_stack.pitch_um(1) + 0.01
        assert abs(got[k, 2] - c[2]) < 0.5 * synth_stack.pitch_um(2)


@pytest.mark.parametrize("seed", range(4))
def test_local_maxima_match_a_library_maximum_filter(seed):
    """The rule as a textbook local maximum of a key that orders pixels by
    pulse height, then earlier first: key = v N + (N - 1 - flat index). A
    grain is a pixel above threshold whose key is the maximum of its
    3 x 3 x 3 block (missing neighbours below every key). scipy's
    maximum_filter and center_of_mass state both steps independently."""
    from scipy import ndimage
    rng = np.random.default_rng(40 + seed)
    nz, ny, nx = 6, 9, 12
    img = rng.integers(0, 256, (nz, ny, nx)).astype(np.uint8)
    if seed % 2:
        img = (img // 32 * 32).astype(np.uint8)   # eight levels: ties everywhere
    n = img.size
    key = img.astype(np.int64) * n + (n - 1 - np.arange(n).reshape(img.shape))
    mx = ndimage.maximum_filter(key, size=3, mode="constant", cval=-1)
    thr = 100
    expect = np.argwhere((img > thr) & (key == mx))
    xyz, pix = find_grains(img, thr)
    assert len(expect) > 0
    assert pix.tolist() == expect.tolist()
    for (z, y, x), c in zip(pix, xyz):
        z0, y0, x0 = max(z - 1, 0), max(y - 1, 0), max(x - 1, 0)
        block = img[z0:z + 2, y0:y + 2, x0:x + 2].astype(np.float64)
        cz, cy, cx = ndimage.center_of_mass(block)
        pos = (x0 + cx, y0 + cy, z0 + cz)
        for m in range(3):
            # nearest 0.01 um of the exact position: within half a unit
            assert abs(c[m] - pos[m] * P_NUM[m] / P_DEN[m]) <= 0.5 + 1e-9
