"""Grain recognition on the GPU through the C ABI against the CPU oracle
(exact: same grains, same order, same integer coordinates), and the
recognised grains feeding the tracking path."""
import sys

import numpy as np
import pytest

from paper_1311_5334_amd import synth_stack
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


@pytest.fixture(scope="module")
def tracker(emt):
    t = emt.Tracker(device=0)
    yield t
    t.close()


@pytest.mark.parametrize("seed,dims", [(1, (64, 48, 12)), (2, (128, 96, 20)), (3, (256, 40, 7)),
                                       (4, (4, 1, 1)), (5, (8, 3, 2)), (6, (196, 77, 33))])
def test_small_stacks_match_oracle(tracker, seed, dims):
    from oracle.grains import find_grains
    n = max(1, dims[0] * dims[1] * dims[2] // 2000)
    st = synth_stack.make_small_stack(seed, dims, n_grains=n)
    ref, _ = find_grains(st.img, st.threshold)
    got = tracker.find_grains(st.img, st.threshold)
    _say(f"stack {dims}: {len(ref)} grains")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed", range(4))
def test_random_stacks_with_ties_match_oracle(tracker, seed):
    from oracle.grains import find_grains
    rng = np.random.default_rng(100 + seed)
    img = rng.integers(0, 256, size=(5, 9, 24)).astype(np.uint8)
    if seed % 2:
        img = (img // 64 * 64).astype(np.uint8)
    for thr in (0, 100, 200, 255):
        ref, _ = find_grains(img, thr)
        got = tracker.find_grains(img, thr)
        assert np.array_equal(got, ref), thr


def test_custom_pitch(tracker):
    from oracle.grains import find_grains
    st = synth_stack.make_small_stack(9, (64, 32, 10), n_grains=12)
    num, den = (7, 65536, 1), (3, 1, 65536)
    ref, _ = find_grains(st.img, st.threshold, num, den)
    got = tracker.find_grains(st.img, st.threshold, pitch_num=num, pitch_den=den)
    assert np.array_equal(got, ref)


def test_full_view_matches_oracle_and_feeds_tracking(emt, tracker, oracle_mod):
    from oracle.grains import find_grains
    st = synth_stack.make_stack(0)
    ref, _ = find_grains(st.img, st.threshold)
    got = tracker.find_grains(st.img, st.threshold)
    _say(f"paper view 1280x1024x40: {len(ref)} grains, {len(st.truth_um)} rendered")
    assert np.array_equal(got, ref)
    assert 0.9 * len(st.truth_um) < len(got) < 1.1 * len(st.truth_um)
    # the recognised grains are the tracking input: GPU tracking of them
    # matches the oracle's tracking of the oracle's grains
    tr = tracker([got])[0]
    assert_view_parity(ref, tr, oracle_mod.track_view(ref))
    assert len(tr["tracks"]) > 20


def test_device_pointers_and_overflow(emt):
    import torch
    from oracle.grains import find_grains
    st = synth_stack.make_small_stack(21, (128, 64, 16), n_grains=40)
    ref, _ = find_grains(st.img, st.threshold)
    dev = torch.from_numpy(st.img).cuda().contiguous()
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as t:
        got = t.find_grains(dev, st.threshold)
        assert np.array_equal(got.cpu().numpy(), ref)
        # too small an output: the first grains, and the count of all
        out = torch.zeros((5, 3), dtype=torch.int32, device="cuda:0")
        with pytest.raises(emt.EmtError) as e:
            t.find_grains(dev, st.threshold, max_out=5, out=out)
        assert e.value.rc == -5
        assert np.array_equal(out.cpu().numpy(), ref[:5])
        # tracking straight from the device-resident grains
        tr = t([got.contiguous()])[0]
    with emt.Tracker(device=0) as h:
        ref_tr = h([ref])[0]
    assert tr["tracks"].tobytes() == ref_tr["tracks"].tobytes()


def test_bad_geometry_is_rejected(emt, tracker):
    import ctypes as C
    lib = emt.load()
    img = np.zeros((2, 3, 8), np.uint8)
    out = np.zeros((4, 3), np.int32)
    n = C.c_uint32()
    for shape, thr, num, rc in [((2, 3, 6), 60, (1, 1, 1), -2), ((2, 3, 8), 300, (1, 1, 1), -2),
                                ((2, 3, 8), 60, (0, 1, 1), -2), ((5000, 3, 8), 60, (1, 1, 1), -2)]:
        g = emt.stack_geom(shape, thr, num, (1, 1, 1))
        assert lib.emt_find_grains(tracker.ctx, img.ctypes.data, C.byref(g), out.ctypes.data, 4,
                                   C.byref(n)) == rc
    g = emt.stack_geom((2, 3, 8), 60)
    assert lib.emt_find_grains(tracker.ctx, None, C.byref(g), out.ctypes.data, 4, C.byref(n)) == -1
    # an all-dark stack has no grains
    assert lib.emt_find_grains(tracker.ctx, img.ctypes.data, C.byref(g), out.ctypes.data, 4,
                               C.byref(n)) == 0 and n.value == 0
