"""The merge's round structure, modelled on the host: prune, reserve and
decide rounds, with candidates that hold at least their threshold of
reservations taking those grains at once, must give exactly what taking the
candidates one by one in key order gives (the paper's exclusive association
with the threshold applied again, Sec. 2). Random small instances with heavy
overlap; no GPU."""
import numpy as np
import pytest


def greedy(cands, thr):
    """cands: list of (key, frozenset of grains) in any order."""
    used, out = set(), {}
    for key, grains in sorted(cands, key=lambda c: c[0]):
        free = grains - used
        if len(free) >= thr[key]:
            used |= free
            out[key] = free
    return out


def rounds(cands, thr):
    """The grid-wide rounds of the library, one candidate at a time within a
    phase but every read taken at the phase's start, as concurrent workgroups
    would see it at worst (a taken grain hidden from a lower-priority reader
    is the only race, and it only hides grains)."""
    owner = {}                      # grain -> 0 (taken) or best key this round
    state = {k: "u" for k, _ in cands}
    members = dict(cands)
    taken = {k: set() for k, _ in cands}
    for _ in range(len(cands) + 2):
        live = [k for k in members if state[k] in ("u", "c")]
        if not live:
            break
        # prune: fewer free grains than the threshold (never a sure one)
        for k in live:
            free = [g for g in members[k] if owner.get(g) != 0]
            if state[k] == "u" and len(free) < thr[k]:
                state[k] = "r"
        # reserve: the best key of the round on every free grain
        res = {}
        for k in live:
            if state[k] == "r":
                continue
            for g in members[k]:
                if owner.get(g) != 0:
                    res[g] = min(res.get(g, k), k)
        for g, k in res.items():
            owner[g] = k
        # decide, from the state at the start of the phase
        snap = dict(owner)
        for k in live:
            if state[k] == "r":
                continue
            free = [g for g in members[k] if snap.get(g) != 0]
            held = [g for g in free if snap.get(g) == k]
            lost = len(free) != len(held)
            if state[k] == "u" and len(free) < thr[k]:
                state[k] = "r"
                continue
            if lost and state[k] == "u" and len(held) < thr[k]:
                continue
            for g in held:
                owner[g] = 0
            taken[k] |= set(held)
            state[k] = "a" if not lost else "c"
        # stale reservations of this round stop counting in the next
        for g in list(owner):
            if owner[g] != 0:
                del owner[g]
    assert all(s in ("a", "r") for s in state.values())
    return {k: taken[k] for k in state if state[k] == "a"}


@pytest.mark.parametrize("seed", range(300))
def test_rounds_with_early_taking_equal_the_one_by_one_reading(seed):
    rng = np.random.default_rng(seed)
    n_grains = int(rng.integers(8, 60))
    n_cands = int(rng.integers(1, 40))
    keys = rng.permutation(10 * n_cands)[:n_cands] + 1  # 0 marks a taken grain
    cands = []
    for k in keys:
        size = int(rng.integers(2, min(16, n_grains) + 1))
        # overlapping "tracks": contiguous stretches with a few strays
        start = int(rng.integers(0, n_grains))
        grains = {(start + i) % n_grains for i in range(size)}
        grains |= set(rng.integers(0, n_grains, int(rng.integers(0, 3))).tolist())
        cands.append((int(k), frozenset(grains)))
    if seed % 3 == 0:
        thr = {k: int(rng.integers(2, 7)) for k, _ in cands}  # per-candidate thresholds
    else:
        n_min = int(rng.integers(2, 7))
        thr = {k: n_min for k, _ in cands}
    want = greedy(cands, thr)
    got = rounds(cands, thr)
    assert got == want
