"""Brute-force statement of the track finding, for tiny views.

Written directly from the tracking paragraph of paper Sec. 2 with no cells,
no early exits and exact integer arithmetic (numpy int64, which is exact
here because tiny views keep every product far below 2^63):

* seeds: all pairs i < j with 0 < |g_j - g_i|^2 < R^2;
* count: grains k with |(g_k - g_i) x d|^2 <= r^2 |d|^2, d = g_j - g_i;
* candidates: count >= n_min, ranked by (count desc, i asc, j asc);
* association: in rank order a candidate keeps its not-yet-used grains and
  becomes a track if at least n_min remain;
* acceptance variants: a finite cylinder (grains projecting at most ext
  beyond a seed grain) and a threshold rising with the seed's angle, used
  in both threshold steps;
* grain order in a track: by ((g_k - g_i).d, k).

It shares nothing with the oracle in ``oracle/`` or with the GPU library.
"""
from __future__ import annotations

import numpy as np


def seeds(g: np.ndarray, R: int):
    out = []
    n = len(g)
    for i in range(n):
        d = g[i + 1:] - g[i]
        D = (d * d).sum(axis=1)
        for j in np.nonzero((D > 0) & (D < R * R))[0]:
            out.append((i, i + 1 + int(j)))
    return out


def line_members(g: np.ndarray, i: int, j: int, r: int, ext: int = -1) -> np.ndarray:
    d = g[j] - g[i]
    D = int(d @ d)
    w = g - g[i]
    c = np.cross(w, d)
    on = (c * c).sum(axis=1) <= r * r * D
    if ext >= 0:
        # finite cylinder: the projection s = w.d / |d| along the line lies
        # in [-ext, |d| + ext]; compared as exact rationals of square roots
        t = w @ d
        keep = []
        for tk in t.tolist():
            lo_ok = tk >= 0 or tk * tk <= ext * ext * D        # s >= -ext
            hi_ok = tk <= D or (tk - D) ** 2 <= ext * ext * D  # s - |d| <= ext
            keep.append(lo_ok and hi_ok)
        on &= np.array(keep, dtype=bool)
    return np.nonzero(on)[0]


def threshold(d, n_min: int, slope=(0, 1), cap: int = 0):
    """n_min + ceil(b tan(theta)), b = slope[0] / slope[1], tan(theta) =
    sqrt(dx^2 + dy^2) / |dz|, capped at cap when cap > 0; dz = 0 gives the
    cap (no cap: unreachable). Closed form with an integer square root:
    ceil(sqrt(X) / K) is ceil(s / K) when X = s^2, else ceil((s + 1) / K)."""
    import math
    num, den = slope
    if num == 0:
        return n_min
    big = cap if cap > 0 else 1 << 62
    dz = abs(int(d[2]))
    if dz == 0:
        return big
    X = num * num * (int(d[0]) ** 2 + int(d[1]) ** 2)
    K = den * dz
    s = math.isqrt(X)
    top = s if s * s == X else s + 1
    return min(big, n_min + -(-top // K))


def track(xyz, R: int = 2500, r: int = 50, n_min: int = 8, ext: int = -1, slope=(0, 1),
          cap: int = 0):
    g = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    cand = []
    mem = {}
    thr = {}
    s = seeds(g, R)
    for i, j in s:
        m = line_members(g, i, j, r, ext)
        thr[(i, j)] = threshold(g[j] - g[i], n_min, slope, cap)
        if len(m) >= thr[(i, j)]:
            cand.append((len(m), i, j))
            mem[(i, j)] = m
    cand.sort(key=lambda t: (-t[0], t[1], t[2]))
    used = np.zeros(len(g), dtype=bool)
    tracks = []
    for n, i, j in cand:
        m = [int(k) for k in mem[(i, j)] if not used[k]]
        if len(m) < thr[(i, j)]:
            continue
        used[m] = True
        d = g[j] - g[i]
        order = sorted(m, key=lambda k: (int((g[k] - g[i]) @ d), k))
        tracks.append((i, j, order))
    cand_arr = np.array([(i, j, n) for n, i, j in cand], dtype=np.int64).reshape(-1, 3)
    return len(s), cand_arr, tracks
