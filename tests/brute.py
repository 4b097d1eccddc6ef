"""Brute-force statement of the track finding, for tiny views.

Written directly from the tracking paragraph of paper Sec. 2 with no cells,
no early exits and exact integer arithmetic (numpy int64, which is exact
here because tiny views keep every product far below 2^63):

* seeds: all pairs i < j with 0 < |g_j - g_i|^2 < R^2;
* count: grains k with |(g_k - g_i) x d|^2 <= r^2 |d|^2, d = g_j - g_i;
* candidates: count >= n_min, ranked by (count desc, i asc, j asc);
* association: in rank order a candidate keeps its not-yet-used grains and
  becomes a track if at least n_min remain;
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


def line_members(g: np.ndarray, i: int, j: int, r: int) -> np.ndarray:
    d = g[j] - g[i]
    D = int(d @ d)
    w = g - g[i]
    c = np.cross(w, d)
    return np.nonzero((c * c).sum(axis=1) <= r * r * D)[0]


def track(xyz, R: int = 2500, r: int = 50, n_min: int = 8):
    g = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    cand = []
    mem = {}
    s = seeds(g, R)
    for i, j in s:
        m = line_members(g, i, j, r)
        if len(m) >= n_min:
            cand.append((len(m), i, j))
            mem[(i, j)] = m
    cand.sort(key=lambda t: (-t[0], t[1], t[2]))
    used = np.zeros(len(g), dtype=bool)
    tracks = []
    for n, i, j in cand:
        m = [int(k) for k in mem[(i, j)] if not used[k]]
        if len(m) < n_min:
            continue
        used[m] = True
        d = g[j] - g[i]
        order = sorted(m, key=lambda k: (int((g[k] - g[i]) @ d), k))
        tracks.append((i, j, order))
    cand_arr = np.array([(i, j, n) for n, i, j in cand], dtype=np.int64).reshape(-1, 3)
    return len(s), cand_arr, tracks
