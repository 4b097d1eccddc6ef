"""Oracle results of named synthetic views, written to an .npz file by a
process of its own, so that slow full-size oracle runs go on beside the GPU
tests (this process never touches a GPU).

    python tests/oracle_worker.py OUT.npz SPEC

SPEC: "c5:I", "c3:I", "c2:I", "c1:I" (view I of that workload) or
"c4fix:I:SIDE_UM:FOG" (synth.make_c4_fixed)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1311_5334_amd import synth  # noqa: E402

TRACK_KEYS = ("i", "j", "grain_offset", "n_grains", "axis", "fit_fp64", "degenerate",
              "slope", "dir", "centroid", "t_begin", "t_end")


def view_of(spec: str) -> np.ndarray:
    parts = spec.split(":")
    if parts[0] == "c4fix":
        return synth.make_c4_fixed(int(parts[1]), float(parts[2]), float(parts[3])).xyz
    return synth.make_view(parts[0], int(parts[1])).xyz


def save(path: str, res) -> None:
    cols = {k: np.array([t[k] for t in res.tracks]) for k in TRACK_KEYS}
    np.savez(path + ".tmp.npz", n_seeds=res.n_seeds, n_tests=res.n_tests, cand=res.cand,
             grains=res.grains, **{"t_" + k: v for k, v in cols.items()})
    os.replace(path + ".tmp.npz", path)


def load(path: str):
    z = np.load(path)
    n = len(z["t_i"])
    tracks = []
    for k in range(n):
        t = {}
        for key in TRACK_KEYS:
            v = z["t_" + key][k]
            t[key] = tuple(float(x) for x in v) if np.ndim(v) else (
                float(v) if key in ("t_begin", "t_end") else int(v))
        tracks.append(t)
    return oracle.OracleResult(int(z["n_seeds"]), int(z["n_tests"]), z["cand"], tracks,
                               z["grains"])


if __name__ == "__main__":
    out, spec = sys.argv[1], sys.argv[2]
    save(out, oracle.track_view(view_of(spec)))
