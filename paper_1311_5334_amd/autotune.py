"""Cell-edge autotuner.

For each grain-density bucket of the library's table, time the whole
tracking path on synthetic views of that density with every candidate cell
geometry, and write the fastest into ``csrc/cell_table.h`` (rebuild the
library afterwards). Results never depend on the cells (every grain is
decided by the exact integer test); only the work does: small cells mean
more cell runs per seed line, large cells more grains tested per hit.

    python -m paper_1311_5334_amd.autotune [--table PATH] [--report PATH]

Needs a GPU. Prints one line per bucket as it goes.
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "cell_table.h")

N_BUCKETS = 8
EDGE0 = 0.75  # grains per 1000 um^3 at the lower edge of bucket 1; doubling
TUNED = range(1, 6)  # buckets swept (up to 24 per 1000 um^3); the others copy the nearest
CX = (100, 150, 200, 250, 350, 500)
CY = (400, 500, 750, 1000, 1500)
CZ = (200, 300, 500, 800)
DEFAULT = (250, 750, 500)


def bucket_center(b: int) -> float:
    """Geometric middle of bucket b's density range (grains per 1000 um^3)."""
    return EDGE0 * 2.0 ** (b - 1) * np.sqrt(2.0)


def time_cells(emt, torch, devs, cell, calls: int = 3) -> float:
    """Median device time (ms, all stages) of one call over the views."""
    with emt.Tracker(device=0, cell=cell,
                     flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS) as tr:
        tr(devs)
        tr(devs)
        ms = []
        for _ in range(calls):
            tr(devs)
            ms.append(tr.stats()["ms_total"])
    return float(np.median(ms))


def write_table(path: str, best: dict, summary: str) -> None:
    rows = [best[min(max(b, min(TUNED)), max(TUNED))] for b in range(N_BUCKETS)]
    body = "\n".join(f"    {{{c[0]}, {c[1]}, {c[2]}}},  // bucket {b}" for b, c in enumerate(rows))
    text = f"""// cell_table.h -- cell edges (units, x y z) per grain-density bucket, used
// when a context leaves its cell edges to the library. Bucket b holds views
// with at least 0.75 * 2^(b-1) grains per 1000 um^3 (b = 0: fewer than
// 0.75). Written by paper_1311_5334_amd/autotune.py from timings of the
// whole path on synthetic views at each bucket's middle density:
{summary}
#ifndef EMT_CELL_TABLE_H
#define EMT_CELL_TABLE_H

namespace emt {{

constexpr int kTunedCells[8][3] = {{
{body}
}};

}}  // namespace emt

#endif
"""
    open(path, "w").write(text)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--table", default=TABLE)
    ap.add_argument("--report", default=None, help="also write a markdown summary here")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_1311_5334_amd import emt, synth

    assert torch.cuda.is_available(), "the autotuner needs a GPU"
    emt.load()
    cands = list(itertools.product(CX, CY, CZ))
    best, lines = {}, []
    t_start = time.time()
    for b in TUNED:
        rho = bucket_center(b)
        views = [synth.make_density_view(0xCE11 + 100 * b + k, rho, 200.0) for k in range(6)]
        views += [synth.make_density_view(0xCE11 + 100 * b + 50 + k, rho, 350.0) for k in range(2)]
        devs = [torch.from_numpy(v.xyz).to("cuda:0").contiguous() for v in views]
        torch.cuda.synchronize()
        grains = sum(v.n for v in views)
        times = {}
        for k, c in enumerate(cands):
            times[c] = time_cells(emt, torch, devs, c)
            if k % 30 == 29:
                print(f"  bucket {b}: {k + 1}/{len(cands)} geometries timed "
                      f"[{time.time() - t_start:.0f} s]", flush=True)
        c_best = min(times, key=times.get)
        best[b] = c_best
        line = (f"bucket {b}: {rho:.2f} grains/1000um^3, {grains} grains in 8 views; "
                f"best {c_best} {times[c_best]:.3f} ms, default {DEFAULT} "
                f"{times[DEFAULT]:.3f} ms, worst {max(times.values()):.3f} ms")
        lines.append(line)
        print(line, f"[{time.time() - t_start:.0f} s]", flush=True)
    summary = "\n".join("//   " + ln for ln in lines)
    write_table(args.table, best, summary)
    print("wrote", args.table, flush=True)
    if args.report:
        with open(args.report, "w") as f:
            f.write("# Cell-edge autotune\n\nCommand: `python -m paper_1311_5334_amd.autotune "
                    f"--report {args.report}`\n\nCandidates: x {CX}, y {CY}, z {CZ} (units of "
                    "0.01 um). Views: 6 of 200x200x50 um and 2 of 350x350x50 um per bucket, "
                    "c4-like tracks plus fog to the bucket's middle density. Time: median "
                    "device time of the whole path (all stages) per call, 3 calls after 2 "
                    "warm-up calls.\n\n")
            for ln in lines:
                f.write(f"- {ln}\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
