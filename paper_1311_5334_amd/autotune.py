"""Autotuner of the cell geometry and of the counting kernel's tiles.

Cells (``--cells``, the default): for each grain-density bucket of the
library's table, time the whole tracking path on synthetic views of that
density with every candidate cell geometry, and write the fastest into
``csrc/cell_table.h``. Results never depend on the cells (every grain is
decided by the exact test); only the work does: small cells mean more cell
runs per seed line, large cells more grains tested per hit.

Tiles: the counting kernel's queue sizes, workgroup shape and refill size
and the cells allowed per grain are compile-time constants. ``--build-tiles
DIR`` (no GPU needed) builds the starting tiles and every one-at-a-time
variation of them into libraries of their own under DIR (``build.build``
with -D overrides). ``--tiles --prebuilt DIR`` (on the GPU) times each of
them in a child process on three workloads (one c2 view, 8 c5 views and 16
c3 views per call), keeps for each constant the value that lowers the mean
of the workloads' times relative to the starting tiles, and writes the
combination into ``csrc/tile_table.h``; a second ``--build-tiles`` then
builds variations around it.

    python -m paper_1311_5334_amd.autotune [--cells] [--report PATH]
    python -m paper_1311_5334_amd.autotune --build-tiles DIR
    python -m paper_1311_5334_amd.autotune --tiles --prebuilt DIR [--report PATH]

Cells and tiles rewrite a header: rebuild the library afterwards. Timing
needs a GPU and prints a line per timed candidate as it goes.
"""
from __future__ import annotations

import argparse
import itertools
import json
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
CY = (500, 750, 1000, 1500, 2000, 3000)
CZ = (200, 300, 500, 800, 1200)
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


TILE_TABLE = os.path.join(HERE, "csrc", "tile_table.h")
# candidate values of each tile constant (see csrc/tile_table.h)
TILE_SPACE = {
    "EMT_COUNT_PIECE": (2, 3, 4),
    "EMT_COUNT_LANE_PIECES": (16, 24, 32),
    "EMT_COUNT_FETCH": (5, 6, 8),
    "EMT_COUNT_REFILL": (24, 32, 48),
    "EMT_FLUSH_UNROLL": (1, 2),
    "EMT_CHUNK_SEEDS": (64, 128, 256),
    "EMT_COUNT_BLOCKS": (1024, 2048),
    "EMT_COUNT_OCCUPANCY": (4, 5),
    "EMT_MERGE_WIDE": (12, 16),
    "EMT_CELLS_PER_GRAIN": (4, 8),
}
TILE_COMMENTS = {
    "EMT_COUNT_PIECE": "grains a flush lane tests per queue entry",
    "EMT_COUNT_LANE_PIECES": "queue entries a lane adds per step",
    "EMT_COUNT_FETCH": "cell pencils a lane fetches per step",
    "EMT_COUNT_REFILL": "lanes waiting for a seed before a wave refills",
    "EMT_FLUSH_UNROLL": "queue words a flush trip loads before testing",
    "EMT_CHUNK_SEEDS": "seeds a wave takes at a time (single views)",
    "EMT_COUNT_BLOCKS": "workgroups of the counting kernel",
    "EMT_COUNT_OCCUPANCY": "waves per SIMD the counting kernel is compiled for",
    "EMT_MERGE_WIDE": "grid-wide merge rounds at most before the per-view tails",
    "EMT_CELLS_PER_GRAIN": "cells a view may use per grain (plus 4096)",
}
WORKLOADS = ("c2", "c5x8", "c3x16")


def read_tiles(path: str = TILE_TABLE) -> dict:
    """The values tile_table.h sets now."""
    import re
    text = open(path).read()
    return {k: int(re.search(rf"#define {k} (\d+)", text).group(1)) for k in TILE_SPACE}


def write_tiles(path: str, tiles: dict, summary: str) -> None:
    lines = []
    for k in TILE_SPACE:
        lines.append(f"#ifndef {k}\n#define {k} {tiles[k]}  // {TILE_COMMENTS[k]}\n#endif")
    body = "\n".join(lines)
    text = f"""// tile_table.h -- queue sizes and launch shapes of the counting kernel and
// the cell budget per grain, chosen by paper_1311_5334_amd/autotune.py
// --tiles from timings of the whole path; -D on the compiler line overrides
// each value.
{summary}
#ifndef EMT_TILE_TABLE_H
#define EMT_TILE_TABLE_H

{body}

// queue capacities that follow from the above
#ifndef EMT_COUNT_PIECE_CAP
#define EMT_COUNT_PIECE_CAP (128 * EMT_COUNT_LANE_PIECES)
#endif
#ifndef EMT_COUNT_RUN_CAP
#define EMT_COUNT_RUN_CAP (64 * EMT_COUNT_FETCH)
#endif

#endif
"""
    open(path, "w").write(text)


def _workload_views(path: str) -> None:
    """The tile workloads' views, generated once and saved for the children."""
    from paper_1311_5334_amd import synth
    arrs = {"c2_0": synth.make_c2(0).xyz}
    for i in range(8):
        arrs[f"c5_{i}"] = synth.make_c5(i).xyz
    for i in range(16):
        arrs[f"c3_{i}"] = synth.make_c3(i).xyz
    np.savez(path, **arrs)


def time_library(lib: str, views_path: str, calls: int = 3) -> dict:
    """Child-process mode: load one library build and time the workloads
    (median device time of the whole path per call, ms)."""
    import torch
    from paper_1311_5334_amd import emt
    emt.load(lib)
    z = np.load(views_path)
    groups = {"c2": [z["c2_0"]], "c5x8": [z[f"c5_{i}"] for i in range(8)],
              "c3x16": [z[f"c3_{i}"] for i in range(16)]}
    out = {}
    for name in WORKLOADS:
        devs = [torch.from_numpy(x).to("cuda:0").contiguous() for x in groups[name]]
        torch.cuda.synchronize()
        with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS) as tr:
            tr(devs)
            tr(devs)
            ms = []
            for _ in range(calls):
                tr(devs)
                ms.append(tr.stats()["ms_total"])
        out[name] = float(np.median(ms))
    return out


def _tag(tiles: dict) -> str:
    return "_".join(f"{k[4:].lower()}{v}" for k, v in sorted(tiles.items()))


def tile_candidates(start: dict) -> list:
    """The starting tiles and every one-at-a-time variation of them."""
    out = [dict(start)]
    for k, values in TILE_SPACE.items():
        for v in values:
            if v != start[k]:
                out.append(dict(start, **{k: v}))
    return out


def build_tiles(outdir: str) -> int:
    """CPU step: build each candidate into outdir/<tag>/libemt.so, and list
    them in outdir/candidates.json."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1311_5334_amd import build
    os.makedirs(outdir, exist_ok=True)
    cands = tile_candidates(read_tiles())

    def one(tiles):
        d = os.path.join(outdir, _tag(tiles))
        build.build(lib=os.path.join(d, "libemt.so"), defines=tiles, objdir=os.path.join(d, "obj"))
        print("built", _tag(tiles), flush=True)
        return {"tiles": tiles, "lib": os.path.join(_tag(tiles), "libemt.so")}

    with ThreadPoolExecutor(4) as ex:
        listed = list(ex.map(one, cands))
    json.dump(listed, open(os.path.join(outdir, "candidates.json"), "w"), indent=1)
    return 0


def tune_tiles(prebuilt: str, report: str | None) -> int:
    """GPU step: time the prebuilt candidates; per constant keep the value
    with the lowest mean time ratio against the starting tiles."""
    import subprocess
    import tempfile
    listed = json.load(open(os.path.join(prebuilt, "candidates.json")))
    tmp = tempfile.mkdtemp(prefix="emt_tiles_")
    views_path = os.path.join(tmp, "views.npz")
    _workload_views(views_path)
    t_start = time.time()
    times = []
    for item in listed:
        lib = os.path.join(prebuilt, item["lib"])
        r = subprocess.run([sys.executable, "-m", "paper_1311_5334_amd.autotune",
                            "--time-lib", lib, views_path], capture_output=True, text=True,
                           timeout=600)
        if r.returncode != 0:
            sys.stderr.write(r.stdout[-2000:] + r.stderr[-2000:])
            raise RuntimeError(f"timing of {item['lib']} failed")
        res = json.loads(r.stdout.strip().splitlines()[-1])
        times.append((item["tiles"], res))
        print(f"  {item['tiles']}: " + ", ".join(f"{k} {v:.3f} ms" for k, v in res.items()) +
              f" [{time.time() - t_start:.0f} s]", flush=True)
    start, base = times[0]

    def score(res: dict) -> float:
        return sum(res[w] / base[w] for w in WORKLOADS) / len(WORKLOADS)

    chosen = dict(start)
    for k in TILE_SPACE:
        best_v, best_s = start[k], 1.0
        for tiles, res in times:
            diff = [m for m in tiles if tiles[m] != start[m]]
            if diff == [k] and score(res) < best_s - 0.01:
                best_v, best_s = tiles[k], score(res)
        chosen[k] = best_v
    lines = [f"starting tiles {start}: " + ", ".join(f"{w} {base[w]:.3f} ms" for w in WORKLOADS),
             f"chosen tiles {chosen} (each constant's best one-at-a-time variation)",
             f"{len(times)} builds timed"]
    write_tiles(TILE_TABLE, chosen, "\n".join("//   " + ln for ln in lines))
    print("wrote", TILE_TABLE, flush=True)
    if report:
        with open(report, "w") as f:
            f.write("# Tile autotune\n\nCommands: `python -m paper_1311_5334_amd.autotune "
                    "--build-tiles DIR` (CPU), then `python -m paper_1311_5334_amd.autotune "
                    f"--tiles --prebuilt DIR --report {report}` (GPU)\n\nSpace: {TILE_SPACE}. "
                    "Workloads: c2 view 0 alone, c5 views 0-7 in one call, c3 views 0-15 in one "
                    "call (device-resident); time: median device time of the whole path per "
                    "call, 3 calls after 2 warm-up calls, each candidate a library of its own. "
                    "One-at-a-time variations of the starting tiles; each constant takes its "
                    "best variation (by the mean time ratio to the start, if better by 1 %).\n\n")
            for ln in lines:
                f.write(f"- {ln}\n")
            f.write("\n| tiles | " + " | ".join(WORKLOADS) + " | ratio |\n|---|" +
                    "---:|" * (len(WORKLOADS) + 1) + "\n")
            for tiles, res in times:
                f.write(f"| {tiles} | " + " | ".join(f"{res[w]:.3f}" for w in WORKLOADS) +
                        f" | {score(res):.3f} |\n")
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    mode = ap.add_mutually_exclusive_group()
    mode.add_argument("--cells", action="store_true", help="tune the cell table (default)")
    mode.add_argument("--tiles", action="store_true",
                      help="time prebuilt tile candidates (--prebuilt) and write the tile table")
    mode.add_argument("--build-tiles", metavar="DIR",
                      help="build the tile candidates into DIR (no GPU needed)")
    mode.add_argument("--time-lib", nargs=2, metavar=("LIB", "VIEWS"), help=argparse.SUPPRESS)
    ap.add_argument("--prebuilt", metavar="DIR", help="directory written by --build-tiles")
    ap.add_argument("--table", default=TABLE)
    ap.add_argument("--report", default=None, help="also write a markdown summary here")
    ap.add_argument("--lib", default=None,
                    help="--cells: time this build of the library instead of the in-tree one")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    if args.time_lib:
        print(json.dumps(time_library(*args.time_lib)), flush=True)
        return 0
    if args.build_tiles:
        return build_tiles(args.build_tiles)
    if args.tiles:
        if not args.prebuilt:
            ap.error("--tiles needs --prebuilt DIR (made by --build-tiles)")
        return tune_tiles(args.prebuilt, args.report)
    import torch
    from paper_1311_5334_amd import emt, synth

    assert torch.cuda.is_available(), "the autotuner needs a GPU"
    emt.load(args.lib or emt.LIB_PATH)
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
