"""Parity sweep: the GPU library against the CPU oracle over many seeded
views of every workload. Needs a GPU; pytest does not collect this file.

    python tests/parity_sweep.py [--out FILE] [--procs 16] [--scale 1.0]

Views (at --scale 1): c1 100, c2 32, c3 512 (8 calls of 64), c4 300 (tracked
in calls of 16 views and, separately, as one stream through the server;
the two must agree byte for byte), c5 32 (one call). Every view is compared
with the oracle by tests/parity.py. Also 16 filtered stacks of the paper's
1280x1024x40 view (fog 0.5-4 per 1000 um^3, thresholds 40-120) go through
the grain recognition, whose grain lists must equal the oracle's exactly,
and the c1 views and 8 c2 views are tracked again under three acceptance
variants (n_min 6; a 5 um finite cylinder; an angle-dependent threshold).
The oracle runs in a pool of worker processes forked before the GPU is
touched; the summary also gives the oracle's whole-pool tracking rate
(grains per second of wall time on those cores).
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from paper_1311_5334_amd import synth  # noqa: E402

COUNTS = {"c5": 32, "c4": 300, "c3": 512, "c2": 32, "c1": 100}
N_STACKS = 16
VARIANTS = {"n_min_6": dict(min_grains=6), "cyl_5um": dict(cyl_ext=500),
            "slope_1_cap_20": dict(thr_slope=(1, 1), thr_max=20)}
N_VARIANT_C2 = 8


def _variant_job(job):
    from oracle import oracle
    name, cfg, idx = job
    v = synth.make_view(cfg, idx)
    c = VARIANTS[name]
    ref = oracle.track_view(v.xyz, n_min=c.get("min_grains", 8), cyl_ext=c.get("cyl_ext", -1),
                            thr_slope=c.get("thr_slope", (0, 1)), thr_max=c.get("thr_max", 0))
    return name, cfg, idx, ref


def _stack(i):
    from paper_1311_5334_amd import synth_stack
    st = synth_stack.make_stack(i, fog_per_1000_um3=0.5 + 3.5 * (i % 4) / 3.0)
    st.threshold = (40, 60, 90, 120)[(i // 4) % 4]
    return st


def _stack_job(i):
    from oracle.grains import find_grains
    st = _stack(i)
    ref, _ = find_grains(st.img, st.threshold)
    return i, ref


def _oracle_job(job):
    from oracle import oracle
    cfg, idx = job
    v = synth.make_view(cfg, idx)
    t0 = time.perf_counter()
    ref = oracle.track_view(v.xyz)
    return cfg, idx, v.n, ref, time.perf_counter() - t0


def _gpu_all(jobs):
    """GPU results per (config, index): batched calls per config, plus the
    c4 views through the server."""
    from paper_1311_5334_amd import emt
    emt.load()
    by_cfg = {}
    for cfg, idx in jobs:
        by_cfg.setdefault(cfg, []).append(idx)
    got, served = {}, {}
    per_call = {"c1": 100, "c2": 32, "c3": 64, "c4": 16, "c5": 32}
    t0 = time.perf_counter()
    with emt.Tracker(device=0) as tr:
        for cfg, idxs in by_cfg.items():
            views = [synth.make_view(cfg, i) for i in idxs]
            for k in range(0, len(views), per_call[cfg]):
                part = views[k:k + per_call[cfg]]
                res = tr([v.xyz for v in part])
                for i, r in zip(idxs[k:k + per_call[cfg]], res):
                    got[(cfg, i)] = r
            print(f"gpu: {cfg} {len(views)} views tracked [{time.perf_counter() - t0:.1f} s]",
                  flush=True)
            if cfg == "c4":
                with emt.Server(n_pipes=2, max_batch_views=16, device=0) as srv:
                    for i, v in zip(idxs, views):
                        srv.submit(v.xyz, view_id=i)
                    while len(served) < len(views):
                        for r in srv.poll(wait_ms=200):
                            served[("c4", r["view_id"])] = r
                print(f"gpu: c4 {len(views)} views served [{time.perf_counter() - t0:.1f} s]",
                      flush=True)
    return got, served


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="also write the summary to this file")
    ap.add_argument("--procs", type=int, default=16)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of each view count")
    args = ap.parse_args()
    jobs = [(cfg, i) for cfg, n in COUNTS.items() for i in range(max(1, int(n * args.scale)))]
    # workers fork before this process touches the GPU
    ctx = mp.get_context("fork")
    pool = ctx.Pool(args.procs)
    t_pool = time.perf_counter()
    it = pool.imap_unordered(_oracle_job, jobs, chunksize=1)
    n_st = max(1, int(N_STACKS * args.scale))
    it_st = pool.imap_unordered(_stack_job, range(n_st), chunksize=1)
    vjobs = [(name, cfg, i) for name in VARIANTS
             for cfg, n in (("c1", COUNTS["c1"]), ("c2", N_VARIANT_C2))
             for i in range(max(1, int(n * args.scale)))]
    it_var = pool.imap_unordered(_variant_job, vjobs, chunksize=1)
    got, served = _gpu_all(jobs)
    from paper_1311_5334_amd import emt
    st_fail, st_grains = 0, 0
    with emt.Tracker(device=0) as tr:
        st_got = {}
        for i in range(n_st):
            st = _stack(i)
            st_got[i] = tr.find_grains(st.img, st.threshold)
    print(f"gpu: {n_st} stacks recognised", flush=True)
    var_got = {}
    for name, c in VARIANTS.items():
        with emt.Tracker(device=0, **c) as tr:
            for cfg in ("c1", "c2"):
                idxs = [i for (nm, cf, i) in vjobs if nm == name and cf == cfg]
                res = tr([synth.make_view(cfg, i).xyz for i in idxs])
                for i, r in zip(idxs, res):
                    var_got[(name, cfg, i)] = r
    print(f"gpu: {len(var_got)} variant views tracked", flush=True)
    stats = {cfg: {"views": 0, "grains": 0, "cpu_s": 0.0, "fail": 0, "first": "", "tracks": 0}
             for cfg in COUNTS}
    serve_mismatch = 0
    done = 0
    t_said = time.perf_counter()
    for cfg, idx, n, ref, sec in it:
        st = stats[cfg]
        st["views"] += 1
        st["grains"] += n
        st["cpu_s"] += sec
        st["tracks"] += len(ref.tracks)
        v = synth.make_view(cfg, idx)
        from parity import assert_view_parity
        try:
            assert_view_parity(v.xyz, got[(cfg, idx)], ref)
        except AssertionError as e:
            st["fail"] += 1
            st["first"] = st["first"] or f"{cfg}[{idx}]: {e!r}"[:200]
        if cfg == "c4":
            a, b = got[(cfg, idx)], served[(cfg, idx)]
            if (b["status"] != 0 or a["tracks"].tobytes() != b["tracks"].tobytes()
                    or not np.array_equal(a["grains"], b["grains"])):
                serve_mismatch += 1
        done += 1
        if done % 50 == 0 or done == len(jobs) or time.perf_counter() - t_said > 30:
            t_said = time.perf_counter()
            print(f"oracle: {done}/{len(jobs)} views compared "
                  f"[{time.perf_counter() - t_pool:.0f} s]", flush=True)
    wall = time.perf_counter() - t_pool
    for i, ref in it_st:
        st_grains += len(ref)
        if not np.array_equal(st_got[i], ref):
            st_fail += 1
    print(f"oracle: {n_st} stacks compared", flush=True)
    var_fail, var_first = 0, ""
    from parity import assert_view_parity as _avp
    for name, cfg, idx, ref in it_var:
        try:
            _avp(synth.make_view(cfg, idx).xyz, var_got[(name, cfg, idx)], ref)
        except AssertionError as e:
            var_fail += 1
            var_first = var_first or f"{name} {cfg}[{idx}]: {e!r}"[:200]
    print(f"oracle: {len(vjobs)} variant views compared", flush=True)
    pool.close()
    pool.join()
    fails = sum(st["fail"] for st in stats.values())
    lines = ["# Parity sweep: GPU library vs CPU oracle", "",
             f"Command (repo root, one MI355X): `python tests/parity_sweep.py --procs {args.procs}"
             + (f" --scale {args.scale}" if args.scale != 1.0 else "")
             + (" --out <this file>" if args.out else "") + "`", "",
             "Every view below was tracked on the GPU (calls of 100 c1, 32 c2, 64 c3, 16 c4 and "
             "32 c5 views) and compared with the oracle: seed counts, candidate counts, track "
             "seeds, order, grain lists and grain order, fit axis and FP64 flag exactly; "
             "slopes, direction, centroid and extent within the tolerances of tests/parity.py. "
             "The c4 views also went through the server as one stream (two pipelines, up to "
             "16 views a batch) and had to match the batched results byte for byte.", "",
             "| config | views | grains | tracks | mismatches | oracle CPU s |",
             "|---|---:|---:|---:|---:|---:|"]
    for cfg in ("c1", "c2", "c3", "c4", "c5"):
        st = stats[cfg]
        lines.append(f"| {cfg} | {st['views']} | {st['grains']:,} | {st['tracks']:,} | "
                     f"{st['fail']} | {st['cpu_s']:.0f} |")
    tot_g = sum(st["grains"] for st in stats.values())
    tot_cpu = sum(st["cpu_s"] for st in stats.values())
    lines += ["", f"Served c4 stream vs batched c4: {serve_mismatch} mismatching views of "
              f"{stats['c4']['views']}.", "",
              f"Grain recognition: {n_st} stacks of 1280x1024x40 pixels, {st_grains:,} grains; "
              f"{st_fail} stacks differ from the oracle's grain list.", "",
              f"Acceptance variants ({', '.join(VARIANTS)}): {len(vjobs)} views (all c1 views "
              f"and {N_VARIANT_C2} c2 views under each, one call per variant and config); "
              f"{var_fail} differ from the oracle." + (f" First: {var_first}" if var_first else ""),
              "",
              f"Oracle: {tot_g:,} grains in {tot_cpu:.0f} s of single-thread CPU time "
              f"({tot_g / tot_cpu:,.0f} grains/s per core); {args.procs} worker processes "
              f"finished in {wall:.0f} s of wall time ({tot_g / wall:,.0f} grains/s for the "
              f"pool, host CPU count {os.cpu_count()})."]
    for cfg in COUNTS:
        if stats[cfg]["first"]:
            lines.append(f"First mismatch: {stats[cfg]['first']}")
    text = "\n".join(lines) + "\n"
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        open(args.out, "w").write(text)
    print(text, flush=True)
    return 1 if fails or serve_mismatch or st_fail or var_fail else 0


if __name__ == "__main__":
    sys.exit(main())
