"""Throughput of the 4pi track finder on one MI355X.

One step = one whole pass of the tracking path (bin, seeds, count, members,
merge, fit, copy-out) over one batch of the largest single-GPU workload: 32
dense star-topology views per call (350 x 350 x 50 um each, 10 vertices of
3-8 prongs, 200 tracks, fog 10 grains per 1000 um^3, about 70k grains a
view), all through one sequence of launches. The grains are resident in HBM
before the timed region starts (device-pointer input); results are copied
back to the host inside it.

Prints one JSON line: grains/s (value), mm^2/hour, per-call latency p50/p99,
the counting kernel's roofline (HIP events on the library's stream) and the
binning stage's HBM rate, and the CPU oracle timed on this host (one core and
the whole box). The same line carries the other forms: the plain path on one
c2 view, 64 uneven c3 views per call, the served c4 stream, grain
recognition, filtering, the module workload and the acceptance variants.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU peak for 32-bit lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic operations per (seed, grain) cylinder test: cross product
# g_k x d - g_i x d (6 multiplies, 6 subtractions), squared norm (3
# multiplies, 2 adds), one compare.
OPS_PER_TEST = 18
HBM_PEAK_GBS = 8000.0
# the counting kernel's code and the tables that shape its work
COUNT_KERNEL_SRCS = [os.path.join(ROOT, "paper_1311_5334_amd", "csrc", f)
                     for f in ("kernels.hip", "cell_table.h", "tile_table.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "count_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "count_valu.json")
BIN_BYTES_PER_GRAIN = 44
GRAIN_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grain_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in COUNT_KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_for_current_kernel(per_launch_tests: float):
    """HBM bytes per launch of the counting kernel from the committed PMC
    summary, only if it was taken on the current kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def grain_traffic_for_current_kernel():
    """HBM bytes per stack of the grain-recognition kernels from the
    committed PMC summary, only if it was taken on the current source."""
    try:
        rec = json.load(open(GRAIN_TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_stack")


def valu_counters_for_current_kernel():
    """The counting kernel's VALU issue rate and lane use from the committed
    PMC summary, only if it was taken on the current kernel source."""
    try:
        rec = json.load(open(VALU_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    keys = ("workload", "valu_issue_frac", "lane_util", "lane_ops_frac_of_peak",
            "valu_lane_ops_per_test", "lds_active_frac", "lds_bank_conflict_frac",
            "lds_insts_per_test", "lds_bytes_per_s_frac_of_measured")
    return {k: rec[k] for k in keys if k in rec}


def _lscpu() -> dict:
    """Host CPU model and core counts as lscpu reports them."""
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        txt = ""
    f = {}
    for line in txt.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            f[k.strip()] = v.strip()

    def num(key, default):
        try:
            return int(f.get(key, default))
        except ValueError:
            return default
    cpus = num("CPU(s)", os.cpu_count() or 1)
    tpc = max(1, num("Thread(s) per core", 1))
    per_socket = num("Core(s) per socket", 0)
    physical = per_socket * max(1, num("Socket(s)", 1)) if per_socket else max(1, cpus // tpc)
    return {"model": f.get("Model name", "unknown"), "physical_cores": physical,
            "logical_cpus": cpus, "threads_per_core": tpc}


def c5_quarter(view_index: int, quarter: int) -> np.ndarray:
    """One quarter (175 x 175 um) of a c5 view: a bounded sample of the
    benchmark workload for the CPU oracle."""
    from paper_1311_5334_amd import synth
    x = synth.make_c5(view_index).xyz
    qx, qy = quarter % 2, quarter // 2
    keep = ((x[:, 0] >= qx * 17500) & (x[:, 0] < (qx + 1) * 17500) &
            (x[:, 1] >= qy * 17500) & (x[:, 1] < (qy + 1) * 17500))
    return np.ascontiguousarray(x[keep])


def _oracle_crop_worker(view_index: int, quarter: int) -> None:
    """Child-process mode: time the oracle on one c5 quarter, print JSON."""
    from oracle import oracle
    xyz = c5_quarter(view_index, quarter)
    t0 = time.perf_counter()
    oracle.track_view(xyz)
    dt = time.perf_counter() - t0
    print(json.dumps({"grains": int(len(xyz)), "seconds": dt}), flush=True)


def cpu_baseline() -> dict:
    """The oracle (single-threaded C, as it stands) on quarters of c5 views,
    timed on this host before the GPU is touched: one process on one core,
    then P processes at once, P = the physical cores available (at most the
    cores this process may run on), each on its own quarter."""
    import subprocess
    from oracle import oracle
    oracle.build()
    info = _lscpu()
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else info["logical_cpus"]
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    P = max(1, min(info["physical_cores"], allowed, share if share > 0 else allowed))

    def run(jobs):
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-crop",
                                   str(v), str(q)], stdout=subprocess.PIPE, text=True)
                 for v, q in jobs]
        t0 = time.perf_counter()
        outs = [json.loads(p.communicate(timeout=600)[0].strip().splitlines()[-1]) for p in procs]
        return outs, time.perf_counter() - t0

    one, _ = run([(0, 0)])
    box, box_wall = run([(1 + k // 4, k % 4) for k in range(P)])
    g1, s1 = one[0]["grains"], one[0]["seconds"]
    gb = sum(o["grains"] for o in box)
    slowest = max(o["seconds"] for o in box)
    return {"value": round(g1 / s1, 1), "unit": "grains/s", "cores": 1, "kind": "oracle",
            "sample": f"one quarter (175x175 um) of c5 view 0, {g1} grains, "
                      f"single-threaded C oracle, {s1:.2f} s of tracking",
            "host": info,
            "whole_box": {"value": round(gb / slowest, 1), "unit": "grains/s", "cores": P,
                          "sample": f"{P} processes at once, each on its own quarter of c5 "
                                    f"views 1..{(P - 1) // 4 + 1} ({gb} grains); rate over the "
                                    f"slowest process's {slowest:.2f} s of tracking",
                          "wall_s_with_generation": round(box_wall, 2)}}


def measure_batch(emt, torch, views, calls: int, warmup: int) -> dict:
    """Whole-batch calls on device-resident views: throughput, per-call
    latency, and the counting kernel's share from one call with stage events."""
    devs = [torch.from_numpy(v.xyz).to("cuda:0").contiguous() for v in views]
    grains = sum(v.n for v in views)
    area = sum(v.area_mm2 for v in views)
    torch.cuda.synchronize()
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as tr:
        for _ in range(warmup):
            tr(devs)
        lat = []
        t0 = time.perf_counter()
        for _ in range(calls):
            t1 = time.perf_counter()
            tr(devs)
            lat.append(time.perf_counter() - t1)
        wall = time.perf_counter() - t0
        st0 = tr.stats()
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS) as tr:
        tr(devs)
        tr(devs)
        st = tr.stats()
    lat_ms = np.array(lat) * 1e3
    count_s = st["ms"]["count"] * 1e-3
    achieved = st["n_tests"] * OPS_PER_TEST / count_s / 1e12
    return {"views_per_call": len(views), "grains_per_call": grains,
            "grains_per_s": round(grains * calls / wall, 1),
            "mm2_per_hour": round(area * calls / wall * 3600.0, 2),
            "ms_per_call": round(wall / calls * 1e3, 3),
            "call_latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                                "p99": round(float(np.percentile(lat_ms, 99)), 3)},
            "stage_ms": {k: round(v, 3) for k, v in st["ms"].items()},
            "work": {"seeds": st0["n_seeds"], "tests": st0["n_tests"],
                     "candidates": st0["n_candidates"], "tracks": st0["n_tracks"],
                     "merge_rounds": st0["merge_rounds"]},
            "count_roofline": {"achieved": round(achieved, 3), "unit": "Tops/s",
                               "frac": round(achieved / (VALU_PEAK_OPS / 1e12), 4)},
            # binning: two reads of the 12-byte grains, one 16-byte sorted
            # write and the cell counters, about 44 bytes a grain
            "bin_roofline": {"achieved": round(BIN_BYTES_PER_GRAIN * grains /
                                               (st["ms"]["bin"] * 1e-3) / 1e9, 1),
                             "unit": "GB/s", "bytes_per_grain": BIN_BYTES_PER_GRAIN,
                             "frac": round(BIN_BYTES_PER_GRAIN * grains / (st["ms"]["bin"] * 1e-3)
                                           / 1e9 / HBM_PEAK_GBS, 4)}}


def measured_copy_gbs(torch, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """A plain device-to-device copy of nbytes, timed with events: bytes
    read plus bytes written per second, the streaming rate HBM gives a
    simple kernel on this GPU."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2.0 * nbytes / sec / 1e9


def measure_served(emt, views, n_req: int, warmup: int, batch: int = 16,
                   fracs=(0.5, 0.9), seed: int = 0x5E4FE, n_pipes: int = 2,
                   max_batch: int = 16) -> dict:
    """The served form on a pool of c4 views (host arrays, as a microscope
    hands them over). First the batched capacity mu_b (views/s through
    emt_track_views, batch views per call) and the plain one-view-per-call
    rate; then a Poisson stream at each fraction of mu_b through the server,
    with latency = completion - submission per view."""
    import threading
    xyzs = [v.xyz for v in views]
    area = np.array([v.area_mm2 for v in views])
    ngr = np.array([v.n for v in views])
    out = {"pool_views": len(views), "pool_mean_grains": round(float(ngr.mean()), 1)}
    with emt.Tracker(device=0) as tr:
        for k in range(0, len(xyzs), batch):
            tr(xyzs[k:k + batch])
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            for k in range(0, len(xyzs), batch):
                tr(xyzs[k:k + batch])
        mu_b = reps * len(xyzs) / (time.perf_counter() - t0)
    # the counting kernel on the same batches the server forms at load,
    # timed stage by stage (a separate pass, so mu_b is not slowed by events)
    tests, count_s = 0, 0.0
    with emt.Tracker(device=0, flags=emt.EMT_F_STATS) as tr:
        for k in range(0, len(xyzs), batch):
            tr(xyzs[k:k + batch])
            st = tr.stats()
            tests += st["n_tests"]
            count_s += st["ms"]["count"] * 1e-3
    if count_s > 0:
        ach = tests * OPS_PER_TEST / count_s / 1e12
        out["count_roofline"] = {"achieved": round(ach, 3), "unit": "Tops/s",
                                 "peak": round(VALU_PEAK_OPS / 1e12, 2),
                                 "frac": round(ach / (VALU_PEAK_OPS / 1e12), 4),
                                 "note": "k_count over the pool in batches of the served "
                                         "size, 18 ops per (seed, grain) test"}
    with emt.Tracker(device=0) as tr:
        lat = []
        t0 = time.perf_counter()
        for x in xyzs:
            t1 = time.perf_counter()
            tr([x])
            lat.append(time.perf_counter() - t1)
        plain_rate = len(xyzs) / (time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    out["batched_capacity_views_per_s"] = round(mu_b, 1)
    out["plain"] = {"views_per_s": round(plain_rate, 1),
                    "grains_per_s": round(plain_rate * float(ngr.mean()), 1),
                    "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                   "p99": round(float(np.percentile(lat, 99)), 3)}}
    rng = np.random.default_rng(seed)
    runs = []
    for frac in fracs:
        lam = frac * mu_b
        total = n_req + warmup
        pick = rng.integers(0, len(xyzs), total)
        gaps = rng.exponential(1.0 / lam, total)
        with emt.Server(n_pipes=n_pipes, max_batch_views=max_batch, device=0) as srv:
            def feed():
                t_next = time.perf_counter()
                for k in range(total):
                    t_next += gaps[k]
                    dt = t_next - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    srv.submit(xyzs[pick[k]], view_id=k)
            th = threading.Thread(target=feed)
            th.start()
            res = {}
            while len(res) < total:
                for r in srv.poll(wait_ms=50):
                    res[r["view_id"]] = (r["status"], r["t_submit_ms"], r["t_done_ms"],
                                         r["batch_views"])
            th.join()
            st = srv.stats()
        ks = np.arange(warmup, total)
        bad = sum(1 for k in ks if res[k][0] != 0)
        sub = np.array([res[k][1] for k in ks])
        done = np.array([res[k][2] for k in ks])
        lat = done - sub
        win_s = (done.max() - sub.min()) * 1e-3
        runs.append({"lambda_frac_of_mu_b": frac, "lambda_views_per_s": round(lam, 1),
                     "microscopes_at_5hz": round(lam / 5.0, 1),
                     "requests": int(n_req), "warmup": int(warmup), "errors": int(bad),
                     "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                    "p99": round(float(np.percentile(lat, 99)), 3)},
                     "grains_per_s": round(float(ngr[pick[ks]].sum()) / win_s, 1),
                     "mm2_per_hour": round(float(area[pick[ks]].sum()) / win_s * 3600.0, 2),
                     "mean_batch_views": round(float(np.mean([res[k][3] for k in ks])), 2),
                     "device_busy_frac": round(st["busy_ms"] / st["elapsed_ms"], 3),
                     "two_batches_on_device_frac": round(st["overlap_ms"] / st["elapsed_ms"], 3)})
    out["served"] = runs
    return out


def measure_grains(emt, torch, stacks, calls: int = 20) -> dict:
    """Grain recognition on device-resident filtered stacks of the paper's
    view (1280 x 1024 x 40 pixels): device time per stack from the library's
    events, the rate of stack bytes through it against the HBM peak."""
    devs = [torch.from_numpy(st.img).to("cuda:0").contiguous() for st in stacks]
    torch.cuda.synchronize()
    ms, grains = [], 0
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS) as tr:
        out = torch.empty((1 << 20, 3), dtype=torch.int32, device="cuda:0")
        for d, st in zip(devs, stacks):
            tr.find_grains(d, st.threshold, max_out=out.shape[0], out=out)
        t0 = time.perf_counter()
        for k in range(calls):
            d, st = devs[k % len(devs)], stacks[k % len(stacks)]
            g = tr.find_grains(d, st.threshold, max_out=out.shape[0], out=out)
            ms.append(tr.stats()["ms_total"])
            grains += g.shape[0]
        wall = time.perf_counter() - t0
    nbytes = devs[0].numel()
    dev_ms = float(np.median(ms))
    # algorithmic bytes: the stack read once, the grains written once
    achieved = (nbytes + 12.0 * grains / calls) / (dev_ms * 1e-3) / 1e9
    return {"stacks": len(stacks), "pixels_per_stack": nbytes,
            "grains_per_stack": round(grains / calls, 1),
            "device_ms_per_stack": round(dev_ms, 4),
            "call_ms_per_stack": round(wall / calls * 1e3, 4),
            "stacks_per_s": round(1e3 / dev_ms, 1),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": grain_traffic_for_current_kernel(),
                         "note": "stack bytes read once and 12 bytes written per grain "
                                 "(algorithmic), over the device time of the whole "
                                 "recognition: clear, find and place kernels"}}


def measure_filter(emt, torch, raws, calls: int = 20) -> dict:
    """Image filtering of device-resident raw stacks of the paper's view
    (1280 x 1024 x 40 pixels) with their per-pixel maps, then grain
    recognition of the filtered stack: device time of each from the
    library's events, the filtering's HBM rate against the peak."""
    dev = [(torch.from_numpy(r.raw).to("cuda:0").contiguous(),
            torch.from_numpy(r.gain.view(np.int16)).to("cuda:0").contiguous(),
            torch.from_numpy(r.thr).to("cuda:0").contiguous()) for r in raws]
    torch.cuda.synchronize()
    f_ms, g_ms, grains = [], [], 0
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS) as tr:
        filt = torch.empty_like(dev[0][0])
        out = torch.empty((1 << 20, 3), dtype=torch.int32, device="cuda:0")
        for raw, gain, thr in dev:
            tr.filter_stack(raw, gain, thr, out=filt)
            tr.find_grains(filt, 40, max_out=out.shape[0], out=out)
        for k in range(calls):
            raw, gain, thr = dev[k % len(dev)]
            tr.filter_stack(raw, gain, thr, out=filt)
            f_ms.append(tr.stats()["ms_total"])
            g = tr.find_grains(filt, 40, max_out=out.shape[0], out=out)
            g_ms.append(tr.stats()["ms_total"])
            grains += g.shape[0]
    npix = dev[0][0].numel()
    plane = dev[0][2].numel()
    fm, gm = float(np.median(f_ms)), float(np.median(g_ms))
    nbytes = 2 * npix + 3 * plane  # raw read, filtered written, maps read once
    achieved = nbytes / (fm * 1e-3) / 1e9
    return {"stacks": len(raws), "pixels_per_stack": npix,
            "filter_device_ms_per_stack": round(fm, 4),
            "recognition_device_ms_per_stack": round(gm, 4),
            "raw_to_grains_device_ms_per_stack": round(fm + gm, 4),
            "grains_per_stack": round(grains / calls, 1),
            "roofline": {"kernel": "k_filter", "bound": "hbm", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "note": "raw stack read and filtered stack written once, gain and "
                                 "threshold maps read once (algorithmic bytes), over the "
                                 "filtering kernel's device time"}}


def measure_module(emt, seed: int = 0, calls: int = 3) -> dict:
    """The efficiency and fake-rate method of Sec. 3 on a synthetic module
    of four layers, each scanned in 8 x 8 views of 300 x 250 um: all 256
    views tracked in calls of 64 (host arrays, as a microscope hands them
    over), then the layers' tracks matched on the host."""
    from paper_1311_5334_amd import module
    m = module.make_module(seed)
    views = [v.xyz for v in m.views]
    n_grains = sum(len(v) for v in views)
    walls = []
    with emt.Tracker(device=0) as tr:
        res = []
        for k in range(0, len(views), 64):
            tr(views[k:k + 64])
        for _ in range(calls):
            res = []
            t0 = time.perf_counter()
            for k in range(0, len(views), 64):
                res += tr(views[k:k + 64])
            walls.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    eff = module.measure_efficiency(m, module.layer_tracks(m, res))
    match_s = time.perf_counter() - t0
    wall = float(np.median(walls))
    return {"views": len(views), "grains": n_grains, "tracking_s": round(wall, 4),
            "views_per_s": round(len(views) / wall, 1), "grains_per_s": round(n_grains / wall, 1),
            "matching_s": round(match_s, 3), "efficiency": round(eff.efficiency, 4),
            "references": int(eff.selected.sum()), "fake_rate": round(eff.fake_rate, 4),
            "fake_references": int(eff.fake_selected.sum()),
            "by_tan_theta": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                             for r in eff.table()]}


def measure_variants(emt, torch, view, calls: int = 20) -> dict:
    """The plain path on the benchmark view under the acceptance variants:
    device time per view and the candidates and tracks each leaves."""
    dev = torch.from_numpy(view.xyz).to("cuda:0").contiguous()
    torch.cuda.synchronize()
    out = {}
    for name, cfg in (("default", {}), ("paper_n_gt_5", {"min_grains": 6}),
                      ("cylinder_5um", {"cyl_ext": 500}), ("segment_only", {"cyl_ext": 0}),
                      ("angle_threshold_b1", {"thr_slope": (1, 1)})):
        with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS, **cfg) as tr:
            for _ in range(3):
                r = tr([dev])[0]
            ms, cnt = [], []
            for _ in range(calls):
                r = tr([dev])[0]
                st = tr.stats()
                ms.append(sum(st["ms"].values()))
                cnt.append(st["ms"]["count"])
        out[name] = {"config": {k: list(v) if isinstance(v, tuple) else v for k, v in cfg.items()},
                     "device_ms_per_view": round(float(np.median(ms)), 4),
                     "count_ms": round(float(np.median(cnt)), 4),
                     "grains_per_s": round(view.n / (float(np.median(ms)) * 1e-3), 1),
                     "candidates": int(r["n_candidates"]), "tracks": int(len(r["tracks"]))}
    return out


def measure_plain(emt, torch, view, steps: int, warmup: int) -> dict:
    """The plain path: one c2 view per call, device-resident, with stage
    events; the same loop without events and with host arrays beside it."""
    dev = torch.from_numpy(view.xyz).to("cuda:0").contiguous()
    torch.cuda.synchronize()
    tr = emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS)
    for _ in range(warmup):
        tr([dev])
    torch.cuda.synchronize()
    lat, stage_ms = [], []
    stats = None
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        tr([dev])
        lat.append(time.perf_counter() - t0)
        stats = tr.stats()
        stage_ms.append(stats["ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    tr.close()
    # one graph launch per call (no stage events): the library's own rate
    with emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS) as tq:
        for _ in range(3):
            tq([dev])
        torch.cuda.synchronize()
        t_q = time.perf_counter()
        for _ in range(steps):
            tq([dev])
        torch.cuda.synchronize()
        wall_q = time.perf_counter() - t_q
    # the view as a host array: PCIe copies of grains and tracks in each call
    with emt.Tracker(device=0) as th:
        for _ in range(3):
            th([view.xyz])
        h_lat = []
        for _ in range(steps):
            t0 = time.perf_counter()
            th([view.xyz])
            h_lat.append(time.perf_counter() - t0)
    h_lat_ms = np.array(h_lat) * 1e3
    lat_ms = np.array(lat) * 1e3
    ms = {k: float(np.mean([st[k] for st in stage_ms])) for k in stage_ms[0]}
    count_s = ms["count"] * 1e-3
    if count_s <= 0:
        raise RuntimeError("the library reported no device time for the counting stage")
    tests = stats["n_tests"]
    achieved = tests * OPS_PER_TEST / count_s / 1e12
    peak = VALU_PEAK_OPS / 1e12
    return {
        "workload": "c2: one full 350x350x50 um view per call, 300 tracks, fog 3/1000 um^3",
        "grains_per_view": view.n,
        "grains_per_s": round(view.n * steps / wall, 1),
        "mm2_per_hour": round(view.area_mm2 * steps / wall * 3600.0, 2),
        "ms_per_view": round(wall / steps * 1e3, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "stage_ms": {k: round(v, 4) for k, v in ms.items()},
        "work": {"seeds": stats["n_seeds"], "tests": tests, "hits": stats["n_hits"],
                 "tests_per_hit": round(tests / max(1, stats["n_hits"]), 3),
                 "candidates": stats["n_candidates"], "tracks": stats["n_tracks"],
                 "merge_rounds": stats["merge_rounds"], "fp64_fits": stats["n_fp64_fits"]},
        "roofline": {"kernel": "k_count", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(peak, 2), "unit": "Tops/s",
                     "frac": round(achieved / peak, 4)},
        "without_stage_events": {"grains_per_s": round(view.n * steps / wall_q, 1),
                                 "ms_per_view": round(wall_q / steps * 1e3, 4)},
        "host_input": {"grains_per_s": round(view.n / (float(h_lat_ms.mean()) * 1e-3), 1),
                       "latency_ms": {"p50": round(float(np.percentile(h_lat_ms, 50)), 4),
                                      "p99": round(float(np.percentile(h_lat_ms, 99)), 4)},
                       "note": "the c2 view as a host array: PCIe copies of grains and "
                               "results inside each call"},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="c2,c3,c4,stacks,raw,module,variants",
                    help="other forms to add to the line (comma list of c2 plain, c3 "
                         "batched, c4 served, stacks for grain recognition, raw for "
                         "filtering, module for the efficiency method and variants for the "
                         "acceptance variants; '' for none)")
    ap.add_argument("--served-requests", type=int, default=5000)
    ap.add_argument("--served-warmup", type=int, default=500)
    ap.add_argument("--form-calls", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy, the reference "
                         "for scaling FETCH_SIZE/WRITE_SIZE counters")
    ap.add_argument("--oracle-crop", nargs=2, type=int, metavar=("VIEW", "QUARTER"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_crop:
        _oracle_crop_worker(*args.oracle_crop)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); views are "
              "independent, so N GPUs would each run this same per-GPU workload", file=sys.stderr)
        return 2

    # the CPU oracle first, before anything touches the GPU
    base = None if args.no_cpu_baseline else cpu_baseline()

    import torch
    from paper_1311_5334_amd import emt, synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the headline: 32 c5 views per call, device-resident, stage events on
    views = [synth.make_c5(i) for i in range(32)]
    devs = [torch.from_numpy(v.xyz).to("cuda:0").contiguous() for v in views]
    grains = sum(v.n for v in views)
    area = sum(v.area_mm2 for v in views)
    torch.cuda.synchronize()
    tr = emt.Tracker(device=0, flags=emt.EMT_F_DEVICE_PTRS | emt.EMT_F_STATS)
    for _ in range(args.warmup):
        tr(devs)
    torch.cuda.synchronize()
    lat, stage_ms = [], []
    stats = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        tr(devs)
        lat.append(time.perf_counter() - t0)
        stats = tr.stats()
        stage_ms.append(stats["ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    tr.close()
    lat_ms = np.array(lat) * 1e3
    ms = {k: float(np.mean([st[k] for st in stage_ms])) for k in stage_ms[0]}
    count_s, bin_s = ms["count"] * 1e-3, ms["bin"] * 1e-3
    if count_s <= 0 or bin_s <= 0:
        raise RuntimeError("the library reported no device time for a stage")
    tests = stats["n_tests"]
    achieved = tests * OPS_PER_TEST / count_s / 1e12
    peak = VALU_PEAK_OPS / 1e12
    bin_gbs = BIN_BYTES_PER_GRAIN * grains / bin_s / 1e9
    out = {
        "metric": "grains/s and mm^2/hour per GPU, batched+served vs plain; p50/p99 view latency",
        "value": round(grains * args.steps / wall, 1),
        "unit": "grains/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "c5 batched: 32 dense views per call, each 350x350x50 um with "
                               "10 vertices of 3-8 prongs (0.3-1.0 grains/um, 3-200 um), 200 "
                               "tracks, fog 10/1000 um^3; R=25 um, r=0.5 um, n_min=8",
                   "form": "batched", "views_per_step": len(views), "grains_per_step": grains},
        "mm2_per_hour": round(area * args.steps / wall * 3600.0, 2),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "note": "per call of 32 views (all views of a call finish together)"},
        "stage_ms": {k: round(v, 4) for k, v in ms.items()},
        "work": {"seeds": stats["n_seeds"], "tests": tests, "hits": stats["n_hits"],
                 "tests_per_hit": round(tests / max(1, stats["n_hits"]), 3),
                 "tests_per_seed": round(tests / max(1, stats["n_seeds"]), 3),
                 "candidates": stats["n_candidates"], "tracks": stats["n_tracks"],
                 "merge_rounds": stats["merge_rounds"], "fp64_fits": stats["n_fp64_fits"]},
        "roofline": {"kernel": "k_count", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(peak, 2), "unit": "Tops/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": traffic_for_current_kernel(tests),
                     "counters": valu_counters_for_current_kernel(),
                     "note": "18 integer/FP32 lane operations per (seed, grain) test over "
                             "k_count's device time from HIP events on the library stream"},
        "bin_roofline": {"achieved": round(bin_gbs, 1), "unit": "GB/s",
                         "bytes_per_grain": BIN_BYTES_PER_GRAIN, "peak": HBM_PEAK_GBS,
                         "frac": round(bin_gbs / HBM_PEAK_GBS, 4)},
    }
    forms = {}
    for f in [x for x in args.forms.split(",") if x]:
        if f == "c2":
            forms["plain_c2"] = measure_plain(emt, torch, synth.make_c2(0), args.steps,
                                              args.warmup)
        elif f == "c3":
            vs = [synth.make_c3(i) for i in range(64)]
            forms["batched_c3"] = measure_batch(emt, torch, vs, args.form_calls, 2)
            forms["batched_c3"]["workload"] = ("c3: 64 views per call, 2k-40k grains each "
                                               "(log-uniform), 50-500 tracks, fog 1-5/1000 um^3")
        elif f == "stacks":
            from paper_1311_5334_amd import synth_stack
            sts = [synth_stack.make_stack(i) for i in range(2)]
            forms["grain_recognition"] = measure_grains(emt, torch, sts)
            forms["grain_recognition"]["workload"] = (
                "filtered 1280x1024x40 8-bit stacks of the paper's 300x250x50 um view, 60 "
                "tracks and fog 1/1000 um^3 rendered as spots, threshold 60")
        elif f == "raw":
            from paper_1311_5334_amd import synth_stack
            raws = [synth_stack.make_raw_stack(i) for i in range(2)]
            forms["filtering"] = measure_filter(emt, torch, raws)
            forms["filtering"]["workload"] = (
                "raw 1280x1024x40 bright-field stacks of the paper's view from a modelled "
                "camera with column and pixel gain spread, per-pixel gain (1/256 units) and "
                "pedestal maps; grains recognised at threshold 40 on the filtered stack")
        elif f == "module":
            forms["module_efficiency"] = measure_module(emt)
            forms["module_efficiency"]["workload"] = (
                "four 50 um layers (two detectors of 200 um base) of 2.4 x 2.0 mm, 8 x 8 views of "
                "300 x 250 um each, cosmic rays 150/mm^2 at 42 grains/100 um, cos^3 zenith "
                "angles to tan 2.5, fog 3/1000 um^3, 2 electrons a view; layers 0, 1, 3 "
                "predict layer 2; fakes with layer 2 displaced by 1 mm")
        elif f == "variants":
            forms["acceptance_variants"] = measure_variants(emt, torch, synth.make_c2(0))
            forms["acceptance_variants"]["workload"] = (
                "the c2 view under each acceptance variant; device time of the "
                "whole path per view")
        elif f == "c4":
            vs = [synth.make_c4(i) for i in range(96)]
            forms["served_c4"] = measure_served(emt, vs, args.served_requests, args.served_warmup)
            forms["served_c4"]["workload"] = (
                "c4: Poisson stream drawn from 96 views of 100^2, 200^2 or 350^2 x 50 um, "
                "fog 1-10/1000 um^3, 2449 tracks/mm^2")
    # the streaming rate a plain copy gets, beside the 8 TB/s specification
    copy_gbs = measured_copy_gbs(torch)
    out["hbm_copy_measured_GBs"] = round(copy_gbs, 1)
    # the library's own microbenchmarks of the units the kernels are bound by
    pk = emt.emt_measure_peaks(0)
    out["peaks_measured"] = {
        "int32_lane_Tops": round(pk["int_lane_ops"] / 1e12, 2),
        "fp32_fma_lane_Tops": round(pk["fp32_lane_ops"] / 1e12, 2),
        "lds_read_TBs": round(pk["lds_bytes"] / 1e12, 2),
        "hbm_copy_TBs": round(pk["hbm_copy_bytes"] / 1e12, 3),
        "compute_units": pk["compute_units"], "clock_mhz": pk["clock_khz"] / 1e3,
        "spec_derived": {"lane_Tops": round(VALU_PEAK_OPS / 1e12, 2),
                         "lds_TBs": round(256 * 128 * 2.4e9 / 1e12, 1), "hbm_TBs": 8.0}}
    meas = max(pk["int_lane_ops"], pk["fp32_lane_ops"]) / 1e12
    out["roofline"]["measured_peak"] = round(meas, 2)
    out["roofline"]["frac_of_measured"] = round(achieved / meas, 4)
    out["bin_roofline"]["frac_of_measured"] = round(bin_gbs / copy_gbs, 4)
    for key in ("grain_recognition", "filtering"):
        if key in forms:
            rf = forms[key]["roofline"]
            rf["measured_peak"] = round(copy_gbs, 1)
            rf["frac_of_measured"] = round(rf["achieved"] / copy_gbs, 4)
    if forms:
        out["forms"] = forms
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
