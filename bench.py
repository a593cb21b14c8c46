"""Benchmark: TPC clusters tracked per second on one MI355X, with p50/p99 latency.

A step is one call of the whole hot path (hit grid, neighbours, cleaner,
chains, Kalman tracklet construction, selection) over one batch that is
already resident in HBM: by default a continuous-readout slice of 50 min-bias
Pb-Pb collisions (36 sector units, ~23 M clusters), generated synthetically
with a fixed seed.  The timed steps replay the call from a HIP graph; the
per-kernel times come from a separate pass with events between the kernels.

Prints ONE JSON line (rank 0).  Besides the contract fields it carries:
  roofline      the dominant kernel: algorithmic bytes per launch / its mean
                duration from HIP events recorded on the library's stream;
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload;
  plain_per_sector  the same work as one call per sector (the plain form);
  collisions    the assignment of the frame's tracks to collisions, after
                tracking and outside the timed step: the call's device time
                (HIP graph replays) and its physics on the 50-collision frame
                of the physical generator against MC truth;
  compression   hit removal and track-model compression of the frame's
                clusters after tracking: device time, HBM roofline, entropy
                of the codes against plain positions;
  clusterizer   raw ADC digits of the frame's clusters to clusters, outside
                the timed step: the call's device time, its HBM roofline and
                the oracle on a sample of units.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC clusters tracked/sec on 1 MI355X; p50/p99 time-frame latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cluster of each kernel family: every array the method
# defines is written once and read once per consuming step at its narrowest
# type (hit grid 24, neighbours 14, cleaner 12, tracklet constructor 27,
# selector 17: 94 in total).
B_ALG = {"grid": 24, "neighbours": 14, "cleaner": 12, "constructor": 27, "selector": 17}
B_ALG_TOTAL = sum(B_ALG.values())
# VALU issue: 256 CUs x 4 SIMDs; a wave64 VALU instruction holds a 16-lane SIMD 4 cycles
N_SIMD = 1024
CLOCK_GHZ = 2.4
# FP32 vector peak of MI355X (256 CUs x 128 FP32 lanes x 2 (FMA) x 2.4 GHz)
FP32_PEAK_TFLOPS = 157.3
# FP32 operations the method defines per Kalman hit update of the tracklet
# constructor (counted on the update's formulas, each FMA as 2, each
# division or square root as 1): parameter transport to the row 24 (with 3
# square roots and 1 division), Jacobian and parameter step 35 (3
# divisions), covariance transport F C F^T on the 15 stored entries 102,
# measurement update with gain, state, covariance and chi2 119 (1 division)
FIT_OPS_PER_UPDATE = 24 + 3 + 1 + 35 + 3 + 102 + 119 + 1
# collision assignment, algorithmic bytes per track: z' kernel reads the state
# (20), x_ref (4) and unit (4) and writes z' (8); the assignment kernel reads
# z' (8), unit (4) and q/pT (4) and writes the candidate (4)
COL_BYTES_PER_TRACK = 20 + 4 + 4 + 8 + 8 + 4 + 4 + 4
# clusterizer, algorithmic bytes: each digit (time 2, charge 2) read once,
# each pad's offset (8) read once, each cluster (y, z, pad, time 4 each, row
# 2, qtot 4, qmax 2) written once
CLU_BYTES_PER_DIGIT, CLU_BYTES_PER_PAD, CLU_BYTES_PER_CLUSTER = 4, 8, 24
# hit removal and compression, algorithmic bytes: per cluster its position and
# row (10) and track index (4) read, class and codes (9) written; per track
# its state at x_ref (24) read once
CMP_BYTES_PER_CLUSTER, CMP_BYTES_PER_TRACK = 23, 24
COL_KERNEL_BYTES = {"k_col_clear": None, "k_col_zdca": 36, "k_col_flags": None, "k_col_number": None,
                    "k_col_assign": 20, "k_col_finish": None}
SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM",
               "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY")
KERNEL_FAMILY = {
    "k_init": None, "k_units": None, "k_tile_hist": "grid", "k_seg_plan": "grid",
    "k_cell_base": "grid", "k_tile_offsets": "grid", "k_tile_scatter": "grid", "k_bin_sort": "grid",
    "k_neighbours": "neighbours", "k_neighbours_wide": "neighbours", "k_clean": "cleaner", "k_scan_blocks": "cleaner",
    "k_compact_starts": "cleaner", "k_chains": "constructor", "k_compact_seeds": "constructor",
    "k_fit": "constructor", "k_select_emit": "selector",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _hip():
    import torch  # noqa: F401 -- the runtime torch loaded
    lib = ctypes.CDLL("libamdhip64.so.7")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def make_workload(name, seed=None):
    import synth
    t = time.time()
    ev = synth.WORKLOADS[name]() if seed is None else synth.WORKLOADS[name](seed)
    log("bench: generated %s: %d clusters in %d units (%.1f s)" % (name, ev.n, ev.n_units, time.time() - t))
    return ev


def col_digest(*names):
    """Digest of kernel sources (default: the collision kernels)."""
    h = hashlib.sha256()
    for name in names or ("tpc_collisions.hip",):
        with open(os.path.join(ROOT, "paper_2106_03636_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def src_digest():
    """Digest of the tracker's kernel sources (its file and the filter header)."""
    return col_digest("tpc_track.hip", "tpc_kalman.h")


def measured_counters(kernel, workload):
    """Counter figures of a kernel (HBM bytes per launch, VALU busy) from the
    committed rocprofv3 runs, if they were taken on the current kernel source;
    else {}."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    try:
        d = json.load(open(p))
    except ValueError:
        return {}
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("src_digest") != src_digest():
        return {}
    return e


def _short(name):
    n = name.replace("(anonymous namespace)::", "")
    if "neg_kernel" in n:
        return "copy_calib"
    return n.split("(")[0].strip()


def _csv(pattern_dir, suffix):
    import csv
    import glob
    paths = sorted(glob.glob(os.path.join(pattern_dir, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit("no *%s under %s" % (suffix, pattern_dir))
    with open(paths[0], newline="") as f:
        return [{k.lower(): v for k, v in r.items()} for r in csv.DictReader(f)]


def _counter_means(d, counter):
    """Mean per dispatch of one counter (summed over its dimensions), by kernel name."""
    per, names = {}, {}
    for r in _csv(d, "counter_collection.csv"):
        if r["counter_name"] != counter:
            continue
        key = r["dispatch_id"]
        per[key] = per.get(key, 0.0) + float(r["counter_value"])
        names[key] = _short(r["kernel_name"])
    acc = {}
    for key, v in per.items():
        acc.setdefault(names[key], []).append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_profiles(prof_dir, workload):
    """Turn rocprofv3 runs of this script into the committed summaries.

    prof_dir holds trace/ (--kernel-trace --stats), fetch/ (--pmc FETCH_SIZE)
    and write/ (--pmc WRITE_SIZE), each from a run with --calib-copy and
    --output-format csv, a cmd.txt with the command line and bench.json with
    the run's output line.  FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are
    scaled by what they read for the 1 GiB-in / 1 GiB-out copy kernel.
    Writes profiles/<workload>_kernels.txt and profiles/traffic.json."""
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stats = {_short(r["name"]): r for r in _csv(os.path.join(prof_dir, "trace"), "kernel_stats.csv")}
    fetch = _counter_means(os.path.join(prof_dir, "fetch"), "FETCH_SIZE")
    write = _counter_means(os.path.join(prof_dir, "write"), "WRITE_SIZE")
    gib_kib = float(1 << 20)
    f_fac = fetch["copy_calib"] / gib_kib
    w_fac = write["copy_calib"] / gib_kib
    sq_dir = os.path.join(prof_dir, "sq")
    sq = {}
    if os.path.isdir(sq_dir):
        for cn in SQ_COUNTERS:
            for k, v in _counter_means(sq_dir, cn).items():
                sq.setdefault(k, {})[cn] = v
    run = json.loads(open(os.path.join(prof_dir, "trace", "bench.json")).read().strip().splitlines()[-1])
    n = run["config"]["clusters"]
    digest = src_digest()
    lines = ["rocprofv3 summary: %s (%d clusters per launch), kernel source digest %s" % (workload, n, digest), ""]
    for sub in ("trace", "fetch", "write") + (("sq",) if sq else ()):
        lines.append("%-5s: %s" % (sub, open(os.path.join(prof_dir, sub, "cmd.txt")).read().strip()))
    lines.append("summary: python bench.py --summarize-profiles <dir of the runs above> --workload %s" % workload)
    lines += ["", "copy kernel (1 GiB read, 1 GiB written): FETCH_SIZE %.6g KiB -> scale %.4f, "
              "WRITE_SIZE %.6g KiB -> scale %.4f" % (fetch["copy_calib"], f_fac, write["copy_calib"], w_fac), "",
              "VALU%: wave64 VALU instructions x 4 cycles / (duration x 1024 SIMDs x " + "%.1f GHz)" % CLOCK_GHZ, "",
              "%-18s %6s %10s %10s %10s %8s %8s %8s %9s %9s %6s" % (
                  "kernel", "calls", "avg_us", "fetch_MB", "write_MB", "B/clus", "GB/s", "alg_B/c", "waves",
                  "valu/wave", "VALU%")]
    traffic = {}
    for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
        if k not in KERNEL_FAMILY:
            continue
        avg_us = float(r["averagens"]) / 1e3
        fb = fetch.get(k, 0.0) * 1024 / f_fac
        wb = write.get(k, 0.0) * 1024 / w_fac
        alg = B_ALG.get(KERNEL_FAMILY[k], 0) if KERNEL_FAMILY[k] else 0
        q = sq.get(k, {})
        waves = q.get("SQ_WAVES", 0.0)
        valu = q.get("SQ_INSTS_VALU", 0.0)
        busy = 100.0 * valu * 4 / (avg_us * 1e-6 * N_SIMD * CLOCK_GHZ * 1e9) if avg_us else 0.0
        lines.append("%-18s %6s %10.1f %10.1f %10.1f %8.2f %8.0f %8s %9.0f %9.0f %6.1f" % (
            k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / n, (fb + wb) / 1e3 / avg_us, alg or "-",
            waves, valu / waves if waves else 0.0, busy))
        traffic[k] = dict(src_digest=digest, bytes_per_launch=fb + wb, fetch_bytes=fb, write_bytes=wb,
                          avg_us=avg_us)
        if q:
            traffic[k].update(valu_insts=valu, valu_busy=busy / 100.0)
    col = run.get("collisions")
    if col:
        nt = col["tracks"]
        lines += ["", "collision assignment (tpc_assign_collisions) over the %d tracks of the frame; one of the "
                  "calls runs on the physical frame's tracks instead" % nt,
                  "%-18s %6s %10s %10s %10s %8s %8s %8s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB",
                                                             "B/track", "GB/s", "alg_B/t")]
        for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
            if k not in COL_KERNEL_BYTES:
                continue
            avg_us = float(r["averagens"]) / 1e3
            fb = fetch.get(k, 0.0) * 1024 / f_fac
            wb = write.get(k, 0.0) * 1024 / w_fac
            lines.append("%-18s %6s %10.1f %10.2f %10.2f %8.1f %8.0f %8s" % (
                k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / nt, (fb + wb) / 1e3 / avg_us,
                COL_KERNEL_BYTES[k] or "-"))
            traffic[k] = dict(src_digest=col_digest(), bytes_per_launch=fb + wb, fetch_bytes=fb, write_bytes=wb,
                              avg_us=avg_us)
    cmpr = run.get("compression")
    if cmpr:
        lines += ["", "hit removal and compression (tpc_compress) over the %d clusters of the frame" % cmpr["clusters"],
                  "%-18s %6s %10s %10s %10s %8s %8s %8s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB",
                                                             "B/clus", "GB/s", "alg_B/c")]
        for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
            if not k.startswith("k_cmp_"):
                continue
            avg_us = float(r["averagens"]) / 1e3
            fb = fetch.get(k, 0.0) * 1024 / f_fac
            wb = write.get(k, 0.0) * 1024 / w_fac
            lines.append("%-18s %6s %10.1f %10.2f %10.2f %8.2f %8.0f %8s" % (
                k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / cmpr["clusters"], (fb + wb) / 1e3 / avg_us,
                CMP_BYTES_PER_CLUSTER if k == "k_cmp_codes" else "-"))
            traffic[k] = dict(src_digest=col_digest("tpc_compress.hip"), bytes_per_launch=fb + wb,
                              fetch_bytes=fb, write_bytes=wb, avg_us=avg_us)
    rft = run.get("refit")
    if rft:
        nt, nh = rft["tracks"], rft["track_hits"]
        lines += ["", "track refit (tpc_refit_tracks) of the %d tracks (%d hits) of the frame" % (nt, nh),
                  "%-18s %6s %10s %10s %10s %8s %8s %9s %9s %6s" % ("kernel", "calls", "avg_us", "fetch_MB",
                                                                    "write_MB", "B/hit", "GB/s", "waves",
                                                                    "valu/wave", "VALU%")]
        for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
            if not k.startswith("k_rf_"):
                continue
            avg_us = float(r["averagens"]) / 1e3
            fb = fetch.get(k, 0.0) * 1024 / f_fac
            wb = write.get(k, 0.0) * 1024 / w_fac
            q = sq.get(k, {})
            waves = q.get("SQ_WAVES", 0.0)
            valu = q.get("SQ_INSTS_VALU", 0.0)
            busy = 100.0 * valu * 4 / (avg_us * 1e-6 * N_SIMD * CLOCK_GHZ * 1e9) if avg_us else 0.0
            lines.append("%-18s %6s %10.1f %10.2f %10.2f %8.2f %8.0f %9.0f %9.0f %6.1f" % (
                k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / max(1, nh), (fb + wb) / 1e3 / avg_us,
                waves, valu / waves if waves else 0.0, busy))
            traffic[k] = dict(src_digest=col_digest("tpc_refit.hip", "tpc_kalman.h"), bytes_per_launch=fb + wb,
                              fetch_bytes=fb, write_bytes=wb, avg_us=avg_us)
            if q:
                traffic[k].update(valu_insts=valu, valu_busy=busy / 100.0)
    mrg = run.get("merge")
    if mrg:
        nt = mrg["tracks"]
        lines += ["", "segment merging (tpc_merge_tracks) and chain fit (tpc_fit_chains) of the %d tracks of the frame: "
                  "%d pairs, %d links, %d chains" % (nt, mrg["pairs"], mrg["links"], mrg["chains"]),
                  "%-18s %6s %10s %10s %10s %8s %9s %9s %6s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB",
                                                               "GB/s", "waves", "valu/wave", "VALU%")]
        for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
            if not (k.startswith("k_mg_") or k.startswith("k_ch_")):
                continue
            avg_us = float(r["averagens"]) / 1e3
            fb = fetch.get(k, 0.0) * 1024 / f_fac
            wb = write.get(k, 0.0) * 1024 / w_fac
            q = sq.get(k, {})
            waves = q.get("SQ_WAVES", 0.0)
            valu = q.get("SQ_INSTS_VALU", 0.0)
            busy = 100.0 * valu * 4 / (avg_us * 1e-6 * N_SIMD * CLOCK_GHZ * 1e9) if avg_us else 0.0
            lines.append("%-18s %6s %10.1f %10.2f %10.2f %8.0f %9.0f %9.0f %6.1f" % (
                k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / 1e3 / avg_us, waves,
                valu / waves if waves else 0.0, busy))
            src = ("tpc_merge.hip",) if k.startswith("k_mg_") else ("tpc_refit.hip", "tpc_kalman.h")
            traffic[k] = dict(src_digest=col_digest(*src), bytes_per_launch=fb + wb, fetch_bytes=fb, write_bytes=wb,
                              avg_us=avg_us)
    clu = run.get("clusterizer")
    if clu:
        nd = clu["digits"]
        lines += ["", "clusterizer (tpc_clusterize) over the %d raw ADC digits of the frame's clusters (%d clusters)"
                  % (nd, clu["clusters"]),
                  "%-18s %6s %10s %10s %10s %8s %8s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB",
                                                       "B/digit", "GB/s")]
        for k, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["totaldurationns"])):
            if not k.startswith("k_clu_"):
                continue
            avg_us = float(r["averagens"]) / 1e3
            fb = fetch.get(k, 0.0) * 1024 / f_fac
            wb = write.get(k, 0.0) * 1024 / w_fac
            lines.append("%-18s %6s %10.1f %10.2f %10.2f %8.2f %8.0f" % (
                k, r["calls"], avg_us, fb / 1e6, wb / 1e6, (fb + wb) / nd, (fb + wb) / 1e3 / avg_us))
            traffic[k] = dict(src_digest=col_digest("tpc_clusterize.hip"), bytes_per_launch=fb + wb,
                              fetch_bytes=fb, write_bytes=wb, avg_us=avg_us)
        lines.append("algorithmic: %d B per digit, %d per pad, %d per cluster; %.3g GB per call"
                     % (CLU_BYTES_PER_DIGIT, CLU_BYTES_PER_PAD, CLU_BYTES_PER_CLUSTER,
                        clu["roofline"]["algorithmic_bytes_per_launch"] / 1e9))
    txt = os.path.join(out_dir, "%s_kernels.txt" % workload)
    open(txt, "w").write("\n".join(lines) + "\n")
    tj = os.path.join(out_dir, "traffic.json")
    d = json.load(open(tj)) if os.path.exists(tj) else {}
    d[workload] = traffic
    json.dump(d, open(tj, "w"), indent=1, sort_keys=True)
    print("\n".join(lines))


def serving_bench(dev, n_frames, n_main, n_sweep, loads, budget_gb, max_in_flight, params, seed=5001,
                  n_capacity=256, batch_clusters=0):
    """Time frames arriving over time (Poisson) at the native server.

    A pool of frames is generated (80% Pb-Pb slices of 10-50 collisions, 20%
    pp frames) and staged on the device and in pinned host memory; requests
    draw frames from it uniformly (seeded), so the server does the full work
    every time.  First the server's capacity is measured in a closed loop,
    then open loops run at fractions of it.  Latency = arrival to the results
    being in host memory, on the client's clock.  The plain form (one tracking
    call per sector unit, then the results copied back) is timed per frame
    and put through the same arrival sequence (first come, first served)."""
    import queue
    import threading
    import numpy as np
    import torch
    import synth
    import paper_2106_03636_amd as T
    from paper_2106_03636_amd.runtime import Batch, Tracker
    from paper_2106_03636_amd.server import Server, TPC_REQ_BORROW_HOST, TPC_REQ_DEVICE

    t = time.time()
    frames = synth.serving_pool(seed, n_frames=n_frames)
    sizes = np.array([f.n for f in frames], np.float64)
    log("bench: serving pool of %d frames, %.1f M clusters mean (%.1f-%.1f M), %.1f s" % (
        len(frames), sizes.mean() / 1e6, sizes.min() / 1e6, sizes.max() / 1e6, time.time() - t))
    dpool = [(torch.as_tensor(f.y).to(dev), torch.as_tensor(f.z).to(dev),
              torch.as_tensor(f.row.view(np.int16)).to(dev)) for f in frames]
    hpool = [tuple(torch.as_tensor(a).pin_memory().numpy() for a in (f.y, f.z, f.row.view(np.int16)))
             for f in frames]
    torch.cuda.synchronize(dev)
    rng = np.random.default_rng(seed + 1)
    srv = Server(frames[0].row_x, frames[0].bz, budget_bytes=int(budget_gb * (1 << 30)),
                 max_in_flight=max_in_flight, queue_depth=64, params=params,
                 max_batch_clusters=int(batch_clusters))

    def submit(i, host):
        f = frames[i]
        if host:
            y, z, r = hpool[i]
            return srv.submit(y, z, r.view(np.uint16), f.unit_offsets, flags=TPC_REQ_BORROW_HOST)
        return srv.submit(*dpool[i], f.unit_offsets, flags=TPC_REQ_DEVICE)

    def run(ids, gaps, host):
        """gaps: inter-arrival times (s), or None for a closed loop."""
        done = [None] * len(ids)
        q = queue.Queue()

        cpu = {}

        def collect():
            c0 = time.thread_time()
            for _ in range(len(ids)):
                k, tk, ta = q.get()
                r = srv.poll(tk, arrays=False)
                done[k] = (time.perf_counter() - ta, r)
                srv.release(tk)
            cpu["collect"] = time.thread_time() - c0
        th = threading.Thread(target=collect)
        s0 = srv.stats()["host_cpu_s"]
        c_sub = time.thread_time()
        th.start()
        t0 = time.perf_counter()
        ta = t0
        busy = 0
        for k, i in enumerate(ids):
            if gaps is not None:
                ta += gaps[k]
                while True:
                    now = time.perf_counter()
                    if now >= ta:
                        break
                    if ta - now > 2e-3:
                        time.sleep(ta - now - 1e-3)
            else:
                ta = time.perf_counter()
            while True:
                st, tk = submit(int(i), host)
                if st == 0:
                    break
                if st != T.TPC_E_BUSY:
                    raise RuntimeError("submit: %s" % T.tpc_status_string(st))
                busy += 1
                time.sleep(2e-4)
            q.put((k, tk, ta))
        c_sub = time.thread_time() - c_sub
        th.join()
        wall = time.perf_counter() - t0
        server_cpu = srv.stats()["host_cpu_s"] - s0
        lat = np.array([d[0] for d in done]) * 1e3
        bad = [d[1]["status"] for d in done if d[1]["status"] != 0]
        if bad:
            raise RuntimeError("served requests failed: %s" % bad[:4])
        ncl = float(sizes[ids].sum())
        batches = np.array([d[1]["batch_requests"] for d in done], np.float64)
        # host cores: the server's own thread, and the client's submit and
        # collect threads (paper §3.1.1 counts the cores that drive a GPU)
        return dict(requests=len(ids), clusters=ncl, wall_s=wall, throughput=ncl / wall,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_batch_requests=float(batches.mean()), busy_retries=busy,
                    host_cores=dict(server_thread=server_cpu / wall,
                                    client_threads=(c_sub + cpu.get("collect", 0.0)) / wall))

    def arrivals(n, load, cap):
        ids = rng.integers(0, len(frames), n)
        rate = load * cap / sizes.mean()  # frames per second
        return ids, rng.exponential(1.0 / rate, n)

    # warm up, then the closed-loop capacity
    run(rng.integers(0, len(frames), 8), None, False)
    capr = run(rng.integers(0, len(frames), n_capacity), None, False)
    cap = capr["throughput"]
    log("bench: served capacity %.3g clusters/s (mean %.2f requests per batch, server thread %.2f cores)"
        % (cap, capr["mean_batch_requests"], capr["host_cores"]["server_thread"]))
    out = dict(pool=dict(frames=len(frames), mean_clusters=float(sizes.mean()), min_clusters=float(sizes.min()),
                         max_clusters=float(sizes.max()), pbpb_share=float(np.mean(
                             [f.name.startswith("pbpb") for f in frames])), seed=seed),
               budget_gb=budget_gb, max_in_flight=max_in_flight, max_batch_clusters=int(batch_clusters),
               grid_shape={k: params[k] for k in ("bin_y_q", "bin_occ", "bin_zmin_q")},
               capacity=dict(clusters_per_s=cap, frames_per_s=cap / sizes.mean(),
                             mean_batch_requests=capr["mean_batch_requests"], host_cores=capr["host_cores"]))
    res = []
    main_ids = main_gaps = None
    for j, load in enumerate(loads):
        n = n_main if j == 0 else n_sweep
        ids, gaps = arrivals(n, load, cap)
        if j == 0:
            main_ids, main_gaps = ids, gaps
        r = run(ids, gaps, False)
        r.update(load=load, offered=load * cap)
        log("bench: served load %.1f: %.3g clusters/s, p50 %.1f ms, p99 %.1f ms, %.2f requests per batch"
            % (load, r["throughput"], r["p50_ms"], r["p99_ms"], r["mean_batch_requests"]))
        res.append(r)
    out["device_inputs"] = res
    ids, gaps = arrivals(n_sweep, loads[0], cap)
    r = run(ids, gaps, True)
    r.update(load=loads[0], offered=loads[0] * cap)
    log("bench: served from host memory, load %.1f: p50 %.1f ms, p99 %.1f ms" % (loads[0], r["p50_ms"], r["p99_ms"]))
    out["host_inputs"] = [r]
    srv.close()

    # the plain form: one call per sector unit, results copied back
    per_unit = max(int(np.diff(f.unit_offsets).max()) for f in frames)
    tr = Tracker(per_unit, 1, len(frames[0].row_x), params, device=dev)
    units = [[Batch.from_device(dpool[i][0][a:b], dpool[i][1][a:b], dpool[i][2][a:b], [0, b - a], f.row_x, f.bz)
              for a, b in zip(f.unit_offsets[:-1], f.unit_offsets[1:])] for i, f in enumerate(frames)]
    svc = np.zeros(len(frames))
    for rep in range(2):
        for i in range(len(frames)):
            torch.cuda.synchronize(dev)
            t1 = time.perf_counter()
            for b in units[i]:
                tr.launch(b)
                r = tr.result()
                r["cluster_track"].cpu(), r["hits"].cpu(), r["params"].cpu()
            svc[i] = time.perf_counter() - t1
    plain_cap = float(sizes.sum() / svc.sum())

    def fifo(ids, gaps):
        t_arr = np.cumsum(gaps)
        end = 0.0
        lat = np.empty(len(ids))
        for k, i in enumerate(ids):
            start = max(t_arr[k], end)
            end = start + svc[i]
            lat[k] = end - t_arr[k]
        return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    throughput=float(sizes[ids].sum() / (end - 0.0)))
    plain = dict(capacity_clusters_per_s=plain_cap, calls_per_frame=len(frames[0].unit_offsets) - 1)
    plain["at_served_main_load"] = fifo(main_ids, main_gaps)
    plain["at_served_main_load"]["stable"] = bool(loads[0] * cap < plain_cap)
    # both forms at a load the plain form sustains
    srv = Server(frames[0].row_x, frames[0].bz, budget_bytes=int(budget_gb * (1 << 30)),
                 max_in_flight=max_in_flight, queue_depth=64, params=params,
                 max_batch_clusters=int(batch_clusters))
    ids, gaps = arrivals(max(32, n_sweep // 2), 0.7, plain_cap)
    low = run(ids, gaps, False)
    srv.close()
    plain["at_0.7_of_plain_capacity"] = dict(offered=0.7 * plain_cap, plain=fifo(ids, gaps),
                                             served=dict(p50_ms=low["p50_ms"], p99_ms=low["p99_ms"],
                                                         throughput=low["throughput"]))
    log("bench: plain per-sector capacity %.3g clusters/s; at 0.7 of it: plain p99 %.1f ms, served p99 %.1f ms"
        % (plain_cap, plain["at_0.7_of_plain_capacity"]["plain"]["p99_ms"], low["p99_ms"]))
    out["plain_per_sector"] = plain
    return out


def batched_bench(dev, reps, retune=False):
    """512 sector chunks of uneven occupancy (1e3-1e5 clusters, pp and Pb-Pb
    generators): one call over all of them, eager with the default grid shape
    and replayed from a HIP graph with the autotuned shape (the autotune
    cache's entry for this batch class; tuned and cached when missing or when
    retune), against the plain form of one call per chunk.  Every form gives
    the same tracks."""
    import numpy as np
    import torch
    from paper_2106_03636_amd import autotune
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    from paper_2106_03636_amd.runtime import Batch, GraphRunner, Tracker

    ev = make_workload("uneven_chunks_512")
    batch = Batch.from_event(ev, dev)
    sizes = np.diff(ev.unit_offsets)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) / k

    tr = Tracker(batch.n, batch.n_units, batch.n_rows, device=dev)
    eager_ms = timed(lambda: tr.launch(batch), reps)
    ref = tr.result()
    n_tracks = ref["n_tracks"]
    del tr
    key = autotune.cache_key(batch)
    table = []
    if retune or key not in autotune.load_cache():
        best, table = autotune.tune(batch, reps=3, log=None)
        autotune.store(batch, best, table)
    best = autotune.tuned_params(batch)
    shape = {k: best[k] for k in autotune.SPACE}
    trt = Tracker(batch.n, batch.n_units, batch.n_rows, best, device=dev)
    g = GraphRunner(trt, batch)
    graph_ms = timed(g.replay, reps)
    res = g.result()
    if res["n_tracks"] != n_tracks:
        raise RuntimeError("tuned graph form found %d tracks, eager %d" % (res["n_tracks"], n_tracks))
    del g, trt
    subs = [Batch.from_device(batch.y[a:b], batch.z[a:b], batch.row[a:b], [0, b - a], ev.row_x, ev.bz)
            for a, b in zip(ev.unit_offsets[:-1], ev.unit_offsets[1:])]
    trp = Tracker(int(sizes.max()), 1, batch.n_rows, device=dev)

    def plain():
        for sb in subs:
            trp.launch(sb)
    plain_ms = timed(plain, max(1, reps // 4))
    plain_tracks = 0
    for sb in subs:  # same tracks as the single call (units are independent)
        trp.launch(sb)
        plain_tracks += trp.result()["n_tracks"]
    if plain_tracks != n_tracks:
        raise RuntimeError("per-chunk calls found %d tracks, one call %d" % (plain_tracks, n_tracks))
    del trp
    n = float(batch.n)
    out = dict(workload="uneven_chunks_512", clusters=int(batch.n), units=int(batch.n_units),
               unit_clusters=dict(min=int(sizes.min()), median=int(np.median(sizes)), max=int(sizes.max())),
               tracks=int(n_tracks),
               graph_tuned=dict(value=n / graph_ms * 1e3, ms=graph_ms, grid_shape=shape),
               eager_default=dict(value=n / eager_ms * 1e3, ms=eager_ms,
                                  grid_shape={k: DEFAULT_PARAMS[k] for k in shape}),
               plain_per_chunk=dict(value=n / plain_ms * 1e3, ms=plain_ms, calls=int(batch.n_units)),
               autotune_key=key, autotune=[dict(r) for r in table], unit="clusters/s")
    log("bench: 512 chunks: graph+tuned %.3g, eager default %.3g, plain per chunk %.3g clusters/s"
        % (out["graph_tuned"]["value"], out["eager_default"]["value"], out["plain_per_chunk"]["value"]))
    return out


def event_bench(dev, reps, params, name):
    """One event (a central Pb-Pb collision: 36 sector units, ~2.6 M clusters;
    or one pp sector): the whole event as one graph-replayed call against one
    eager call per sector unit."""
    import numpy as np
    import torch
    from paper_2106_03636_amd.runtime import Batch, GraphRunner, Tracker

    ev = make_workload(name)
    batch = Batch.from_event(ev, dev)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) / k

    tr = Tracker(batch.n, batch.n_units, batch.n_rows, params, device=dev)
    g = GraphRunner(tr, batch)
    one_ms = timed(g.replay, reps)
    n_tracks = g.result()["n_tracks"]
    del g, tr
    sizes = np.diff(ev.unit_offsets)
    subs = [Batch.from_device(batch.y[a:b], batch.z[a:b], batch.row[a:b], [0, b - a], ev.row_x, ev.bz)
            for a, b in zip(ev.unit_offsets[:-1], ev.unit_offsets[1:])]
    trp = Tracker(int(sizes.max()), 1, batch.n_rows, params, device=dev)

    def plain():
        for sb in subs:
            trp.launch(sb)
    plain_ms = timed(plain, reps)
    n = float(batch.n)
    out = dict(workload=name, clusters=int(batch.n), units=int(batch.n_units), tracks=int(n_tracks),
               one_call_graph=dict(value=n / one_ms * 1e3, ms=one_ms),
               plain_per_sector=dict(value=n / plain_ms * 1e3, ms=plain_ms, calls=int(batch.n_units)),
               unit="clusters/s")
    log("bench: %s: one call %.3g, one call per sector %.3g clusters/s"
        % (name, out["one_call_graph"]["value"], out["plain_per_sector"]["value"]))
    return out


def collision_bench(dev, tr, ev, reps, workload):
    """Collision assignment (tpc_assign_collisions) after tracking: the time
    of one call over the tracks of `ev` (the tracker's last result), and its
    physics on the physical 50-collision frame (one vertex per collision,
    helices end at the outer wall) against MC truth."""
    import numpy as np
    import torch
    import synth
    import paper_2106_03636_amd as T
    from paper_2106_03636_amd import mctruth
    from paper_2106_03636_amd.runtime import Batch, CollisionAssigner
    cp = T.make_collision_params(v_drift=synth.V_DRIFT, outer_radius=synth.R_EXIT)
    side = torch.as_tensor(np.where(np.asarray(ev.unit_sector) < 18, 1, -1).astype(np.int32)).to(dev)
    ca = CollisionAssigner(tr, cp)
    for _ in range(3):
        ca.launch(side, ev.bz)
    g = {k: v.clone() if torch.is_tensor(v) else v for k, v in ca.result().items()}
    n_tracks = int(tr.o_counts[0].item())
    # the call captured in a HIP graph and replayed back to back, so that the
    # host's launch overhead does not show in the device time
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ca.launch(side, ev.bz)
    torch.cuda.synchronize(dev)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    gr = ca.result()
    if int(gr["n_collisions"]) != int(g["n_collisions"]) or not torch.equal(gr["collision"], g["collision"]):
        raise RuntimeError("graph replay and eager call of the collision assignment disagree")
    del graph
    achieved = n_tracks * COL_BYTES_PER_TRACK / (ms * 1e-3) / 1e9
    out = dict(workload=workload, tracks=n_tracks, candidates=int(g["n_collisions"]), ms_per_call=ms,
               tracks_per_s=n_tracks / (ms * 1e-3), launches=6,
               roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=achieved / HBM_PEAK_GBS, algorithmic_bytes_per_track=COL_BYTES_PER_TRACK,
                             traffic=None))
    t = time.time()
    evp = synth.event_pbpb_timeframe(3001, physical=True)
    log("bench: generated the physical frame: %d clusters (%.1f s)" % (evp.n, time.time() - t))
    bp = Batch.from_event(evp, dev)
    tr.launch(bp)
    ca.launch(side, evp.bz)
    res = tr.result()
    gp = ca.result()
    p = res["params"].cpu().numpy()
    kcurv = float(np.float32(-np.float32(synth.KAPPA) * np.float32(evp.bz)))
    trk_side = side.cpu().numpy()[res["unit"].cpu().numpy()]
    out["physics"] = dict(workload="pbpb_timeframe_50 physical (seed 3001)", clusters=int(evp.n),
                          tracks=int(res["n_tracks"]),
                          **mctruth.collision_report(evp.label, evp.tracks.t0, evp.tracks.vz,
                                                     res["n_hits"].cpu().numpy(), res["hits"].cpu().numpy(),
                                                     trk_side, np.abs(kcurv * p[:, 4]) < cp.c_max,
                                                     gp["collision"].cpu().numpy(), gp["side"].cpu().numpy(),
                                                     gp["t0"].cpu().numpy(), synth.V_DRIFT))
    log("bench: collisions " + json.dumps(out))
    return out


def _entropy_bits(counts):
    import numpy as np
    c = np.asarray(counts, np.float64)
    c = c[c > 0]
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum()) if len(p) else 0.0


def compression_bench(dev, tr, batch, reps, workload):
    """Hit removal and track-model compression (tpc_compress) of the tracker's
    last batch: the call's device time from HIP graph replays, the HBM
    roofline, and the entropy of the codes against that of plain positions."""
    import numpy as np
    import torch
    from paper_2106_03636_amd import make_compress_params
    from paper_2106_03636_amd.runtime import Compressor
    cp = make_compress_params()
    c = Compressor(tr, cp)
    for _ in range(2):
        c.launch(batch)
    r = c.result()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        c.launch(batch)
    torch.cuda.synchronize(dev)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    r2 = c.result()
    if not np.array_equal(r2["counts"], r["counts"]):
        raise RuntimeError("graph replay and eager call of the compression disagree")
    del graph
    n_tracks = int(tr.o_counts[0].item())
    alg = CMP_BYTES_PER_CLUSTER * batch.n + CMP_BYTES_PER_TRACK * n_tracks
    achieved = alg / (ms * 1e-3) / 1e9
    # entropy of the codes (what an entropy coder would need) against plain positions
    cls = r["cls"].cpu().numpy()
    cy, cz = r["code_y"].cpu().numpy(), r["code_z"].cpu().numpy()
    keep = cls != 2
    step = float(np.float32(cp.step))
    py = np.rint(batch.y.cpu().numpy().astype(np.float64) / step).astype(np.int64)
    pz = np.rint(batch.z.cpu().numpy().astype(np.float64) / step).astype(np.int64)
    h_pos = sum(_entropy_bits(np.unique(v[keep], return_counts=True)[1]) for v in (py, pz))
    res = cls == 1
    other = keep & ~res
    h_res = _entropy_bits(r["hist_y"]) + _entropy_bits(r["hist_z"])
    h_oth = sum(_entropy_bits(np.unique(v[other], return_counts=True)[1]) for v in (cy, cz)) if other.any() else 0.0
    bits_model = (res.sum() * h_res + other.sum() * h_oth) / max(1, batch.n)
    bits_plain = h_pos * keep.sum() / max(1, batch.n)
    out = dict(workload=workload, clusters=int(batch.n), tracks=n_tracks, ms_per_call=ms,
               clusters_per_s=batch.n / (ms * 1e-3), launches=2,
               classes=dict(no_track=int(r["counts"][0]), residual=int(r["counts"][1]), removed=int(r["counts"][2]),
                            no_model=int(r["counts"][3])),
               removed_fraction=float(r["counts"][2]) / max(1, batch.n),
               entropy_bits_per_cluster=dict(positions_of_kept=bits_plain, track_model=bits_model,
                                             residual_y_z=h_res, raw_float_y_z=64.0),
               roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=achieved / HBM_PEAK_GBS, algorithmic_bytes_per_launch=int(alg), traffic=None))
    log("bench: compression " + json.dumps(out))
    return out


def refit_bench(dev, tr, batch, reps, workload):
    """Track refit (tpc_refit_tracks) of the tracker's last batch: the call's
    device time from HIP graph replays, and its FP32 issue rate against the
    vector peak at the method's operation count per Kalman hit update."""
    import numpy as np
    import torch
    from paper_2106_03636_amd.runtime import Refitter
    if tr._last is not batch:
        raise RuntimeError("the refit leg needs the tracker's last batch")
    rf = Refitter(tr)
    n_tracks = int(tr.o_counts[0].item())
    n_hits = int(tr.o_counts[1].item())
    for _ in range(2):
        rf.launch(batch)
    r = {k: v.cpu().numpy() for k, v in rf.result(n_tracks).items()}
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rf.launch(batch)
    torch.cuda.synchronize(dev)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    r2 = {k: v.cpu().numpy() for k, v in rf.result(n_tracks).items()}
    if not all(np.array_equal(r[k], r2[k]) for k in r):
        raise RuntimeError("graph replay and eager call of the refit disagree")
    del graph
    ok = r["ok"].astype(bool)
    nh = tr.o_n_hits[:n_tracks].cpu().numpy()
    updates = int(2 * nh[ok].sum())  # every hit is updated once per pass
    flops = updates * FIT_OPS_PER_UPDATE
    tfs = flops / (ms * 1e-3) / 1e12
    chi2_ndf = r["chi2"][ok] / np.maximum(1, 2 * nh[ok] - 5)
    out = dict(workload=workload, tracks=n_tracks, track_hits=n_hits, ms_per_call=ms,
               tracks_per_s=n_tracks / (ms * 1e-3), hits_per_s=n_hits / (ms * 1e-3), launches=7,
               refitted_fraction=float(ok.mean()) if n_tracks else 0.0,
               chi2_per_ndf_median=float(np.median(chi2_ndf)) if ok.any() else None,
               roofline=dict(bound="alu", kernel="k_rf_fit (whole call timed)", achieved=tfs,
                             peak=FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=tfs / FP32_PEAK_TFLOPS,
                             hit_updates_per_launch=updates, ops_per_update=FIT_OPS_PER_UPDATE,
                             algorithmic_flops_per_launch=flops, traffic=None))
    log("bench: refit " + json.dumps(out))
    return out


def merge_bench(dev, tr, batch, ev, reps, workload):
    """Segment merging (tpc_merge_tracks) of the tracker's last batch after
    its refit: the merge call's device time from HIP graph replays (the refit
    runs once before), the pairs, candidates and links, and the links'
    purity against MC truth."""
    import numpy as np
    import torch
    import synth
    from paper_2106_03636_amd import mctruth
    from paper_2106_03636_amd.runtime import Merger, Refitter
    if tr._last is not batch:
        raise RuntimeError("the merge leg needs the tracker's last batch")
    rf = Refitter(tr)
    rf.launch(batch)
    # unit angles and sides on the device before the graph is captured
    alpha = torch.as_tensor(np.array([synth.sector_alpha(int(s)) for s in ev.unit_sector], np.float32)).to(dev)
    side = torch.as_tensor(np.where(np.asarray(ev.unit_sector) < 18, 1, -1).astype(np.int32)).to(dev)
    mg = Merger(rf, len(alpha))
    n_tracks = int(tr.o_counts[0].item())
    for _ in range(2):
        mg.launch(batch, alpha, side)
    r = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in mg.result(n_tracks).items()}
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        mg.launch(batch, alpha, side)
    torch.cuda.synchronize(dev)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    r2 = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in mg.result(n_tracks).items()}
    if not np.array_equal(r["next"], r2["next"]):
        raise RuntimeError("graph replay and eager call of the merger disagree")
    del graph
    res = tr.result(sync=False)
    maj = mctruth.majority_particle(ev.label, res["n_hits"].cpu().numpy(), res["hits"].cpu().numpy())
    a = np.nonzero(r["next"] >= 0)[0]
    b = r["next"][a]
    unit = res["unit"].cpu().numpy()
    out = dict(workload=workload, tracks=n_tracks, ms_per_call=ms, tracks_per_s=n_tracks / (ms * 1e-3), launches=10,
               pairs=r["n_pairs"], candidates=r["n_candidates"], links=r["n_links"],
               links_across_sectors=int((unit[a] != unit[b]).sum()),
               link_purity=float(((maj[a] == maj[b]) & (maj[a] >= 0)).mean()) if len(a) else None,
               chains=int(((r["prev"] < 0) & (r["next"] >= 0)).sum()))
    # the fit of the merged chains across frames
    from paper_2106_03636_amd.runtime import ChainFitter
    cfit = ChainFitter(tr)
    for _ in range(2):
        cfit.launch(batch, mg, alpha)
    c = {k: v.cpu().numpy() for k, v in cfit.result(n_tracks).items()}
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cfit.launch(batch, mg, alpha)
    torch.cuda.synchronize(dev)
    graph.replay()
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    cms = e0.elapsed_time(e1) / reps
    c2 = {k: v.cpu().numpy() for k, v in cfit.result(n_tracks).items()}
    if not all(np.array_equal(c[k], c2[k]) for k in c):
        raise RuntimeError("graph replay and eager call of the chain fit disagree")
    del graph
    heads = np.nonzero(c["n_hits"] > 0)[0]
    ok = c["ok"][heads].astype(bool)
    h = heads[ok]
    chi2_ndf = c["chi2"][h] / np.maximum(1, 2 * c["n_hits"][h] - 5)
    cupd = int(2 * c["n_hits"][h].sum())  # every hit is updated once per pass
    cflops = cupd * FIT_OPS_PER_UPDATE
    ctfs = cflops / (cms * 1e-3) / 1e12
    # q/pT against the generated particle: the chain fit and its head segment's own refit
    p = maj[h]
    g = p >= 0
    true_qpt = ev.tracks.q[p[g]] / ev.tracks.pt[p[g]]
    seg = rf.result(n_tracks, sync=False)["params"].cpu().numpy()
    out["chain_fit"] = dict(ms_per_call=cms, chains=int(len(heads)), launches=8,
                            fitted_fraction=float(ok.mean()) if len(heads) else None,
                            hits=int(c["n_hits"][heads].sum()), chi2_per_ndf_median=float(np.median(chi2_ndf)) if len(h) else None,
                            qpt_rel_error_median=dict(chain=float(np.median(np.abs(c["params"][h][g, 4] / true_qpt - 1))),
                                                      head_segment=float(np.median(np.abs(seg[h][g, 4] / true_qpt - 1)))),
                            # the method's FP32 operations per hit update, as for the refit; every
                            # chain's wave is resident at once, so the longest chains' dependent
                            # steps (latency) set the time, not the issue rate
                            roofline=dict(bound="alu", kernel="k_ch_fit (whole call timed)", achieved=ctfs,
                                          peak=FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=ctfs / FP32_PEAK_TFLOPS,
                                          hit_updates_per_launch=cupd, ops_per_update=FIT_OPS_PER_UPDATE,
                                          algorithmic_flops_per_launch=cflops, traffic=None,
                                          limited_by="latency of the longest chains"))
    log("bench: merge " + json.dumps(out))
    return out


def clusterizer_bench(dev, ev, reps, workload, cpu_units=2):
    """Clusterizer (tpc_clusterize) on the raw ADC digits of `ev` (generated
    from its clusters): the call's device time from HIP graph replays, the
    HBM roofline at the algorithmic bytes, and the oracle on cpu_units units
    of the same digits (one core)."""
    import numpy as np
    import torch
    import synth
    import oracle
    from paper_2106_03636_amd.runtime import Clusterizer
    t = time.time()
    d = synth.event_digits(ev, 7)
    log("bench: generated %d digits of %s (%.1f s)" % (d.n, workload, time.time() - t))
    pw, tb, zoff = (float(np.float32(v)) for v in (synth.PAD_W, synth.TIME_BIN, synth.Z_OFF))
    tt, qq, off = Clusterizer.upload(d, dev)
    c = Clusterizer(synth.PAD_HALF, pw, tb, zoff, d.n_units, d.n, device=dev)
    for _ in range(2):
        c.launch(tt, qq, off, d.n_units)
    n_clusters = c.result()["n"]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        c.launch(tt, qq, off, d.n_units)
    torch.cuda.synchronize(dev)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    if c.result()["n"] != n_clusters:
        raise RuntimeError("graph replay and eager call of the clusterizer disagree")
    del graph
    n_pads = d.n_units * synth.PADS_TOTAL
    alg = CLU_BYTES_PER_DIGIT * d.n + CLU_BYTES_PER_PAD * n_pads + CLU_BYTES_PER_CLUSTER * n_clusters
    achieved = alg / (ms * 1e-3) / 1e9
    # the oracle on a sample of units, one thread
    nu = min(cpu_units, d.n_units)
    pads = nu * synth.PADS_TOTAL
    sub_off = d.pad_offsets[:pads + 1]
    n_sub = int(sub_off[-1])
    t = time.time()
    oracle.clusterize(synth.PAD_HALF, sub_off, d.time[:n_sub], d.q[:n_sub], nu, 10, pw, tb, zoff)
    cpu_s = time.time() - t
    out = dict(workload=workload, digits=int(d.n), clusters=int(n_clusters), pads=int(n_pads),
               ms_per_call=ms, digits_per_s=d.n / (ms * 1e-3), launches=4,
               roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=achieved / HBM_PEAK_GBS, algorithmic_bytes_per_launch=int(alg), traffic=None),
               cpu_oracle=dict(value=n_sub / cpu_s, unit="digits/s", cores=1,
                               sample="%d of %d units (%d digits), %.1f s" % (nu, d.n_units, n_sub, cpu_s)))
    log("bench: clusterizer " + json.dumps(out))
    del tt, qq, off, c
    torch.cuda.empty_cache()
    return out


def cpu_baseline(ev, n_units_sample, values, single_core_units=2):
    """The CPU oracle, as it stands, on the first n_units_sample units with all
    its threads, and on single_core_units units with one thread (the paper
    compares against one CPU core, section 3.2)."""
    import oracle
    sub = ev.subset_units(list(range(n_units_sample)))
    oracle.build()
    threads = oracle.num_threads()
    t = time.time()
    r = oracle.run_event(sub, values)
    dt = time.time() - t
    out = dict(value=sub.n / dt, unit="clusters/s", cores=threads, kind="oracle",
               sample="%d of %d sector units of the same workload (%d clusters), one call, %.1f s"
                      % (n_units_sample, ev.n_units, sub.n, dt),
               seconds=dt, n_tracks=int(r["n_tracks"]))
    if single_core_units > 0:
        one = ev.subset_units(list(range(single_core_units)))
        oracle.set_threads(1)
        t = time.time()
        oracle.run_event(one, values)
        d1 = time.time() - t
        oracle.set_threads(threads)
        out["single_core"] = dict(value=one.n / d1, unit="clusters/s", cores=1,
                                  sample="%d sector units (%d clusters), %.1f s" % (single_core_units, one.n, d1))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pbpb_timeframe_50")
    ap.add_argument("--cpu-units", type=int, default=-1,
                    help="units in the CPU-oracle sample (-1: all, 0: skip)")
    ap.add_argument("--no-tune", action="store_true", help="default grid shape instead of the autotuned one")
    ap.add_argument("--retune", action="store_true",
                    help="tune the grid shape for this workload and store it in the autotune cache first")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-chunk batched measurement")
    ap.add_argument("--serve-frames", type=int, default=64, help="frames in the serving pool")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests at the main load")
    ap.add_argument("--serve-sweep", type=int, default=200, help="requests at each other load")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0, help="the server's device memory")
    ap.add_argument("--serve-inflight", type=int, default=3, help="batches the server keeps on the GPU")
    ap.add_argument("--serve-capacity-requests", type=int, default=256,
                    help="requests of the closed loop that measures the served capacity")
    ap.add_argument("--serve-batch-clusters", type=float, default=5e7,
                    help="clusters packed into one batch at most (0: as many as the arena holds)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 runs of this script and exit")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-call-per-sector comparison")
    ap.add_argument("--no-collisions", action="store_true", help="skip the collision-assignment measurement")
    ap.add_argument("--no-clusterizer", action="store_true", help="skip the clusterizer measurement")
    ap.add_argument("--no-compression", action="store_true", help="skip the compression measurement")
    ap.add_argument("--no-refit", action="store_true", help="skip the track refit measurement")
    ap.add_argument("--no-merge", action="store_true", help="skip the segment merging measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.workload)
        return
    if args.gpus != 1:
        print("bench.py measures one MI355X; --gpus %d is not supported (sector units are independent, "
              "so several GPUs would each take whole time frames or a share of a frame's units)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2106_03636_amd as T
    from paper_2106_03636_amd.runtime import Batch, Tracker

    ev = make_workload(args.workload)
    dev = torch.device("cuda:0")
    batch = Batch.from_event(ev, dev)
    # grid shape (speed only; the tuner checks that every shape gives the same
    # tracks): the autotuner's cached choice for this batch class
    from paper_2106_03636_amd import autotune
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    params = dict(DEFAULT_PARAMS)
    shape_source = "default"
    if not args.no_tune:
        if args.retune:
            t = time.time()
            autotune.tuned_params(batch, force=True, log=None)
            log("bench: tuned the grid shape in %.1f s" % (time.time() - t))
            torch.cuda.empty_cache()
        key = autotune.cache_key(batch)
        if key in autotune.load_cache():
            params = autotune.tuned_params(batch)
            shape_source = "autotune cache " + key
    shape = {k: params[k] for k in autotune.SPACE}
    log("bench: grid shape %s (%s)" % (shape, shape_source))
    tr = Tracker(batch.n, batch.n_units, batch.n_rows, params, device=dev)
    log("bench: workspace %.2f GB" % (tr.ws_bytes / 1e9))
    stream = torch.cuda.current_stream(dev)

    # a plain device copy (1 GiB read, 1 GiB written): the HBM rate a streaming
    # kernel reaches here, and the known size that scales the byte counters
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3 if args.calib_copy else 5
    torch.cuda.synchronize(dev)
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize(dev)
    copy_gbs = 2.0 * a.numel() * 4 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()

    # warmup
    for _ in range(args.warmup):
        tr.launch(batch)
    res = tr.result()
    log("bench: %d tracklets, %d tracks, %d assigned clusters" %
        (res["n_tracklets"], res["n_tracks"], res["n_track_hits"]))

    # timed region: K steps, each one replay of the call captured in a HIP
    # graph, with an event pair around every step on the replay stream
    from paper_2106_03636_amd.runtime import GraphRunner
    g = GraphRunner(tr, batch)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize(dev)
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev_s[k].record()
        g.replay()
        ev_e[k].record()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    assert tr.status() == T.TPC_OK
    gres = g.result()
    if gres["n_tracks"] != res["n_tracks"] or gres["n_track_hits"] != res["n_track_hits"]:
        raise RuntimeError("graph replay and eager call disagree")
    step_ms = np.array([ev_s[k].elapsed_time(ev_e[k]) for k in range(args.steps)])
    del g

    # per-kernel times: a separate pass of eager calls with HIP events between
    # the kernels, on the stream the library launches on
    hip = _hip()
    nk = T.tpc_kernel_count()
    names = [T.tpc_kernel_name(i) for i in range(nk)]
    evs = []
    for _ in range(args.steps):
        row = []
        for _ in range(nk + 1):
            e = ctypes.c_void_p()
            assert hip.hipEventCreate(ctypes.byref(e)) == 0
            row.append(e.value)
        evs.append(row)
    torch.cuda.synchronize(dev)
    for k in range(args.steps):
        tr.launch_profiled(batch, evs[k])
    torch.cuda.synchronize(dev)
    assert tr.status() == T.TPC_OK

    def el(a, b):
        ms = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return ms.value

    kern_ms = np.array([[el(evs[k][i], evs[k][i + 1]) for i in range(nk)] for k in range(args.steps)])
    profiled_step_ms = float(np.mean([el(evs[k][0], evs[k][nk]) for k in range(args.steps)]))
    for row in evs:
        for e in row:
            hip.hipEventDestroy(ctypes.c_void_p(e))
    mean_k = kern_ms.mean(axis=0)
    per_kernel = {}
    for i, n in enumerate(names):
        key, j = n, 2
        while key in per_kernel:
            key, j = "%s_%d" % (n, j), j + 1
        per_kernel[key] = round(float(mean_k[i]), 4)
    dom = int(np.argmax(mean_k))
    dom_name = names[dom]
    fam = KERNEL_FAMILY.get(dom_name)
    algo_bytes = (B_ALG[fam] if fam else 0) * batch.n
    achieved = algo_bytes / (mean_k[dom] * 1e-3) / 1e9
    ms_per_step = wall / args.steps * 1e3
    value = batch.n * args.steps / wall
    counters = measured_counters(dom_name, args.workload)
    traffic = counters.get("bytes_per_launch")
    hbm = dict(achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
               algorithmic_bytes_per_launch=algo_bytes, traffic=traffic)
    if dom_name == "k_fit":
        # the constructor is bound by FP32 instruction issue, not by HBM: price it
        # at the FP32 operations its Kalman updates define (both passes)
        K = res["n_seeds"]
        nfit = tr.inspect(T.TPC_VIEW_TRK_NFIT).cpu().numpy()[:K].astype(np.int64)
        p1n = tr.inspect(T.TPC_VIEW_TRK_P1N).cpu().numpy()[:K].astype(np.int64)
        fitted = nfit > 0
        updates = int(nfit[fitted].sum() + p1n[fitted].sum())
        flops = updates * FIT_OPS_PER_UPDATE
        tfs = flops / (mean_k[dom] * 1e-3) / 1e12
        roofline = dict(bound="alu", kernel=dom_name, achieved=tfs, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=tfs / FP32_PEAK_TFLOPS, traffic=traffic, valu_busy=counters.get("valu_busy"),
                        hit_updates_per_launch=updates, ops_per_update=FIT_OPS_PER_UPDATE,
                        algorithmic_flops_per_launch=flops, mean_ms=float(mean_k[dom]), hbm=hbm)
    else:
        roofline = dict(bound="hbm", kernel=dom_name, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=achieved / HBM_PEAK_GBS, traffic=traffic, valu_busy=counters.get("valu_busy"),
                        algorithmic_bytes_per_launch=algo_bytes, mean_ms=float(mean_k[dom]))
    # physics performance of the GPU result against MC truth, and the
    # workspace the call needs as the input grows
    from paper_2106_03636_amd import mctruth
    physics = mctruth.report(ev.label, ev.unit_offsets, ev.tracks.pt, res["first_hit"].cpu().numpy(),
                             res["n_hits"].cpu().numpy(), res["hits"].cpu().numpy(), pt_min=0.2)
    memory = dict(workspace_bytes=int(tr.ws_bytes), workspace_bytes_per_cluster=tr.ws_bytes / batch.n,
                  vs_n=[dict(clusters=int(nn), units=36,
                             workspace_bytes=int(T.tpc_workspace_size(int(nn), 36, batch.n_rows, tr.params)))
                        for nn in (1e4, 1e5, 1e6, 5e6, 2e7, 5e7, 1e8)])
    for e in memory["vs_n"]:
        e["bytes_per_cluster"] = e["workspace_bytes"] / e["clusters"]
    log("bench: per-kernel ms " + json.dumps(per_kernel))
    compression = None if args.no_compression else compression_bench(dev, tr, batch, max(20, args.steps),
                                                                     args.workload)
    # the refit and the merger read the tracker's last batch: they run before
    # the collision leg, which tracks the physical frame with the same tracker
    refit = None if args.no_refit else refit_bench(dev, tr, batch, max(20, args.steps), args.workload)
    merge = None if args.no_merge else merge_bench(dev, tr, batch, ev, max(20, args.steps), args.workload)
    collisions = None if args.no_collisions else collision_bench(dev, tr, ev, max(50, args.steps), args.workload)

    out = dict(
        metric=METRIC, value=value, unit="clusters/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32+i64", data="synthetic",
        config=dict(workload=args.workload, clusters=batch.n, units=batch.n_units, rows=batch.n_rows,
                    bz_tesla=batch.bz, collisions=50 if args.workload.startswith("pbpb_timeframe") else None,
                    grid_shape=dict(shape, source=shape_source)),
        p50_ms=float(np.percentile(step_ms, 50)), p99_ms=float(np.percentile(step_ms, 99)),
        roofline=roofline,
        pipeline_roofline=dict(bytes_per_cluster=B_ALG_TOTAL,
                               achieved=B_ALG_TOTAL * value / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=B_ALG_TOTAL * value / 1e9 / HBM_PEAK_GBS,
                               measured_copy_gbs=copy_gbs,
                               frac_of_copy=B_ALG_TOTAL * value / 1e9 / copy_gbs),
        kernel_ms=per_kernel, profiled_step_ms=profiled_step_ms,
        tracks=res["n_tracks"], tracklets=res["n_tracklets"], physics=physics, memory=memory,
    )
    if collisions is not None:
        out["collisions"] = collisions
    if compression is not None:
        out["compression"] = compression
    if refit is not None:
        out["refit"] = refit
    if merge is not None:
        out["merge"] = merge

    # the plain form: one call per sector unit, same stream, same work
    if not args.no_plain:
        subs = [Batch.from_event(ev.subset_units([u]), dev) for u in range(ev.n_units)]
        trp = Tracker(max(s.n for s in subs), 1, batch.n_rows, params, device=dev)
        for s in subs[:2]:
            trp.launch(s)
        torch.cuda.synchronize(dev)
        reps = max(1, min(5, args.steps))
        t0 = time.perf_counter()
        for _ in range(reps):
            for s in subs:
                trp.launch(s)
        torch.cuda.synchronize(dev)
        dtp = (time.perf_counter() - t0) / reps
        out["plain_per_sector"] = dict(value=batch.n / dtp, unit="clusters/s", ms_per_step=dtp * 1e3,
                                       calls_per_step=len(subs))
        del trp

    del tr
    torch.cuda.empty_cache()
    if not args.no_clusterizer:
        out["clusterizer"] = clusterizer_bench(dev, ev, max(20, args.steps), args.workload)
    if not args.no_batched:
        out["central"] = event_bench(dev, max(4, args.steps), params, "pbpb_central")
        out["pp_sector"] = event_bench(dev, max(4, args.steps), params, "pp_sector")
        out["batched"] = batched_bench(dev, max(4, args.steps), retune=args.retune)
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = serving_bench(dev, args.serve_frames, args.serve_requests, args.serve_sweep,
                                       (0.7, 0.3, 0.5, 0.9), args.serve_budget_gb, args.serve_inflight, params,
                                       n_capacity=args.serve_capacity_requests,
                                       batch_clusters=args.serve_batch_clusters)

    if args.cpu_units != 0:
        from paper_2106_03636_amd.params import DEFAULT_PARAMS
        nu = ev.n_units if args.cpu_units < 0 else min(args.cpu_units, ev.n_units)
        log("bench: timing the CPU oracle on %d units" % nu)
        out["cpu_baseline"] = cpu_baseline(ev, nu, DEFAULT_PARAMS)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
