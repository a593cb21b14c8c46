"""Autotuner for the hit-grid shape.

The grid's bin shape (y bin width, target occupancy of the adaptive z bins,
shortest z bin) changes only the speed of the neighbour search and of the
pickups: links are chosen by (score, cluster ids), never by bin, so every
candidate must give the same tracks.  The tuner times each candidate with HIP
events on the launch stream, checks that its cluster-to-track partition equals
the baseline's, and caches the fastest shape per (GPU arch, batch size bucket,
unit count bucket, hits-per-row bucket) in a JSON file.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

import numpy as np
import torch

from .params import DEFAULT_PARAMS
from .runtime import Batch, Tracker

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

SPACE = dict(bin_y_q=(384, 768, 1536), bin_occ=(1, 2, 4), bin_zmin_q=(128, 512))


def _bucket(v):
    return int(round(math.log2(max(1, v)) * 2))


def cache_key(batch: Batch) -> str:
    arch = torch.cuda.get_device_properties(batch.y.device).gcnArchName.split(":")[0]
    per_row = batch.n / max(1, batch.n_units * batch.n_rows)
    return "%s/n%d/u%d/r%d" % (arch, _bucket(batch.n), _bucket(batch.n_units), _bucket(per_row))


def _partition_key(tr: Tracker, res):
    """cluster -> id of its track's first hit (independent of grid order)."""
    import paper_2106_03636_amd as T
    ct = res["cluster_track"].cpu().numpy()
    if res["n_tracks"] == 0:
        return ct
    keep = tr.tracklet_field(T.TPC_VIEW_TRK_KEEP)
    start = tr.inspect(T.TPC_VIEW_TRK_START).cpu().numpy()[:res["n_tracklets"]]
    perm = tr.inspect(T.TPC_VIEW_PERM).cpu().numpy()
    first = perm[start[np.nonzero(keep)[0]]]
    out = np.full(len(ct), -1, np.int64)
    m = ct >= 0
    out[m] = first[ct[m]]
    return out


def _time(tr: Tracker, batch: Batch, reps: int) -> float:
    tr.launch(batch)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        tr.launch(batch)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def tune(batch: Batch, base=None, space=None, reps=3, verify=True, log=None):
    """Time every grid shape of `space` on `batch`; return (best params dict, table)."""
    base = dict(DEFAULT_PARAMS if base is None else base)
    space = dict(SPACE if space is None else space)
    names = sorted(space)
    table = []
    ref_key = None
    best = None
    for combo in itertools.product(*[space[k] for k in names]):
        cand = dict(base, **dict(zip(names, combo)))
        tr = Tracker(batch.n, batch.n_units, batch.n_rows, cand, device=batch.y.device)
        ms = _time(tr, batch, reps)
        res = tr.result()
        if verify:
            key = _partition_key(tr, res)
            if ref_key is None:
                ref_key = key
            elif not np.array_equal(key, ref_key):
                raise AssertionError("grid shape %s changed the tracks" % (dict(zip(names, combo)),))
        row = dict(zip(names, combo), ms=ms)
        table.append(row)
        if log:
            log("autotune %s: %.3f ms" % (dict(zip(names, combo)), ms))
        if best is None or ms < best[1]:
            best = (cand, ms)
        del tr
    return best[0], table


def load_cache(path=None):
    path = path or os.environ.get("TPC_AUTOTUNE_CACHE", CACHE_PATH)
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except ValueError:
            return {}
    return {}


def tuned_params(batch: Batch, base=None, path=None, tune_if_missing=False, force=False, log=None):
    """Cached grid shape for this batch class, merged into `base`; tuned (and
    cached) when missing and tune_if_missing, or always when force.  The
    cache file is TPC_AUTOTUNE_CACHE if set, else the one next to this file."""
    path = path or os.environ.get("TPC_AUTOTUNE_CACHE", CACHE_PATH)
    base = dict(DEFAULT_PARAMS if base is None else base)
    cache = load_cache(path)
    key = cache_key(batch)
    if key in cache and not force:
        return dict(base, **{k: cache[key][k] for k in SPACE})
    if not (tune_if_missing or force):
        return base
    best, table = tune(batch, base, log=log)
    store(batch, best, table, path)
    return best


def store(batch: Batch, best, table, path=None):
    """Record a tuning result for this batch class in the cache file."""
    path = path or os.environ.get("TPC_AUTOTUNE_CACHE", CACHE_PATH)
    cache = load_cache(path)
    cache[cache_key(batch)] = dict({k: best[k] for k in SPACE}, ms=min(r["ms"] for r in table),
                                   tuned_at=time.time())
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
