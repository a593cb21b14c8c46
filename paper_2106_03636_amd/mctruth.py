"""Physics performance against Monte-Carlo truth (synthetic events only).

A generated particle is *findable* in a unit when at least `min_hits` of its
clusters lie in that unit (a sector crossing counts per sector).  A track is
*matched* to the (unit, particle) that owns at least `purity` of its
clusters, else it is a *fake*; a second or later track matched to the same
(unit, particle) is a *clone*.  Efficiency = matched findable / findable,
reported overall and in bins of the particle's pT.  The paper names
efficiency at high occupancy as the concern of the synchronous tracking
(§2.3) but gives no figures; these are reported beside the throughput.
"""
from __future__ import annotations

import numpy as np

PT_EDGES = (0.1, 0.2, 0.3, 0.5, 1.0, 2.0, 5.0, 1e9)


def report(label, unit_offsets, pt, track_first_hit, track_n_hits, track_hits, min_hits=40, purity=0.9,
           pt_min=0.0):
    """label[n] particle index per cluster (-1 noise); pt[n_particles] GeV;
    track_* the track output (cluster ids of each track's hits)."""
    label = np.asarray(label, np.int64)
    n_units = len(unit_offsets) - 1
    unit_of = np.repeat(np.arange(n_units, dtype=np.int64), np.diff(np.asarray(unit_offsets)))
    shift = np.int64(1) << np.int64(32)
    # findable (unit, particle) pairs
    m = label >= 0
    keys, cnt = np.unique(unit_of[m] * shift + label[m], return_counts=True)
    findable = keys[(cnt >= min_hits) & (np.asarray(pt)[keys % shift] > pt_min)]
    # majority (unit, particle) of each track
    nt = len(track_first_hit)
    th = np.asarray(track_hits, np.int64)
    tid = np.repeat(np.arange(nt, dtype=np.int64), np.asarray(track_n_hits, np.int64))
    lab = label[th]
    good = lab >= 0
    tk = tid[good] * (np.int64(1) << np.int64(34)) + unit_of[th[good]] * (np.int64(1) << np.int64(24)) + lab[good]
    if np.any(lab[good] >= (1 << 24)) or n_units >= (1 << 10):
        raise ValueError("too many particles or units for the packed keys")
    uk, uc = np.unique(tk, return_counts=True)
    t_of = uk >> np.int64(34)
    order = np.lexsort((-uc, t_of))  # per track, largest count first
    first = np.ones(len(order), bool)
    first[1:] = t_of[order][1:] != t_of[order][:-1]
    best = order[first]
    best_t = t_of[best]
    best_key = ((uk[best] >> np.int64(24)) & np.int64((1 << 10) - 1)) * shift + (uk[best] & np.int64((1 << 24) - 1))
    nh = np.asarray(track_n_hits, np.int64)
    matched_t = np.zeros(nt, bool)
    match_key = np.full(nt, -1, np.int64)
    ok = uc[best] >= purity * nh[best_t]
    matched_t[best_t[ok]] = True
    match_key[best_t[ok]] = best_key[ok]
    mk = match_key[matched_t]
    uniq, mult = np.unique(mk, return_counts=True)
    clones = int((mult - 1).sum())
    found = np.isin(findable, uniq)
    out = dict(findable=int(len(findable)), tracks=int(nt), efficiency=float(found.mean()) if len(findable) else 0.0,
               fake_rate=float((~matched_t).sum()) / max(1, nt), clone_rate=clones / max(1, int(matched_t.sum())),
               min_hits=min_hits, purity=purity)
    fpt = np.asarray(pt)[findable % shift]
    bins = []
    for lo, hi in zip(PT_EDGES[:-1], PT_EDGES[1:]):
        sel = (fpt >= lo) & (fpt < hi)
        if sel.any():
            bins.append(dict(pt_lo=lo, pt_hi=None if hi > 1e8 else hi, findable=int(sel.sum()),
                             efficiency=float(found[sel].mean())))
    out["vs_pt"] = bins
    return out
