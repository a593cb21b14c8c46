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


def majority_particle(label, track_n_hits, track_hits):
    """Per track, the particle that generated most of its clusters (ties: the
    lower index; -1 when only noise)."""
    label = np.asarray(label, np.int64)
    nh = np.asarray(track_n_hits, np.int64)
    nt = len(nh)
    out = np.full(nt, -1, np.int64)
    if nt == 0:
        return out
    tid = np.repeat(np.arange(nt, dtype=np.int64), nh)
    lab = label[np.asarray(track_hits, np.int64)[:int(nh.sum())]]
    span = int(lab.max()) + 2
    u, cnt = np.unique(tid * span + (lab + 1), return_counts=True)
    ut, ul = u // span, u % span - 1
    order = np.lexsort((-cnt, ut))
    first = np.ones(len(order), bool)
    first[1:] = ut[order][1:] != ut[order][:-1]
    out[ut[order][first]] = ul[order][first]
    return out


def collision_report(label, particle_t0, particle_vz, track_n_hits, track_hits, track_side, track_forming,
                     collision, c_side, c_t0, v_drift, min_tracks=100):
    """Collision assignment against MC truth.  A track's true collision is the
    t0 of its majority particle.  A candidate's collision is the majority over
    its tracks; forming tracks (the ones that define candidates) are
    *assigned* when they join a candidate and *pure* when that candidate's
    collision is theirs.  A (collision, side) with at least min_tracks forming
    tracks, and no other collision within 3 cm of its z' on that side, is
    *found* when some candidate on that side has it as its collision."""
    truth = majority_particle(label, track_n_hits, track_hits)
    ok = truth >= 0
    t0t = np.where(ok, np.asarray(particle_t0)[np.maximum(truth, 0)], np.nan)
    col = np.asarray(collision)
    form = np.asarray(track_forming, bool)
    side = np.asarray(track_side)
    nc = len(c_side)
    cmaj = np.full(nc, np.nan)
    sel = (col >= 0) & ok
    if sel.any():  # per candidate, the most frequent true t0 (ties: the earlier one)
        t0u, t0i = np.unique(t0t[sel], return_inverse=True)
        u, cnt = np.unique(col[sel].astype(np.int64) * len(t0u) + t0i, return_counts=True)
        uc = u // len(t0u)
        order = np.lexsort((-cnt, uc))
        first = np.ones(len(order), bool)
        first[1:] = uc[order][1:] != uc[order][:-1]
        cmaj[uc[order][first]] = t0u[u[order][first] % len(t0u)]
    assigned = (col >= 0) & ok & form
    pure = assigned & (cmaj[np.maximum(col, 0)] == t0t)
    resid = np.abs(np.asarray(c_t0) - cmaj)[~np.isnan(cmaj)]
    pt0, pvz = np.asarray(particle_t0), np.asarray(particle_vz)
    found = findable = 0
    for s in (1, -1):
        zs = {}
        for t0 in np.unique(pt0):
            zs[t0] = np.median(pvz[pt0 == t0]) - s * v_drift * t0
        zall = np.array(list(zs.values()))
        have = set(cmaj[(np.asarray(c_side) == s) & ~np.isnan(cmaj)].tolist())
        for t0, z in zs.items():
            if ((t0t == t0) & (side == s) & form).sum() < min_tracks or (np.abs(zall - z) < 3.0).sum() > 1:
                continue
            findable += 1
            found += t0 in have
    return dict(candidates=int(nc), candidates_a=int((np.asarray(c_side) == 1).sum()),
                candidates_c=int((np.asarray(c_side) == -1).sum()),
                collisions_found=int(found), collisions_findable=int(findable),
                forming_assigned=float(assigned.sum() / max(1, (ok & form).sum())),
                forming_purity=float(pure.sum() / max(1, assigned.sum())),
                all_assigned=float(((col >= 0) & ok).sum() / max(1, ok.sum())),
                t0_resid_us_p50=float(np.percentile(resid, 50)) if len(resid) else None,
                t0_resid_us_p90=float(np.percentile(resid, 90)) if len(resid) else None,
                min_tracks=min_tracks)
