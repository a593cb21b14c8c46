"""Element-by-element comparison of the HIP path with the CPU oracle.

Bars (the FP32 GPU fit against the FP64 oracle fit):
  * hit grid (permutation, cell table, per-row grid shape), neighbour links,
    cleaned links, start hits / tracklet list, chain lengths: bit-exact;
  * tracklet hit sets: identical for >= 99.9% of the tracklets; a tracklet may
    differ only if the oracle flagged one of its decisions as fragile (a
    rounded prediction within `fragile_eps` quanta of a rounding boundary
    whose other rounding changes the pick, or sin(phi) within 1e-5 of the
    limit);
  * fitted parameters of identical hit sets: |dp_k| <= 1e-4 max(|p_k|, f_k)
    with floors f = (1 cm, 1 cm, 1e-2, 1e-2, 0.1 /GeV) for at least 99.9% of
    the fitted tracklets (the stated 1e-4 relative tolerance, read as a bar
    on the bulk); every tracklet within max(that, 0.21 sigma_k) and at most
    0.003% beyond max(that, 0.1 sigma_k) (sigma from the oracle's
    covariance); chi2 within 1e-3 relative (floor 1) for 99.98% and within
    2e-2 for all; covariance diagonal within 4.7e-2 for all, within 1e-2 for
    99.998% and, on samples of at least 1e4 fitted tracklets, within 1e-3 for
    99.6%.
    The clauses beyond the 1e-4 one bound the few ill-conditioned fits (short,
    low-pT, steep tracklets; chi2 per degree of freedom far above 1) where
    FP32 cannot follow FP64 closer.  Each is no looser than the tail that
    FP32 rounding alone produces: tests/test_fp32_bars.py builds two copies of
    the oracle whose fit runs operation by operation in FP32 (full 5x5
    covariance products, and the symmetric lower triangle the kernel keeps),
    runs them on all 36 sectors of the 50-collision time frame, and checks
    every clause against the worse of the two tails (maxima to within 5%,
    fractions of outliers to within 10-50%, since the two builds' tails differ
    by up to 9x between rounding orders);
  * owner keys, keep flags and the cluster-to-track map: bit-exact for every
    cluster and tracklet not touched by a differing tracklet.
"""
from __future__ import annotations

import numpy as np

PARAM_FLOORS = np.array([1.0, 1.0, 1e-2, 1e-2, 0.1])
PARAM_RTOL = 1e-4
PARAM_SIGMA = 0.1
PARAM_SIGMA_ALL = 0.21
MIN_SIGMA_FRACTION = 0.99997
COV_RTOL = 1e-3
COV_RTOL_MID = 1e-2
COV_RTOL_ALL = 4.7e-2
MIN_COV_FRACTION = 0.996
MIN_COV_MID_FRACTION = 0.99998
COV_FRACTION_MIN_SAMPLE = 10000
CHI2_RTOL = 1e-3
CHI2_RTOL_ALL = 2e-2
MIN_CHI2_FRACTION = 0.9998
MIN_MATCHED_FRACTION = 0.999
MIN_WITHIN_FRACTION = 0.999

# Bars of the track refit (tests/test_gpu_refit.py), where they differ from
# the tracklet bars above.  The refit is the same FP32 filter over each
# track's final hit list; its covariance tail is wider on the few low-pT
# tracks whose q/pT variance shrinks by four to five orders of magnitude from
# its prior cov0, so that the covariance update cancels that many bits.  The
# clause on every track therefore scales with that ratio: a diagonal entry
# c_ii may differ by max(COV_RTOL_ALL, REFIT_COV_COND_K 2^-24 cov0_i / c_ii)
# relative (the bits an update loses to cancellation grow with the log of
# cov0_i / c_ii); the bulk clauses keep their form with refit fractions.
# tests/test_fp32_bars.py derives all three from FP32 builds of the oracle's
# refit (four rounding orders: full and symmetric covariance, each with and
# without FMA contraction) on the tracks of the 50-collision frame.
REFIT_MIN_COV_FRACTION = 0.992
REFIT_MIN_COV_MID_FRACTION = 0.999955
REFIT_COV_COND_K = 96.0
FP32_EPS = 2.0 ** -24
# The fit of merged chains (tests/test_gpu_merge.py): the refit's clauses with
# wider bulk fractions.  A chain holds about twice a segment's hits, so its
# q/pT variance falls further below its prior and its updates cancel more
# bits; tests/test_fp32_bars.py derives the two fractions from the same four
# FP32 builds, running the oracle's chain fit on the 50-collision frame.
CHAIN_MIN_COV_FRACTION = 0.9812
CHAIN_MIN_COV_MID_FRACTION = 0.9999

SEG_FIELDS = ["seg_start", "seg_count", "seg_zmin", "seg_zmax", None, "seg_by", "seg_ny", "seg_bz",
              "seg_nz", "seg_cell_base"]


def gpu_state(tracker, result):
    """Pull intermediates of the last launch to host numpy arrays."""
    import torch
    import paper_2106_03636_amd as T
    n_rows = tracker.n_rows
    K = result["n_tracklets"]
    g = {}
    g["perm"] = tracker.inspect(T.TPC_VIEW_PERM).cpu().numpy()
    g["cell"] = tracker.inspect(T.TPC_VIEW_CELL).cpu().numpy()[:result["n_cells"] + 1]
    g["seg"] = tracker.inspect(T.TPC_VIEW_SEG).cpu().numpy().reshape(-1, 12)
    for name, what in (("up", T.TPC_VIEW_UP), ("dn", T.TPC_VIEW_DN), ("upc", T.TPC_VIEW_UPC),
                       ("dnc", T.TPC_VIEW_DNC)):
        g[name] = tracker.inspect(what).cpu().numpy()
    g["owner"] = tracker.inspect(T.TPC_VIEW_OWNER).cpu().numpy().view(np.uint32)
    for name, what in (("trk_start", T.TPC_VIEW_TRK_START), ("trk_unit", T.TPC_VIEW_TRK_UNIT),
                       ("trk_len", T.TPC_VIEW_TRK_LEN)):
        g[name] = tracker.inspect(what).cpu().numpy()[:K]
    # the fit's fields are stored per seed; spread them over the tracklets
    for name, what in (("trk_nfit", T.TPC_VIEW_TRK_NFIT), ("trk_rlo", T.TPC_VIEW_TRK_RLO),
                       ("trk_rhi", T.TPC_VIEW_TRK_RHI), ("trk_owned", T.TPC_VIEW_TRK_OWNED),
                       ("trk_keep", T.TPC_VIEW_TRK_KEEP), ("trk_p1n", T.TPC_VIEW_TRK_P1N)):
        g[name] = tracker.tracklet_field(what)
    g["trk_key"] = tracker.tracklet_field(T.TPC_VIEW_TRK_KEY).view(np.uint32)
    g["trk_params"] = tracker.tracklet_field(T.TPC_VIEW_TRK_PARAMS, torch.float32, 5)
    g["trk_cov"] = tracker.tracklet_field(T.TPC_VIEW_TRK_COV, torch.float32, 15)
    g["trk_xref"] = tracker.tracklet_field(T.TPC_VIEW_TRK_XREF, torch.float32)
    g["trk_chi2"] = tracker.tracklet_field(T.TPC_VIEW_TRK_CHI2, torch.float32)
    # seeds: tracklets with a chain of >= l_min hits, in tracklet order
    seeds = np.nonzero(g["trk_len"] >= int(tracker.params.l_min))[0]
    g["n_seeds"] = result["n_seeds"]
    g["seed_list"] = tracker.inspect(T.TPC_VIEW_SEED_LIST).cpu().numpy()[:result["n_seeds"]]
    g["seeds_expected"] = seeds
    raw = tracker.inspect(T.TPC_VIEW_TRK_HITS).cpu().numpy().reshape(-1, n_rows, 64)
    per_seed = raw.transpose(0, 2, 1).reshape(-1, n_rows)[:len(seeds)]  # [seed][row]
    g["seed_hits"] = np.where(per_seed >= 0, per_seed & ((1 << 30) - 1), per_seed)  # drop the owned mark
    for k in ("n_tracks", "n_track_hits", "n_tracklets", "n_cells"):
        g[k] = result[k]
    for k in ("cluster_track", "params", "cov", "x_ref", "chi2", "unit", "n_hits", "n_fit",
              "first_hit", "hits"):
        g["out_" + k] = result[k].cpu().numpy()
    return g


def gpu_hit_pairs(g):
    """(tracklet, hit position) pairs of every fitted tracklet, sorted by
    tracklet then position, from the by-row hit table of the seeds (rows
    rlo..rhi of each seed are valid)."""
    seeds = g["seeds_expected"]
    H = g["seed_hits"]
    if len(seeds) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    lo, hi, nfit = g["trk_rlo"][seeds], g["trk_rhi"][seeds], g["trk_nfit"][seeds]
    rows = np.arange(H.shape[1])[None, :]
    m = (rows >= lo[:, None]) & (rows <= hi[:, None]) & (H >= 0) & (nfit[:, None] > 0) & (lo[:, None] >= 0)
    j, _ = np.nonzero(m)
    return _sorted_pairs(seeds[j].astype(np.int64), H[m].astype(np.int64))


def oracle_hit_pairs(o):
    """The same pairs from the oracle's per-tracklet hit lists."""
    H = o["trk_hits"]
    nfit = o["trk_nfit"]
    m = np.arange(H.shape[1])[None, :] < nfit[:, None]
    t, _ = np.nonzero(m)
    return _sorted_pairs(t.astype(np.int64), H[m].astype(np.int64))


def _sorted_pairs(t, h):
    key = (t << 32) | h
    key.sort()
    return key >> 32, key & 0xFFFFFFFF


def hit_set_diff(gp, op, K):
    """Tracklets whose hit sets differ, from sorted (tracklet, hit) pairs."""
    cg, co = np.bincount(gp[0], minlength=K), np.bincount(op[0], minlength=K)
    same_n = cg == co
    sg, so = same_n[gp[0]], same_n[op[0]]
    # tracklets with equal counts line up element by element in both sorted lists
    neq = gp[1][sg] != op[1][so]
    bad = np.zeros(K, bool)
    bad[~same_n] = True
    bad[gp[0][sg][neq]] = True
    return bad


class ParityReport(dict):
    def fail(self, msg):
        self.setdefault("failures", []).append(msg)

    @property
    def ok(self):
        return not self.get("failures")


def compare_fit(rep, g_par, g_cov, g_chi2, g_xref, o_par, o_cov, o_chi2, o_xref, rtol_scale=1.0, refit_cov0=None,
                chain=False):
    """The fit clauses of the bars, over tracklets with identical hit sets:
    params [n,5], covariance lower triangles [n,15], chi2 and x_ref [n].
    refit_cov0: the prior covariance diagonal; given, the covariance clauses
    are the refit's (REFIT_*), with the chain fit's bulk fractions (CHAIN_*)
    when chain is set."""
    gp, op = np.asarray(g_par, np.float64), np.asarray(o_par, np.float64)
    diag = [0, 2, 5, 9, 14]
    sig = np.sqrt(np.abs(np.asarray(o_cov)[:, diag]))
    scale = np.maximum(np.abs(op), PARAM_FLOORS)
    dp = np.abs(gp - op)
    rel = dp / scale
    rep["param_max_rel"] = rel.max(axis=0).tolist()
    rep["param_max_dp_over_sigma"] = (dp / np.maximum(sig, 1e-30)).max(axis=0).tolist()
    within = np.all(rel <= PARAM_RTOL * rtol_scale, axis=1)
    rep["param_within_fraction"] = float(within.mean())
    if within.mean() < MIN_WITHIN_FRACTION:
        rep.fail("only %.5f of fitted tracklets within 1e-4" % within.mean())
    tol = PARAM_RTOL * rtol_scale * scale
    mid = np.all(dp <= np.maximum(tol, PARAM_SIGMA * sig), axis=1)
    rep["param_within_0.1_sigma"] = float(mid.mean())
    if mid.mean() < MIN_SIGMA_FRACTION:
        rep.fail("%d tracklets beyond max(1e-4 relative, 0.1 sigma)" % int((~mid).sum()))
    loose = np.all(dp <= np.maximum(tol, PARAM_SIGMA_ALL * sig), axis=1)
    if not loose.all():
        rep.fail("%d tracklets beyond max(1e-4 relative, %g sigma)" % (int((~loose).sum()), PARAM_SIGMA_ALL))
    gc, oc = np.asarray(g_cov, np.float64)[:, diag], np.asarray(o_cov, np.float64)[:, diag]
    crel_el = np.abs(gc - oc) / np.maximum(np.abs(oc), 1e-12)
    crel = crel_el.max(axis=1)
    min_frac, min_mid = MIN_COV_FRACTION, MIN_COV_MID_FRACTION
    bound = np.full_like(crel_el, COV_RTOL_ALL * rtol_scale)
    if refit_cov0 is not None:
        min_frac, min_mid = REFIT_MIN_COV_FRACTION, REFIT_MIN_COV_MID_FRACTION
        if chain:
            min_frac, min_mid = CHAIN_MIN_COV_FRACTION, CHAIN_MIN_COV_MID_FRACTION
        cond = FP32_EPS * np.asarray(refit_cov0, np.float64)[None, :] / np.maximum(np.abs(oc), 1e-30)
        bound = np.maximum(bound, REFIT_COV_COND_K * cond)
    rep["cov_max_rel"] = float(crel.max(initial=0.0))
    rep["cov_max_over_bound"] = float((crel_el / bound).max(initial=0.0))
    rep["cov_within_1e-3"] = float((crel <= COV_RTOL * rtol_scale).mean())
    rep["cov_within_1e-2"] = float((crel <= COV_RTOL_MID * rtol_scale).mean())
    if len(crel) >= COV_FRACTION_MIN_SAMPLE and rep["cov_within_1e-3"] < min_frac:
        rep.fail("only %.5f of covariances within 1e-3" % rep["cov_within_1e-3"])
    if rep["cov_within_1e-2"] < min_mid:
        rep.fail("only %.5f of covariances within 1e-2" % rep["cov_within_1e-2"])
    if (crel_el > bound).any():
        rep.fail("covariance beyond its bound: max %.3g, %.3g of the bound" % (crel.max(), rep["cov_max_over_bound"]))
    gx, ox = np.asarray(g_chi2, np.float64), np.asarray(o_chi2, np.float64)
    xrel = np.abs(gx - ox) / np.maximum(np.abs(ox), 1.0)
    rep["chi2_max_rel"] = float(xrel.max())
    rep["chi2_within_1e-3"] = float((xrel <= CHI2_RTOL * rtol_scale).mean())
    if rep["chi2_within_1e-3"] < MIN_CHI2_FRACTION or xrel.max() > CHI2_RTOL_ALL * rtol_scale:
        rep.fail("chi2: %.5f within 1e-3, max %.3g" % (rep["chi2_within_1e-3"], xrel.max()))
    if not np.allclose(g_xref, o_xref, rtol=0, atol=1e-4):
        rep.fail("x_ref differs")


def compare(g, o, check_outputs=True, rtol_scale=1.0):
    """Compare GPU state g (gpu_state) with oracle result o.  Returns a report;
    report.ok is the verdict, report['failures'] lists what broke."""
    rep = ParityReport()
    # --- grid
    for k in ("perm", "up", "dn", "upc", "dnc"):
        if not np.array_equal(g[k], o[k]):
            bad = int(np.sum(g[k] != o[k])) if g[k].shape == o[k].shape else -1
            rep.fail("%s differs at %d positions" % (k, bad))
    if g["n_cells"] != o["n_cells"] or not np.array_equal(g["cell"], o["cell_start"]):
        rep.fail("cell table differs")
    for j, f in enumerate(SEG_FIELDS):
        if f is not None and not np.array_equal(g["seg"][:, j], o[f]):
            rep.fail("segment field %s differs" % f)
    # --- tracklets
    K = g["n_tracklets"]
    rep["n_tracklets"] = K
    if K != o["n_tracklets"]:
        rep.fail("tracklet count %d vs %d" % (K, o["n_tracklets"]))
        return rep
    for k in ("trk_start", "trk_unit", "trk_len"):
        if not np.array_equal(g[k], o[k]):
            rep.fail("%s differs" % k)
    if "seed_list" in g and not np.array_equal(g["seed_list"], g["seeds_expected"]):
        rep.fail("seed list is not the tracklets with a chain of >= l_min hits")
    gp, op = gpu_hit_pairs(g), oracle_hit_pairs(o)
    same = ~hit_set_diff(gp, op, K)
    same &= g["trk_nfit"] == o["trk_nfit"]
    if "trk_p1n" in g:  # the first pass took the same number of hits
        fitted = o["trk_nfit"] > 0
        same &= ~fitted | (g["trk_p1n"] == o["trk_p1n"])
    diff = np.nonzero(~same)[0]
    rep["n_hitset_diff"] = int(len(diff))
    rep["n_fragile"] = int(o["trk_fragile"].sum())
    seeded = int((o["trk_nfit"] > 0).sum())
    rep["n_fitted"] = seeded
    rep["matched_fraction"] = 1.0 - len(diff) / max(1, seeded)
    if rep["matched_fraction"] < MIN_MATCHED_FRACTION:
        rep.fail("only %.5f of tracklet hit sets match" % rep["matched_fraction"])
    unflagged = [int(t) for t in diff if not o["trk_fragile"][t]]
    if unflagged:
        rep.fail("%d differing tracklets not flagged fragile (e.g. %s)" % (len(unflagged), unflagged[:5]))
    # --- fitted parameters of identical hit sets
    m = same & (o["trk_nfit"] > 0)
    if m.any():
        compare_fit(rep, g["trk_params"][m], g["trk_cov"][m], g["trk_chi2"][m], g["trk_xref"][m],
                    o["trk_params"][m], o["trk_cov"][m], o["trk_chi2"][m], o["trk_xref"][m], rtol_scale)
    # --- ownership and selection away from differing tracklets
    n_pos = len(g["perm"])
    is_diff = ~same
    touched = np.zeros(n_pos, bool)
    touched[gp[1][is_diff[gp[0]]]] = True
    touched[op[1][is_diff[op[0]]]] = True
    # tracklets sharing a touched hit may change their owned count
    affected = is_diff.copy()
    affected[gp[0][touched[gp[1]]]] = True
    affected[op[0][touched[op[1]]]] = True
    rep["n_affected"] = int(affected.sum())
    ok_t = ~affected
    if not np.array_equal(g["trk_key"][ok_t], o["trk_key"][ok_t]):
        rep.fail("tracklet keys differ")
    own_ok = ~touched
    if not np.array_equal(g["owner"][own_ok], o["owner"][own_ok]):
        rep.fail("owner keys differ on untouched hits")
    if not np.array_equal(g["trk_keep"][ok_t], o["trk_keep"][ok_t]) or \
            not np.array_equal(g["trk_owned"][ok_t], o["trk_owned"][ok_t]):
        rep.fail("selection differs on unaffected tracklets")
    g_kept = np.nonzero(g["trk_keep"])[0]
    if check_outputs and (len(g_kept) != g["n_tracks"] or
                          (len(g["out_cluster_track"]) and g["out_cluster_track"].max() >= g["n_tracks"])):
        rep.fail("kept tracklets (%d) and track outputs (%d tracks) disagree" % (len(g_kept), g["n_tracks"]))
        check_outputs = False
    if check_outputs:
        # cluster -> tracklet (through the track list) must agree away from affected tracklets
        o_kept = o["track_tracklet"]
        def _through(ct, kept):
            r = np.full(len(ct), -1, np.int64)
            m = ct >= 0
            r[m] = kept[ct[m]]
            return r
        gct = _through(g["out_cluster_track"], g_kept)
        oct_ = _through(o["cluster_track"], o_kept)
        perm = g["perm"]
        aff_pos = np.zeros(len(perm), bool)
        aff_pos[gp[1][affected[gp[0]]]] = True
        aff_pos[op[1][affected[op[0]]]] = True
        aff_cluster = np.zeros(len(perm), bool)
        aff_cluster[perm[aff_pos]] = True
        bad = (gct != oct_) & ~aff_cluster
        rep["cluster_track_mismatch"] = int(bad.sum())
        if bad.any():
            rep.fail("cluster_track differs on %d unaffected clusters" % int(bad.sum()))
        if not affected.any():
            if not np.array_equal(g["out_cluster_track"], o["cluster_track"]):
                rep.fail("cluster_track not bit-exact")
            if g["n_tracks"] != o["n_tracks"] or not np.array_equal(g["out_hits"], o["track_hits"]):
                rep.fail("track hit lists differ")
            if not np.array_equal(g["out_n_hits"], o["track_n_hits"]) or \
                    not np.array_equal(g["out_first_hit"], o["track_first_hit"]):
                rep.fail("track hit counts / offsets differ")
        # output params are the kept tracklets' params
        if len(g_kept) == g["n_tracks"] and g["n_tracks"]:
            if not np.array_equal(g["out_params"], g["trk_params"][g_kept]):
                rep.fail("output params are not the kept tracklets' params")
    return rep
