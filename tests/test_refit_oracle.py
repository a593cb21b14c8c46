"""Pins of the oracle's track refit (CPU).

The refit fits every selected track again over the hits it kept, with the
two-pass filter of the tracker (whose own pins tie it to the truth of noise-
free helices, to batch least squares and to standard-normal pulls).  What the
refit adds is the plumbing around that filter: gathering a track's clusters
through its hit list, measuring them in quanta of 1/256 cm at the x of their
row, and reporting the state at both ends.  The pins here check each of those
against facts that do not come from the oracle:
  * noise-free helices: the inner state equals the helix at the first hit and
    the outer state the helix at the last hit, to within the small error that
    quantization (at most half a quantum per coordinate) can cause;
  * quantization: moving every cluster by less than half a quantum inside its
    quantum leaves the result unchanged to the last bit, and a cluster exactly
    half-way between two quanta counts as the even one;
  * the refit of a track whose hits the selector left alone agrees with the
    tracker's own fit of it (the two differ only in the pass-1 seed);
  * degenerate tracks (fewer than 3 hits, a helix that leaves |sin(phi)| <
    sinphi_max) are reported as not refitted with zero outputs.
"""
import numpy as np

import oracle
import synth
from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
from test_oracle_pins import K_CURV, _local_states, _some_tracks

DIAG = [0, 2, 5, 9, 14]


def _clusters_of(tracks, rng=None):
    """Clusters of several tracks' noise-free states [(x, p)], in shuffled id
    order, and the tracks' hit lists (increasing row) over those ids."""
    ys, zs, rows, owner = [], [], [], []
    for t, (st, r) in enumerate(tracks):
        ys += [p[0] for _, p in st]
        zs += [p[1] for _, p in st]
        rows += list(r)
        owner += [t] * len(st)
    n = len(ys)
    ids = np.arange(n) if rng is None else rng.permutation(n)  # position j gets cluster id ids[j]
    y = np.zeros(n, np.float32)
    z = np.zeros(n, np.float32)
    row = np.zeros(n, np.uint16)
    y[ids], z[ids], row[ids] = ys, zs, rows
    first, nh, hits = [], [], []
    j = 0
    for st, _ in tracks:
        first.append(len(hits))
        nh.append(len(st))
        hits += list(ids[j:j + len(st)])
        j += len(st)
    return y, z, row, np.array(first), np.array(nh), np.array(hits)


def _noise_free(seed=13, min_len=20):
    tr, xs = _some_tracks(seed=seed)
    out = []
    for t in range(len(tr)):
        st, rows = _local_states(tr, xs, t, 0)
        if len(st) >= min_len:
            out.append((st, rows))
    return out


def test_refit_of_noise_free_helices_gives_the_helix_at_both_ends():
    """Quantization moves a coordinate by at most 1/512 cm (uniform, rms
    1/(256 sqrt 12)); with sigma_y, sigma_z of the fit at the cm-tenths scale
    the fitted states then sit within a few hundredths of their own standard
    deviation of the helix, far inside the 0.1 sigma allowed here, while any
    wrong x, wrong hit or wrong end moves them by many sigma."""
    trk = _noise_free()
    assert len(trk) > 10
    rng = np.random.default_rng(5)
    y, z, row, first, nh, hits = _clusters_of(trk, rng)
    r = oracle.refit_tracks(first, nh, hits, y, z, row, synth.ROW_X, K_CURV, P)
    assert r["ok"].all()
    for t, (st, _) in enumerate(trk):
        sig_in = np.sqrt(r["cov"][t][DIAG])
        sig_out = np.sqrt(r["cov_out"][t][DIAG])
        # the helix at the clusters' FP32 positions: the truth the quanta approximate
        assert r["x_ref"][t] == st[0][0] and r["x_out"][t] == st[-1][0]
        assert np.all(np.abs(r["p"][t] - st[0][1]) <= 0.1 * sig_in), (t, r["p"][t], st[0][1], sig_in)
        assert np.all(np.abs(r["p_out"][t] - st[-1][1]) <= 0.1 * sig_out), (t, r["p_out"][t], st[-1][1])
        # chi2: sum of squared quantization residuals over sigma^2, far below 1 per hit
        assert r["chi2"][t] < 0.01 * len(st)


def test_refit_takes_clusters_in_quanta():
    """Every cluster moved inside its own quantum (by less than half a
    quantum from its centre) gives the same refit to the last bit; a cluster
    exactly half-way between two quanta counts as the even quantum."""
    trk = _noise_free(seed=17)
    y, z, row, first, nh, hits = _clusters_of(trk)
    Y, Z = np.rint(y.astype(np.float64) * 256), np.rint(z.astype(np.float64) * 256)
    base = oracle.refit_tracks(first, nh, hits, (Y / 256).astype(np.float32), (Z / 256).astype(np.float32), row,
                               synth.ROW_X, K_CURV, P)
    rng = np.random.default_rng(3)
    jy = ((Y + rng.uniform(-0.45, 0.45, len(Y))) / 256).astype(np.float32)
    jz = ((Z + rng.uniform(-0.45, 0.45, len(Z))) / 256).astype(np.float32)
    assert np.array_equal(np.rint(jy.astype(np.float64) * 256), Y)  # still inside the quantum
    moved = oracle.refit_tracks(first, nh, hits, jy, jz, row, synth.ROW_X, K_CURV, P)
    for key in ("p", "cov", "chi2", "p_out", "cov_out", "ok"):
        assert np.array_equal(base[key], moved[key]), key
    # half-way clusters: (m + 1/2) / 256 is a float32 value for these |m|;
    # it must count as whichever of m, m + 1 is even
    m = np.floor(y.astype(np.float64) * 256)
    half_y = ((m + 0.5) / 256).astype(np.float32)
    assert np.array_equal(half_y.astype(np.float64) * 256, m + 0.5)
    even = np.where(m % 2 == 0, m, m + 1)
    a = oracle.refit_tracks(first, nh, hits, half_y, z, row, synth.ROW_X, K_CURV, P)
    b = oracle.refit_tracks(first, nh, hits, (even / 256).astype(np.float32), z, row, synth.ROW_X, K_CURV, P)
    odd = np.where(m % 2 == 0, m + 1, m)
    c = oracle.refit_tracks(first, nh, hits, (odd / 256).astype(np.float32), z, row, synth.ROW_X, K_CURV, P)
    assert np.array_equal(a["p"], b["p"]) and np.array_equal(a["chi2"], b["chi2"])
    assert not np.array_equal(a["p"], c["p"])


def test_refit_agrees_with_the_trackers_fit_where_no_hit_was_removed():
    """Lone smeared primaries: the tracker's output tracks that kept every hit
    of their tracklet's fit are refitted over the same hits; the two fits
    differ only in the pass-1 seed (the tracker seeds from its chain), which
    reaches the result through the finite pass-2 prior: within 0.1 sigma,
    diagonal covariance within 1e-2, chi2 within 1e-3."""
    rng = np.random.default_rng(31)
    tr = synth.primaries_pp_sector(rng, 60, 0, pt_range=(1.0, 10.0))
    xs = synth.helix_crossings(tr, 0.5)
    ys, zs, rows = [], [], []
    for t in range(len(tr)):
        st, r = _local_states(tr, xs, t, 0)
        if len(st) < 40:
            continue
        ys += [p[0] for _, p in st]
        zs += [p[1] for _, p in st]
        rows += list(r)
    y = (np.array(ys) + rng.normal(0, synth.SIGMA_Y, len(ys))).astype(np.float32)
    z = (np.array(zs) + rng.normal(0, synth.SIGMA_Z, len(zs))).astype(np.float32)
    row = np.array(rows, np.uint16)
    res = oracle.run(y, z, row, [0, len(y)], synth.ROW_X_F32, 0.5, P)
    T = int(res["n_tracks"])
    assert T > 20
    r = oracle.refit_tracks(res["track_first_hit"], res["track_n_hits"], res["track_hits"], y, z, row,
                            synth.ROW_X_F32, K_CURV, P)
    tl = res["track_tracklet"]
    full = np.nonzero(res["trk_nfit"][tl] == res["track_n_hits"])[0]
    assert len(full) > 20
    for t in full:
        sig = np.sqrt(r["cov"][t][DIAG])
        assert r["ok"][t]
        assert np.all(np.abs(res["trk_params"][tl[t]] - r["p"][t]) <= 0.1 * sig)
        assert np.all(np.abs(res["trk_cov"][tl[t]][DIAG] / r["cov"][t][DIAG] - 1) <= 1e-2)
        assert abs(res["trk_chi2"][tl[t]] / r["chi2"][t] - 1) <= 1e-3
        assert r["x_ref"][t] == res["trk_xref"][tl[t]]


def test_refit_degenerate_tracks():
    """Fewer than 3 hits, and a helix the seed puts beyond the sin(phi) limit,
    are not refitted; their outputs are zero and other tracks are unaffected."""
    trk = _noise_free(seed=19)
    y, z, row, first, nh, hits = _clusters_of(trk)
    # track A: the first two hits of track 0; track B: three hits of a steep
    # circle (sin(phi) about 0.995 at its first point)
    x3 = synth.ROW_X[[0, 1, 2]]
    yB = np.array([0.0, 10.0 * (x3[1] - x3[0]), 10.0 * (x3[2] - x3[0])], np.float32)  # dy/dx = 10
    y2 = np.concatenate([y, yB])
    z2 = np.concatenate([z, np.zeros(3, np.float32)])
    row2 = np.concatenate([row, np.array([0, 1, 2], np.uint16)])
    idB = np.arange(len(y), len(y) + 3)
    first2 = np.concatenate([first, [len(hits), len(hits) + 2]])
    nh2 = np.concatenate([nh, [2, 3]])
    hits2 = np.concatenate([hits, hits[first[0]:first[0] + 2], idB])
    a = oracle.refit_tracks(first, nh, hits, y, z, row, synth.ROW_X, K_CURV, P)
    b = oracle.refit_tracks(first2, nh2, hits2, y2, z2, row2, synth.ROW_X, K_CURV, P)
    assert list(b["ok"][-2:]) == [0, 0]
    for key in ("p", "cov", "x_ref", "chi2", "p_out", "cov_out", "x_out"):
        assert not np.any(b[key][-2:]), key
        assert np.array_equal(a[key], b[key][:-2]), key
