"""Pins of the oracle's segment merger (CPU).

The merger turns a segment's outer state into the frame of a neighbouring
sector, carries it to the next segment's first hit, and links segments whose
states agree (chi2 over the five parameters) and that are each other's best
match.  Pins, each against facts that do not come from the oracle:
  * the turn and the helix transport reproduce the generator's closed-form
    helix: the state of a helix at its last row in one sector, turned into
    the next sector and carried to its first row there, is the state the
    generator computes in that sector;
  * the turn's Jacobian matches finite differences of the turn followed by
    the transport back to the turned plane;
  * a hand-worked set of straight segments with unit covariances gives the
    chi2 values and links derived by hand: best matches both ways, ties to
    the smaller index, the row, z, y, side and angle rules;
  * MC truth on a central Pb-Pb collision: links join segments of one
    particle, and most particles that the tracker split are joined.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import cached_event, cached_oracle
from paper_2106_03636_amd.params import DEFAULT_PARAMS as P

K_CURV = -synth.KAPPA * 0.5
DALPHA = math.radians(20.0)


def _boundary_crossings(seed=21, n=400):
    """(state in sector A at its last row, x, state in B at its first row, x,
    alpha_B - alpha_A) for helices that leave sector A through its side and
    enter the neighbouring sector B on the same side."""
    rng = np.random.default_rng(seed)
    tr = synth.primaries_pp_sector(rng, n, 0, pt_range=(0.3, 2.0))
    xs = synth.helix_crossings(tr, 0.5)
    out = []
    for t in range(len(tr)):
        m = np.nonzero((xs["track"] == t) & (xs["cosphi"] > 0))[0]
        if len(m) < 2:
            continue
        m = m[np.argsort(xs["s"][m])]  # along the helix
        sec, row = xs["sector"][m], xs["row"][m]
        for j in range(len(m) - 1):
            a, b = m[j], m[j + 1]
            if sec[j] == sec[j + 1] or row[j + 1] <= row[j]:
                continue
            if (sec[j] < 18) != (sec[j + 1] < 18):
                continue
            d = math.remainder(synth.sector_alpha(int(sec[j + 1])) - synth.sector_alpha(int(sec[j])), 2 * math.pi)
            if abs(abs(d) - DALPHA) > 1e-9:
                continue
            qpt = tr.q[t] / tr.pt[t]
            pa = np.array([xs["y"][a], xs["z"][a], xs["sinphi"][a], tr.tgl[t], qpt])
            pb = np.array([xs["y"][b], xs["z"][b], xs["sinphi"][b], tr.tgl[t], qpt])
            out.append((pa, synth.ROW_X[row[j]], pb, synth.ROW_X[row[j + 1]], d))
            break
    return out


def test_turn_and_transport_reproduce_the_helix_in_the_next_sector():
    cases = _boundary_crossings()
    assert len(cases) > 30
    both_ways = set()
    for pa, xa, pb, xb, d in cases:
        r = oracle.rotate(pa, xa, d, K_CURV)
        assert r is not None
        q, x1 = r
        p = oracle.propagate(q, x1, xb, K_CURV)
        assert p is not None
        assert np.allclose(p, pb, rtol=0, atol=1e-8), (p, pb, d)
        both_ways.add(d > 0)
    assert both_ways == {True, False}  # tracks of both charges leave through both edges


@pytest.mark.parametrize("case", [([3.0, -20.0, 0.3, 0.7, -2.5], 120.0, 0.35),
                                  ([-15.0, 100.0, -0.2, -1.1, 4.0], 200.0, -0.35),
                                  ([20.0, 5.0, 0.6, 0.2, 0.8], 90.0, 0.1)])
def test_turn_jacobian_matches_finite_differences(case):
    p0, x, d = case
    p0 = np.array(p0)
    base, x1, J = oracle.rotate(p0, x, d, K_CURV, jacobian=True)

    def g(p):
        q, xq = oracle.rotate(p, x, d, K_CURV)
        return oracle.propagate(q, xq, x1, K_CURV)  # back to the nominal turned plane

    assert np.allclose(g(p0), base, atol=1e-12)
    h = 1e-6
    num = np.zeros((5, 5))
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        num[:, j] = (g(p0 + e) - g(p0 - e)) / (2 * h)
    assert np.allclose(num, J, rtol=1e-6, atol=1e-7), (num, J)


def _seg(y, z=0.0, s=0.0):
    return np.array([y, z, s, 0.0, 0.0])


def _hand(units, rows, p_in, p_out, x_in=None, x_out=None, alpha=(0.0, DALPHA, 2 * DALPHA, 0.0),
          side=(1, 1, 1, -1), **kw):
    """Segments with unit covariances on straight lines (k = 0); by default
    every segment's ends lie at x = 100, so the transport is the identity and
    chi2 = |p_b - p_a|^2 / 2."""
    T = len(units)
    eye = np.zeros(15)
    eye[[0, 2, 5, 9, 14]] = 1.0
    x_in = np.full(T, 100.0) if x_in is None else np.asarray(x_in, float)
    x_out = np.full(T, 100.0) if x_out is None else np.asarray(x_out, float)
    refit = dict(ok=np.ones(T, np.int8), p=np.array(p_in, float), cov=np.tile(eye, (T, 1)), x_ref=x_in,
                 p_out=np.array(p_out, float), cov_out=np.tile(eye, (T, 1)), x_out=x_out)
    return oracle.merge(units, [r[0] for r in rows], [r[1] for r in rows], refit, alpha, side, 152, 0.0, **kw)


def test_hand_worked_links():
    """One unit; A0 ends at row 10, A1 at row 12, B2 spans rows 20-60, B3
    rows 25-70 (so neither B continues the other, nor A1 A0).  Outer ends
    A0 (y, z) = (0, 0), A1 (0, 1); inner ends B2 (1, 1), B3 (sqrt 3.75,
    -0.5): chi2(A0,B2) = 1, chi2(A1,B2) = 0.5, chi2(A0,B3) = 2,
    chi2(A1,B3) = 3.  Best outward: A0 -> B2, A1 -> B2; best inward: B2 <- A1,
    B3 <- A0.  The one mutual pair is A1 -> B2."""
    units = [0, 0, 0, 0]
    rows = [(0, 10), (0, 12), (20, 60), (25, 70)]
    p_out = [_seg(0.0, 0.0), _seg(0.0, 1.0), _seg(0.0), _seg(0.0)]
    p_in = [_seg(0.0), _seg(0.0), _seg(1.0, 1.0), _seg(math.sqrt(3.75), -0.5)]
    m = _hand(units, rows, p_in, p_out)
    assert m["n_candidates"] == 4
    assert m["next"].tolist() == [-1, 2, -1, -1] and m["prev"].tolist() == [-1, -1, 1, -1]
    assert abs(m["link_chi2"][1] - 0.5) < 1e-12
    # a tie: A0 and A1 both at chi2 0.5 to B2; B2 takes the smaller index, A0
    m = _hand(units, rows, p_in, [_seg(0.0, 1.0), _seg(0.0, 1.0), _seg(0.0), _seg(0.0)])
    assert m["prev"][2] == 0 and m["next"][0] == 2 and m["next"][1] == -1
    # the cut: only chi2(A1,B2) = 0.5 stays below 0.75
    m = _hand(units, rows, p_in, p_out, chi2_max=0.75)
    assert m["n_candidates"] == 1 and m["next"][1] == 2


def test_hand_worked_rules():
    """Row, gap, z, y, side and angle rules, on segments whose states agree."""
    p = [_seg(0.0)] * 2
    # B must start after A ends, at most max_gap (32) rows after
    assert _hand([0, 0], [(0, 10), (10, 40)], p, p)["next"][0] == -1
    assert _hand([0, 0], [(0, 10), (11, 40)], p, p)["next"][0] == 1
    assert _hand([0, 0], [(0, 10), (42, 80)], p, p)["next"][0] == 1
    assert _hand([0, 0], [(0, 10), (43, 80)], p, p)["next"][0] == -1
    # the inner z' of B within dz_max (64 cm) of A's outer z' (the chi2 cut lifted)
    far = [_seg(0.0), _seg(0.0, 64.0)]
    assert _hand([0, 0], [(0, 10), (11, 40)], far, p, chi2_max=1e30)["next"][0] == 1
    far = [_seg(0.0), _seg(0.0, 64.5)]
    assert _hand([0, 0], [(0, 10), (11, 40)], far, p, chi2_max=1e30)["next"][0] == -1
    # the inner y of B within dy_max (2 cm) of A's state carried to B's x
    assert _hand([0, 0], [(0, 10), (11, 40)], [_seg(0.0), _seg(2.0)], p, chi2_max=1e30)["next"][0] == 1
    assert _hand([0, 0], [(0, 10), (11, 40)], [_seg(0.0), _seg(-2.25)], p, chi2_max=1e30)["next"][0] == -1
    # unit 3 lies on the other side at unit 0's angle: identical states, no link
    assert _hand([0, 3], [(0, 10), (11, 40)], p, p)["next"][0] == -1
    # the straight line y = 0 of a unit at angle a2, seen from a unit at angle a1
    for w, linked in ((1, True), (2, False)):  # 20 degrees apart: neighbours; 40: not
        d = w * DALPHA
        pa, xa = oracle.rotate(_seg(0.0), 100.0, -d, 0.0)
        m = _hand([0, w], [(0, 10), (11, 40)], [_seg(0.0), _seg(0.0)], [pa, _seg(0.0)], x_out=[xa, 100.0])
        assert (m["next"][0] == 1) == linked, w
        assert m["n_candidates"] == (1 if linked else 0)
        if linked:
            assert m["link_chi2"][0] < 1e-20


def _maj(labels, first, nh, hits):
    out = np.full(len(nh), -1, np.int64)
    for t, (f, n) in enumerate(zip(first, nh)):
        lab = labels[hits[f:f + n]]
        lab = lab[lab >= 0]
        if len(lab):
            out[t] = np.bincount(lab).argmax()
    return out


def merge_event(name):
    """The oracle tracker's tracks of an event, refitted and merged, with the
    inputs rounded to FP32 as the GPU path stores them."""
    ev = cached_event(name)
    o = cached_oracle(name)
    k = float(np.float32(-np.float32(synth.KAPPA) * np.float32(ev.bz)))
    first, nh, hits = o["track_first_hit"], o["track_n_hits"], o["track_hits"]
    r = oracle.refit_tracks(first, nh, hits, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), k, P)
    for key in ("p", "cov", "x_ref", "p_out", "cov_out", "x_out"):
        r[key] = r[key].astype(np.float32).astype(np.float64)
    unit = o["trk_unit"][o["track_tracklet"]]
    fr, lr = oracle.segment_rows(first, nh, hits, ev.row)
    alpha = np.array([float(np.float32(synth.sector_alpha(int(s)))) for s in ev.unit_sector])
    side = np.where(np.asarray(ev.unit_sector) < 18, 1, -1).astype(np.int32)
    m = oracle.merge(unit, fr, lr, r, alpha, side, len(ev.row_x), k)
    return ev, o, r, unit, fr, lr, alpha, side, m


def test_links_on_a_central_collision_follow_the_particles():
    ev, o, r, unit, fr, lr, alpha, side, m = merge_event("pbpb_central")
    first, nh, hits = o["track_first_hit"], o["track_n_hits"], o["track_hits"]
    maj = _maj(ev.label, first, nh, hits)
    a = np.nonzero(m["next"] >= 0)[0]
    b = m["next"][a]
    assert len(a) > 5000
    assert ((maj[a] == maj[b]) & (maj[a] >= 0)).mean() > 0.995
    assert (unit[a] != unit[b]).mean() > 0.9  # mostly sector crossings
    # chi2 of the links: five degrees of freedom (median 4.35 for a chi2(5))
    assert 3.5 < np.median(m["link_chi2"][a]) < 7.0
    # efficiency: segment pairs of one particle on the same turn of its helix
    # that the rules admit, the outer one being the particle's next segment
    # after the inner one's last row.  The throughput workloads follow each
    # helix for two turns, so a particle's later pass through the chamber
    # shows up as more segments; a segment one turn later carries z' off by
    # the turn's z advance 2 pi R tan(lambda) and is no continuation.
    tr = ev.tracks
    turn_dz = 2 * np.pi * tr.pt / (synth.KAPPA * ev.bz) * np.abs(tr.tgl)
    ok = r["ok"].astype(bool)
    z = ev.z.astype(np.float64)
    wanted = linked = 0
    for p in np.unique(maj[ok & (maj >= 0)]):
        ts = np.nonzero(ok & (maj == p))[0]
        for A in ts:
            zA = z[hits[first[A] + nh[A] - 1]]
            after = [B for B in ts if fr[B] > lr[A] and fr[B] - lr[A] <= 32 and side[unit[B]] == side[unit[A]]
                     and abs(z[hits[first[B]]] - zA) < 0.5 * turn_dz[p]]
            if not after:
                continue
            B = min(after, key=lambda q: (fr[q], q))
            wanted += 1
            linked += m["next"][A] == B
    assert wanted > 5000 and linked / wanted > 0.9, (wanted, linked)


# ----------------------------------------------------------------------------
# fit of merged chains across frames

def _crossing_chains(seed=23, n=400):
    """Generator helices that cross from one sector into its neighbour on the
    same side: their first-leg crossings in the first sector, then in the
    second, as (rows_a, states_a, rows_b, states_b, sector_a, sector_b)."""
    rng = np.random.default_rng(seed)
    tr = synth.primaries_pp_sector(rng, n, 0, pt_range=(0.3, 2.0))
    xs = synth.helix_crossings(tr, 0.5)
    out = []
    for t in range(len(tr)):
        m = np.nonzero((xs["track"] == t) & (xs["cosphi"] > 0))[0]
        if len(m) < 20:
            continue
        m = m[np.argsort(xs["s"][m])]
        sec = xs["sector"][m]
        if len(np.unique(sec)) != 2 or np.any(np.diff(xs["row"][m]) <= 0):
            continue
        cut = int(np.nonzero(sec != sec[0])[0][0])
        if np.any(sec[cut:] != sec[cut]) or cut < 8 or len(m) - cut < 8:
            continue
        qpt = tr.q[t] / tr.pt[t]
        st = [np.array([xs["y"][j], xs["z"][j], xs["sinphi"][j], tr.tgl[t], qpt]) for j in m]
        out.append((xs["row"][m[:cut]], st[:cut], xs["row"][m[cut:]], st[cut:], int(sec[0]), int(sec[cut])))
    return out


def test_chain_fit_of_helices_across_two_sectors_gives_the_helix():
    """Noise-free helices measured in two sector frames: the chain fit (turns
    at the boundary in both passes) returns the helix's state at the first hit
    within 0.1 sigma (quantization of the positions only) and a chi2 far below
    one per hit."""
    cases = _crossing_chains()
    assert len(cases) > 20
    for ra, sa, rb, sb, seca, secb in cases:
        n = len(ra) + len(rb)
        y = np.array([s[0] for s in sa + sb], np.float32)
        z = np.array([s[1] for s in sa + sb], np.float32)
        row = np.concatenate([ra, rb]).astype(np.uint16)
        units = np.array([0] * len(ra) + [1] * len(rb), np.int32)
        alpha = [synth.sector_alpha(seca), synth.sector_alpha(secb)]
        r = oracle.refit_chains([0], [n], np.arange(n), units, y, z, row, synth.ROW_X, alpha, K_CURV, P)
        assert r["ok"][0] and r["x_ref"][0] == synth.ROW_X[ra[0]]
        sig = np.sqrt(r["cov"][0][[0, 2, 5, 9, 14]])
        assert np.all(np.abs(r["p"][0] - sa[0]) <= 0.1 * sig), (r["p"][0], sa[0], sig)
        assert r["chi2"][0] < 0.01 * n


def test_chain_of_one_frame_is_the_track_refit():
    """A chain whose hits all lie in one unit is fitted exactly as the track
    refit fits the same hit list (no turn happens)."""
    cases = _crossing_chains(seed=29)
    for ra, sa, _, _, seca, _ in cases[:10]:
        n = len(ra)
        y = np.array([s[0] for s in sa], np.float32)
        z = np.array([s[1] for s in sa], np.float32)
        row = ra.astype(np.uint16)
        r = oracle.refit_chains([0], [n], np.arange(n), np.zeros(n, np.int32), y, z, row, synth.ROW_X,
                                [synth.sector_alpha(seca)], K_CURV, P)
        q = oracle.refit_tracks([0], [n], np.arange(n), y, z, row, synth.ROW_X, K_CURV, P)
        for key in ("p", "cov", "chi2", "x_ref", "ok"):
            assert np.array_equal(r[key][0], q[key][0]), key


def test_chains_follow_the_links():
    """oracle.chains: heads are segments with no prev and a next; a chain's
    hit list is its segments' hit lists in link order."""
    nxt = np.array([2, -1, 3, -1, -1])
    prv = np.array([-1, -1, 0, 2, -1])
    first = np.array([0, 3, 5, 9, 12])
    nh = np.array([3, 2, 4, 3, 2])
    hits = np.arange(14) + 100
    unit = np.array([0, 1, 1, 2, 0])
    heads, cf, cn, ch, cu = oracle.chains(nxt, prv, first, nh, hits, unit)
    assert heads.tolist() == [0] and cf.tolist() == [0] and cn.tolist() == [10]
    assert ch.tolist() == [100, 101, 102, 105, 106, 107, 108, 109, 110, 111]
    assert cu.tolist() == [0, 0, 0, 1, 1, 1, 1, 2, 2, 2]


def test_chain_fit_on_a_central_collision():
    """The linked chains of a central collision fitted across frames: almost
    all succeed, chi2 per degree of freedom about 1, and q/pT is measured far
    better than by the chain's first segment alone (a longer lever arm;
    measured 0.16% against 1.84% median relative error)."""
    ev, o, r, unit, fr, lr, alpha, side, m = merge_event("pbpb_central")
    first, nh, hits = o["track_first_hit"], o["track_n_hits"], o["track_hits"]
    heads, cf, cn, ch, cu = oracle.chains(m["next"], m["prev"], first, nh, hits, unit)
    k = float(np.float32(-np.float32(synth.KAPPA) * np.float32(ev.bz)))
    rc = oracle.refit_chains(cf, cn, ch, cu, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), alpha, k, P)
    ok = rc["ok"].astype(bool)
    assert len(heads) > 10000 and ok.mean() > 0.99
    assert 0.9 < np.median(rc["chi2"][ok] / (2 * cn[ok] - 5)) < 1.1
    maj = _maj(ev.label, first, nh, hits)[heads]
    g = ok & (maj >= 0)
    true_qpt = ev.tracks.q[maj[g]] / ev.tracks.pt[maj[g]]
    chain_err = np.median(np.abs(rc["p"][g, 4] / true_qpt - 1))
    head_err = np.median(np.abs(r["p"][heads[g], 4] / true_qpt - 1))
    assert chain_err < head_err / 4, (chain_err, head_err)
