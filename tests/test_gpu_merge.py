"""Segment merging on the GPU (tpc_merge_tracks through the C ABI) against
the oracle (orc_merge), on inputs that do not come from the GPU: the oracle
tracker's output tracks of an event and the oracle's refit of them (rounded
to FP32 as the refit call stores them), uploaded for the GPU; and the
hand-worked segments of the oracle's pins.

Both sides decide in FP64 from the same FP32 inputs, with the same formulas
and contraction off; only the library's cos, sin and asin may differ in the
last bit.  Bars: links (next, prev) identical except on segments the oracle
flags (a chi2 within 1e-9 relative of the cut or of a tie); link chi2 within
1e-9 relative; candidate counts equal when nothing is flagged.  The GPU
tracker -> refit -> merge path (the configuration the benchmark times) is
checked for consistent links.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import cached_event, cached_oracle
from gpu_inputs import DeviceMerged, DeviceRefit, DeviceTracks
from paper_2106_03636_amd.params import DEFAULT_PARAMS as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2106_03636_amd as T
    T.load_library()
    return T


F32 = lambda v: float(np.float32(v))  # noqa: E731
# the merge parameters as the GPU holds them (FP32)
ORACLE_MERGE = dict(sinphi_max=F32(0.95), max_dalpha=F32(0.3665), max_gap=32, dz_max=64.0, dy_max=2.0, chi2_max=30.0)


def _k(bz):
    return float(np.float32(-np.float32(synth.KAPPA) * np.float32(bz)))


def _units(ev):
    alpha = np.array([synth.sector_alpha(int(s)) for s in ev.unit_sector], np.float32)
    side = np.where(np.asarray(ev.unit_sector) < 18, 1, -1).astype(np.int32)
    return alpha, side


def _f32(r):
    r = dict(r)
    for key in ("p", "cov", "x_ref", "chi2", "p_out", "cov_out", "x_out"):
        r[key] = r[key].astype(np.float32).astype(np.float64)
    return r


def _gpu_merge(ev, tracks, refit, alpha, side, params=None):
    from paper_2106_03636_amd.runtime import Batch, Merger
    b = Batch.from_event(ev)
    mg = Merger(refit, len(alpha), params)
    mg.launch(b, alpha, side)
    return mg


def _compare(g, o):
    frag = o["fragile"].astype(bool)
    for f in ("next", "prev"):
        differ = g[f] != o[f]
        assert not (differ & ~frag).any(), (f, np.nonzero(differ & ~frag)[0][:10])
    linked = (g["next"] >= 0) & (g["next"] == o["next"])
    rel = np.abs(g["link_chi2"][linked] - o["link_chi2"][linked]) / np.maximum(o["link_chi2"][linked], 1e-300)
    assert rel.max(initial=0.0) <= 1e-9
    assert not np.any(g["link_chi2"][g["next"] < 0])
    if not frag.any():
        assert g["n_candidates"] == o["n_candidates"]


@pytest.mark.parametrize("name", ["pbpb_central", "pbpb_timeframe_50"])
def test_links_match_the_oracle(T, name):
    ev, ot = cached_event(name), cached_oracle(name)
    first, nh, hits = ot["track_first_hit"], ot["track_n_hits"], ot["track_hits"]
    _say("case merge", name, len(nh), "tracks")
    r = _f32(oracle.refit_tracks(first, nh, hits, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), _k(ev.bz), P))
    alpha, side = _units(ev)
    dt = DeviceTracks.from_oracle(ot)
    mg = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side)
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in mg.result(len(nh)).items()}
    unit = ot["trk_unit"][ot["track_tracklet"]]
    fr, lr = oracle.segment_rows(first, nh, hits, ev.row)
    o = oracle.merge(unit, fr, lr, r, alpha.astype(np.float64), side, len(ev.row_x), _k(ev.bz), **ORACLE_MERGE)
    _say("pairs", g["n_pairs"], "candidates", g["n_candidates"], o["n_candidates"], "links", g["n_links"],
         int((o["next"] >= 0).sum()), "fragile", int(o["fragile"].sum()))
    _compare(g, o)
    assert g["n_links"] == int((g["next"] >= 0).sum()) > 10000


def _hand_tracks(units, rows, p_in, p_out, x_in=None, x_out=None):
    """Segments of two hits each (at their first and last row) with the
    given refit states and unit covariances."""
    n = len(units)
    row = np.array([r for fl in rows for r in fl], np.uint16)
    hits = np.arange(2 * n, dtype=np.int32)
    eye = np.zeros(15)
    eye[[0, 2, 5, 9, 14]] = 1.0
    r = dict(ok=np.ones(n, np.int8), p=np.array(p_in, float), cov=np.tile(eye, (n, 1)),
             x_ref=np.full(n, 100.0) if x_in is None else np.asarray(x_in, float), chi2=np.zeros(n),
             p_out=np.array(p_out, float), cov_out=np.tile(eye, (n, 1)),
             x_out=np.full(n, 100.0) if x_out is None else np.asarray(x_out, float))
    ev = synth.Event(np.zeros(2 * n, np.float32), np.zeros(2 * n, np.float32), row,
                     np.array([0, 2 * n], np.int64), np.zeros(1, np.int16), np.full(2 * n, -1, np.int32), None,
                     0.0, "hand")
    dt = DeviceTracks(2 * n, np.arange(0, 2 * n, 2, dtype=np.int32), np.full(n, 2, np.int32), hits,
                      unit=np.asarray(units, np.int32))
    return ev, dt, r


def test_hand_worked_links_on_the_gpu(T):
    """The oracle pins' hand-worked case (test_merge_oracle.test_hand_worked_links)
    through the C ABI: chi2 1, 0.5, 2, 3; the one mutual pair A1 -> B2."""
    seg = lambda y, z=0.0: [y, z, 0.0, 0.0, 0.0]  # noqa: E731
    units = [0, 0, 0, 0]
    rows = [(0, 10), (0, 12), (20, 60), (25, 70)]
    p_out = [seg(0.0, 0.0), seg(0.0, 1.0), seg(0.0), seg(0.0)]
    p_in = [seg(0.0), seg(0.0), seg(1.0, 1.0), seg(math.sqrt(3.75), -0.5)]
    ev, dt, r = _hand_tracks(units, rows, p_in, p_out)
    alpha = np.array([0.0, math.radians(20.0), math.radians(40.0), 0.0], np.float32)
    side = np.array([1, 1, 1, -1], np.int32)
    g = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side).result(4)
    assert g["next"].cpu().tolist() == [-1, 2, -1, -1] and g["prev"].cpu().tolist() == [-1, -1, 1, -1]
    assert abs(g["link_chi2"][1].item() - 0.5) < 1e-12 and g["n_candidates"] == 4
    # the tie: B2 takes A0
    p_out2 = [seg(0.0, 1.0), seg(0.0, 1.0), seg(0.0), seg(0.0)]
    ev, dt, r = _hand_tracks(units, rows, p_in, p_out2)
    g = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side).result(4)
    assert g["prev"][2].item() == 0 and g["next"][0].item() == 2 and g["next"][1].item() == -1
    # a neighbouring unit's straight line, turned (20 degrees: linked), and two units apart (not)
    for w, linked in ((1, True), (2, False)):
        pa, xa = oracle.rotate(seg(0.0), 100.0, -float(np.float32(w * math.radians(20.0))), 0.0)
        pa = pa.astype(np.float32).astype(np.float64)
        ev, dt, r = _hand_tracks([0, w], [(0, 10), (11, 40)], [seg(0.0), seg(0.0)], [pa, seg(0.0)],
                                 x_out=[float(np.float32(xa)), 100.0])
        g = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side).result(2)
        o = oracle.merge([0, w], [0, 11], [10, 40], r, alpha.astype(np.float64), side, 152, 0.0, **ORACLE_MERGE)
        assert (g["next"][0].item() == 1) == linked and g["next"].cpu().tolist() == o["next"].tolist()


def test_merge_after_tracking_on_the_gpu(T):
    """GPU tracker -> refit -> merge on the 50-collision frame: links join
    refitted segments on one side, in units at most max_dalpha apart, with
    rows increasing; prev and next agree; and the number of links is within
    0.5% of the oracle-input run's."""
    from paper_2106_03636_amd.runtime import Batch, Merger, Refitter, Tracker
    ev = cached_event("pbpb_timeframe_50")
    _say("case merge after tracking", ev.n, "clusters")
    b = Batch.from_event(ev)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows)
    tr.launch(b)
    rf = Refitter(tr)
    rf.launch(b)
    alpha, side = _units(ev)
    mg = Merger(rf, len(alpha))
    mg.launch(b, alpha, side)
    res = tr.result()
    n = res["n_tracks"]
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in mg.result(n).items()}
    ok = rf.result(n)["ok"].cpu().numpy().astype(bool)
    unit = res["unit"].cpu().numpy()
    fr, lr = oracle.segment_rows(res["first_hit"].cpu().numpy(), res["n_hits"].cpu().numpy(),
                                 res["hits"].cpu().numpy(), ev.row)
    a = np.nonzero(g["next"] >= 0)[0]
    bb = g["next"][a]
    assert np.array_equal(g["prev"][bb], a) and (g["prev"] >= 0).sum() == len(a)
    assert ok[a].all() and ok[bb].all()
    assert (fr[bb] > lr[a]).all() and (fr[bb] - lr[a] <= 32).all()
    assert (side[unit[a]] == side[unit[bb]]).all()
    d = np.abs(np.remainder(alpha[unit[bb]].astype(np.float64) - alpha[unit[a]] + np.pi, 2 * np.pi) - np.pi)
    assert (d <= 0.3665 + 1e-6).all()
    assert (g["link_chi2"][a] <= 30.0).all()
    _say("links", len(a), "candidates", g["n_candidates"], "pairs", g["n_pairs"])
    assert len(a) > 100000


def test_merge_edge_cases(T):
    """A failed tracking or refit status passes through; more pairs than
    cap_pairs gives TPC_E_CAPACITY with the count; a unit without a side,
    and a track whose hits lie outside the hit list, give TPC_E_INVALID; no
    tracks."""
    from paper_2106_03636_amd import make_merge_params
    from paper_2106_03636_amd.runtime import TrackingError
    seg = lambda y: [y, 0.0, 0.0, 0.0, 0.0]  # noqa: E731
    p = [seg(0.0)] * 3
    alpha = np.zeros(1, np.float32)
    side = np.ones(1, np.int32)
    ev, dt, r = _hand_tracks([0, 0, 0], [(0, 10), (11, 40), (12, 50)], p, p)
    g = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side).result(3)
    assert g["n_pairs"] == 2 and g["next"][0].item() == 1  # a tie: the smaller index
    with pytest.raises(TrackingError) as e:
        _gpu_merge(ev, dt, DeviceRefit(dt, r, status=T.TPC_E_CAPACITY), alpha, side).result(3)
    assert e.value.status == T.TPC_E_CAPACITY
    mg = _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, side, make_merge_params(cap_pairs=1))
    with pytest.raises(TrackingError) as e:
        mg.result(3)
    assert e.value.status == T.TPC_E_CAPACITY and int(mg.o_counts[0].item()) == 2
    with pytest.raises(TrackingError) as e:
        _gpu_merge(ev, dt, DeviceRefit(dt, r), alpha, np.zeros(1, np.int32)).result(3)
    assert e.value.status == T.TPC_E_INVALID
    for f2, n2 in ((5, 2), (-1, 2), (4, -1)):  # a track's hits outside the hit list
        dtb = DeviceTracks(ev.n, np.array([0, 2, f2]), np.array([2, 2, n2]), np.arange(6), unit=np.zeros(3))
        with pytest.raises(TrackingError) as e:
            _gpu_merge(ev, dtb, DeviceRefit(dtb, r), alpha, side).result(3)
        assert e.value.status == T.TPC_E_INVALID, (f2, n2)
    ev0, dt0, r0 = _hand_tracks([], [], np.zeros((0, 5)), np.zeros((0, 5)))
    g = _gpu_merge(ev0, dt0, DeviceRefit(dt0, r0), alpha, side).result(0)
    assert g["n_links"] == 0 and len(g["next"]) == 0


@pytest.mark.parametrize("name", ["pbpb_central", "pbpb_timeframe_50"])
def test_chain_fit_matches_the_oracle(T, name):
    """The chains of the oracle merger's links over the oracle tracker's
    tracks, fitted across frames on the GPU (FP32) and by the oracle (FP64):
    fitted flags identical, the states at the refit's bars with the chain
    fit's bulk covariance fractions (parity.CHAIN_*, derived from FP32 builds
    of the oracle's chain fit in tests/test_fp32_bars.py)."""
    import torch
    from parity import ParityReport, compare_fit
    from paper_2106_03636_amd.runtime import Batch, ChainFitter
    ev, ot = cached_event(name), cached_oracle(name)
    first, nh, hits = ot["track_first_hit"], ot["track_n_hits"], ot["track_hits"]
    r = _f32(oracle.refit_tracks(first, nh, hits, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), _k(ev.bz), P))
    alpha, side = _units(ev)
    unit = ot["trk_unit"][ot["track_tracklet"]]
    fr, lr = oracle.segment_rows(first, nh, hits, ev.row)
    m = oracle.merge(unit, fr, lr, r, alpha.astype(np.float64), side, len(ev.row_x), _k(ev.bz), **ORACLE_MERGE)
    heads, cf, cn, ch, cu = oracle.chains(m["next"], m["prev"], first, nh, hits, unit)
    _say("case chain fit", name, len(heads), "chains")
    o = oracle.refit_chains(cf, cn, ch, cu, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), alpha.astype(np.float64),
                            _k(ev.bz), P)
    b = Batch.from_event(ev)
    dt = DeviceTracks.from_oracle(ot)
    cfit = ChainFitter(dt)
    cfit.launch(b, DeviceMerged(m["next"], m["prev"]), torch.as_tensor(alpha).cuda())
    g = {k: v.cpu().numpy() for k, v in cfit.result(len(nh)).items()}
    assert np.array_equal(np.nonzero(g["n_hits"])[0], heads) and np.array_equal(g["n_hits"][heads], cn)
    gok, ook = g["ok"][heads].astype(bool), o["ok"].astype(bool)
    assert np.array_equal(gok, ook), int((gok != ook).sum())
    assert ook.mean() > 0.99
    both = gok & ook
    cov0 = [float(np.float32(v)) for v in P["cov0"]]
    rep = ParityReport()
    compare_fit(rep, g["params"][heads][both], g["cov"][heads][both], g["chi2"][heads][both],
                g["x_ref"][heads][both], o["p"][both], o["cov"][both], o["chi2"][both], o["x_ref"][both],
                refit_cov0=cov0, chain=True)
    _say({k: v for k, v in rep.items() if k != "failures"})
    assert rep.ok, rep.get("failures")



def _chain_fit(ev, dt, next_, prev, alpha, status=0):
    import torch
    from paper_2106_03636_amd.runtime import Batch, ChainFitter
    cf = ChainFitter(dt)
    cf.launch(Batch.from_event(ev), DeviceMerged(np.asarray(next_), np.asarray(prev), status=status),
              torch.as_tensor(np.asarray(alpha, np.float32)).cuda())
    return cf


def _chain_status(ev, dt, next_, prev, alpha, status=0):
    from paper_2106_03636_amd.runtime import TrackingError
    try:
        _chain_fit(ev, dt, next_, prev, alpha, status).result(dt.T)
    except TrackingError as e:
        return e.status
    return 0


def test_chain_fit_edge_cases(T):
    """Straight segments of two hits (no field): a chain of three is fitted as
    the oracle fits it and the other tracks are no heads; unlinked tracks and
    no tracks at all give no chains.  A failed tracking or merging status
    passes through.  Links that are not mutual, name no track of the call,
    close a loop, or make a chain of more than 64 segments (64 is fine), a
    chain segment without hits, a linked track's unit out of range, a track's
    hits outside the hit list and a hit naming no cluster give
    TPC_E_INVALID."""
    seg = [0.0] * 5
    ev, dt, _ = _hand_tracks([0, 0, 0], [(0, 10), (11, 40), (50, 60)], [seg] * 3, [seg] * 3)
    alpha = [0.0]
    g = {k: v.cpu().numpy() for k, v in _chain_fit(ev, dt, [1, 2, -1], [-1, 0, 1], alpha).result(3).items()}
    assert g["n_hits"].tolist() == [6, 0, 0] and g["ok"].tolist() == [1, 0, 0]
    first, nh, hits = np.arange(0, 6, 2), np.full(3, 2), np.arange(6)
    heads, cf, cn, ch, cu = oracle.chains(np.array([1, 2, -1]), np.array([-1, 0, 1]), first, nh, hits, np.zeros(3))
    o = oracle.refit_chains(cf, cn, ch, cu, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), np.zeros(1), 0.0, P)
    assert heads.tolist() == [0] and o["ok"].tolist() == [1]
    assert np.allclose(g["params"][0], o["p"][0], rtol=0, atol=1e-5)
    assert np.allclose(g["cov"][0], o["cov"][0], rtol=1e-3, atol=1e-9)
    assert g["x_ref"][0] == np.float32(o["x_ref"][0])
    assert not np.any(g["params"][1:]) and not np.any(g["cov"][1:])
    g = {k: v.cpu().numpy() for k, v in _chain_fit(ev, dt, [-1] * 3, [-1] * 3, alpha).result(3).items()}
    assert not np.any(g["n_hits"]) and not np.any(g["ok"])
    ev0, dt0, _ = _hand_tracks([], [], np.zeros((0, 5)), np.zeros((0, 5)))
    assert all(len(v) == 0 for v in _chain_fit(ev0, dt0, [], [], alpha).result(0).values())
    # statuses passed through
    assert _chain_status(ev, dt, [1, 2, -1], [-1, 0, 1], alpha, status=T.TPC_E_CAPACITY) == T.TPC_E_CAPACITY
    dtc = DeviceTracks(ev.n, first, nh, hits, unit=np.zeros(3), status=T.TPC_E_CAPACITY)
    assert _chain_status(ev, dtc, [1, 2, -1], [-1, 0, 1], alpha) == T.TPC_E_CAPACITY
    # malformed links
    bad = T.TPC_E_INVALID
    assert _chain_status(ev, dt, [1, -1, 1], [-1, 0, -1], alpha) == bad  # 2 -> 1, but 1 continues 0
    assert _chain_status(ev, dt, [5, -1, -1], [-1, -1, -1], alpha) == bad  # a link to no track
    assert _chain_status(ev, dt, [-1, -1, -1], [-1, -1, 7], alpha) == bad
    assert _chain_status(ev, dt, [1, 0, -1], [1, 0, -1], alpha) == bad  # 0 -> 1 -> 0: no head
    for n_seg, want in ((64, 0), (65, bad)):
        evl, dtl, _ = _hand_tracks([0] * n_seg, [(0, 1)] * n_seg, [seg] * n_seg, [seg] * n_seg)
        nx = list(range(1, n_seg)) + [-1]
        pv = [-1] + list(range(n_seg - 1))
        assert _chain_status(evl, dtl, nx, pv, alpha) == want, n_seg
    # a linked track's unit out of range (an unlinked one is not read)
    dtu = DeviceTracks(ev.n, first, nh, hits, unit=np.array([0, 1, 5]))
    assert _chain_status(ev, dtu, [1, -1, -1], [-1, 0, -1], alpha) == bad
    assert _chain_status(ev, dtu, [-1, -1, -1], [-1, -1, -1], alpha) == 0
    # hits outside the list, a hit naming no cluster
    for f2, n2 in ((5, 2), (-1, 2), (0, -1)):
        dth = DeviceTracks(ev.n, np.array([0, 2, f2]), np.array([2, 2, n2]), hits, unit=np.zeros(3))
        assert _chain_status(ev, dth, [1, -1, -1], [-1, 0, -1], alpha) == bad, (f2, n2)
    dtx = DeviceTracks(ev.n, first, nh, np.array([0, 1, 2, 99, 4, 5]), unit=np.zeros(3))
    assert _chain_status(ev, dtx, [1, -1, -1], [-1, 0, -1], alpha) == bad
    # a chain segment without hits (at the head, inside, at the tail); unlinked, it is fine
    dte = DeviceTracks(ev.n, np.array([0, 2, 2]), np.array([2, 0, 4]), hits, unit=np.zeros(3))
    for nx, pv in (([1, 2, -1], [-1, 0, 1]), ([2, -1, 1], [-1, 2, 0]), ([-1, 0, -1], [1, -1, -1])):
        assert _chain_status(ev, dte, nx, pv, alpha) == bad, (nx, pv)
    assert _chain_status(ev, dte, [2, -1, -1], [-1, -1, 0], alpha) == 0
