"""Track refit on the GPU (tpc_refit_tracks through the C ABI) against the
oracle (orc_refit_tracks), on hit lists that do not come from the GPU: the
generator's truth tracks, and the oracle tracker's own output tracks.

Both sides fit the same hits, the GPU in FP32 with the tracker's filter, the
oracle in FP64.  Bars:
  * ok flags identical, except where the oracle flags a transport within
    1e-5 of the sin(phi) limit;
  * for the tracks both refit: the fit clauses of the tracker's parity bars
    (parity.compare_fit, FP32 against FP64 of the same filter) with the
    refit's covariance clauses (parity.REFIT_*, derived from FP32 builds of
    the oracle's refit in tests/test_fp32_bars.py) on the inner state (pass 2
    at the first hit, with its chi2) and on the outer state (pass 1 at the
    last hit); x_ref and x_out are the rows' FP32 x exactly;
  * tracks not refitted: every output zero.
The refit of the GPU tracker's own output is checked against the refit of
the same hit lists uploaded from the host (bit-exact: same kernel, same
inputs), which ties the tracker's output layout to the refit's input.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import cached_event, cached_oracle
from gpu_inputs import DeviceTracks, truth_tracks
from paper_2106_03636_amd.params import DEFAULT_PARAMS
from parity import ParityReport, compare_fit

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


def _k(bz):
    return float(np.float32(-np.float32(synth.KAPPA) * np.float32(bz)))


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _gpu_refit(ev, first, nh, hits, status=0):
    from paper_2106_03636_amd.runtime import Batch, Refitter
    b = Batch.from_event(ev)
    dt = DeviceTracks(b.n, first, nh, hits, status=status)
    rf = Refitter(dt)
    rf.launch(b)
    return rf, len(nh)


def _oracle_refit(ev, first, nh, hits):
    return oracle.refit_tracks(first, nh, hits, ev.y, ev.z, ev.row, ev.row_x.astype(np.float64), _k(ev.bz),
                               DEFAULT_PARAMS)


def _compare(g, o, min_ok=0.99):
    """min_ok: the fraction of tracks both sides must refit (truth tracks include
    legs the state cannot describe: inward-bound return legs, |sin(phi)| beyond
    the limit; their ok flags are still compared)."""
    ok_g, ok_o = g["ok"].astype(bool), o["ok"].astype(bool)
    differ = ok_g != ok_o
    assert not (differ & ~o["fragile"].astype(bool)).any(), np.nonzero(differ & ~o["fragile"].astype(bool))[0][:10]
    both = ok_g & ok_o
    assert both.mean() >= min_ok, both.mean()
    for f in ("params", "cov", "x_ref", "chi2", "params_out", "cov_out", "x_out"):
        assert not np.any(g[f][~ok_g]), f
    cov0 = [float(np.float32(v)) for v in DEFAULT_PARAMS["cov0"]]
    rep = ParityReport()
    compare_fit(rep, g["params"][both], g["cov"][both], g["chi2"][both], g["x_ref"][both], o["p"][both],
                o["cov"][both], o["chi2"][both], o["x_ref"][both], refit_cov0=cov0)
    assert rep.ok, dict(rep)
    zero = np.zeros(int(both.sum()))
    rep_out = ParityReport()
    compare_fit(rep_out, g["params_out"][both], g["cov_out"][both], zero, g["x_out"][both], o["p_out"][both],
                o["cov_out"][both], zero, o["x_out"][both], refit_cov0=cov0)
    assert rep_out.ok, dict(rep_out)
    assert np.array_equal(g["x_ref"][both], o["x_ref"][both].astype(np.float32))
    assert np.array_equal(g["x_out"][both], o["x_out"][both].astype(np.float32))
    return rep, rep_out


@pytest.mark.parametrize("name", ["pp_sector", "pbpb_central", "pbpb_timeframe_50"])
def test_refit_of_truth_tracks_matches_the_oracle(T, name):
    ev = cached_event(name)
    first, nh, hits, _ = truth_tracks(ev)
    _say("case refit truth", name, len(nh), "tracks", len(hits), "hits")
    rf, n = _gpu_refit(ev, first, nh, hits)
    g = _host(rf.result(n))
    o = _oracle_refit(ev, first, nh, hits)
    rep, rep_out = _compare(g, o, min_ok=0.75)
    _say("inner", {k: rep[k] for k in ("param_within_fraction", "cov_max_rel", "chi2_max_rel")},
         "outer", {k: rep_out[k] for k in ("param_within_fraction", "cov_max_rel")})
    # a sane fit: chi2 per degree of freedom near 1 on the bulk (the clusters are Gaussian-smeared)
    ok = g["ok"].astype(bool)
    ndf = 2 * nh[ok] - 5
    assert 0.5 < np.median(g["chi2"][ok] / ndf) < 2.0


@pytest.mark.parametrize("name", ["pp_sector", "pbpb_central", "pbpb_timeframe_50"])
def test_refit_of_the_oracle_trackers_tracks_matches_the_oracle(T, name):
    ev, o_trk = cached_event(name), cached_oracle(name)
    first, nh, hits = o_trk["track_first_hit"], o_trk["track_n_hits"], o_trk["track_hits"]
    _say("case refit of tracker output", name, len(nh), "tracks")
    rf, n = _gpu_refit(ev, first, nh, hits)
    g = _host(rf.result(n))
    _compare(g, _oracle_refit(ev, first, nh, hits))


@pytest.mark.parametrize("name", ["pbpb_central", "pbpb_timeframe_50"])
def test_refit_reads_the_trackers_output(T, name):
    """GPU tracker -> GPU refit (the configuration the benchmark times) gives
    the refit of the same hit lists uploaded from the host, bit for bit."""
    from paper_2106_03636_amd.runtime import Batch, Refitter, Tracker
    ev = cached_event(name)
    _say("case refit after tracking", name, ev.n, "clusters")
    b = Batch.from_event(ev)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows)
    tr.launch(b)
    rf = Refitter(tr)
    rf.launch(b)
    res = tr.result()
    n = res["n_tracks"]
    g = _host(rf.result(n))
    first, nh, hits = (res[f].cpu().numpy() for f in ("first_hit", "n_hits", "hits"))
    rf2, _ = _gpu_refit(ev, first, nh, hits)
    g2 = _host(rf2.result(n))
    for f in g:
        assert np.array_equal(g[f], g2[f]), f
    assert g["ok"].mean() > 0.99
    _say("refitted", int(g["ok"].sum()), "of", n)


def test_refit_edge_cases(T):
    """Tracks of 0, 1 and 2 hits are not refitted; a failed tracking call's
    status passes through; a hit that names no cluster, and a track whose
    hits lie outside the hit list, give TPC_E_INVALID; no tracks at all is
    fine."""
    from paper_2106_03636_amd.runtime import TrackingError
    ev = cached_event("pp_sector")
    first, nh, hits, _ = truth_tracks(ev)
    # three short tracks (0, 1 and 2 hits, over the first two list entries) in front of the real ones
    hits2 = np.concatenate([hits[:2], hits]).astype(np.int32)
    nh2 = np.concatenate([[0, 1, 2], nh]).astype(np.int32)
    first2 = np.concatenate([[0, 0, 0], first + 2]).astype(np.int32)
    rf, n = _gpu_refit(ev, first2, nh2, hits2)
    g = _host(rf.result(n))
    assert list(g["ok"][:3]) == [0, 0, 0]
    for f in g:
        assert not np.any(g[f][:3]), f
    o = _oracle_refit(ev, first2, nh2, hits2)
    _compare(g, o, min_ok=0.9)
    rf, n = _gpu_refit(ev, first, nh, hits, status=T.TPC_E_CAPACITY)
    with pytest.raises(TrackingError) as e:
        rf.result(n)
    assert e.value.status == T.TPC_E_CAPACITY
    bad = hits.copy()
    bad[len(bad) // 2] = ev.n + 5
    rf, n = _gpu_refit(ev, first, nh, bad)
    with pytest.raises(TrackingError) as e:
        rf.result(n)
    assert e.value.status == T.TPC_E_INVALID
    # a track whose hits lie outside the hit list (past its end, a negative start or count)
    assert first[-1] + nh[-1] == len(hits)
    for f2, n2 in ((first[-1] + 1, nh[-1]), (-1, nh[-1]), (first[-1], -1)):
        fb, nb = first.copy(), nh.copy()
        fb[-1], nb[-1] = f2, n2
        rf, n = _gpu_refit(ev, fb, nb, hits)
        with pytest.raises(TrackingError) as e:
            rf.result(n)
        assert e.value.status == T.TPC_E_INVALID, (f2, n2)
    rf, n = _gpu_refit(ev, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert n == 0 and all(len(v) == 0 for v in _host(rf.result(0)).values())
