"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU."""
import json
import os
import sys

import numpy as np
import pytest

from conftest import cached_event, cached_oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def _run(T, ev, params=None, **kw):
    from paper_2106_03636_amd.runtime import Batch, Tracker
    b = Batch.from_event(ev)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows, params, **kw)
    tr.launch(b)
    res = tr.result()
    return tr, res


def _compare(T, ev, o, params=None):
    import parity
    tr, res = _run(T, ev, params)
    g = parity.gpu_state(tr, res)
    rep = parity.compare(g, o)
    _say("parity", ev.name, {k: v for k, v in rep.items() if k != "failures"})
    assert rep.ok, rep.get("failures")
    return g, rep


class _Ev:
    """Minimal event from arrays."""

    def __init__(self, y, z, row, off, row_x, bz, name="toy"):
        self.y, self.z = np.asarray(y, np.float32), np.asarray(z, np.float32)
        self.row = np.asarray(row, np.uint16)
        self.unit_offsets = np.asarray(off, np.int64)
        self.row_x = np.asarray(row_x, np.float32)
        self.bz = bz
        self.name = name

    @property
    def n(self):
        return len(self.y)

    @property
    def n_units(self):
        return len(self.unit_offsets) - 1


def test_golden_neighbour_rule_gpu(T):
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    g = json.load(open(os.path.join(HERE, "golden", "neighbour_rule.json")))
    c = g["clusters"]
    ev = _Ev(np.asarray(c["Y"]) / 256.0, np.asarray(c["Z"]) / 256.0, c["row"], [0, len(c["row"])],
             g["row_x_cm"], g["bz_tesla"], "golden")
    tr, res = _run(T, ev)
    perm = tr.inspect(T.TPC_VIEW_PERM).cpu().numpy()
    for view, key in ((T.TPC_VIEW_DN, "dn_id"), (T.TPC_VIEW_UP, "up_id"), (T.TPC_VIEW_UPC, "clean_up_id"),
                      (T.TPC_VIEW_DNC, "clean_dn_id")):
        lk = tr.inspect(view).cpu().numpy()
        by_id = np.full(ev.n, -1)
        m = lk >= 0
        by_id[perm[m]] = perm[lk[m]]
        assert by_id.tolist() == g["expected"][key], key
    o = oracle.run_event(ev, P, fragile_eps=0.05)
    _compare(T, ev, o)


def _hand_derived_cases():
    """The hand-derived toy events of the oracle pins: the score weights decide
    a neighbour pair and a pickup, a pickup tie goes to the smaller id, a walk
    crosses max_miss empty rows but not one more (upward, and downward below
    the chain), a track of n_min hits is kept and one of n_min - 1 is not, a
    walk stops where its prediction leaves the sector, and a pickup 0.01
    quanta from a rounding boundary (flagged fragile by the oracle; the GPU
    must still take the same decision)."""
    import synth
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    rx = synth.ROW_X_F32
    cases = [_Ev(np.array([40, 0, 0, 0]) / 256.0, np.array([0, 40, 0, 0]) / 256.0, [0, 0, 1, 2], [0, 4],
                 [100.0, 101.0, 102.0], 0.5, "neighbour_weights")]
    rows = [r for r in range(20) if r != 10] + [10, 10]
    y, z = np.zeros(len(rows)), np.zeros(len(rows))
    y[-2], z[-1] = 240 / 256.0, 240 / 256.0
    cases.append(_Ev(y, z, rows, [0, len(rows)], rx[:20], 0.0, "pickup_weights"))
    y = np.zeros(len(rows))
    y[-2], y[-1] = -200 / 256.0, 200 / 256.0
    cases.append(_Ev(y, np.zeros(len(rows)), rows, [0, len(rows)], rx[:20], 0.0, "pickup_tie"))
    m = P["max_miss"]
    for gap in (m, m + 1):
        rows = list(range(15)) + list(range(15 + gap, 25 + gap))
        cases.append(_Ev(np.zeros(len(rows)), np.zeros(len(rows)), rows, [0, len(rows)], rx[:25 + gap], 0.0,
                         "gap_%d" % gap))
    for n_hits in (P["n_min"], P["n_min"] - 1):
        cases.append(_Ev(np.zeros(n_hits), np.zeros(n_hits), list(range(n_hits)), [0, n_hits], rx[:n_hits + 2],
                         0.0, "keep_%d" % n_hits))
    import test_oracle_pins as pins
    for gap in (m, m + 1):
        (y, z, r, off, row_x), _ = pins.pass2_gap_event(gap)
        cases.append(_Ev(y, z, r, off, row_x, 0.0, "pass2_gap_%d" % gap))
    for far in (True, False):
        (y, z, r, off, row_x), _ = pins.edge_stop_event(with_far_hit=far)
        cases.append(_Ev(y, z, r, off, row_x, 0.0, "edge_stop_%s" % far))
    for x10, yd in ((128.47, 9 - P["ext_win_y_q"]), (127.6, 9 - P["ext_win_y_q"]), (128.47, 9)):
        y, z, r, off, row_x = pins.fragile_event(x10, yd)
        cases.append(_Ev(y, z, r, off, row_x, 0.0, "fragile_%g_%d" % (x10, yd)))
    return cases


def test_parity_hand_derived_cases(T):
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    for ev in _hand_derived_cases():
        _say("case", ev.name, ev.n, "clusters")
        _, rep = _compare(T, ev, oracle.run_event(ev, P, fragile_eps=0.05))
        assert rep["n_hitset_diff"] == 0, ev.name


def test_parity_pp_sector(T):
    _say("case pp_sector")
    _compare(T, cached_event("pp_sector"), cached_oracle("pp_sector"))


def test_parity_pbpb_central(T):
    _say("case pbpb_central")
    _compare(T, cached_event("pbpb_central"), cached_oracle("pbpb_central"))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_parity_tiny_crowded(T, seed):
    import oracle
    from test_oracle_pins import _tiny_inputs
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    row, y, z, row_x = _tiny_inputs(seed)
    ev = _Ev(y, z, row, [0, len(y)], row_x, 0.5, "tiny%d" % seed)
    _say("case tiny", seed)
    _compare(T, ev, oracle.run_event(ev, P, fragile_eps=0.05))


@pytest.mark.parametrize("per_row,z_max", [(8000, 250.0), (20000, 80.0)])
def test_parity_crowded_rows(T, per_row, z_max):
    """Three adjacent rows far denser than any time frame: 8000 hits per row
    over 250 cm (more than a thread block keeps in registers while binning)
    and 20000 over 80 cm (more than the binning's LDS pool, so the bins go
    through the workspace; and neighbour slabs of ~1500 hits, too large for
    LDS, so those chunks take the wide path)."""
    import oracle
    import synth
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    rng = np.random.default_rng(per_row)
    rows = np.repeat(np.arange(10, 13), per_row)
    half = synth.ROW_X_F32[rows].astype(np.float64) * np.tan(np.radians(10.0)) * 0.95
    y = rng.uniform(-1, 1, len(rows)) * half
    z = rng.uniform(0.0, z_max, len(rows))
    order = rng.permutation(len(rows))
    ev = _Ev(y[order], z[order], rows[order], [0, len(rows)], synth.ROW_X_F32, 0.5, "crowded%d" % per_row)
    _say("case crowded rows", per_row)
    _compare(T, ev, oracle.run_event(ev, P, fragile_eps=0.05))


def test_parity_ragged_units(T):
    """Units of very different sizes: empty, single cluster, one row only,
    several tiles with a ragged tail, and a full sector."""
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    full = cached_event("pbpb_central")
    pp = cached_event("pp_sector")
    parts = []
    parts.append((np.zeros(0), np.zeros(0), np.zeros(0)))                       # empty
    parts.append((pp.y[:1], pp.z[:1], pp.row[:1]))                              # one cluster
    one_row = pp.row == 40
    parts.append((pp.y[one_row], pp.z[one_row], pp.row[one_row]))               # one row
    parts.append((pp.y[:4097], pp.z[:4097], pp.row[:4097]))                     # 2 tiles + 1
    s = full.unit(5)
    parts.append((full.y[s], full.z[s], full.row[s]))                           # a Pb-Pb sector
    parts.append((pp.y, pp.z, pp.row))                                          # a pp sector
    parts.append((np.zeros(0), np.zeros(0), np.zeros(0)))                       # empty at the end
    y = np.concatenate([p[0] for p in parts]).astype(np.float32)
    z = np.concatenate([p[1] for p in parts]).astype(np.float32)
    row = np.concatenate([p[2] for p in parts]).astype(np.uint16)
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])])
    ev = _Ev(y, z, row, off, pp.row_x, 0.5, "ragged")
    _say("case ragged")
    _compare(T, ev, oracle.run_event(ev, P, fragile_eps=0.05))


def test_parity_zero_field(T):
    import oracle
    import synth
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    rng = np.random.default_rng(5)
    tr = synth.primaries_pp_sector(rng, 60, 0)
    xs = synth.helix_crossings(tr, 0.0)
    m = xs["sector"] == 0
    y = xs["y"][m] + rng.normal(0, 0.1, m.sum())
    z = xs["z"][m] + rng.normal(0, 0.15, m.sum())
    ev = _Ev(y, z, xs["row"][m], [0, int(m.sum())], synth.ROW_X_F32, 0.0, "bz0")
    _say("case bz0")
    _compare(T, ev, oracle.run_event(ev, P, fragile_eps=0.05))


@pytest.mark.parametrize("bins", [(256, 1, 64), (4096, 8, 128)])
def test_parity_other_bin_sizes(T, bins):
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    q = dict(P, bin_y_q=bins[0], bin_occ=bins[1], bin_zmin_q=bins[2])
    ev = cached_event("pp_sector")
    _say("case bins", bins)
    _compare(T, ev, oracle.run_event(ev, q, fragile_eps=0.05), params=q)


def test_parity_int64_scores(T):
    """S_max at or above 2^48 sends every row to the int64 scoring path (the
    FP64 one is exact only below it): links must still match bit for bit."""
    import oracle
    from paper_2106_03636_amd.params import DEFAULT_PARAMS as P
    ev = cached_event("pp_sector")
    x = np.round(ev.row_x.astype(np.float64) * 256)
    span = int((x[2:] - x[:-2]).min())
    q = dict(P, smax_k=int(2 ** 48 // span ** 2) + 1)
    assert q["smax_k"] < 2 ** 30
    _say("case int64 scores", q["smax_k"])
    _compare(T, ev, oracle.run_event(ev, q, fragile_eps=0.05), params=q)


def test_empty_batch(T):
    import synth
    ev = _Ev(np.zeros(0), np.zeros(0), np.zeros(0), [0, 0], synth.ROW_X_F32, 0.5, "empty")
    tr, res = _run(T, ev)
    assert res["n_tracks"] == 0 and res["n_tracklets"] == 0


def test_invalid_input_reports_status_and_next_call_works(T):
    import torch
    from paper_2106_03636_amd.runtime import Batch, Tracker, TrackingError
    pp = cached_event("pp_sector")
    row = pp.row.copy()
    row[100] = 200  # beyond the 152 rows
    bad = Batch(pp.y, pp.z, row, pp.unit_offsets, pp.row_x, pp.bz)
    tr = Tracker(pp.n, 1)
    tr.launch(bad)
    with pytest.raises(TrackingError) as e:
        tr.result()
    assert e.value.status == T.TPC_E_INVALID
    y = pp.y.copy()
    y[7] = np.nan
    tr.launch(Batch(y, pp.z, pp.row, pp.unit_offsets, pp.row_x, pp.bz))
    with pytest.raises(TrackingError):
        tr.result()
    good = Batch.from_event(pp)
    tr.launch(good)
    res = tr.result()
    assert res["n_tracks"] == cached_oracle("pp_sector")["n_tracks"]


def test_capacity_exceeded_then_retry(T):
    from paper_2106_03636_amd.runtime import Batch, Tracker, TrackingError
    pp = cached_event("pp_sector")
    o = cached_oracle("pp_sector")
    b = Batch.from_event(pp)
    tr = Tracker(pp.n, 1, cap_tracks=5)
    tr.launch(b)
    with pytest.raises(TrackingError) as e:
        tr.result()
    assert e.value.status == T.TPC_E_CAPACITY
    counts = tr.o_counts.cpu().numpy()
    assert counts[0] == o["n_tracks"]  # required size reported
    tr2 = Tracker(pp.n, 1, cap_tracks=int(counts[0]), cap_hits=int(counts[1]))
    tr2.launch(b)
    assert tr2.result()["n_tracks"] == o["n_tracks"]


def test_seed_capacity_exceeded_then_retry(T):
    """A seed capacity below the batch's seeds (n / 64 + 64 for a central Pb-Pb
    collision with about n / 29 seeds) fails with TPC_E_CAPACITY and reports
    the seeds needed in counts[4]; a retry with the divisor derived from it
    gives the oracle's tracks."""
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    from paper_2106_03636_amd.runtime import Batch, Tracker, TrackingError
    ev = cached_event("pbpb_central")
    o = cached_oracle("pbpb_central")
    b = Batch.from_event(ev)
    seeds = int((o["trk_len"] >= DEFAULT_PARAMS["l_min"]).sum())
    tr = Tracker(b.n, b.n_units, params=dict(DEFAULT_PARAMS, tracklet_cap_div=64))
    tr.launch(b)
    with pytest.raises(TrackingError) as e:
        tr.result()
    assert e.value.status == T.TPC_E_CAPACITY
    counts = tr.o_counts.cpu().numpy()
    assert counts[4] == seeds and counts[2] == o["n_tracklets"]
    div = max(2, int(b.n // int(counts[4])))
    tr2 = Tracker(b.n, b.n_units, params=dict(DEFAULT_PARAMS, tracklet_cap_div=div))
    tr2.launch(b)
    r = tr2.result()
    assert r["n_tracks"] == o["n_tracks"] and r["n_seeds"] == seeds


def test_rerun_is_bit_identical(T):
    """Order-independent merges: two runs give identical bits (race check)."""
    import torch
    ev = cached_event("pbpb_central")
    from paper_2106_03636_amd.runtime import Batch, Tracker
    b = Batch.from_event(ev)
    tr = Tracker(b.n, b.n_units)
    outs = []
    for _ in range(2):
        tr.launch(b)
        r = tr.result()
        outs.append({k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in r.items()})
    for k in outs[0]:
        a, c = outs[0][k], outs[1][k]
        if isinstance(a, torch.Tensor):
            assert torch.equal(a, c), k
        else:
            assert a == c, k


def test_profiled_launch_matches_plain(T):
    """The launch that records an event pair around every kernel (used for the
    per-kernel times) computes the same results as the plain launch."""
    import ctypes
    import torch
    from paper_2106_03636_amd.runtime import Batch, Tracker
    ev = cached_event("pbpb_central")
    b = Batch.from_event(ev)
    tr = Tracker(b.n, b.n_units, b.n_rows)
    tr.launch(b)
    ref = {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in tr.result().items()}
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    events = []
    for _ in range(T.tpc_kernel_count() + 1):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        events.append(e.value)
    try:
        tr.launch_profiled(b, events)
        out = tr.result()
        for k, v in ref.items():
            if isinstance(v, torch.Tensor):
                assert torch.equal(v, out[k]), k
            else:
                assert v == out[k], k
        total = 0.0
        for a, c in zip(events, events[1:]):
            ms = ctypes.c_float()
            assert hip.hipEventElapsedTime(ctypes.byref(ms), a, c) == 0
            assert ms.value >= 0.0
            total += ms.value
        assert total > 0.0
    finally:
        for e in events:
            hip.hipEventDestroy(e)


def _unit_tracks(ev, g, units):
    """Per cluster of the given units: (local id of the track's start hit) or -1;
    and per track of those units: its params keyed by the start's local id."""
    perm = g["perm"]
    kept = np.nonzero(g["trk_keep"])[0]
    out_ct, out_params = g["out_cluster_track"], g["out_params"]
    res_ct, res_par = [], {}
    for u in units:
        a, b = int(ev.unit_offsets[u]), int(ev.unit_offsets[u + 1])
        ct = out_ct[a:b]
        key = np.full(b - a, -1, np.int64)
        m = ct >= 0
        starts = g["trk_start"][kept[ct[m]]]
        key[m] = perm[starts] - a
        res_ct.append(key)
        for t_idx, tl in enumerate(kept):
            if g["trk_unit"][tl] == u:
                res_par[(u, int(perm[g["trk_start"][tl]] - a))] = out_params[t_idx]
    return res_ct, res_par


def _full_size_case(T, name, params=None, sample_units=()):
    """Full-size batch on the GPU (as timed by the benchmark) against the
    oracle on every unit of the same batch, at the parity bars.  With
    sample_units, also GPU(full batch) restricted to those units ==
    GPU(batch of those units alone), bit for bit (units are independent)."""
    import oracle
    import parity
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    P = dict(DEFAULT_PARAMS if params is None else params)
    ev = cached_event(name)
    _say("case full-size", name, ev.n, "clusters", ev.n_units, "units",
         {k: P[k] for k in ("bin_y_q", "bin_occ", "bin_zmin_q")})
    trf, resf = _run(T, ev, P)
    gf = parity.gpu_state(trf, resf)
    o = oracle.run_event(ev, P, fragile_eps=0.05)
    rep = parity.compare(gf, o)
    _say("parity", name, "all %d units" % ev.n_units, {k: v for k, v in rep.items() if k != "failures"})
    assert rep.ok, rep.get("failures")
    assert rep["n_fitted"] > 0
    del trf, o
    if len(sample_units):
        sub = ev.subset_units(sample_units)
        trs, ress = _run(T, sub, P)
        gs = parity.gpu_state(trs, ress)
        ct_f, par_f = _unit_tracks(ev, gf, sample_units)
        ct_s, par_s = _unit_tracks(sub, gs, range(len(sample_units)))
        for a, b in zip(ct_f, ct_s):
            assert np.array_equal(a, b)
        assert len(par_f) == len(par_s)
        for (u, k), v in par_f.items():
            j = list(sample_units).index(u)
            assert np.array_equal(v, par_s[(j, k)])


def _tuned(name):
    from paper_2106_03636_amd import autotune
    from paper_2106_03636_amd.runtime import Batch
    ev = cached_event(name)
    b = Batch.from_event(ev)
    key = autotune.cache_key(b)
    if key not in autotune.load_cache():
        pytest.fail("no tuned shape cached for %s (%s)" % (name, key))
    return autotune.tuned_params(b)


def test_parity_timeframe_full_size(T):
    _full_size_case(T, "pbpb_timeframe_50", sample_units=[0, 13, 27])


def test_parity_timeframe_full_size_tuned_shape(T):
    """The grid shape the benchmark runs with (the autotune cache's entry for
    this batch), every unit at the benchmark's full size."""
    _full_size_case(T, "pbpb_timeframe_50", params=_tuned("pbpb_timeframe_50"))


def test_parity_uneven_chunks_full_size(T):
    _full_size_case(T, "uneven_chunks_512", sample_units=list(range(0, 512, 64)))


def test_parity_uneven_chunks_full_size_tuned_shape(T):
    """All 512 chunks at the shape the batched benchmark replays."""
    _full_size_case(T, "uneven_chunks_512", params=_tuned("uneven_chunks_512"))


def test_graph_capture_replays_match_eager(T):
    """The whole call captured in a HIP graph: every replay, with eager work on
    other buffers in between, gives the eager result bit for bit."""
    import torch
    from paper_2106_03636_amd.runtime import Batch, GraphRunner, Tracker
    ev = cached_event("pbpb_central")
    b = Batch.from_event(ev)
    tr = Tracker(b.n, b.n_units)
    tr.launch(b)
    ref = {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in tr.result().items()}
    pp = cached_event("pp_sector")
    b2 = Batch.from_event(pp)
    tr2 = Tracker(b2.n, 1)
    gr = GraphRunner(tr, b)
    for i in range(3):
        tr2.launch(b2)
        assert tr2.result()["n_tracks"] == cached_oracle("pp_sector")["n_tracks"]
        tr.o_cluster_track.fill_(-7)
        gr.replay()
        got = gr.result()
        for k, v in ref.items():
            if isinstance(v, torch.Tensor):
                assert torch.equal(v, got[k]), (i, k)
            else:
                assert v == got[k], (i, k)


def test_autotuner_keeps_tracks_and_picks_a_shape(T, tmp_path):
    from paper_2106_03636_amd import autotune
    from paper_2106_03636_amd.runtime import Batch
    ev = cached_event("pbpb_central")
    b = Batch.from_event(ev)
    space = dict(bin_y_q=(384, 1536), bin_occ=(1, 4), bin_zmin_q=(256,))
    best, table = autotune.tune(b, space=space, reps=1, verify=True)
    assert len(table) == 4 and all(r["ms"] > 0 for r in table)
    assert best["bin_y_q"] in (384, 1536)
