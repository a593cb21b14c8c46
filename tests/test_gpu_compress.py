"""Hit removal and track-model compression on the GPU (tpc_compress through
the C ABI) against the oracle (orc_compress).

Both sides get the same tracks, which do not come from the GPU: the oracle
tracker's output tracks of the event, their FP64 states rounded to FP32 as a
tracking call stores them, uploaded for the GPU.  Both take their decisions
in FP64 from the same FP32 inputs and parameters: the class of every cluster
is identical, and so are the codes except where the oracle flags an
unrounded residual code as within 1e-6 of a half step (the helix through
asin and square roots may round differently in the last bit); position codes
are single correctly rounded quotients, identical everywhere.  The
histograms and counts are checked against the GPU's own codes, also on the
GPU tracker's own output (the configuration the benchmark times).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import cached_event, cached_oracle

pytestmark = pytest.mark.gpu

F32 = lambda v: float(np.float32(v))  # noqa: E731


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


def _compress(ev, tracks, params=None):
    """tpc_compress of ev's clusters with `tracks` (a Tracker after its launch,
    or gpu_inputs.DeviceTracks); host copies of the outputs."""
    from paper_2106_03636_amd.runtime import Batch, Compressor
    b = Batch.from_event(ev)
    cmp = Compressor(tracks, params)
    cmp.launch(b)
    g = cmp.result()
    return cmp, {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}


def _oracle_inputs(ev, o):
    """The oracle tracker's tracks as both sides take them."""
    from gpu_inputs import DeviceTracks
    dt = DeviceTracks.from_oracle(o)
    tl = o["track_tracklet"]
    host = dict(cluster_track=o["cluster_track"], params=o["trk_params"][tl].astype(np.float32),
                x_ref=o["trk_xref"][tl].astype(np.float32))
    return dt, host


def _check_codes(ev, cmp, host, g):
    """GPU codes against the oracle's on the same tracks."""
    cp = cmp.params
    k = F32(np.float32(-np.float32(synth.KAPPA) * np.float32(ev.bz)))
    o = oracle.compress(ev.y, ev.z, ev.row, host["cluster_track"], host["params"], host["x_ref"], ev.row_x, k,
                        F32(cp.step), F32(cp.pt_remove), F32(cp.sinphi_max))
    assert np.array_equal(g["cls"], o["cls"])
    frag = o["fragile"].astype(bool)
    differ = (g["code_y"] != o["code_y"]) | (g["code_z"] != o["code_z"])
    assert not (differ & ~frag).any(), np.nonzero(differ & ~frag)[0][:10]
    assert frag.sum() <= 1e-5 * len(frag) + 5  # residuals within 1e-6 of a half step are rare
    return o


def _check_tallies(cmp, g):
    """Histograms and class counts against the GPU's own codes."""
    h = cmp.params.hist_half
    a = g["cls"] == 1
    for f, hist, esc in (("code_y", g["hist_y"], g["counts"][4]), ("code_z", g["hist_z"], g["counts"][5])):
        c = g[f][a]
        inside = (c >= -h) & (c < h)
        assert np.array_equal(hist, np.bincount(c[inside] + h, minlength=2 * h))
        assert esc == (~inside).sum()
    assert g["counts"][:4].tolist() == np.bincount(g["cls"], minlength=4).tolist()


@pytest.mark.parametrize("name", ["pp_sector", "pbpb_central", "pbpb_timeframe_50"])
def test_codes_match_the_oracle(T, name):
    ev = cached_event(name)
    _say("case compression", name, ev.n, "clusters")
    dt, host = _oracle_inputs(ev, cached_oracle(name))
    cmp, g = _compress(ev, dt)
    _check_codes(ev, cmp, host, g)
    _check_tallies(cmp, g)
    c = g["counts"]
    _say("classes", c[:4].tolist(), "escapes", c[4:].tolist())
    assert c[1] > 0.5 * ev.n  # most clusters get residual codes
    if name.startswith("pbpb"):
        assert c[2] > 0  # the soft Pb-Pb spectrum has tracks below 0.1 GeV: their clusters go


@pytest.mark.parametrize("name", ["pbpb_central", "pbpb_timeframe_50"])
def test_codes_of_the_gpu_trackers_output(T, name):
    """GPU tracker -> compression, the configuration the benchmark times: the
    tallies match the codes, removal follows the tracks' q/pT, and the
    classes agree with those the oracle's tracks give on all but the few
    clusters whose track differs between the two trackers."""
    from paper_2106_03636_amd.runtime import Batch, Tracker
    ev = cached_event(name)
    _say("case compression after tracking", name, ev.n, "clusters")
    b = Batch.from_event(ev)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows)
    tr.launch(b)
    cmp, g = _compress(ev, tr)
    res = tr.result()
    _check_tallies(cmp, g)
    ct = res["cluster_track"].cpu().numpy()
    qpt = res["params"].cpu().numpy()[:, 4]
    removed = np.zeros(len(ct), bool)
    att = ct >= 0
    removed[att] = np.abs(qpt[ct[att]].astype(np.float64)) * F32(cmp.params.pt_remove) > 1.0
    assert np.array_equal(g["cls"] == 2, removed)
    assert np.array_equal(g["cls"] == 0, ~att)
    dt, host = _oracle_inputs(ev, cached_oracle(name))
    _, go = _compress(ev, dt)
    assert (g["cls"] != go["cls"]).mean() < 1e-3


def test_edge_cases(T):
    """No removal (pt_remove 0), a tiny histogram (most codes escape), a
    failed tracking call (its status passes through), an empty batch."""
    from paper_2106_03636_amd import make_compress_params
    from paper_2106_03636_amd.runtime import Batch, Compressor, Tracker, TrackingError
    ev = cached_event("pp_sector")
    dt, host = _oracle_inputs(ev, cached_oracle("pp_sector"))
    cmp, g = _compress(ev, dt, make_compress_params(pt_remove=0.0, hist_half=2))
    _check_codes(ev, cmp, host, g)
    _check_tallies(cmp, g)
    assert g["counts"][2] == 0 and g["counts"][4] > 0
    b = Batch.from_event(ev)
    small = Tracker(b.n, b.n_units, b.n_rows, cap_tracks=3)  # too small: TPC_E_CAPACITY
    small.launch(b)
    c = Compressor(small)
    c.launch(b)
    with pytest.raises(TrackingError) as e:
        c.result()
    assert e.value.status == T.TPC_E_CAPACITY
    eb = Batch(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.uint16), [0, 0], ev.row_x, ev.bz)
    te = Tracker(1, 1, eb.n_rows)
    te.launch(eb)
    ce = Compressor(te)
    ce.launch(eb)
    r = ce.result()
    assert r["counts"].tolist() == [0] * 6
