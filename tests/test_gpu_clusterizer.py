"""The clusterizer on the GPU (tpc_clusterize through the C ABI) against the
oracle (orc_clusterize): bit for bit, since peaks and charge sums are integer
and the centre and position are the same FP64 expressions rounded once to
FP32.  Cases: the oracle pins' random digit sets full of ties and the
hand-worked maps, digits of a pp sector, of a central Pb-Pb collision and of
the 50-collision slice at full size; edge cases; and the chain digits ->
clusters -> tracks against the oracle's chain."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

Q_MIN = 10
# the geometry reaches the kernels as FP32 values: the oracle gets the same values
PW, TB, ZOFF = (float(np.float32(v)) for v in (synth.PAD_W, synth.TIME_BIN, synth.Z_OFF))


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


def _gpu(half, off, time, q, n_units, cap=None, q_min=Q_MIN):
    import torch
    from paper_2106_03636_amd.runtime import Clusterizer
    c = Clusterizer(half, PW, TB, ZOFF, n_units, cap if cap is not None else max(1, len(time)), q_min=q_min)
    dev = torch.device("cuda")
    t = torch.as_tensor(np.ascontiguousarray(time, np.uint16).view(np.int16)).to(dev)
    qq = torch.as_tensor(np.ascontiguousarray(q, np.uint16).view(np.int16)).to(dev)
    o = torch.as_tensor(np.ascontiguousarray(off, np.int64)).to(dev)
    c.launch(t, qq, o, n_units)
    return c


def _host(r):
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}
    out["row"] = out["row"].view(np.uint16)
    out["qmax"] = out["qmax"].view(np.uint16)
    return out


def _compare(g, o, half, n_units):
    assert g["n"] == o["n"]
    assert np.array_equal(g["row"].astype(np.int32), o["row"])
    assert np.array_equal(g["qmax"].astype(np.int32), o["qmax"])
    assert np.array_equal(g["qtot"], o["q"])
    for a, b in (("pad", "padf"), ("time", "timef"), ("y", "y"), ("z", "z")):
        assert np.array_equal(g[a].view(np.uint32), o[b].view(np.uint32)), a  # bit for bit
    uo = np.searchsorted(o["unit"], np.arange(n_units + 1), side="left")
    assert np.array_equal(g["unit_offsets"], uo)


def _case(half, off, time, q, n_units):
    c = _gpu(half, off, time, q, n_units)
    g = _host(c.result())
    o = oracle.clusterize(half, off, time, q, n_units, Q_MIN, PW, TB, ZOFF)
    _compare(g, o, half, n_units)
    return g


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_digit_sets(T, seed):
    import test_clusterizer_oracle as P
    rng = np.random.default_rng(seed)
    half = rng.integers(2, 4, 3).astype(np.int32)
    digits = set()
    for _ in range(400):
        u, r = int(rng.integers(0, 2)), int(rng.integers(0, 3))
        digits.add((u, r, int(rng.integers(0, 2 * half[r])), int(rng.integers(0, 30))))
    digits = [(u, r, p, t, int(rng.integers(8, 15))) for u, r, p, t in sorted(digits)]
    off, time, q = P._csr(half, 2, digits)
    g = _case(half, off, time, q, 2)
    assert g["n"] > 20


def test_hand_worked_maps(T):
    import test_clusterizer_oracle as P
    half = np.array(P.HALF, np.int32)
    cases = [
        [(0, 0, 2, 5, 40), (0, 0, 1, 5, 10), (0, 0, 3, 5, 10), (0, 0, 2, 4, 12), (0, 0, 2, 6, 12),
         (0, 0, 1, 4, 3), (0, 0, 3, 6, 3)],
        [(0, 0, 1, 3, 20), (0, 0, 1, 4, 20), (0, 0, 2, 3, 20), (0, 0, 2, 4, 20), (0, 1, 1, 8, 30), (0, 1, 2, 9, 30)],
        [(0, 0, 5, 7, 20), (0, 1, 0, 7, 30), (0, 0, 0, 2, 15), (0, 0, 0, 4, 16), (0, 1, 3, 20, 9), (0, 1, 5, 20, 10)],
    ]
    want = [[(0, 2, 5)], [(0, 1, 3), (1, 1, 8)], [(0, 0, 2), (0, 0, 4), (0, 5, 7), (1, 0, 7), (1, 5, 20)]]
    for d, w in zip(cases, want):
        g = _case(half, *P._csr(half, 1, d), 1)
        assert g["n"] == len(w) and g["row"].tolist() == [x[0] for x in w]


@pytest.mark.parametrize("name", ["pp_sector", "pbpb_central", "pbpb_timeframe_50"])
def test_generated_digits(T, name):
    ev = synth.WORKLOADS[name]()
    d = synth.event_digits(ev, 7)
    _say("case clusterizer", name, d.n, "digits", ev.n_units, "units")
    g = _case(synth.PAD_HALF, d.pad_offsets, d.time, d.q, d.n_units)
    _say("clusters", g["n"])
    assert g["n"] > 0.7 * ev.n


def test_edge_cases(T):
    """No digits; empty units between full ones; times that do not increase
    inside a pad (rejected on the device); more clusters than the capacity
    (reported with the count); one clusterizer used twice, the second batch
    smaller."""
    from paper_2106_03636_amd.runtime import TrackingError
    import test_clusterizer_oracle as P
    half = np.array([3, 3], np.int32)
    off = np.zeros(3 * 12 + 1, np.int64)
    g = _host(_gpu(half, off, np.zeros(0, np.uint16), np.zeros(0, np.uint16), 3).result())
    assert g["n"] == 0 and g["unit_offsets"].tolist() == [0, 0, 0, 0]
    d = [(0, 0, 2, 5, 40), (2, 1, 3, 9, 25), (2, 1, 4, 9, 11)]
    g = _case(half, *P._csr(half, 3, d), 3)
    assert g["n"] == 2 and g["unit_offsets"].tolist() == [0, 1, 1, 2]
    off, time, q = P._csr(half, 1, [(0, 0, 2, 5, 40), (0, 0, 2, 6, 30)])
    time = time[::-1].copy()  # 6 then 5 in one pad
    c = _gpu(half, off, time, q, 1)
    with pytest.raises(TrackingError) as e:
        c.result()
    assert e.value.status == T.TPC_E_INVALID
    off, time, q = P._csr(half, 1, [(0, 0, p, t, 20) for p in range(0, 6, 2) for t in range(0, 20, 3)])
    c = _gpu(half, off, time, q, 1, cap=5)
    with pytest.raises(TrackingError) as e:
        c.result()
    assert e.value.status == T.TPC_E_CAPACITY and int(c.o_count.item()) == 21
    import torch
    big = [(0, r, p, t, 20) for r in range(2) for p in range(0, 6, 2) for t in range(0, 40, 3)]
    c = _gpu(half, *P._csr(half, 1, big), 1)
    first = _host(c.result())
    small = big[:10]
    off, time, q = P._csr(half, 1, small)
    dev = torch.device("cuda")
    c.launch(torch.as_tensor(time.view(np.int16)).to(dev), torch.as_tensor(q.view(np.int16)).to(dev),
             torch.as_tensor(off).to(dev), 1)
    second = _host(c.result())
    assert first["n"] == len(big) and second["n"] == 10
    o = oracle.clusterize(half, off, time, q, 1, Q_MIN, PW, TB, ZOFF)
    _compare(second, o, half, 1)


def test_digits_to_tracks_chain(T):
    """The chain on the GPU (clusterize, then track the clusters it wrote, on
    the device) against the oracle's chain (oracle clusters, oracle tracking),
    at the parity bars of the tracker, on the central Pb-Pb collision."""
    import parity
    from paper_2106_03636_amd.params import DEFAULT_PARAMS
    from paper_2106_03636_amd.runtime import Tracker
    ev = synth.WORKLOADS["pbpb_central"]()
    d = synth.event_digits(ev, 7)
    from paper_2106_03636_amd.runtime import Clusterizer
    t, q, off = Clusterizer.upload(d)
    c = Clusterizer(synth.PAD_HALF, PW, TB, ZOFF, d.n_units, d.n)
    c.launch(t, q, off, d.n_units)
    b = c.batch(ev.row_x, ev.bz)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows)
    tr.launch(b)
    res = tr.result()
    oc = oracle.clusterize(synth.PAD_HALF, d.pad_offsets, d.time, d.q, d.n_units, Q_MIN, PW, TB, ZOFF)
    cev = synth.Event(oc["y"], oc["z"], oc["row"].astype(np.uint16),
                      np.searchsorted(oc["unit"], np.arange(d.n_units + 1)).astype(np.int64), ev.unit_sector,
                      np.full(oc["n"], -1, np.int32), ev.tracks, ev.bz, "central_clusters")
    o = oracle.run_event(cev, DEFAULT_PARAMS, fragile_eps=0.05)
    g = parity.gpu_state(tr, res)
    rep = parity.compare(g, o)
    _say("chain parity", {k: v for k, v in rep.items() if k != "failures"})
    assert rep.ok, rep.get("failures")
    assert res["n_tracks"] > 10000
