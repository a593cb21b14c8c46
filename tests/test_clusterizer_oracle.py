"""Pins of the oracle's clusterizer (orc_clusterize in oracle/tpc_oracle.c)
against facts fixed outside it: a dense-map implementation written here with
array shifts (a different algorithm: whole-map comparisons instead of
per-digit neighbour searches) on random digit sets full of ties, hand-worked
maps, and the generator's isolated clusters (one cluster each, centred on the
truth)."""
import numpy as np
import pytest

import oracle
import synth

Q_MIN = 10


def _oracle(half, off, time, q, n_units, q_min=Q_MIN):
    return oracle.clusterize(half, off, time, q, n_units, q_min, synth.PAD_W, synth.TIME_BIN, synth.Z_OFF)


def _csr(half, n_units, digits):
    """digits: list of (unit, row, pad, time, q) -> CSR arrays."""
    half = np.asarray(half, np.int32)
    pads_total = int(2 * half.sum())
    row_base = np.concatenate([[0], np.cumsum(2 * half)])
    digits = sorted(digits, key=lambda d: (d[0], row_base[d[1]] + d[2], d[3]))
    off = np.zeros(n_units * pads_total + 1, np.int64)
    for u, r, p, t, v in digits:
        off[u * pads_total + row_base[r] + p + 1] += 1
    off = np.cumsum(off)
    time = np.array([d[3] for d in digits], np.uint16)
    q = np.array([d[4] for d in digits], np.uint16)
    return off, time, q


def _dense(half, n_units, digits, q_min=Q_MIN):
    """Clusters by whole-map array operations, per (unit, row): a dense
    pads x times map, the peak mask from the eight shifted maps (ties go to the
    earlier digit in (pad, time) order), 3x3 sums by shifted adds."""
    half = np.asarray(half, np.int32)
    out = []
    by = {}
    for u, r, p, t, v in digits:
        by.setdefault((u, r), []).append((p, t, v))
    for (u, r) in sorted(by):
        ds = by[(u, r)]
        np_ = 2 * int(half[r])
        tmax = max(t for _, t, _ in ds) + 3
        M = np.full((np_ + 2, tmax + 2), -1, np.int64)  # -1: no digit; one cell of margin all round
        for p, t, v in ds:
            M[p + 1, t + 1] = v
        core = M[1:-1, 1:-1]
        peak = core >= q_min
        for dp in (-1, 0, 1):
            for dt in (-1, 0, 1):
                if dp == 0 and dt == 0:
                    continue
                N = M[1 + dp:M.shape[0] - 1 + dp, 1 + dt:M.shape[1] - 1 + dt]
                later = dp > 0 or (dp == 0 and dt > 0)
                ok = (N < core) | ((N == core) & later) | (N < 0)
                peak &= ok
        C = np.where(M < 0, 0, M)
        Q = np.zeros_like(core)
        Sp = np.zeros_like(core)
        St = np.zeros_like(core)
        for dp in (-1, 0, 1):
            for dt in (-1, 0, 1):
                N = C[1 + dp:C.shape[0] - 1 + dp, 1 + dt:C.shape[1] - 1 + dt]
                Q += N
                Sp += dp * N
                St += dt * N
        for p, t in zip(*np.nonzero(peak)):
            padf = p + Sp[p, t] / Q[p, t]
            timef = t + St[p, t] / Q[p, t]
            out.append((u, r, int(p), int(t), int(core[p, t]), int(Q[p, t]), int(Sp[p, t]), int(St[p, t]),
                        np.float32(padf), np.float32(timef),
                        np.float32((padf + 0.5 - half[r]) * synth.PAD_W),
                        np.float32((timef + 0.5) * synth.TIME_BIN - synth.Z_OFF)))
    return out


def _as_rows(c):
    return [tuple(x) for x in zip(c["unit"], c["row"], c["pad"], c["time"], c["qmax"], c["q"], c["sp"], c["st"],
                                  c["padf"], c["timef"], c["y"], c["z"])]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_matches_a_dense_map_implementation(seed):
    """Random digits on 2 units x 3 rows of 3-5 pads, charges 8-14 (many equal
    neighbours, plateaus, peaks at pad and row edges)."""
    rng = np.random.default_rng(seed)
    half = rng.integers(2, 4, 3)
    digits = set()
    for _ in range(400):
        u, r = int(rng.integers(0, 2)), int(rng.integers(0, 3))
        digits.add((u, r, int(rng.integers(0, 2 * half[r])), int(rng.integers(0, 30))))
    digits = [(u, r, p, t, int(rng.integers(8, 15))) for u, r, p, t in sorted(digits)]
    off, time, q = _csr(half, 2, digits)
    got = _as_rows(_oracle(half, off, time, q, 2))
    want = sorted(_dense(half, 2, digits), key=lambda c: (c[0], c[1], c[2], c[3]))
    assert len(want) > 20
    assert got == want


HALF = [3, 3]


def test_symmetric_cluster_is_centred():
    """A cross of equal wings around (pad 2, time 5): the centre is exactly the
    peak's pad and time, and y, z' are the pad and time-bin centres."""
    d = [(0, 0, 2, 5, 40), (0, 0, 1, 5, 10), (0, 0, 3, 5, 10), (0, 0, 2, 4, 12), (0, 0, 2, 6, 12),
         (0, 0, 1, 4, 3), (0, 0, 3, 6, 3)]
    c = _oracle(HALF, *_csr(HALF, 1, d), 1)
    assert c["n"] == 1
    assert (c["pad"][0], c["time"][0], c["qmax"][0], c["q"][0], c["sp"][0], c["st"][0]) == (2, 5, 40, 90, 0, 0)
    assert c["padf"][0] == 2.0 and c["timef"][0] == 5.0
    assert c["y"][0] == np.float32((2 + 0.5 - 3) * synth.PAD_W)
    assert c["z"][0] == np.float32((5 + 0.5) * synth.TIME_BIN - synth.Z_OFF)


def test_plateau_and_diagonal_ties_give_one_peak():
    """Equal charges: a 2x2 plateau has one peak, its first digit in (pad,
    time) order; of two equal diagonal neighbours the earlier is the peak."""
    d = [(0, 0, 1, 3, 20), (0, 0, 1, 4, 20), (0, 0, 2, 3, 20), (0, 0, 2, 4, 20),
         (0, 1, 1, 8, 30), (0, 1, 2, 9, 30)]
    c = _oracle(HALF, *_csr(HALF, 1, d), 1)
    assert list(zip(c["row"], c["pad"], c["time"])) == [(0, 1, 3), (1, 1, 8)]
    assert c["q"].tolist() == [80, 60] and c["sp"].tolist() == [40, 30] and c["st"].tolist() == [40, 30]


def test_neighbours_stay_in_their_row_pad_and_time_window():
    """The last pad of row 0 and the first pad of row 1 are next to each other
    in the digit order but not neighbours; digits two time bins apart are not
    neighbours; the peak threshold is q_min, inclusive."""
    d = [(0, 0, 5, 7, 20), (0, 1, 0, 7, 30),      # adjacent in CSR order, different rows: two peaks
         (0, 0, 0, 2, 15), (0, 0, 0, 4, 16),      # same pad, two bins apart: two peaks
         (0, 1, 3, 20, 9), (0, 1, 5, 20, 10)]     # below and at q_min
    c = _oracle(HALF, *_csr(HALF, 1, d), 1)
    got = set(zip(c["row"].tolist(), c["pad"].tolist(), c["time"].tolist()))
    assert got == {(0, 5, 7), (1, 0, 7), (0, 0, 2), (0, 0, 4), (1, 5, 20)}


def test_isolated_generated_clusters():
    """Clusters far apart (one per row), no noise, charge >= 100 ADC:
    each gives exactly one cluster, centred within 0.12 pads and 0.12 time bins
    of the generated position (the 3x3 centre of gravity of a Gaussian of
    width 0.7 bins is pulled towards the peak bin by at most ~0.1 bins), with a
    charge between 85% and 100% of the digits' total."""
    rng = np.random.default_rng(5)
    n = 150
    rows = np.arange(n) % synth.N_ROWS
    y = (rng.uniform(-0.8, 0.8, n) * synth.ROW_X[rows] * synth.TAN_HALF).astype(np.float32)
    z = rng.uniform(-200, 200, n).astype(np.float32)
    ev = synth.Event(y, z, rows.astype(np.uint16), np.array([0, n], np.int64), np.array([0], np.int16),
                     np.arange(n, dtype=np.int32), None, 0.5, "isolated")
    d = synth.event_digits(ev, 9, noise=0.0, charge_min=100.0)  # every peak well above q_min
    c = _oracle(synth.PAD_HALF, d.pad_offsets, d.time, d.q, 1)
    assert c["n"] == n and np.array_equal(c["row"], rows)
    pad_true = y / synth.PAD_W + synth.PAD_HALF[rows] - 0.5
    time_true = (z + synth.Z_OFF) / synth.TIME_BIN - 0.5
    assert np.abs(c["padf"] - pad_true).max() < 0.12
    assert np.abs(c["timef"] - time_true).max() < 0.12
    # each row holds one cluster's digits: its total
    row_of_digit = np.repeat(np.arange(synth.N_ROWS).repeat(2 * synth.PAD_HALF), np.diff(d.pad_offsets))
    totals = np.bincount(row_of_digit, weights=d.q, minlength=synth.N_ROWS)[rows]
    assert np.all(c["q"] <= totals) and np.all(c["q"] >= 0.85 * totals)
