"""Pins of the oracle's hit removal and track-model compression (orc_compress
in oracle/tpc_oracle.c) against facts fixed outside it: clusters on the
generator's closed-form helices have residual code 0 against the helix's own
state, displacements set by hand come back as their codes, the removal cut
and the rounding rule at hand-worked boundaries, and on a tracked event the
residual codes need far fewer bits than the positions."""
import math

import numpy as np
import pytest

import oracle
import synth

K = -synth.KAPPA * 0.5
STEP = 1.0 / 64


def _helix_case(n_tracks=60, seed=21, pt=(0.3, 5.0)):
    """Clusters of noise-free helices in sector 0 (first leg), each track's
    state taken at its innermost crossing."""
    rng = np.random.default_rng(seed)
    tr = synth.primaries_pp_sector(rng, n_tracks, 0, pt_range=pt)
    xs = synth.helix_crossings(tr, 0.5)
    m = (xs["sector"] == 0) & (xs["s"] < 300)
    y, z, row, trk = xs["y"][m], xs["z"][m], xs["row"][m], xs["track"][m]
    sp = xs["sinphi"][m]
    tracks = np.unique(trk)
    params, x_ref = [], []
    ct = np.full(len(y), -1, np.int32)
    for k, t in enumerate(tracks):
        idx = np.nonzero(trk == t)[0]
        i0 = idx[np.argmin(row[idx])]
        params.append([y[i0], z[i0], sp[i0], tr.tgl[t], tr.q[t] / tr.pt[t]])
        x_ref.append(synth.ROW_X[row[i0]])
        ct[idx] = k
    return (y.astype(np.float32), z.astype(np.float32), row.astype(np.uint16), ct,
            np.asarray(params, np.float32), np.asarray(x_ref, np.float32))


def test_clusters_on_the_helix_have_code_zero():
    """The state is rounded to FP32 (1e-7 relative) and so are the positions,
    which moves predictions by far less than half a step (0.0078 cm)."""
    y, z, row, ct, params, x_ref = _helix_case()
    # the states as FP32 values (what a tracking call writes); the generator's
    # z' is exact, so compare against the FP64 helix through the FP32 state
    r = oracle.compress(y, z, row, ct, params, x_ref, synth.ROW_X_F32, K, STEP)
    assert (r["cls"] == 1).all()
    assert np.abs(r["code_y"]).max() == 0 and np.abs(r["code_z"]).max() == 0


def test_displacements_come_back_as_codes():
    y, z, row, ct, params, x_ref = _helix_case(seed=22)
    rng = np.random.default_rng(3)
    dy = rng.integers(-40, 41, len(y))
    dz = rng.integers(-40, 41, len(y))
    # displaced by whole steps plus a fraction well inside the rounding interval
    y2 = (y.astype(np.float64) + (dy + 0.2) * STEP).astype(np.float32)
    z2 = (z.astype(np.float64) + (dz - 0.3) * STEP).astype(np.float32)
    r = oracle.compress(y2, z2, row, ct, params, x_ref, synth.ROW_X_F32, K, STEP)
    assert np.array_equal(r["code_y"], dy) and np.array_equal(r["code_z"], dz)


def test_removal_cut_and_unattached_rounding():
    """pT below pt_remove (0.1 GeV): |q/pT| = 10 stays, 10.01 goes; clusters
    of no track are coded by position, halves to even (2.5 -> 2, 3.5 -> 4)."""
    y = np.array([2.5 * STEP, 3.5 * STEP, -2.5 * STEP, 1.0, 1.0, 1.0], np.float32)
    z = np.array([0.0, -1.5 * STEP, 7.25 * STEP, 2.0, 2.0, 2.0], np.float32)
    row = np.array([0, 0, 0, 10, 10, 10], np.uint16)
    ct = np.array([-1, -1, -1, 0, 1, 2], np.int32)
    params = np.array([[1.0, 2.0, 0.0, 0.0, 10.0], [1.0, 2.0, 0.0, 0.0, 10.01], [1.0, 2.0, 0.0, 0.0, -10.01]],
                      np.float32)
    x_ref = np.full(3, synth.ROW_X_F32[10], np.float32)
    r = oracle.compress(y, z, row, ct, params, x_ref, synth.ROW_X_F32, K, STEP)
    assert r["cls"].tolist() == [0, 0, 0, 1, 2, 2]
    assert r["code_y"][:3].tolist() == [2, 4, -2] and r["code_z"][:3].tolist() == [0, -2, 7]
    assert r["code_y"][3] == 0 and r["code_z"][3] == 0  # its own plane: the state itself


def test_unreachable_row_and_fragile_flag():
    """A track that turns back before the cluster's row is coded by position
    (class 3).  A residual code within eps of a half step on a row the helix
    is carried to is flagged; one on the state's own plane (nothing carried)
    and a position code (one correctly rounded quotient) never are."""
    y = np.array([0.3, 5.5 * STEP, 1.0 + 2.5 * STEP, 1.0 + 2.5 * STEP], np.float32)
    z = np.array([0.0, 0.0, 2.0, 2.0], np.float32)
    row = np.array([150, 0, 10, 20], np.uint16)
    ct = np.array([0, -1, 1, 1], np.int32)
    params = np.array([[0.0, 0.0, 0.9, 0.0, -5.0],  # C = +0.0075/cm: sin(phi) passes 0.999 on the way
                       [1.0, 2.0, 0.0, 0.0, 0.0]], np.float32)  # straight, along x
    x_ref = np.array([synth.ROW_X_F32[0], synth.ROW_X_F32[10]], np.float32)
    r = oracle.compress(y, z, row, ct, params, x_ref, synth.ROW_X_F32, K, STEP, eps=1e-3)
    assert r["cls"].tolist() == [3, 0, 1, 1]
    assert r["code_y"][0] == round(0.3 / STEP)
    assert r["code_y"][2:].tolist() == [2, 2]  # 2.5 steps from the line, half to even
    assert r["fragile"].tolist() == [0, 0, 0, 1]


def _entropy(codes):
    _, c = np.unique(codes, return_counts=True)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def test_residuals_need_fewer_bits_than_positions():
    """Tracked pp sector: the residual codes of attached clusters carry under
    half the entropy of their position codes, in y and in z."""
    from conftest import cached_event, cached_oracle
    ev = cached_event("pp_sector")
    o = cached_oracle("pp_sector")
    kept = o["track_tracklet"]
    ct = np.full(ev.n, -1, np.int32)
    for t in range(o["n_tracks"]):
        hs = o["track_hits"][o["track_first_hit"][t]:o["track_first_hit"][t] + o["track_n_hits"][t]]
        ct[hs] = t
    r = oracle.compress(ev.y, ev.z, ev.row, ct, o["trk_params"][kept].astype(np.float32),
                        o["trk_xref"][kept].astype(np.float32), synth.ROW_X_F32, K, STEP)
    a = r["cls"] == 1
    assert a.sum() > 0.5 * ev.n
    pos = oracle.compress(ev.y, ev.z, ev.row, np.full(ev.n, -1, np.int32), np.zeros((0, 5), np.float32),
                          np.zeros(0, np.float32), synth.ROW_X_F32, K, STEP)
    for f in ("code_y", "code_z"):
        assert _entropy(r[f][a]) < 0.5 * _entropy(pos[f][a]), f
