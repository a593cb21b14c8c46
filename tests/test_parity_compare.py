"""The element-by-element comparison itself (tests/parity.py), on the CPU: a
GPU-shaped state built from the oracle's own result passes every clause, and
each kind of planted difference (a hit set, an owner key, the cluster-to-track
map, a link, the grid order) is reported."""
import numpy as np
import pytest

from conftest import cached_event, cached_oracle
from paper_2106_03636_amd.params import DEFAULT_PARAMS as P


def state_from_oracle(o, n_rows):
    """The oracle's result laid out the way parity.gpu_state lays out the GPU's."""
    K = o["n_tracklets"]
    g = {k: o[k].copy() for k in ("perm", "up", "dn", "upc", "dnc", "owner")}
    g["cell"] = o["cell_start"].copy()
    S = len(o["seg_start"])
    seg = np.zeros((S, 12), np.int32)
    for j, f in enumerate(["seg_start", "seg_count", "seg_zmin", "seg_zmax", None, "seg_by", "seg_ny",
                           "seg_bz", "seg_nz", "seg_cell_base"]):
        if f is not None:
            seg[:, j] = o[f]
    g["seg"] = seg
    for k in ("trk_start", "trk_unit", "trk_len", "trk_nfit", "trk_p1n", "trk_owned", "trk_keep", "trk_key"):
        g[k] = o[k].copy()
    g["trk_params"] = o["trk_params"].astype(np.float32)
    g["trk_cov"] = o["trk_cov"].astype(np.float32)
    g["trk_xref"] = o["trk_xref"].astype(np.float32)
    g["trk_chi2"] = o["trk_chi2"].astype(np.float32)
    seeds = np.nonzero(o["trk_len"] >= P["l_min"])[0]
    g["seed_list"] = seeds.copy()
    g["seeds_expected"] = seeds
    # row of each sorted position: segments are (unit, row) ranges in order
    row_of = np.repeat(np.tile(np.arange(n_rows), S // n_rows), o["seg_count"])
    hits = np.full((len(seeds), n_rows), -1, np.int32)
    rlo = np.full(K, -1, np.int32)
    rhi = np.full(K, -1, np.int32)
    for j, t in enumerate(seeds):
        h = o["trk_hits"][t, :o["trk_nfit"][t]]
        if len(h):
            r = row_of[h]
            hits[j, r] = h
            rlo[t], rhi[t] = r.min(), r.max()
    g["seed_hits"] = hits
    g["trk_rlo"], g["trk_rhi"] = rlo, rhi
    for k in ("n_tracks", "n_track_hits", "n_tracklets", "n_cells"):
        g[k] = o[k]
    kept = o["track_tracklet"]
    g["out_cluster_track"] = o["cluster_track"].copy()
    g["out_params"] = g["trk_params"][kept]
    g["out_hits"] = o["track_hits"].copy()
    g["out_n_hits"] = o["track_n_hits"].copy()
    g["out_first_hit"] = o["track_first_hit"].copy()
    return g


@pytest.fixture(scope="module")
def case():
    ev = cached_event("pbpb_central")
    sub = ev.subset_units([3, 20])
    import oracle
    o = oracle.run_event(sub, P, fragile_eps=0.05)
    return o, sub.row_x.shape[0]


def test_oracle_state_passes(case):
    import parity
    o, nr = case
    rep = parity.compare(state_from_oracle(o, nr), o)
    assert rep.ok, rep.get("failures")
    assert rep["n_hitset_diff"] == 0 and rep["matched_fraction"] == 1.0 and rep["n_affected"] == 0
    assert rep["n_fitted"] > 1000


def _unflagged_fitted(o, n=1):
    t = np.nonzero((o["trk_nfit"] > 5) & (o["trk_fragile"] == 0) & (o["trk_keep"] == 1))[0]
    return t[:n]


def test_planted_hit_set_difference_is_reported(case):
    import parity
    o, nr = case
    g = state_from_oracle(o, nr)
    t = int(_unflagged_fitted(o)[0])
    j = int(np.searchsorted(g["seeds_expected"], t))
    row = int(np.nonzero(g["seed_hits"][j] >= 0)[0][2])
    g["seed_hits"][j, row] = -1  # one hit dropped, nfit unchanged
    rep = parity.compare(g, o)
    assert not rep.ok and rep["n_hitset_diff"] == 1
    assert any("not flagged fragile" in f for f in rep["failures"])
    # a different hit in the same row, same count
    g = state_from_oracle(o, nr)
    g["seed_hits"][j, row] += 1
    rep = parity.compare(g, o)
    assert not rep.ok and rep["n_hitset_diff"] == 1


def test_planted_first_pass_count_difference_is_reported(case):
    import parity
    o, nr = case
    g = state_from_oracle(o, nr)
    t = int(_unflagged_fitted(o)[0])
    g["trk_p1n"][t] += 1  # same final hits, a different first pass
    rep = parity.compare(g, o)
    assert not rep.ok and rep["n_hitset_diff"] == 1


def test_planted_ownership_and_output_differences_are_reported(case):
    import parity
    o, nr = case
    g = state_from_oracle(o, nr)
    h = int(o["track_hits"][0])
    pos = int(np.nonzero(o["perm"] == h)[0][0])
    g["owner"][pos] ^= 1
    rep = parity.compare(g, o)
    assert not rep.ok and any("owner" in f for f in rep["failures"])
    g = state_from_oracle(o, nr)
    g["out_cluster_track"][h] = -1
    rep = parity.compare(g, o)
    assert not rep.ok and any("cluster_track" in f for f in rep["failures"])
    g = state_from_oracle(o, nr)
    g["trk_keep"][int(o["track_tracklet"][0])] = 0
    rep = parity.compare(g, o)
    assert not rep.ok and any("selection" in f for f in rep["failures"])


def test_planted_grid_and_link_differences_are_reported(case):
    import parity
    o, nr = case
    for k in ("perm", "up", "upc"):
        g = state_from_oracle(o, nr)
        i = int(np.nonzero(g[k] >= 0)[0][5])
        g[k][i], g[k][i + 1] = g[k][i + 1], g[k][i]
        if g[k][i] == g[k][i + 1]:
            g[k][i] = -1
        rep = parity.compare(g, o)
        assert not rep.ok and any(k in f for f in rep["failures"]), k
    g = state_from_oracle(o, nr)
    g["cell"][10] += 1
    assert not parity.compare(g, o).ok
