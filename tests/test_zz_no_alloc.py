"""The entry point that allocates nothing (tpc_track_sectors_noalloc, through
the C ABI): its outputs equal those of tpc_track_sectors with a caller
workspace, bit for bit, on two calls in a row (the second one smaller, so
the scratch array holds the first call's contents when it starts); a batch
whose workspace exceeds the scratch array is refused with TPC_E_NOMEM and
the next call still works."""
import sys

import numpy as np
import pytest

from conftest import cached_event

pytestmark = pytest.mark.gpu

OUT_KEYS = ("cluster_track", "params", "cov", "x_ref", "chi2", "unit", "n_hits", "n_fit", "first_hit",
            "hits")


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


def _host(res):
    out = {k: res[k].cpu().numpy().copy() for k in OUT_KEYS}
    for k in ("n_tracks", "n_track_hits", "n_tracklets", "n_cells"):
        out[k] = res[k]
    return out


def _reference(ev):
    from paper_2106_03636_amd.runtime import Batch, Tracker
    b = Batch.from_event(ev)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows)
    tr.launch(b)
    return _host(tr.result())


def _fits(T, ev):
    from paper_2106_03636_amd import make_params
    need = T.tpc_workspace_size(ev.n, ev.n_units, len(ev.row_x), make_params())
    return 0 < need <= T.TPC_SCRATCH_BYTES


def test_noalloc_matches_the_workspace_entry_point(T):
    import torch
    from paper_2106_03636_amd.runtime import Batch, Tracker
    central = cached_event("pbpb_central")
    units = [0]
    while _fits(T, central.subset_units(units + [len(units)])):
        units.append(len(units))
    big = central.subset_units(units)
    small = cached_event("pp_sector")
    assert _fits(T, big) and small.n < big.n
    refs = [_reference(big), _reference(small)]
    nt = Tracker(big.n, big.n_units, len(big.row_x), workspace=False)
    assert nt.workspace is None
    for ev, ref in zip((big, small), refs):
        _say("noalloc call:", ev.name, ev.n, "clusters", ev.n_units, "units")
        b = Batch.from_event(ev)
        nt.o_cluster_track.fill_(-7)
        nt.launch(b)
        got = _host(nt.result())
        assert ref["n_tracks"] > 0
        for k, v in ref.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, got[k]), (ev.name, k)
            else:
                assert v == got[k], (ev.name, k)
    torch.cuda.synchronize()


def test_noalloc_refuses_a_batch_beyond_the_scratch_array(T):
    from paper_2106_03636_amd.runtime import Batch, Tracker, TrackingError
    central = cached_event("pbpb_central")
    assert not _fits(T, central)
    b = Batch.from_event(central)
    nt = Tracker(b.n, b.n_units, b.n_rows, workspace=False)
    with pytest.raises(TrackingError) as e:
        nt.launch(b)
    assert e.value.status == T.TPC_E_NOMEM
    small = cached_event("pp_sector")
    ref = _reference(small)
    nt.launch(Batch.from_event(small))
    got = _host(nt.result())
    assert np.array_equal(ref["cluster_track"], got["cluster_track"]) and ref["n_tracks"] == got["n_tracks"]
