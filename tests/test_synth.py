"""The seeded input generators (shared by the GPU path and the oracle): shapes
and determinism of the serving frame pool."""
import numpy as np

import synth


def _small_pool(seed=7):
    return synth.serving_pool(seed, n_frames=6, pbpb_collisions=(1, 2), pp_collisions=20, lib_pbpb=3, lib_pp=40)


def test_serving_pool_shapes():
    frames = _small_pool()
    assert len(frames) == 6
    for f in frames:
        assert f.n_units == synth.N_SECTORS
        assert f.unit_offsets[0] == 0 and f.unit_offsets[-1] == f.n
        assert np.all(np.diff(f.unit_offsets) >= 0)
        assert f.y.dtype == np.float32 and f.z.dtype == np.float32 and f.row.dtype == np.uint16
        assert int(f.row.max()) < synth.N_ROWS
        # clusters stay inside the sector acceptance of their row (smearing aside)
        hw = synth.ROW_X[f.row] * synth.TAN_HALF
        assert np.all(np.abs(f.y) <= hw + 1.0)
        sig = f.label >= 0
        assert 0.04 * sig.sum() <= (~sig).sum() <= 0.06 * sig.sum() + synth.N_SECTORS


def test_serving_pool_is_deterministic():
    a, b = _small_pool(11), _small_pool(11)
    for fa, fb in zip(a, b):
        assert fa.name == fb.name
        np.testing.assert_array_equal(fa.y, fb.y)
        np.testing.assert_array_equal(fa.z, fb.z)
        np.testing.assert_array_equal(fa.row, fb.row)


def test_composed_frame_shifts_z_by_drift_time():
    """A collision placed at time t0 appears at z - side * v_drift * t0."""
    rng = np.random.default_rng(3)
    lib = synth.collision_library(rng, [5])
    f = synth.compose_timeframe(np.random.default_rng(4), lib, [0], slice_us=100.0)
    t0 = np.random.default_rng(4).uniform(0.0, 100.0, 1)[0]
    for u in (0, 20):
        side = 1.0 if u < 18 else -1.0
        s = f.unit(u)
        m = f.label[s] >= 0
        a, b = lib.offsets[u], lib.offsets[u + 1]
        np.testing.assert_allclose(f.z[s][m], lib.z[a:b] - np.float32(side * synth.V_DRIFT * t0), rtol=0, atol=1e-3)
