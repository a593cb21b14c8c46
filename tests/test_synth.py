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


def _helix_radius_at(tr, t, s, bz=0.5):
    """Distance from the beam axis at transverse arc length s (the generator's
    closed form of the helix, written out again here)."""
    C = tr.curvature(bz)[t]
    if C == 0.0:
        return np.hypot(tr.vx[t] + s * np.cos(tr.phi0[t]), tr.vy[t] + s * np.sin(tr.phi0[t]))
    R = 1.0 / C
    cx, cy = tr.vx[t] - R * np.sin(tr.phi0[t]), tr.vy[t] + R * np.cos(tr.phi0[t])
    phi = tr.phi0[t] + C * s
    return np.hypot(cx + R * np.sin(phi), cy - R * np.cos(phi))


def test_exit_at_the_outer_wall():
    """With r_exit the crossings are exactly those of the default (two turns)
    that come before the helix first leaves the cylinder r = r_exit, found by
    a scan of the distance along the helix; loopers that stay inside keep both
    turns.  The default is unchanged."""
    rng = np.random.default_rng(21)
    tr = synth.primaries_pbpb(rng, 400)
    full = synth.helix_crossings(tr, 0.5)
    cut = synth.helix_crossings(tr, 0.5, r_exit=synth.R_EXIT)
    again = synth.helix_crossings(tr, 0.5, r_exit=0.0)
    for k in full:
        np.testing.assert_array_equal(full[k], again[k])
    kept = set(zip(cut["track"].tolist(), cut["sector"].tolist(), cut["row"].tolist(), np.round(cut["s"], 9)))
    n_loopers = n_cut = 0
    for t in range(len(tr)):
        m = full["track"] == t
        if not m.any():
            continue
        s_max = full["s"][m].max()
        ss = np.arange(0.0, s_max + 0.05, 0.02)
        out = np.nonzero(_helix_radius_at(tr, t, ss) > synth.R_EXIT)[0]
        s_exit = ss[out[0]] if len(out) else np.inf
        for i in np.nonzero(m)[0]:
            key = (t, int(full["sector"][i]), int(full["row"][i]), np.round(full["s"][i], 9))
            if abs(full["s"][i] - s_exit) < 0.05:
                continue  # within the scan's step of the exit
            assert (key in kept) == (full["s"][i] < s_exit), (t, full["s"][i], s_exit)
        n_loopers += not len(out)
        n_cut += (full["s"][m] > s_exit).any()
    assert n_loopers > 50 and n_cut > 20
    assert len(cut["s"]) < len(full["s"])


def test_physical_frame_has_one_vertex_per_collision():
    ev = synth.event_pbpb_timeframe(5, n_collisions=3, physical=True)
    tr = ev.tracks
    for t0 in np.unique(tr.t0):
        m = tr.t0 == t0
        assert np.ptp(tr.vz[m]) == 0.0 and np.ptp(tr.vx[m]) == 0.0
    assert len(np.unique(tr.vz)) == 3
