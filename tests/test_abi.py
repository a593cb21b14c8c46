"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/tpc_track.h declares, sizes workspaces sanely and rejects bad
arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2106_03636_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tpc_track.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = T.load_library()
    names = _declared_functions()
    assert {"tpc_track_sectors", "tpc_workspace_size", "tpc_status_string", "tpc_inspect"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the structs have the sizes and field offsets the C
    compiler gives the header's structs."""
    import subprocess
    from paper_2106_03636_amd import server as S
    structs = {"tpc_clusters_t": T.tpc_clusters_t, "tpc_geometry_t": T.tpc_geometry_t,
               "tpc_field_t": T.tpc_field_t, "tpc_params_t": T.tpc_params_t,
               "tpc_tracks_t": T.tpc_tracks_t, "tpc_view_t": T.tpc_view_t,
               "tpc_collision_params_t": T.tpc_collision_params_t, "tpc_collisions_t": T.tpc_collisions_t,
               "tpc_pad_geometry_t": T.tpc_pad_geometry_t, "tpc_digits_t": T.tpc_digits_t,
               "tpc_clusterizer_params_t": T.tpc_clusterizer_params_t, "tpc_cluster_out_t": T.tpc_cluster_out_t,
               "tpc_compress_params_t": T.tpc_compress_params_t, "tpc_compressed_t": T.tpc_compressed_t,
               "tpc_refit_t": T.tpc_refit_t, "tpc_merge_params_t": T.tpc_merge_params_t,
               "tpc_merged_t": T.tpc_merged_t, "tpc_chain_fit_t": T.tpc_chain_fit_t,
               "tpc_server_config_t": S.tpc_server_config_t, "tpc_request_t": S.tpc_request_t,
               "tpc_result_t": S.tpc_result_t, "tpc_server_stats_t": S.tpc_server_stats_t}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tpc_track.h"', 'int main(void){']
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(cls, f).offset, (name, f)


def test_server_host_checks():
    """Serving calls that fail before any device work: bad configuration,
    footprint of impossible shapes."""
    from paper_2106_03636_amd import server as S
    p = T.make_params()
    assert S.tpc_server_footprint(1000, 1, 152, p) > S.tpc_server_footprint(10, 1, 152, p) > 0
    assert S.tpc_server_footprint(-1, 1, 152, p) == 0
    cfg = S.tpc_server_config_t()
    cfg.budget_bytes = 0  # no arena
    cfg.max_in_flight = 1
    cfg.queue_depth = 1
    cfg.n_rows = 152
    cfg.params = p
    st, h = S.tpc_server_create(cfg)
    assert st == T.TPC_E_INVALID and not h.value


def test_workspace_size_monotone_and_rejects_bad_shapes():
    p = T.make_params()
    a = T.tpc_workspace_size(1000, 1, 152, p)
    b = T.tpc_workspace_size(100000, 1, 152, p)
    c = T.tpc_workspace_size(100000, 36, 152, p)
    assert 0 < a < b < c
    assert T.tpc_workspace_size(0, 1, 152, p) > 0
    assert T.tpc_workspace_size(-1, 1, 152, p) == 0
    assert T.tpc_workspace_size(10, 0, 152, p) == 0
    assert T.tpc_workspace_size(10, 1, 2, p) == 0
    assert T.tpc_workspace_size(10, 1, 256, p) == 0
    assert T.tpc_workspace_size(1 << 30, 1, 152, p) == 0
    bad = T.make_params()
    bad.version = 99
    assert T.tpc_workspace_size(10, 1, 152, bad) == 0


def test_invalid_arguments_rejected_on_host():
    p = T.make_params()
    c, g, f, o = T.tpc_clusters_t(), T.tpc_geometry_t(), T.tpc_field_t(), T.tpc_tracks_t()
    assert T.tpc_track_sectors(c, g, f, p, o, 0, 0, 0) == T.TPC_E_INVALID
    c.n, c.n_units, c.unit_offsets = 10, 1, 0x1000
    c.y = c.z = c.row = 0x2000
    g.n_rows, g.row_x = 152, 0x3000
    f.bz_tesla = 0.5
    o.counts, o.status, o.cluster_track = 0x4000, 0x5000, 0x6000
    # misaligned workspace
    assert T.tpc_track_sectors(c, g, f, p, o, 0x7001, 1 << 30, 0) == T.TPC_E_INVALID
    # too small workspace
    assert T.tpc_track_sectors(c, g, f, p, o, 0x7000, 16, 0) == T.TPC_E_NOMEM
    bad = T.make_params(sinphi_max=1.5)
    assert T.tpc_track_sectors(c, g, f, bad, o, 0x7000, 1 << 30, 0) == T.TPC_E_INVALID
    g.n_rows = 300
    assert T.tpc_track_sectors(c, g, f, p, o, 0x7000, 1 << 30, 0) == T.TPC_E_INVALID


def test_collision_call_host_checks():
    """Workspace sizes and the arguments tpc_assign_collisions rejects before
    any device work."""
    cp = T.make_collision_params()
    ws = T.tpc_collisions_workspace_size(cp)
    assert ws >= 2 * 8192 * 16  # two int32 and one int64 per bin, 8192 bins per side
    assert T.tpc_collisions_workspace_size(T.make_collision_params(bin_width=2.0)) < ws
    for bad in (dict(bin_width=0.0), dict(z_range=-1.0), dict(bin_width=0.01, z_range=4096.0),
                dict(z_range=2.0e6, bin_width=100.0)):
        assert T.tpc_collisions_workspace_size(T.make_collision_params(**bad)) == 0, bad
    trk, out, f = T.tpc_tracks_t(), T.tpc_collisions_t(), T.tpc_field_t()
    f.bz_tesla = 0.5
    assert T.tpc_assign_collisions(trk, 0x1000, 36, f, cp, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    trk.params = trk.x_ref = trk.unit = trk.counts = trk.status = 0x2000
    trk.cap_tracks = 100
    out.cap = 16
    out.zdca = out.collision = out.side = out.bin = out.count = out.n_form = out.z = out.t0 = 0x3000
    out.n_collisions = out.status = 0x4000
    assert T.tpc_assign_collisions(trk, 0x1000, 36, f, cp, out, 0x8001, ws, 0) == T.TPC_E_INVALID  # misaligned
    assert T.tpc_assign_collisions(trk, 0x1000, 36, f, cp, out, 0x8000, ws - 1, 0) == T.TPC_E_NOMEM
    assert T.tpc_assign_collisions(trk, 0x1000, 0, f, cp, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    for bad in (dict(v_drift=0.0), dict(n_min=0), dict(reach=65), dict(reach=-1)):
        assert T.tpc_assign_collisions(trk, 0x1000, 36, f, T.make_collision_params(**bad), out, 0x8000,
                                       1 << 20, 0) == T.TPC_E_INVALID, bad


def test_clusterizer_host_checks():
    """Workspace sizes and the arguments tpc_clusterize rejects before any
    device work."""
    g = T.tpc_pad_geometry_t()
    g.n_rows, g.pads_total, g.half = 152, 14982, 0x1000
    g.pad_width, g.time_bin, g.z_offset = 0.6, 0.516, 4096.0
    ws = T.tpc_clusterize_workspace_size(36, g)
    assert ws >= 36 * 14982 * 4 and T.tpc_clusterize_workspace_size(1, g) < ws
    assert T.tpc_clusterize_workspace_size(0, g) == 0
    p = T.tpc_clusterizer_params_t()
    p.q_min = 10
    d, o = T.tpc_digits_t(), T.tpc_cluster_out_t()
    assert T.tpc_clusterize(d, g, p, o, 0x8000, ws, 0) == T.TPC_E_INVALID
    d.n, d.n_units, d.pad_offsets, d.time, d.q = 100, 36, 0x2000, 0x3000, 0x3000
    o.cap, o.unit_offsets, o.count, o.status = 10, 0x4000, 0x4000, 0x4000
    o.y = o.z = o.row = o.qtot = o.qmax = o.pad = o.time = 0x5000
    assert T.tpc_clusterize(d, g, p, o, 0x8001, ws, 0) == T.TPC_E_INVALID  # misaligned
    assert T.tpc_clusterize(d, g, p, o, 0x8000, ws - 1, 0) == T.TPC_E_NOMEM
    p.q_min = 0
    assert T.tpc_clusterize(d, g, p, o, 0x8000, ws, 0) == T.TPC_E_INVALID
    p.q_min = 10
    g.pad_width = 0.0
    assert T.tpc_clusterize(d, g, p, o, 0x8000, ws, 0) == T.TPC_E_INVALID


def test_refit_host_checks():
    """Workspace sizes and the arguments tpc_refit_tracks rejects before any
    device work."""
    ws = T.tpc_refit_workspace_size(100, 1000, 50000)
    assert ws >= 100 * 8 + 1000 * 4 + 50000 * 8
    assert T.tpc_refit_workspace_size(100, 1000, 40000) < ws and T.tpc_refit_workspace_size(0, 0, 0) > 0
    assert T.tpc_refit_workspace_size(200, 1000, 50000) > ws
    assert T.tpc_refit_workspace_size(10, -1, 10) == 0 and T.tpc_refit_workspace_size(10, 10, 1 << 40) == 0
    assert T.tpc_refit_workspace_size(1 << 30, 10, 10) == 0
    c, g, f, trk, out = T.tpc_clusters_t(), T.tpc_geometry_t(), T.tpc_field_t(), T.tpc_tracks_t(), T.tpc_refit_t()
    p = T.make_params()
    f.bz_tesla = 0.5
    c.n, c.n_units, c.y, c.z, c.row = 100, 1, 0x1000, 0x1000, 0x1000
    g.n_rows, g.row_x = 152, 0x1000
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    trk.cap_tracks, trk.cap_hits = 1000, 50000
    trk.n_hits = trk.first_hit = trk.hits = trk.counts = trk.status = 0x2000
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0x8000, ws, 0) == T.TPC_E_INVALID  # no outputs
    out.params = out.cov = out.x_ref = out.chi2 = out.params_out = out.cov_out = out.x_out = 0x3000
    out.ok = out.status = 0x4000
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0x8001, ws, 0) == T.TPC_E_INVALID  # misaligned
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0, ws, 0) == T.TPC_E_INVALID
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0x8000, ws - 1, 0) == T.TPC_E_NOMEM
    for bad in (dict(sinphi_max=1.0), dict(sigma_y=0.0), dict(cov0=[1.0, 1.0, 0.0, 1.0, 1.0])):
        assert T.tpc_refit_tracks(c, g, f, T.make_params(**bad), trk, out, 0x8000, ws, 0) == T.TPC_E_INVALID, bad
    g.n_rows = 2
    assert T.tpc_refit_tracks(c, g, f, p, trk, out, 0x8000, ws, 0) == T.TPC_E_INVALID


def test_merge_host_checks():
    """Workspace sizes and the arguments tpc_merge_tracks rejects before any
    device work."""
    mp = T.make_merge_params(cap_pairs=1000)
    ws = T.tpc_merge_workspace_size(36, 152, 5000, mp)
    assert ws >= 36 * 152 * 8 + 5000 * 36 + 1000 * 16
    assert T.tpc_merge_workspace_size(36, 152, 4000, mp) < ws
    assert T.tpc_merge_workspace_size(36, 152, 5000, T.make_merge_params(cap_pairs=2000)) > ws
    assert T.tpc_merge_workspace_size(0, 152, 5000, mp) == 0 and T.tpc_merge_workspace_size(36, 2, 5000, mp) == 0
    assert T.tpc_merge_workspace_size(36, 152, -1, mp) == 0
    c, g, f, trk, rf, out = (T.tpc_clusters_t(), T.tpc_geometry_t(), T.tpc_field_t(), T.tpc_tracks_t(),
                             T.tpc_refit_t(), T.tpc_merged_t())
    f.bz_tesla = 0.5
    c.n, c.row = 100, 0x1000
    g.n_rows, g.row_x = 152, 0x1000
    trk.cap_tracks = 5000
    trk.n_hits = trk.first_hit = trk.hits = trk.unit = trk.counts = trk.status = 0x2000
    for name in ("params", "cov", "x_ref", "params_out", "cov_out", "x_out", "ok", "status"):
        setattr(rf, name, 0x3000)
    args = lambda ws_ptr, ws_bytes, params=mp, n_units=36: (c, g, f, trk, rf, 0x4000, 0x4000, n_units, params, out,  # noqa: E731
                                                           ws_ptr, ws_bytes, 0)
    assert T.tpc_merge_tracks(*args(0x8000, ws)) == T.TPC_E_INVALID  # no outputs
    out.next = out.prev = out.link_chi2 = out.counts = out.status = 0x5000
    assert T.tpc_merge_tracks(*args(0x8001, ws)) == T.TPC_E_INVALID  # misaligned
    assert T.tpc_merge_tracks(*args(0, ws)) == T.TPC_E_INVALID
    assert T.tpc_merge_tracks(*args(0x8000, ws - 1)) == T.TPC_E_NOMEM
    assert T.tpc_merge_tracks(*args(0x8000, ws, n_units=0)) == T.TPC_E_INVALID
    for bad in (dict(max_gap=0), dict(max_gap=256), dict(chi2_max=0.0), dict(sinphi_max=1.0), dict(dz_max=-1.0),
                dict(dy_max=-1.0), dict(max_dalpha=-0.1)):
        assert T.tpc_merge_tracks(*args(0x8000, 1 << 30, params=T.make_merge_params(cap_pairs=1000, **bad))) == \
            T.TPC_E_INVALID, bad


def test_chain_fit_host_checks():
    """The arguments tpc_fit_chains rejects before any device work."""
    c, g, f, trk, mg, out = (T.tpc_clusters_t(), T.tpc_geometry_t(), T.tpc_field_t(), T.tpc_tracks_t(),
                             T.tpc_merged_t(), T.tpc_chain_fit_t())
    p = T.make_params()
    f.bz_tesla = 0.5
    c.n, c.y, c.z, c.row = 100, 0x1000, 0x1000, 0x1000
    g.n_rows, g.row_x = 152, 0x1000
    trk.cap_tracks = 50
    trk.n_hits = trk.first_hit = trk.hits = trk.unit = trk.counts = trk.status = 0x2000
    mg.next = mg.prev = mg.status = 0x3000
    trk.cap_hits = 2000
    ws = T.tpc_refit_workspace_size(100, 50, 2000)
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0x4000, 36, out, 0x8000, ws, 0) == T.TPC_E_INVALID  # no outputs
    out.params = out.cov = out.x_ref = out.chi2 = out.n_hits = out.ok = out.status = 0x5000
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0x4000, 0, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0, 36, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0x4000, 36, out, 0x8001, ws, 0) == T.TPC_E_INVALID  # misaligned
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0x4000, 36, out, 0x8000, ws - 1, 0) == T.TPC_E_NOMEM
    mg.prev = 0
    assert T.tpc_fit_chains(c, g, f, p, trk, mg, 0x4000, 36, out, 0x8000, ws, 0) == T.TPC_E_INVALID
    mg.prev = 0x3000
    for bad in (dict(sinphi_max=1.0), dict(sigma_z=0.0), dict(cov0=[1.0, 0.0, 1.0, 1.0, 1.0])):
        assert T.tpc_fit_chains(c, g, f, T.make_params(**bad), trk, mg, 0x4000, 36, out, 0x8000, ws, 0) == \
            T.TPC_E_INVALID, bad


def test_status_strings():
    for s in (T.TPC_OK, T.TPC_E_INVALID, T.TPC_E_CAPACITY, T.TPC_E_NOMEM, T.TPC_E_HIP, T.TPC_E_BUSY):
        assert T.tpc_status_string(s) and T.tpc_status_string(s) != "unknown status"
    assert T.tpc_status_string(12345) == "unknown status"


def test_product_path_has_no_oracle_dependency():
    """The library and its binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2106_03636_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn
                assert "tpc_oracle" not in txt, fn
