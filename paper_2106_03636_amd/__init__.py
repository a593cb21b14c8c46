"""MI355X TPC sector track finder: Python binding of the C ABI in include/tpc_track.h.

The functions here carry the C names and only marshal arguments: every step
of the tracking runs in the HIP kernels of `_tpctrack.so`.  torch provides
device memory and streams.  There is no CPU fallback: if the library is not
built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

from .params import DEFAULT_PARAMS

HERE = os.path.dirname(os.path.abspath(__file__))
# TPC_TRACK_LIB: another build of the library to load instead of the in-tree one
LIB_PATH = os.environ.get("TPC_TRACK_LIB") or os.path.join(HERE, "_tpctrack.so")

TPC_PARAMS_VERSION = 1
TPC_OK, TPC_E_INVALID, TPC_E_CAPACITY, TPC_E_NOMEM, TPC_E_HIP, TPC_E_BUSY = 0, -1, -2, -3, -4, -5
TPC_SCRATCH_BYTES = 64 << 20

(TPC_VIEW_PERM, TPC_VIEW_CELL, TPC_VIEW_SEG, TPC_VIEW_UP, TPC_VIEW_DN, TPC_VIEW_UPC, TPC_VIEW_DNC,
 TPC_VIEW_OWNER, TPC_VIEW_TRK_START, TPC_VIEW_TRK_UNIT, TPC_VIEW_TRK_LEN, TPC_VIEW_TRK_NFIT,
 TPC_VIEW_TRK_RLO, TPC_VIEW_TRK_RHI, TPC_VIEW_TRK_KEY, TPC_VIEW_TRK_OWNED, TPC_VIEW_TRK_KEEP,
 TPC_VIEW_TRK_PARAMS, TPC_VIEW_TRK_COV, TPC_VIEW_TRK_XREF, TPC_VIEW_TRK_CHI2,
 TPC_VIEW_TRK_HITS, TPC_VIEW_SEED_LIST, TPC_VIEW_TRK_P1N) = range(1, 25)

_vp = ctypes.c_void_p


class tpc_clusters_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_units", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("unit_offsets", _vp), ("y", _vp), ("z", _vp), ("row", _vp)]


class tpc_geometry_t(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("reserved", ctypes.c_int32), ("row_x", _vp)]


class tpc_field_t(ctypes.Structure):
    _fields_ = [("bz_tesla", ctypes.c_float)]


class tpc_params_t(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("q_shift", ctypes.c_int32),
                ("tan_half_q16", ctypes.c_int32), ("bin_y_q", ctypes.c_int32),
                ("bin_occ", ctypes.c_int32), ("bin_zmin_q", ctypes.c_int32),
                ("win_y_q", ctypes.c_int32), ("win_z_q", ctypes.c_int32),
                ("w_y", ctypes.c_int32), ("w_z", ctypes.c_int32), ("smax_k", ctypes.c_int64),
                ("l_min", ctypes.c_int32), ("ext_win_y_q", ctypes.c_int32),
                ("ext_win_z_q", ctypes.c_int32), ("ext_edge_q", ctypes.c_int32),
                ("max_miss", ctypes.c_int32), ("n_min", ctypes.c_int32),
                ("f_min_q8", ctypes.c_int32), ("tracklet_cap_div", ctypes.c_int32),
                ("sinphi_max", ctypes.c_float), ("sigma_y", ctypes.c_float),
                ("sigma_z", ctypes.c_float), ("cov0", ctypes.c_float * 5),
                ("reserved", ctypes.c_int32)]


class tpc_tracks_t(ctypes.Structure):
    _fields_ = [("cap_tracks", ctypes.c_int64), ("cap_hits", ctypes.c_int64),
                ("cluster_track", _vp), ("params", _vp), ("cov", _vp), ("x_ref", _vp),
                ("chi2", _vp), ("unit", _vp), ("n_hits", _vp), ("n_fit", _vp),
                ("first_hit", _vp), ("hits", _vp), ("counts", _vp), ("status", _vp)]


class tpc_collision_params_t(ctypes.Structure):
    _fields_ = [("v_drift", ctypes.c_float), ("bin_width", ctypes.c_float), ("z_range", ctypes.c_float),
                ("c_max", ctypes.c_float), ("n_min", ctypes.c_int32), ("reach", ctypes.c_int32)]


class tpc_collisions_t(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("zdca", _vp), ("collision", _vp), ("side", _vp), ("bin", _vp),
                ("count", _vp), ("n_form", _vp), ("z", _vp), ("t0", _vp), ("n_collisions", _vp),
                ("status", _vp)]


class tpc_pad_geometry_t(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("pads_total", ctypes.c_int32), ("half", _vp),
                ("pad_width", ctypes.c_float), ("time_bin", ctypes.c_float), ("z_offset", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class tpc_digits_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_units", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pad_offsets", _vp), ("time", _vp), ("q", _vp)]


class tpc_clusterizer_params_t(ctypes.Structure):
    _fields_ = [("q_min", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tpc_cluster_out_t(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("y", _vp), ("z", _vp), ("row", _vp), ("qtot", _vp), ("qmax", _vp),
                ("pad", _vp), ("time", _vp), ("unit_offsets", _vp), ("count", _vp), ("status", _vp)]


class tpc_compress_params_t(ctypes.Structure):
    _fields_ = [("step", ctypes.c_float), ("pt_remove", ctypes.c_float), ("sinphi_max", ctypes.c_float),
                ("hist_half", ctypes.c_int32)]


class tpc_compressed_t(ctypes.Structure):
    _fields_ = [("cls", _vp), ("code_y", _vp), ("code_z", _vp), ("hist", _vp), ("counts", _vp), ("status", _vp)]


class tpc_refit_t(ctypes.Structure):
    _fields_ = [("params", _vp), ("cov", _vp), ("x_ref", _vp), ("chi2", _vp), ("params_out", _vp),
                ("cov_out", _vp), ("x_out", _vp), ("ok", _vp), ("status", _vp)]


class tpc_merge_params_t(ctypes.Structure):
    _fields_ = [("cap_pairs", ctypes.c_int64), ("max_dalpha", ctypes.c_float), ("max_gap", ctypes.c_int32),
                ("dz_max", ctypes.c_float), ("dy_max", ctypes.c_float), ("chi2_max", ctypes.c_float),
                ("sinphi_max", ctypes.c_float)]


class tpc_merged_t(ctypes.Structure):
    _fields_ = [("next", _vp), ("prev", _vp), ("link_chi2", _vp), ("counts", _vp), ("status", _vp)]


class tpc_chain_fit_t(ctypes.Structure):
    _fields_ = [("params", _vp), ("cov", _vp), ("x_ref", _vp), ("chi2", _vp), ("n_hits", _vp), ("ok", _vp),
                ("status", _vp)]


class tpc_view_t(ctypes.Structure):
    _fields_ = [("ptr", _vp), ("count", ctypes.c_int64), ("elem_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def load_library():
    """Load the HIP library.  Raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built (run __graft_entry__.build() or "
                               "python paper_2106_03636_amd/build.py)" % LIB_PATH)
        import torch  # noqa: F401  -- share torch's HIP runtime
        lib = ctypes.CDLL(LIB_PATH)
        lib.tpc_workspace_size.restype = ctypes.c_size_t
        lib.tpc_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(tpc_params_t)]
        lib.tpc_track_sectors.restype = ctypes.c_int
        lib.tpc_track_sectors.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                          ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_params_t),
                                          ctypes.POINTER(tpc_tracks_t), _vp, ctypes.c_size_t, _vp]
        lib.tpc_track_sectors_profiled.restype = ctypes.c_int
        lib.tpc_track_sectors_profiled.argtypes = lib.tpc_track_sectors.argtypes + [
            ctypes.POINTER(_vp), ctypes.c_int32]
        lib.tpc_track_sectors_noalloc.restype = ctypes.c_int
        lib.tpc_track_sectors_noalloc.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                                  ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_params_t),
                                                  ctypes.POINTER(tpc_tracks_t), _vp]
        lib.tpc_kernel_count.restype = ctypes.c_int32
        lib.tpc_kernel_name.restype = ctypes.c_char_p
        lib.tpc_kernel_name.argtypes = [ctypes.c_int32]
        lib.tpc_status_string.restype = ctypes.c_char_p
        lib.tpc_status_string.argtypes = [ctypes.c_int]
        lib.tpc_collisions_workspace_size.restype = ctypes.c_size_t
        lib.tpc_collisions_workspace_size.argtypes = [ctypes.POINTER(tpc_collision_params_t)]
        lib.tpc_assign_collisions.restype = ctypes.c_int
        lib.tpc_assign_collisions.argtypes = [ctypes.POINTER(tpc_tracks_t), _vp, ctypes.c_int32,
                                              ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_collision_params_t),
                                              ctypes.POINTER(tpc_collisions_t), _vp, ctypes.c_size_t, _vp]
        lib.tpc_clusterize_workspace_size.restype = ctypes.c_size_t
        lib.tpc_clusterize_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(tpc_pad_geometry_t)]
        lib.tpc_clusterize.restype = ctypes.c_int
        lib.tpc_clusterize.argtypes = [ctypes.POINTER(tpc_digits_t), ctypes.POINTER(tpc_pad_geometry_t),
                                       ctypes.POINTER(tpc_clusterizer_params_t), ctypes.POINTER(tpc_cluster_out_t),
                                       _vp, ctypes.c_size_t, _vp]
        lib.tpc_compress.restype = ctypes.c_int
        lib.tpc_compress.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                     ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_tracks_t),
                                     ctypes.POINTER(tpc_compress_params_t), ctypes.POINTER(tpc_compressed_t), _vp]
        lib.tpc_refit_workspace_size.restype = ctypes.c_size_t
        lib.tpc_refit_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.tpc_refit_tracks.restype = ctypes.c_int
        lib.tpc_refit_tracks.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                         ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_params_t),
                                         ctypes.POINTER(tpc_tracks_t), ctypes.POINTER(tpc_refit_t), _vp,
                                         ctypes.c_size_t, _vp]
        lib.tpc_merge_workspace_size.restype = ctypes.c_size_t
        lib.tpc_merge_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.POINTER(tpc_merge_params_t)]
        lib.tpc_merge_tracks.restype = ctypes.c_int
        lib.tpc_merge_tracks.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                         ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_tracks_t),
                                         ctypes.POINTER(tpc_refit_t), _vp, _vp, ctypes.c_int32,
                                         ctypes.POINTER(tpc_merge_params_t), ctypes.POINTER(tpc_merged_t), _vp,
                                         ctypes.c_size_t, _vp]
        lib.tpc_fit_chains.restype = ctypes.c_int
        lib.tpc_fit_chains.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.POINTER(tpc_geometry_t),
                                       ctypes.POINTER(tpc_field_t), ctypes.POINTER(tpc_params_t),
                                       ctypes.POINTER(tpc_tracks_t), ctypes.POINTER(tpc_merged_t), _vp,
                                       ctypes.c_int32, ctypes.POINTER(tpc_chain_fit_t), _vp, ctypes.c_size_t, _vp]
        lib.tpc_inspect.restype = ctypes.c_int
        lib.tpc_inspect.argtypes = [ctypes.POINTER(tpc_clusters_t), ctypes.c_int32,
                                    ctypes.POINTER(tpc_params_t), _vp, ctypes.c_int,
                                    ctypes.POINTER(tpc_view_t)]
        _lib = lib
    return _lib


def make_params(values: dict | None = None, **overrides) -> tpc_params_t:
    """C parameter block from a dict of values (defaults: DEFAULT_PARAMS)."""
    v = dict(DEFAULT_PARAMS if values is None else values)
    v.update(overrides)
    p = tpc_params_t()
    p.version = TPC_PARAMS_VERSION
    for name in ("q_shift", "tan_half_q16", "bin_y_q", "bin_occ", "bin_zmin_q", "win_y_q", "win_z_q",
                 "w_y", "w_z", "smax_k", "l_min", "ext_win_y_q", "ext_win_z_q", "ext_edge_q",
                 "max_miss", "n_min", "f_min_q8"):
        setattr(p, name, int(v[name]))
    p.tracklet_cap_div = int(v.get("tracklet_cap_div", 16))
    p.sinphi_max = float(v["sinphi_max"])
    p.sigma_y = float(v["sigma_y"])
    p.sigma_z = float(v["sigma_z"])
    for i, c in enumerate(v["cov0"]):
        p.cov0[i] = float(c)
    return p


# --- C names ---------------------------------------------------------------------

def tpc_workspace_size(n_clusters: int, n_units: int, n_rows: int, params: tpc_params_t) -> int:
    return int(load_library().tpc_workspace_size(n_clusters, n_units, n_rows, ctypes.byref(params)))


def tpc_track_sectors(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t,
                      params: tpc_params_t, out: tpc_tracks_t, workspace: int, workspace_bytes: int,
                      stream: int) -> int:
    return int(load_library().tpc_track_sectors(ctypes.byref(clusters), ctypes.byref(geometry),
                                                ctypes.byref(field), ctypes.byref(params),
                                                ctypes.byref(out), workspace, workspace_bytes, stream))


def tpc_track_sectors_noalloc(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t,
                              params: tpc_params_t, out: tpc_tracks_t, stream: int) -> int:
    return int(load_library().tpc_track_sectors_noalloc(ctypes.byref(clusters), ctypes.byref(geometry),
                                                        ctypes.byref(field), ctypes.byref(params),
                                                        ctypes.byref(out), stream))


def tpc_track_sectors_profiled(clusters, geometry, field, params, out, workspace, workspace_bytes,
                               stream, events) -> int:
    arr = (_vp * len(events))(*events)
    return int(load_library().tpc_track_sectors_profiled(
        ctypes.byref(clusters), ctypes.byref(geometry), ctypes.byref(field), ctypes.byref(params),
        ctypes.byref(out), workspace, workspace_bytes, stream, arr, len(events)))


def tpc_kernel_count() -> int:
    return int(load_library().tpc_kernel_count())


def tpc_kernel_name(i: int) -> str:
    return load_library().tpc_kernel_name(i).decode()


def tpc_status_string(status: int) -> str:
    return load_library().tpc_status_string(status).decode()


def tpc_collisions_workspace_size(params: tpc_collision_params_t) -> int:
    return int(load_library().tpc_collisions_workspace_size(ctypes.byref(params)))


def tpc_assign_collisions(tracks: tpc_tracks_t, unit_side: int, n_units: int, field: tpc_field_t,
                          params: tpc_collision_params_t, out: tpc_collisions_t, workspace: int,
                          workspace_bytes: int, stream: int) -> int:
    return int(load_library().tpc_assign_collisions(ctypes.byref(tracks), unit_side, n_units, ctypes.byref(field),
                                                    ctypes.byref(params), ctypes.byref(out), workspace,
                                                    workspace_bytes, stream))


def tpc_clusterize_workspace_size(n_units: int, geometry: tpc_pad_geometry_t) -> int:
    return int(load_library().tpc_clusterize_workspace_size(n_units, ctypes.byref(geometry)))


def tpc_clusterize(digits: tpc_digits_t, geometry: tpc_pad_geometry_t, params: tpc_clusterizer_params_t,
                   out: tpc_cluster_out_t, workspace: int, workspace_bytes: int, stream: int) -> int:
    return int(load_library().tpc_clusterize(ctypes.byref(digits), ctypes.byref(geometry), ctypes.byref(params),
                                             ctypes.byref(out), workspace, workspace_bytes, stream))


def tpc_compress(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t, tracks: tpc_tracks_t,
                 params: tpc_compress_params_t, out: tpc_compressed_t, stream: int) -> int:
    return int(load_library().tpc_compress(ctypes.byref(clusters), ctypes.byref(geometry), ctypes.byref(field),
                                           ctypes.byref(tracks), ctypes.byref(params), ctypes.byref(out), stream))


def tpc_refit_workspace_size(n_clusters: int, cap_tracks: int, cap_hits: int) -> int:
    return int(load_library().tpc_refit_workspace_size(n_clusters, cap_tracks, cap_hits))


def tpc_refit_tracks(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t, params: tpc_params_t,
                     tracks: tpc_tracks_t, out: tpc_refit_t, workspace: int, workspace_bytes: int, stream: int) -> int:
    return int(load_library().tpc_refit_tracks(ctypes.byref(clusters), ctypes.byref(geometry), ctypes.byref(field),
                                               ctypes.byref(params), ctypes.byref(tracks), ctypes.byref(out),
                                               workspace, workspace_bytes, stream))


def tpc_merge_workspace_size(n_units: int, n_rows: int, cap_tracks: int, params: tpc_merge_params_t) -> int:
    return int(load_library().tpc_merge_workspace_size(n_units, n_rows, cap_tracks, ctypes.byref(params)))


def tpc_merge_tracks(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t, tracks: tpc_tracks_t,
                     refit: tpc_refit_t, unit_alpha: int, unit_side: int, n_units: int, params: tpc_merge_params_t,
                     out: tpc_merged_t, workspace: int, workspace_bytes: int, stream: int) -> int:
    return int(load_library().tpc_merge_tracks(ctypes.byref(clusters), ctypes.byref(geometry), ctypes.byref(field),
                                               ctypes.byref(tracks), ctypes.byref(refit), unit_alpha, unit_side,
                                               n_units, ctypes.byref(params), ctypes.byref(out), workspace,
                                               workspace_bytes, stream))


def tpc_fit_chains(clusters: tpc_clusters_t, geometry: tpc_geometry_t, field: tpc_field_t, params: tpc_params_t,
                   tracks: tpc_tracks_t, merged: tpc_merged_t, unit_alpha: int, n_units: int, out: tpc_chain_fit_t,
                   workspace: int, workspace_bytes: int, stream: int) -> int:
    return int(load_library().tpc_fit_chains(ctypes.byref(clusters), ctypes.byref(geometry), ctypes.byref(field),
                                             ctypes.byref(params), ctypes.byref(tracks), ctypes.byref(merged),
                                             unit_alpha, n_units, ctypes.byref(out), workspace, workspace_bytes,
                                             stream))


def make_merge_params(cap_pairs=1 << 22, max_dalpha=0.3665, max_gap=32, dz_max=64.0, dy_max=2.0, chi2_max=30.0,
                      sinphi_max=0.95) -> tpc_merge_params_t:
    """Defaults: neighbouring sectors 20 degrees apart (21 allowed), 32 rows,
    64 cm in z', 2 cm in the carried y, chi2 30 over five parameters."""
    mp = tpc_merge_params_t()
    mp.cap_pairs, mp.max_dalpha, mp.max_gap = int(cap_pairs), max_dalpha, int(max_gap)
    mp.dz_max, mp.dy_max, mp.chi2_max, mp.sinphi_max = dz_max, dy_max, chi2_max, sinphi_max
    return mp


def make_compress_params(step=1.0 / 64, pt_remove=0.1, sinphi_max=0.999, hist_half=1024) -> tpc_compress_params_t:
    cp = tpc_compress_params_t()
    cp.step, cp.pt_remove, cp.sinphi_max, cp.hist_half = step, pt_remove, sinphi_max, int(hist_half)
    return cp


def make_collision_params(v_drift=2.58, bin_width=1.0, z_range=4096.0, c_max=None, n_min=10, reach=2,
                          outer_radius=None) -> tpc_collision_params_t:
    """Defaults: 1 cm bins over +-4096 cm, 10 forming tracks per candidate,
    reach 2 bins; c_max = 2 / outer_radius when that is given, else c_max
    (None: every track forms candidates)."""
    cp = tpc_collision_params_t()
    cp.v_drift, cp.bin_width, cp.z_range = v_drift, bin_width, z_range
    if c_max is None:
        c_max = 2.0 / outer_radius if outer_radius else float("inf")
    cp.c_max = c_max
    cp.n_min, cp.reach = int(n_min), int(reach)
    return cp


def tpc_inspect(clusters: tpc_clusters_t, n_rows: int, params: tpc_params_t, workspace: int,
                what: int) -> tpc_view_t:
    v = tpc_view_t()
    st = load_library().tpc_inspect(ctypes.byref(clusters), n_rows, ctypes.byref(params), workspace,
                                    what, ctypes.byref(v))
    if st != TPC_OK:
        raise ValueError("tpc_inspect: %s" % tpc_status_string(st))
    return v


# --- torch convenience ---------------------------------------------------------------

def __getattr__(name):
    # the torch-side helpers load on first use, so that importing the package
    # (e.g. for its parameter values) does not import torch
    if name in ("Tracker", "track", "CollisionAssigner", "Clusterizer", "Compressor", "Refitter", "Merger",
                "ChainFitter"):
        from . import runtime
        return getattr(runtime, name)
    raise AttributeError(name)
