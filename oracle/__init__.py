"""CPU reference (oracle) for TPC sector track finding -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It loads `oracle/_oracle.so`, built from
`oracle/tpc_oracle.c` (plain C, FP64 fit, int64 decisions), and shares nothing
with the HIP library: it is handed the same input arrays and the same
parameter values (a plain dict) and computes everything itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(HERE, "tpc_oracle.c")
# TPC_ORACLE_LIB: another build of the same source (the sanitizer test uses it)
_LIB = os.environ.get("TPC_ORACLE_LIB") or os.path.join(HERE, "_oracle.so")


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-D_POSIX_C_SOURCE=200809L",
                               "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("q_shift", ctypes.c_int32), ("tan_half_q16", ctypes.c_int32),
        ("bin_y_q", ctypes.c_int32), ("bin_occ", ctypes.c_int32), ("bin_zmin_q", ctypes.c_int32),
        ("win_y_q", ctypes.c_int32), ("win_z_q", ctypes.c_int32),
        ("w_y", ctypes.c_int32), ("w_z", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("smax_k", ctypes.c_int64),
        ("l_min", ctypes.c_int32), ("ext_win_y_q", ctypes.c_int32), ("ext_win_z_q", ctypes.c_int32),
        ("ext_edge_q", ctypes.c_int32), ("max_miss", ctypes.c_int32), ("n_min", ctypes.c_int32),
        ("f_min_q8", ctypes.c_int32), ("brute", ctypes.c_int32),
        ("sinphi_max", ctypes.c_double), ("sigma_y", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("cov0", ctypes.c_double * 5), ("fragile_eps", ctypes.c_double),
    ]


_I32P = ctypes.POINTER(ctypes.c_int32)
_U32P = ctypes.POINTER(ctypes.c_uint32)
_F64P = ctypes.POINTER(ctypes.c_double)


class _Result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_units", ctypes.c_int64), ("n_rows", ctypes.c_int64),
        ("n_seg", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("n_tracklets", ctypes.c_int64),
        ("n_tracks", ctypes.c_int64), ("n_track_hits", ctypes.c_int64),
        ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("perm", _I32P), ("up", _I32P), ("dn", _I32P), ("upc", _I32P), ("dnc", _I32P),
        ("owner", _U32P), ("cluster_track", _I32P),
        ("seg_start", _I32P), ("seg_count", _I32P), ("seg_zmin", _I32P), ("seg_zmax", _I32P),
        ("seg_ny", _I32P), ("seg_nz", _I32P), ("seg_by", _I32P), ("seg_bz", _I32P),
        ("seg_cell_base", _I32P), ("cell_start", _I32P),
        ("trk_start", _I32P), ("trk_unit", _I32P), ("trk_len", _I32P), ("trk_nfit", _I32P),
        ("trk_p1n", _I32P), ("trk_owned", _I32P), ("trk_keep", _I32P), ("trk_fragile", _I32P),
        ("trk_key", _U32P),
        ("trk_params", _F64P), ("trk_cov", _F64P), ("trk_xref", _F64P), ("trk_chi2", _F64P),
        ("trk_hits", _I32P),
        ("track_tracklet", _I32P), ("track_first_hit", _I32P), ("track_n_hits", _I32P),
        ("track_hits", _I32P),
        ("time_s", ctypes.c_double * 8),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int64, vp,
                                ctypes.c_float, ctypes.POINTER(Params), ctypes.POINTER(_Result)]
        lib.orc_free.argtypes = [ctypes.POINTER(_Result)]
        lib.orc_propagate.restype = ctypes.c_int
        lib.orc_propagate.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, vp, vp]
        lib.orc_seed.restype = ctypes.c_int
        lib.orc_seed.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp]
        lib.orc_fit_two_pass.restype = ctypes.c_int
        lib.orc_fit_two_pass.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_double,
                                         ctypes.POINTER(Params), vp, vp, vp, vp]
        lib.orc_kf_update.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, vp]
        lib.orc_zdca.restype = ctypes.c_double
        lib.orc_zdca.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp, vp]
        lib.orc_collisions.restype = ctypes.c_int64
        lib.orc_collisions.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_double] + [vp] * 10
        lib.orc_clusterize.restype = ctypes.c_int64
        lib.orc_clusterize.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double] + [vp] * 12
        lib.orc_compress.restype = None
        lib.orc_compress.argtypes = [ctypes.c_int64] + [vp] * 7 + [ctypes.c_double] * 5 + [vp] * 4
        lib.orc_refit_tracks.restype = None
        lib.orc_refit_tracks.argtypes = [ctypes.c_int64] + [vp] * 7 + [ctypes.c_double, ctypes.POINTER(Params)] + [vp] * 9
        lib.orc_rotate.restype = ctypes.c_int
        lib.orc_rotate.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        lib.orc_merge.restype = ctypes.c_int64
        lib.orc_merge.argtypes = ([ctypes.c_int64] + [vp] * 10 + [ctypes.c_int32, vp, vp, ctypes.c_int32] +
                                  [ctypes.c_double] * 3 + [ctypes.c_int32] + [ctypes.c_double] * 4 + [vp] * 4)
        lib.orc_refit_chains.restype = None
        lib.orc_refit_chains.argtypes = ([ctypes.c_int64] + [vp] * 9 + [ctypes.c_int32, ctypes.c_double,
                                          ctypes.POINTER(Params)] + [vp] * 5)
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def make_params(values: dict, brute: bool = False, fragile_eps: float = 0.0) -> Params:
    """Oracle parameter block from a plain dict of parameter values."""
    p = Params()
    for name in ("q_shift", "tan_half_q16", "bin_y_q", "bin_occ", "bin_zmin_q", "win_y_q",
                 "win_z_q", "w_y", "w_z", "smax_k", "l_min", "ext_win_y_q", "ext_win_z_q",
                 "ext_edge_q", "max_miss", "n_min", "f_min_q8"):
        setattr(p, name, int(values[name]))
    # float parameters are float32 values; the oracle reads their exact doubles
    for name in ("sinphi_max", "sigma_y", "sigma_z"):
        setattr(p, name, float(np.float32(values[name])))
    for i, v in enumerate(values["cov0"]):
        p.cov0[i] = float(np.float32(v))
    p.brute = 1 if brute else 0
    p.fragile_eps = float(fragile_eps)
    return p


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(int(n),)).astype(dtype, copy=True)


def run(y, z, row, unit_offsets, row_x, bz, values: dict, brute=False, fragile_eps=0.0):
    """Run the reference on host arrays.  Returns a dict of numpy arrays (see
    orc_result_t in tpc_oracle.c), or raises ValueError on invalid input."""
    lib = _load()
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    row = np.ascontiguousarray(row, np.uint16)
    off = np.ascontiguousarray(unit_offsets, np.int64)
    rx = np.ascontiguousarray(row_x, np.float32)
    P = make_params(values, brute, fragile_eps)
    R = _Result()
    st = lib.orc_run(len(y), len(off) - 1, off.ctypes.data, y.ctypes.data, z.ctypes.data,
                     row.ctypes.data, len(rx), rx.ctypes.data, ctypes.c_float(bz),
                     ctypes.byref(P), ctypes.byref(R))
    if st != 0:
        lib.orc_free(ctypes.byref(R))
        raise ValueError("oracle: invalid input (status %d)" % st)
    n, S, C, K, T, TH, NR = (R.n, R.n_seg, R.n_cells, R.n_tracklets, R.n_tracks, R.n_track_hits,
                             R.n_rows)
    out = dict(n=n, n_seg=S, n_cells=C, n_tracklets=K, n_tracks=T, n_track_hits=TH,
               time_s=np.array(R.time_s[:]))
    for f in ("perm", "up", "dn", "upc", "dnc"):
        out[f] = _arr(getattr(R, f), n, np.int32)
    out["owner"] = _arr(R.owner, n, np.uint32)
    out["cluster_track"] = _arr(R.cluster_track, n, np.int32)
    for f in ("seg_start", "seg_count", "seg_zmin", "seg_zmax", "seg_ny", "seg_nz", "seg_by",
              "seg_bz", "seg_cell_base"):
        out[f] = _arr(getattr(R, f), S, np.int32)
    out["cell_start"] = _arr(R.cell_start, C + 1, np.int32)
    for f in ("trk_start", "trk_unit", "trk_len", "trk_nfit", "trk_p1n", "trk_owned", "trk_keep",
              "trk_fragile"):
        out[f] = _arr(getattr(R, f), K, np.int32)
    out["trk_key"] = _arr(R.trk_key, K, np.uint32)
    out["trk_params"] = _arr(R.trk_params, K * 5, np.float64).reshape(K, 5)
    out["trk_cov"] = _arr(R.trk_cov, K * 15, np.float64).reshape(K, 15)
    out["trk_xref"] = _arr(R.trk_xref, K, np.float64)
    out["trk_chi2"] = _arr(R.trk_chi2, K, np.float64)
    out["trk_hits"] = _arr(R.trk_hits, K * NR, np.int32).reshape(K, NR)
    for f in ("track_tracklet", "track_first_hit", "track_n_hits"):
        out[f] = _arr(getattr(R, f), T, np.int32)
    out["track_hits"] = _arr(R.track_hits, TH, np.int32)
    lib.orc_free(ctypes.byref(R))
    return out


def run_event(ev, values: dict, **kw):
    return run(ev.y, ev.z, ev.row, ev.unit_offsets, ev.row_x, ev.bz, values, **kw)


# ---- single-step helpers used by the pins ---------------------------------------

def propagate(p, x1, x2, k, sinphi_max=0.95, jacobian=False):
    lib = _load()
    p = np.ascontiguousarray(p, np.float64)
    out = np.zeros(5)
    F = np.zeros(25)
    st = lib.orc_propagate(p.ctypes.data, x1, x2, k, sinphi_max, out.ctypes.data,
                           F.ctypes.data if jacobian else None)
    if st != 0:
        return None if not jacobian else (None, None)
    return (out, F.reshape(5, 5)) if jacobian else out


def seed(x, y, z, k, sinphi_max=0.95):
    lib = _load()
    x, y, z = (np.ascontiguousarray(a, np.float64) for a in (x, y, z))
    p = np.zeros(5)
    st = lib.orc_seed(x.ctypes.data, y.ctypes.data, z.ctypes.data, k, sinphi_max, p.ctypes.data)
    return p if st == 0 else None


def fit_two_pass(x, y, z, k, values: dict):
    lib = _load()
    x, y, z = (np.ascontiguousarray(a, np.float64) for a in (x, y, z))
    P = make_params(values)
    p = np.zeros(5)
    cov = np.zeros(15)
    chi2 = np.zeros(1)
    p1 = np.zeros(5)
    st = lib.orc_fit_two_pass(len(x), x.ctypes.data, y.ctypes.data, z.ctypes.data, k,
                              ctypes.byref(P), p.ctypes.data, cov.ctypes.data, chi2.ctypes.data,
                              p1.ctypes.data)
    if st != 0:
        return None
    return dict(p=p, cov=cov, chi2=float(chi2[0]), p_pass1=p1)


def kf_update(p, cov15, my, mz, sy, sz):
    lib = _load()
    p = np.array(p, np.float64)
    c = np.array(cov15, np.float64)
    chi2 = np.zeros(1)
    lib.orc_kf_update(p.ctypes.data, c.ctypes.data, my, mz, sy, sz, chi2.ctypes.data)
    return p, c, float(chi2[0])


def zdca(p, x, k):
    """z' at the transverse point of closest approach to the beam axis and the
    arc length to it, for the state p at plane x (curvature k p[4])."""
    lib = _load()
    p = np.ascontiguousarray(p, np.float64)
    sT, turn = np.zeros(1), np.zeros(1)
    z = lib.orc_zdca(p.ctypes.data, float(x), float(k), sT.ctypes.data, turn.ctypes.data)
    return float(z), float(sT[0])


def collisions(params, x_ref, unit, unit_side, k, v_drift, width=1.0, zmax=4096.0, c_max=None, n_min=10,
               reach=2, eps=0.0):
    """Collision candidates of tracks (see orc_collisions in tpc_oracle.c).
    c_max defaults to no cut (every track forms candidates)."""
    lib = _load()
    params = np.ascontiguousarray(params, np.float64).reshape(-1, 5)
    n = len(params)
    x_ref = np.ascontiguousarray(x_ref, np.float64)
    unit = np.ascontiguousarray(unit, np.int32)
    unit_side = np.ascontiguousarray(unit_side, np.int32)
    zd, t0 = np.zeros(n), np.zeros(n)
    col, frag = np.zeros(n, np.int32), np.zeros(n, np.int32)
    cap = 2 * int(np.ceil(2 * zmax / width)) + 1
    cs, cb, cc, cf = (np.zeros(cap, np.int32) for _ in range(4))
    cz, ct = np.zeros(cap), np.zeros(cap)
    nc = lib.orc_collisions(n, params.ctypes.data, x_ref.ctypes.data, unit.ctypes.data, unit_side.ctypes.data,
                            float(k), float(v_drift), float(width), float(zmax),
                            float("inf") if c_max is None else float(c_max), int(n_min), int(reach), float(eps),
                            zd.ctypes.data, t0.ctypes.data, col.ctypes.data, frag.ctypes.data, cs.ctypes.data,
                            cb.ctypes.data, cc.ctypes.data, cf.ctypes.data, cz.ctypes.data, ct.ctypes.data)
    return dict(zdca=zd, t0=t0, collision=col, fragile=frag, n_collisions=int(nc), side=cs[:nc], bin=cb[:nc],
                count=cc[:nc], n_form=cf[:nc], c_zdca=cz[:nc], c_t0=ct[:nc])


def clusterize(half, pad_offsets, time, q, n_units, q_min, pw, tb, zoff):
    """Clusters of zero-suppressed digits (see orc_clusterize in tpc_oracle.c).
    half: half the pad count per row; pad_offsets: CSR over (unit, row, pad)."""
    lib = _load()
    half = np.ascontiguousarray(half, np.int32)
    off = np.ascontiguousarray(pad_offsets, np.int64)
    time = np.ascontiguousarray(time, np.uint16)
    q = np.ascontiguousarray(q, np.uint16)
    cap = max(1, len(time))
    ints = {k: np.zeros(cap, np.int32) for k in ("unit", "row", "pad", "time", "qmax", "q", "sp", "st")}
    flts = {k: np.zeros(cap, np.float32) for k in ("padf", "timef", "y", "z")}
    n = lib.orc_clusterize(int(n_units), len(half), half.ctypes.data, off.ctypes.data, time.ctypes.data,
                           q.ctypes.data, int(q_min), float(pw), float(tb), float(zoff),
                           *[ints[k].ctypes.data for k in ("unit", "row", "pad", "time", "qmax", "q", "sp", "st")],
                           *[flts[k].ctypes.data for k in ("padf", "timef", "y", "z")])
    out = {k: v[:n] for k, v in ints.items()}
    out.update({k: v[:n] for k, v in flts.items()})
    out["n"] = int(n)
    return out


def compress(y, z, row, cluster_track, params, x_ref, row_x, k, step=1.0 / 64, pt_remove=0.1, sinphi_max=0.999,
             eps=1e-6):
    """Hit removal and residual codes of clusters (see orc_compress in tpc_oracle.c)."""
    lib = _load()
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    row = np.ascontiguousarray(row, np.uint16)
    ct = np.ascontiguousarray(cluster_track, np.int32)
    params = np.ascontiguousarray(params, np.float32).reshape(-1)
    x_ref = np.ascontiguousarray(x_ref, np.float32)
    row_x = np.ascontiguousarray(row_x, np.float32)
    n = len(y)
    cls = np.zeros(n, np.uint8)
    cy, cz = np.zeros(n, np.int32), np.zeros(n, np.int32)
    frag = np.zeros(n, np.uint8)
    if len(params) == 0:
        params = np.zeros(5, np.float32)
        x_ref = np.zeros(1, np.float32)
    lib.orc_compress(n, y.ctypes.data, z.ctypes.data, row.ctypes.data, ct.ctypes.data, params.ctypes.data,
                     x_ref.ctypes.data, row_x.ctypes.data, float(k), float(step), float(pt_remove),
                     float(sinphi_max), float(eps), cls.ctypes.data, cy.ctypes.data, cz.ctypes.data, frag.ctypes.data)
    return dict(cls=cls, code_y=cy, code_z=cz, fragile=frag)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of later calls (timing only: results do not depend on it)."""
    _load().orc_set_threads(int(n))


def unpack_cov(c15):
    """15 packed lower-triangle entries (row-major, (i,j<=i)) -> symmetric 5x5."""
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = c15[k]
            k += 1
    return M


def refit_tracks(first_hit, n_hits, hits, y, z, row, row_x, k, values: dict):
    """Two-pass refit of selected tracks over their hit lists (see
    orc_refit_tracks in tpc_oracle.c).  row_x as the tracker sees it (pass the
    FP32 values to compare with FP32 code)."""
    lib = _load()
    first = np.ascontiguousarray(first_hit, np.int32)
    nh = np.ascontiguousarray(n_hits, np.int32)
    hits = np.ascontiguousarray(hits, np.int32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    row = np.ascontiguousarray(row, np.uint16)
    row_x = np.ascontiguousarray(row_x, np.float64)
    T = len(nh)
    assert len(first) == T
    if T:
        assert first.min() >= 0 and (first.astype(np.int64) + nh).max() <= len(hits)
    if len(hits):
        assert hits.min() >= 0 and hits.max() < len(y) and row[hits].max() < len(row_x)
    P = make_params(values)
    out = dict(p=np.zeros((T, 5)), cov=np.zeros((T, 15)), x_ref=np.zeros(T), chi2=np.zeros(T),
               p_out=np.zeros((T, 5)), cov_out=np.zeros((T, 15)), x_out=np.zeros(T),
               ok=np.zeros(T, np.int8), fragile=np.zeros(T, np.int8))
    lib.orc_refit_tracks(T, first.ctypes.data, nh.ctypes.data, hits.ctypes.data, y.ctypes.data, z.ctypes.data,
                         row.ctypes.data, row_x.ctypes.data, float(k), ctypes.byref(P),
                         *[out[key].ctypes.data for key in ("p", "cov", "x_ref", "chi2", "p_out", "cov_out",
                                                            "x_out", "ok", "fragile")])
    return out


def rotate(p, x, d, k, sinphi_max=0.95, jacobian=False):
    """A state at plane x of one sector frame turned by angle d into another
    (see orc_rotate): (state, x') or None; with jacobian, also the 5x5 Jacobian."""
    lib = _load()
    p = np.ascontiguousarray(p, np.float64)
    out = np.zeros(5)
    xo = np.zeros(1)
    J = np.zeros(25)
    st = lib.orc_rotate(p.ctypes.data, float(x), float(d), float(k), float(sinphi_max), out.ctypes.data,
                        xo.ctypes.data, J.ctypes.data)
    if st != 0:
        return None
    return (out, float(xo[0]), J.reshape(5, 5)) if jacobian else (out, float(xo[0]))


def segment_rows(first_hit, n_hits, hits, row):
    """First and last hit row of each track (hit lists in increasing row order)."""
    first_hit = np.asarray(first_hit, np.int64)
    n_hits = np.asarray(n_hits, np.int64)
    row = np.asarray(row)
    hits = np.asarray(hits, np.int64)
    fr = np.zeros(len(n_hits), np.int32)
    lr = np.zeros(len(n_hits), np.int32)
    has = n_hits > 0
    fr[has] = row[hits[first_hit[has]]]
    lr[has] = row[hits[first_hit[has] + n_hits[has] - 1]]
    return fr, lr


def merge(unit, first_row, last_row, refit, unit_alpha, unit_side, n_rows, k, sinphi_max=0.95,
          max_dalpha=0.3665, max_gap=32, dz_max=64.0, dy_max=2.0, chi2_max=30.0, eps=1e-9):
    """Links between refitted segments (see orc_merge).  refit: a dict as
    refit_tracks returns (ok, p, cov, x_ref, p_out, cov_out, x_out)."""
    lib = _load()
    T = len(unit)
    unit = np.ascontiguousarray(unit, np.int32)
    fr = np.ascontiguousarray(first_row, np.int32)
    lr = np.ascontiguousarray(last_row, np.int32)
    ok = np.ascontiguousarray(refit["ok"], np.int8)
    arrs = [np.ascontiguousarray(refit[key], np.float64) for key in ("p", "cov", "x_ref", "p_out", "cov_out", "x_out")]
    ua = np.ascontiguousarray(unit_alpha, np.float64)
    us = np.ascontiguousarray(unit_side, np.int32)
    if T:
        assert unit.min() >= 0 and unit.max() < len(ua) and fr.min() >= 0 and lr.max() < n_rows
    nxt = np.zeros(T, np.int32)
    prv = np.zeros(T, np.int32)
    lc = np.zeros(T)
    frag = np.zeros(T, np.int8)
    n_cand = lib.orc_merge(T, unit.ctypes.data, fr.ctypes.data, lr.ctypes.data, ok.ctypes.data,
                           *[a.ctypes.data for a in arrs], len(ua), ua.ctypes.data, us.ctypes.data, int(n_rows),
                           float(k), float(sinphi_max), float(max_dalpha), int(max_gap), float(dz_max),
                           float(dy_max), float(chi2_max), float(eps),
                           nxt.ctypes.data, prv.ctypes.data, lc.ctypes.data, frag.ctypes.data)
    return dict(next=nxt, prev=prv, link_chi2=lc, fragile=frag, n_candidates=int(n_cand))


def chains(next_, prev, first_hit, n_hits, hits, unit):
    """The merged chains of linked segments (prev = -1, next >= 0 at the head):
    per chain its head, its hit list (the segments' hit lists in chain order)
    and each hit's unit.  Returns (heads, chain_first, chain_n, chain_hits,
    hit_unit)."""
    next_ = np.asarray(next_)
    heads = np.nonzero((np.asarray(prev) < 0) & (next_ >= 0))[0]
    cf, cn, ch, cu = [], [], [], []
    pos = 0
    for h in heads:
        cf.append(pos)
        t = int(h)
        n = 0
        while t >= 0:
            f, m = int(first_hit[t]), int(n_hits[t])
            ch.append(np.asarray(hits[f:f + m]))
            cu.append(np.full(m, unit[t], np.int32))
            n += m
            t = int(next_[t])
        cn.append(n)
        pos += n
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return (heads.astype(np.int64), np.array(cf, np.int32), np.array(cn, np.int32), cat(ch, np.int32),
            cat(cu, np.int32))


def refit_chains(chain_first, chain_n, chain_hits, hit_unit, y, z, row, row_x, unit_alpha, k, values: dict):
    """Two-pass fit of merged chains across frames (see orc_fit_chain)."""
    lib = _load()
    cf = np.ascontiguousarray(chain_first, np.int32)
    cn = np.ascontiguousarray(chain_n, np.int32)
    ch = np.ascontiguousarray(chain_hits, np.int32)
    cu = np.ascontiguousarray(hit_unit, np.int32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    row = np.ascontiguousarray(row, np.uint16)
    row_x = np.ascontiguousarray(row_x, np.float64)
    ua = np.ascontiguousarray(unit_alpha, np.float64)
    C = len(cn)
    if len(ch):
        assert ch.min() >= 0 and ch.max() < len(y) and cu.min() >= 0 and cu.max() < len(ua)
    P = make_params(values)
    out = dict(p=np.zeros((C, 5)), cov=np.zeros((C, 15)), x_ref=np.zeros(C), chi2=np.zeros(C), ok=np.zeros(C, np.int8))
    lib.orc_refit_chains(C, cf.ctypes.data, cn.ctypes.data, ch.ctypes.data, cu.ctypes.data, y.ctypes.data,
                         z.ctypes.data, row.ctypes.data, row_x.ctypes.data, ua.ctypes.data, len(ua), float(k),
                         ctypes.byref(P),
                         *[out[key].ctypes.data for key in ("p", "cov", "x_ref", "chi2", "ok")])
    return out

