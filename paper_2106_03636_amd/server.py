"""Python binding of the serving calls (tpc_server_* in include/tpc_track.h).

Argument marshalling only: admission, batching, streams, copies and tracking
all run in the library (its host thread and its kernels).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import (TPC_E_BUSY, TPC_OK, load_library, make_params, tpc_params_t, tpc_status_string)

TPC_REQ_COPY, TPC_REQ_BORROW_HOST, TPC_REQ_DEVICE = 0, 1, 2

_vp = ctypes.c_void_p


class tpc_server_config_t(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_in_flight", ctypes.c_int32),
                ("queue_depth", ctypes.c_int32), ("max_batch_clusters", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("row_x", _vp), ("bz_tesla", ctypes.c_float), ("device", ctypes.c_int32),
                ("params", tpc_params_t)]


class tpc_request_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_units", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("unit_offsets", _vp), ("y", _vp), ("z", _vp), ("row", _vp)]


class tpc_result_t(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n", ctypes.c_int64),
                ("n_tracks", ctypes.c_int64), ("n_track_hits", ctypes.c_int64),
                ("cluster_track", _vp), ("params", _vp), ("cov", _vp), ("x_ref", _vp), ("chi2", _vp),
                ("unit", _vp), ("n_hits", _vp), ("n_fit", _vp), ("first_hit", _vp), ("hits", _vp),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("batch_id", ctypes.c_int64), ("batch_requests", ctypes.c_int32),
                ("reserved2", ctypes.c_int32)]


class tpc_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected_busy", ctypes.c_int64), ("rejected_nomem", ctypes.c_int64),
                ("rejected_invalid", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("pending", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("host_cpu_s", ctypes.c_double)]


_bound = False


def _lib():
    global _bound
    lib = load_library()
    if not _bound:
        lib.tpc_server_create.restype = ctypes.c_int
        lib.tpc_server_create.argtypes = [ctypes.POINTER(tpc_server_config_t), ctypes.POINTER(_vp)]
        lib.tpc_server_submit.restype = ctypes.c_int
        lib.tpc_server_submit.argtypes = [_vp, ctypes.POINTER(tpc_request_t), ctypes.POINTER(ctypes.c_uint64)]
        lib.tpc_server_poll.restype = ctypes.c_int
        lib.tpc_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(tpc_result_t), ctypes.c_int64]
        lib.tpc_server_release.restype = ctypes.c_int
        lib.tpc_server_release.argtypes = [_vp, ctypes.c_uint64]
        lib.tpc_server_stats.restype = ctypes.c_int
        lib.tpc_server_stats.argtypes = [_vp, ctypes.POINTER(tpc_server_stats_t)]
        lib.tpc_server_destroy.restype = ctypes.c_int
        lib.tpc_server_destroy.argtypes = [_vp]
        lib.tpc_server_footprint.restype = ctypes.c_size_t
        lib.tpc_server_footprint.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(tpc_params_t)]
        _bound = True
    return lib


def tpc_server_create(config: tpc_server_config_t):
    h = _vp()
    st = _lib().tpc_server_create(ctypes.byref(config), ctypes.byref(h))
    return st, h


def tpc_server_submit(server, request: tpc_request_t):
    t = ctypes.c_uint64()
    st = _lib().tpc_server_submit(server, ctypes.byref(request), ctypes.byref(t))
    return st, int(t.value)


def tpc_server_poll(server, ticket: int, wait_us: int = -1):
    r = tpc_result_t()
    st = _lib().tpc_server_poll(server, ticket, ctypes.byref(r), wait_us)
    return st, r


def tpc_server_release(server, ticket: int) -> int:
    return int(_lib().tpc_server_release(server, ticket))


def tpc_server_stats(server) -> tpc_server_stats_t:
    s = tpc_server_stats_t()
    _lib().tpc_server_stats(server, ctypes.byref(s))
    return s


def tpc_server_destroy(server) -> int:
    return int(_lib().tpc_server_destroy(server))


def tpc_server_footprint(n, n_units, n_rows, params) -> int:
    return int(_lib().tpc_server_footprint(n, n_units, n_rows, ctypes.byref(params)))


def _np(ptr, n, dtype, shape=None):
    if n == 0 or not ptr:
        a = np.zeros(0, dtype)
    else:
        a = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dtype))),
                                  shape=(int(n),)).copy()
    return a.reshape(shape) if shape is not None else a


class Server:
    """Owns a tpc_server_t.  submit() takes host numpy arrays (copied, or
    borrowed when flags says so) or device tensors (flags=TPC_REQ_DEVICE)."""

    def __init__(self, row_x, bz, budget_bytes, max_in_flight=2, queue_depth=64, max_batch_clusters=0,
                 max_batch_requests=0, params=None, device=0):
        self._row_x = np.ascontiguousarray(row_x, np.float32)
        cfg = tpc_server_config_t()
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_in_flight = int(max_in_flight)
        cfg.queue_depth = int(queue_depth)
        cfg.max_batch_clusters = int(max_batch_clusters)
        cfg.max_batch_requests = int(max_batch_requests)
        cfg.n_rows = len(self._row_x)
        cfg.row_x = self._row_x.ctypes.data
        cfg.bz_tesla = float(bz)
        cfg.device = int(device)
        cfg.params = make_params(params)
        self.params = cfg.params
        self.n_rows = cfg.n_rows
        st, self._h = tpc_server_create(cfg)
        if st != TPC_OK:
            raise RuntimeError("tpc_server_create: %s" % tpc_status_string(st))
        self._keep = {}

    def footprint(self, n, n_units):
        return tpc_server_footprint(n, n_units, self.n_rows, self.params)

    def submit(self, y, z, row, unit_offsets, flags=TPC_REQ_COPY):
        """Returns (status, ticket).  Status TPC_E_BUSY means back pressure."""
        off = np.ascontiguousarray(unit_offsets, np.int64)
        req = tpc_request_t()
        req.n = int(off[-1])
        req.n_units = len(off) - 1
        req.flags = int(flags)
        req.unit_offsets = off.ctypes.data
        if flags == TPC_REQ_DEVICE:
            req.y, req.z, req.row = y.data_ptr(), z.data_ptr(), row.data_ptr()
            keep = (y, z, row)
        else:
            y = np.ascontiguousarray(y, np.float32)
            z = np.ascontiguousarray(z, np.float32)
            row = np.ascontiguousarray(row, np.uint16)
            req.y, req.z, req.row = y.ctypes.data, z.ctypes.data, row.ctypes.data
            keep = (y, z, row)
        st, t = tpc_server_submit(self._h, req)
        if st == TPC_OK and flags != TPC_REQ_COPY:
            self._keep[t] = keep  # borrowed arrays stay alive until released
        return st, t

    def poll(self, ticket, wait_us=-1, arrays=True):
        """None while running (wait_us >= 0), else a dict: status, counts and
        times, plus copies of the result arrays unless arrays is False."""
        st, r = tpc_server_poll(self._h, ticket, wait_us)
        if st == TPC_E_BUSY:
            return None
        if st != TPC_OK:
            raise KeyError("unknown ticket %d" % ticket)
        T, H, n = r.n_tracks, r.n_track_hits, r.n
        out = dict(status=r.status, n=n, n_tracks=T, n_track_hits=H,
                   t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done,
                   batch_id=r.batch_id, batch_requests=r.batch_requests)
        if r.status == TPC_OK and arrays:
            out.update(cluster_track=_np(r.cluster_track, n, np.int32),
                       params=_np(r.params, 5 * T, np.float32, (T, 5)),
                       cov=_np(r.cov, 15 * T, np.float32, (T, 15)),
                       x_ref=_np(r.x_ref, T, np.float32), chi2=_np(r.chi2, T, np.float32),
                       unit=_np(r.unit, T, np.int32), n_hits=_np(r.n_hits, T, np.int32),
                       n_fit=_np(r.n_fit, T, np.int32), first_hit=_np(r.first_hit, T, np.int32),
                       hits=_np(r.hits, H, np.int32))
        return out

    def release(self, ticket):
        self._keep.pop(ticket, None)
        return tpc_server_release(self._h, ticket)

    def stats(self):
        s = tpc_server_stats(self._h)
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if self._h:
            tpc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
