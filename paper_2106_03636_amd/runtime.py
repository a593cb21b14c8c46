"""torch-side plumbing around the C ABI: device buffers and streams only.

`Tracker` owns the workspace and output buffers for batches up to a given
size and calls `tpc_track_sectors` on a torch stream.  Nothing here computes
any step of the method.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import (DEFAULT_PARAMS, TPC_OK, tpc_clusters_t, tpc_field_t, tpc_geometry_t, tpc_inspect,
               tpc_status_string, tpc_track_sectors, tpc_tracks_t, tpc_workspace_size, make_params)

_VIEW_DTYPE = {
    "float": torch.float32, "int": torch.int32,
}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


class TrackingError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class Batch:
    """Clusters of one batch resident on the device (what the C ABI consumes)."""

    def __init__(self, y, z, row, unit_offsets, row_x, bz, device="cuda"):
        dev = torch.device(device)
        self.y = torch.as_tensor(np.ascontiguousarray(y, np.float32)).to(dev)
        self.z = torch.as_tensor(np.ascontiguousarray(z, np.float32)).to(dev)
        self.row = torch.as_tensor(np.ascontiguousarray(row, np.uint16).view(np.int16)).to(dev)
        self.unit_offsets = torch.as_tensor(np.ascontiguousarray(unit_offsets, np.int64)).to(dev)
        self.row_x = torch.as_tensor(np.ascontiguousarray(row_x, np.float32)).to(dev)
        self.n = int(len(y))
        self.n_units = int(len(unit_offsets) - 1)
        self.n_rows = int(len(row_x))
        self.bz = float(bz)

    @staticmethod
    def from_event(ev, device="cuda"):
        return Batch(ev.y, ev.z, ev.row, ev.unit_offsets, ev.row_x, ev.bz, device)

    @staticmethod
    def from_device(y, z, row, unit_offsets, row_x, bz):
        """A batch over device tensors that are already resident (no copies of
        y, z, row: float32, float32, int16 holding the uint16 rows)."""
        b = Batch.__new__(Batch)
        dev = y.device
        b.y, b.z, b.row = y, z, row
        b.unit_offsets = torch.as_tensor(np.ascontiguousarray(unit_offsets, np.int64)).to(dev)
        b.row_x = torch.as_tensor(np.ascontiguousarray(row_x, np.float32)).to(dev)
        b.n = int(y.numel())
        b.n_units = int(len(unit_offsets) - 1)
        b.n_rows = int(len(row_x))
        b.bz = float(bz)
        return b

    def clusters_struct(self):
        c = tpc_clusters_t()
        c.n = self.n
        c.n_units = self.n_units
        c.unit_offsets = _ptr(self.unit_offsets)
        c.y, c.z, c.row = _ptr(self.y), _ptr(self.z), _ptr(self.row)
        return c

    def geometry_struct(self):
        g = tpc_geometry_t()
        g.n_rows = self.n_rows
        g.row_x = _ptr(self.row_x)
        return g


class Tracker:
    """Workspace + outputs for batches of up to max_n clusters / max_units units."""

    def __init__(self, max_n, max_units, n_rows=152, params=None, device="cuda", cap_tracks=None,
                 cap_hits=None, workspace=True):
        """workspace=False: no workspace is allocated and launches go through
        tpc_track_sectors_noalloc (the library's fixed device scratch array;
        no intermediate arrays to inspect)."""
        self.values = dict(DEFAULT_PARAMS if params is None else params)
        self.params = make_params(self.values)
        self.device = torch.device(device)
        self.max_n, self.max_units, self.n_rows = int(max_n), int(max_units), int(n_rows)
        ws = tpc_workspace_size(self.max_n, self.max_units, self.n_rows, self.params)
        if ws == 0:
            raise ValueError("invalid batch shape or parameters")
        self.ws_bytes = ws
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device) if workspace else None
        n_min = max(1, int(self.values["n_min"]))
        self.cap_tracks = int(cap_tracks if cap_tracks is not None else self.max_n // n_min + 1)
        self.cap_hits = int(cap_hits if cap_hits is not None else self.max_n)
        d, i32, f32 = self.device, torch.int32, torch.float32
        ct = max(1, self.cap_tracks)
        self.o_cluster_track = torch.empty(max(1, self.max_n), dtype=i32, device=d)
        self.o_params = torch.empty((ct, 5), dtype=f32, device=d)
        self.o_cov = torch.empty((ct, 15), dtype=f32, device=d)
        self.o_x_ref = torch.empty(ct, dtype=f32, device=d)
        self.o_chi2 = torch.empty(ct, dtype=f32, device=d)
        self.o_unit = torch.empty(ct, dtype=i32, device=d)
        self.o_n_hits = torch.empty(ct, dtype=i32, device=d)
        self.o_n_fit = torch.empty(ct, dtype=i32, device=d)
        self.o_first_hit = torch.empty(ct, dtype=i32, device=d)
        self.o_hits = torch.empty(max(1, self.cap_hits), dtype=i32, device=d)
        self.o_counts = torch.zeros(5, dtype=torch.int64, device=d)
        self.o_status = torch.zeros(1, dtype=i32, device=d)
        self._last = None

    def tracks_struct(self):
        o = tpc_tracks_t()
        o.cap_tracks, o.cap_hits = self.cap_tracks, self.cap_hits
        o.cluster_track = _ptr(self.o_cluster_track)
        o.params, o.cov = _ptr(self.o_params), _ptr(self.o_cov)
        o.x_ref, o.chi2 = _ptr(self.o_x_ref), _ptr(self.o_chi2)
        o.unit, o.n_hits, o.n_fit = _ptr(self.o_unit), _ptr(self.o_n_hits), _ptr(self.o_n_fit)
        o.first_hit, o.hits = _ptr(self.o_first_hit), _ptr(self.o_hits)
        o.counts, o.status = _ptr(self.o_counts), _ptr(self.o_status)
        return o

    def launch(self, batch: Batch, stream=None):
        """Enqueue tracking of `batch` on `stream` (default: torch's current stream)."""
        if batch.n > self.max_n or batch.n_units > self.max_units or batch.n_rows != self.n_rows:
            raise ValueError("batch larger than this tracker was sized for")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        c, g = batch.clusters_struct(), batch.geometry_struct()
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        o = self.tracks_struct()
        if self.workspace is None:
            from . import tpc_track_sectors_noalloc
            st = tpc_track_sectors_noalloc(c, g, f, self.params, o, s.cuda_stream)
            name = "tpc_track_sectors_noalloc"
        else:
            st = tpc_track_sectors(c, g, f, self.params, o, self.workspace.data_ptr(), self.ws_bytes,
                                   s.cuda_stream)
            name = "tpc_track_sectors"
        if st != TPC_OK:
            raise TrackingError(st, "%s: %s" % (name, tpc_status_string(st)))
        self._last = batch
        return st

    def launch_profiled(self, batch: Batch, events, stream=None):
        """As launch, recording `events` (raw hipEvent_t handles, tpc_kernel_count()+1
        of them) around every kernel on the same stream."""
        from . import tpc_track_sectors_profiled
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        c, g = batch.clusters_struct(), batch.geometry_struct()
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        o = self.tracks_struct()
        st = tpc_track_sectors_profiled(c, g, f, self.params, o, self.workspace.data_ptr(),
                                        self.ws_bytes, s.cuda_stream, events)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_track_sectors_profiled: %s" % tpc_status_string(st))
        self._last = batch
        return st

    def status(self):
        return int(self.o_status.item())

    def result(self, sync=True):
        """Trimmed outputs of the last launch (synchronizes)."""
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        counts = self.o_counts.cpu().numpy()
        if st != TPC_OK:
            raise TrackingError(st, "tracking failed on the device: %s (counts %s)"
                                % (tpc_status_string(st), counts.tolist()))
        T, H = int(counts[0]), int(counts[1])
        n = self._last.n
        return dict(n_tracks=T, n_track_hits=H, n_tracklets=int(counts[2]), n_cells=int(counts[3]),
                    n_seeds=int(counts[4]),
                    cluster_track=self.o_cluster_track[:n], params=self.o_params[:T], cov=self.o_cov[:T],
                    x_ref=self.o_x_ref[:T], chi2=self.o_chi2[:T], unit=self.o_unit[:T],
                    n_hits=self.o_n_hits[:T], n_fit=self.o_n_fit[:T], first_hit=self.o_first_hit[:T],
                    hits=self.o_hits[:H])

    def tracklet_field(self, what, dtype=torch.int32, width=1):
        """A per-seed view (NFIT, RLO, ..., PARAMS) of the last launch spread over
        all its tracklets (host numpy; tracklets that are not seeds get 0, and -1
        for RLO / RHI)."""
        from . import TPC_VIEW_SEED_LIST, TPC_VIEW_TRK_RLO, TPC_VIEW_TRK_RHI
        counts = self.o_counts.cpu().numpy()
        K, S = int(counts[2]), int(counts[4])
        seeds = self.inspect(TPC_VIEW_SEED_LIST).cpu().numpy()[:S]
        v = self.inspect(what, dtype).cpu().numpy().reshape(-1, width)[:S]
        fill = -1 if what in (TPC_VIEW_TRK_RLO, TPC_VIEW_TRK_RHI) else 0
        out = np.full((K, width), fill, v.dtype)
        out[seeds] = v
        return out if width > 1 else out[:, 0]

    def inspect(self, what, dtype=torch.int32, shape=None):
        """Copy of an intermediate workspace array of the last launch (tpc_inspect)."""
        if self.workspace is None:
            raise ValueError("a tracker without a workspace has no intermediate arrays")
        b = self._last
        v = tpc_inspect(b.clusters_struct(), b.n_rows, self.params, self.workspace.data_ptr(), what)
        base = self.workspace.data_ptr()
        off = v.ptr - base
        nbytes = v.count * v.elem_bytes
        raw = self.workspace[off:off + nbytes]
        t = raw.view(dtype)
        if shape is not None:
            t = t.view(*shape)
        return t.clone()


def track(y, z, row, unit_offsets, row_x, bz, params=None, device="cuda"):
    """One-shot convenience: track host arrays on the GPU, return host numpy arrays."""
    b = Batch(y, z, row, unit_offsets, row_x, bz, device)
    tr = Tracker(max(1, b.n), b.n_units, b.n_rows, params, device)
    tr.launch(b)
    r = tr.result()
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in r.items()}


class GraphRunner:
    """One tracking call over a resident batch, captured once into a HIP graph
    (through torch's graph capture on a side stream) and replayed: the whole
    pipeline becomes a single graph launch.  The call allocates nothing and
    records no memset, so it is capturable as is."""

    def __init__(self, tracker: Tracker, batch: Batch):
        self.tracker, self.batch = tracker, batch
        tracker.launch(batch)
        torch.cuda.synchronize(tracker.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            tracker.launch(batch)
        torch.cuda.synchronize(tracker.device)

    def replay(self):
        self.graph.replay()
        self.tracker._last = self.batch

    def result(self):
        return self.tracker.result()


class CollisionAssigner:
    """Workspace and outputs of tpc_assign_collisions for the tracks of a
    Tracker (same device, same stream order)."""

    def __init__(self, tracker: Tracker, params=None, cap=4096):
        from . import make_collision_params, tpc_collisions_workspace_size
        self.params = params if params is not None else make_collision_params()
        self.tracker = tracker
        self.device = tracker.device
        ws = tpc_collisions_workspace_size(self.params)
        if ws == 0:
            raise ValueError("invalid collision parameters")
        self.ws_bytes = ws
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.cap = int(cap)
        d, ct, c = self.device, max(1, tracker.cap_tracks), max(1, self.cap)
        self.o_zdca = torch.empty(ct, dtype=torch.float64, device=d)
        self.o_collision = torch.empty(ct, dtype=torch.int32, device=d)
        self.o_side = torch.empty(c, dtype=torch.int32, device=d)
        self.o_bin = torch.empty(c, dtype=torch.int32, device=d)
        self.o_count = torch.empty(c, dtype=torch.int32, device=d)
        self.o_n_form = torch.empty(c, dtype=torch.int32, device=d)
        self.o_z = torch.empty(c, dtype=torch.float64, device=d)
        self.o_t0 = torch.empty(c, dtype=torch.float64, device=d)
        self.o_n = torch.zeros(1, dtype=torch.int64, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)
        self._side = None

    def out_struct(self):
        from . import tpc_collisions_t
        o = tpc_collisions_t()
        o.cap = self.cap
        o.zdca, o.collision = _ptr(self.o_zdca), _ptr(self.o_collision)
        o.side, o.bin, o.count, o.n_form = _ptr(self.o_side), _ptr(self.o_bin), _ptr(self.o_count), _ptr(self.o_n_form)
        o.z, o.t0 = _ptr(self.o_z), _ptr(self.o_t0)
        o.n_collisions, o.status = _ptr(self.o_n), _ptr(self.o_status)
        return o

    def launch(self, unit_side, bz, stream=None):
        """Enqueue the assignment of the tracker's last tracks; unit_side: +1 / -1
        per unit (host sequence or device int32 tensor)."""
        from . import tpc_assign_collisions
        if not torch.is_tensor(unit_side):
            unit_side = torch.as_tensor(np.ascontiguousarray(unit_side, np.int32)).to(self.device)
        self._side = unit_side
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        f = tpc_field_t()
        f.bz_tesla = float(bz)
        st = tpc_assign_collisions(self.tracker.tracks_struct(), _ptr(unit_side), int(unit_side.numel()), f,
                                   self.params, self.out_struct(), self.workspace.data_ptr(), self.ws_bytes,
                                   s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_assign_collisions: %s" % tpc_status_string(st))
        return st

    def result(self, sync=True):
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        n = int(self.o_n.item())
        if st != TPC_OK:
            raise TrackingError(st, "collision assignment failed on the device: %s (candidates %d)"
                                % (tpc_status_string(st), n))
        T = int(self.tracker.o_counts[0].item())
        return dict(n_collisions=n, zdca=self.o_zdca[:T], collision=self.o_collision[:T], side=self.o_side[:n],
                    bin=self.o_bin[:n], count=self.o_count[:n], n_form=self.o_n_form[:n], z=self.o_z[:n],
                    t0=self.o_t0[:n])


class Clusterizer:
    """Workspace and outputs of tpc_clusterize for digit batches of up to
    max_units units and cap clusters.  half: half the pad count of each row;
    pad_width, time_bin, z_offset as in tpc_pad_geometry_t."""

    def __init__(self, half, pad_width, time_bin, z_offset, max_units, cap, q_min=10, device="cuda"):
        from . import tpc_clusterize_workspace_size, tpc_clusterizer_params_t, tpc_pad_geometry_t
        self.device = torch.device(device)
        half = np.ascontiguousarray(half, np.int32)
        self.half = torch.as_tensor(half).to(self.device)
        self.geometry = tpc_pad_geometry_t()
        self.geometry.n_rows = len(half)
        self.geometry.pads_total = int(2 * half.sum())
        self.geometry.half = _ptr(self.half)
        self.geometry.pad_width, self.geometry.time_bin, self.geometry.z_offset = pad_width, time_bin, z_offset
        self.params = tpc_clusterizer_params_t()
        self.params.q_min = int(q_min)
        self.max_units, self.cap = int(max_units), int(cap)
        ws = tpc_clusterize_workspace_size(self.max_units, self.geometry)
        if ws == 0:
            raise ValueError("invalid pad geometry")
        self.ws_bytes = ws
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        d, c = self.device, max(1, self.cap)
        self.o_y = torch.empty(c, dtype=torch.float32, device=d)
        self.o_z = torch.empty(c, dtype=torch.float32, device=d)
        self.o_row = torch.empty(c, dtype=torch.int16, device=d)  # uint16 rows
        self.o_qtot = torch.empty(c, dtype=torch.int32, device=d)
        self.o_qmax = torch.empty(c, dtype=torch.int16, device=d)  # uint16 charges
        self.o_pad = torch.empty(c, dtype=torch.float32, device=d)
        self.o_time = torch.empty(c, dtype=torch.float32, device=d)
        self.o_unit_offsets = torch.zeros(self.max_units + 1, dtype=torch.int64, device=d)
        self.o_count = torch.zeros(1, dtype=torch.int64, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)
        self._n_units = 0

    @staticmethod
    def upload(digits, device="cuda"):
        """Host digits (time, q: uint16; pad_offsets: int64) to device tensors."""
        dev = torch.device(device)
        t = torch.as_tensor(np.ascontiguousarray(digits.time, np.uint16).view(np.int16)).to(dev)
        q = torch.as_tensor(np.ascontiguousarray(digits.q, np.uint16).view(np.int16)).to(dev)
        off = torch.as_tensor(np.ascontiguousarray(digits.pad_offsets, np.int64)).to(dev)
        return t, q, off

    def launch(self, time, q, pad_offsets, n_units, stream=None):
        """Enqueue the clusterization of device digits (time, q as int16 views
        of uint16, pad_offsets int64) of n_units units."""
        from . import tpc_cluster_out_t, tpc_clusterize, tpc_digits_t
        if n_units > self.max_units:
            raise ValueError("more units than this clusterizer was sized for")
        if pad_offsets.numel() != n_units * self.geometry.pads_total + 1:
            raise ValueError("pad_offsets must have n_units * pads_total + 1 entries")
        dg = tpc_digits_t()
        dg.n = int(time.numel())
        dg.n_units = int(n_units)
        dg.pad_offsets = _ptr(pad_offsets)
        dg.time, dg.q = _ptr(time), _ptr(q)
        o = tpc_cluster_out_t()
        o.cap = self.cap
        o.y, o.z, o.row = _ptr(self.o_y), _ptr(self.o_z), _ptr(self.o_row)
        o.qtot, o.qmax, o.pad, o.time = _ptr(self.o_qtot), _ptr(self.o_qmax), _ptr(self.o_pad), _ptr(self.o_time)
        o.unit_offsets, o.count, o.status = _ptr(self.o_unit_offsets), _ptr(self.o_count), _ptr(self.o_status)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = tpc_clusterize(dg, self.geometry, self.params, o, self.workspace.data_ptr(), self.ws_bytes, s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_clusterize: %s" % tpc_status_string(st))
        self._n_units = int(n_units)
        return st

    def result(self, sync=True):
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        n = int(self.o_count.item())
        if st != TPC_OK:
            raise TrackingError(st, "clusterization failed on the device: %s (clusters %d)" % (tpc_status_string(st), n))
        return dict(n=n, y=self.o_y[:n], z=self.o_z[:n], row=self.o_row[:n], qtot=self.o_qtot[:n],
                    qmax=self.o_qmax[:n], pad=self.o_pad[:n], time=self.o_time[:n],
                    unit_offsets=self.o_unit_offsets[:self._n_units + 1])

    def batch(self, row_x, bz):
        """The last result as a tracking Batch over the same device arrays
        (synchronizes once, for the cluster count)."""
        r = self.result()
        b = Batch.__new__(Batch)
        b.y, b.z, b.row = r["y"], r["z"], r["row"]
        b.unit_offsets = r["unit_offsets"]
        b.row_x = torch.as_tensor(np.ascontiguousarray(row_x, np.float32)).to(self.device)
        b.n = r["n"]
        b.n_units = self._n_units
        b.n_rows = int(len(row_x))
        b.bz = float(bz)
        return b


class Compressor:
    """Outputs of tpc_compress for the clusters of a Tracker's last batch."""

    def __init__(self, tracker: Tracker, params=None):
        from . import make_compress_params
        self.params = params if params is not None else make_compress_params()
        self.tracker = tracker
        self.device = tracker.device
        d, n = self.device, max(1, tracker.max_n)
        self.o_cls = torch.empty(n, dtype=torch.uint8, device=d)
        self.o_code_y = torch.empty(n, dtype=torch.int32, device=d)
        self.o_code_z = torch.empty(n, dtype=torch.int32, device=d)
        self.o_hist = torch.zeros(4 * self.params.hist_half, dtype=torch.int64, device=d)
        self.o_counts = torch.zeros(6, dtype=torch.int64, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)

    def launch(self, batch: Batch, stream=None):
        """Enqueue the codes of `batch`, the batch of the tracker's last call."""
        from . import tpc_compress, tpc_compressed_t
        o = tpc_compressed_t()
        o.cls, o.code_y, o.code_z = _ptr(self.o_cls), _ptr(self.o_code_y), _ptr(self.o_code_z)
        o.hist, o.counts, o.status = _ptr(self.o_hist), _ptr(self.o_counts), _ptr(self.o_status)
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = tpc_compress(batch.clusters_struct(), batch.geometry_struct(), f, self.tracker.tracks_struct(),
                          self.params, o, s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_compress: %s" % tpc_status_string(st))
        self._n = batch.n
        return st

    def result(self, sync=True):
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        if st != TPC_OK:
            raise TrackingError(st, "compression failed on the device: %s" % tpc_status_string(st))
        n, h = self._n, self.params.hist_half
        hist = self.o_hist.cpu().numpy()
        return dict(cls=self.o_cls[:n], code_y=self.o_code_y[:n], code_z=self.o_code_z[:n],
                    hist_y=hist[:2 * h], hist_z=hist[2 * h:], counts=self.o_counts.cpu().numpy())


class Refitter:
    """Outputs of tpc_refit_tracks for the tracks of a Tracker's last batch."""

    def __init__(self, tracker: Tracker):
        from . import tpc_refit_workspace_size
        self.tracker = tracker
        self.device = d = tracker.device
        T, H = max(1, tracker.cap_tracks), max(1, tracker.cap_hits)
        self.o_params = torch.empty((T, 5), dtype=torch.float32, device=d)
        self.o_cov = torch.empty((T, 15), dtype=torch.float32, device=d)
        self.o_xref = torch.empty(T, dtype=torch.float32, device=d)
        self.o_chi2 = torch.empty(T, dtype=torch.float32, device=d)
        self.o_params_out = torch.empty((T, 5), dtype=torch.float32, device=d)
        self.o_cov_out = torch.empty((T, 15), dtype=torch.float32, device=d)
        self.o_xout = torch.empty(T, dtype=torch.float32, device=d)
        self.o_ok = torch.empty(T, dtype=torch.uint8, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)
        N = max(1, tracker.max_n)
        self.ws_bytes = tpc_refit_workspace_size(N, T, H)
        if self.ws_bytes == 0:
            raise ValueError("tpc_refit_workspace_size rejected %d clusters, capacities %d tracks, %d hits" % (N, T, H))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d)

    def launch(self, batch: Batch, stream=None):
        """Enqueue the refit of the tracks of `batch`, the batch of the tracker's last call."""
        from . import tpc_refit_t, tpc_refit_tracks
        o = tpc_refit_t()
        o.params, o.cov, o.x_ref, o.chi2 = _ptr(self.o_params), _ptr(self.o_cov), _ptr(self.o_xref), _ptr(self.o_chi2)
        o.params_out, o.cov_out, o.x_out = _ptr(self.o_params_out), _ptr(self.o_cov_out), _ptr(self.o_xout)
        o.ok, o.status = _ptr(self.o_ok), _ptr(self.o_status)
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = tpc_refit_tracks(batch.clusters_struct(), batch.geometry_struct(), f, self.tracker.params,
                              self.tracker.tracks_struct(), o, self.workspace.data_ptr(), self.ws_bytes,
                              s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_refit_tracks: %s" % tpc_status_string(st))
        return st

    def result(self, n_tracks: int, sync=True):
        """Device tensors of the first n_tracks tracks (the tracker's result count)."""
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        if st != TPC_OK:
            raise TrackingError(st, "refit failed on the device: %s" % tpc_status_string(st))
        T = n_tracks
        return dict(params=self.o_params[:T], cov=self.o_cov[:T], x_ref=self.o_xref[:T], chi2=self.o_chi2[:T],
                    params_out=self.o_params_out[:T], cov_out=self.o_cov_out[:T], x_out=self.o_xout[:T],
                    ok=self.o_ok[:T])

    def struct(self):
        """The tpc_refit_t of this refitter's outputs (the merger reads them)."""
        from . import tpc_refit_t
        o = tpc_refit_t()
        o.params, o.cov, o.x_ref, o.chi2 = _ptr(self.o_params), _ptr(self.o_cov), _ptr(self.o_xref), _ptr(self.o_chi2)
        o.params_out, o.cov_out, o.x_out = _ptr(self.o_params_out), _ptr(self.o_cov_out), _ptr(self.o_xout)
        o.ok, o.status = _ptr(self.o_ok), _ptr(self.o_status)
        return o


class Merger:
    """Outputs of tpc_merge_tracks for the tracks of a Tracker's last batch and
    their refit (a Refitter launched on the same batch)."""

    def __init__(self, refitter: Refitter, n_units: int, params=None):
        from . import make_merge_params, tpc_merge_workspace_size
        self.params = params if params is not None else make_merge_params()
        self.refitter = refitter
        self.tracker = refitter.tracker
        self.device = d = self.tracker.device
        T = max(1, self.tracker.cap_tracks)
        self.n_units = int(n_units)
        self.o_next = torch.empty(T, dtype=torch.int32, device=d)
        self.o_prev = torch.empty(T, dtype=torch.int32, device=d)
        self.o_chi2 = torch.empty(T, dtype=torch.float64, device=d)
        self.o_counts = torch.zeros(3, dtype=torch.int64, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)
        n_rows = self.tracker.n_rows if hasattr(self.tracker, "n_rows") else 152
        self.ws_bytes = tpc_merge_workspace_size(self.n_units, n_rows, self.tracker.cap_tracks, self.params)
        if self.ws_bytes == 0:
            raise ValueError("tpc_merge_workspace_size rejected the arguments")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d)

    def launch(self, batch: Batch, unit_alpha, unit_side, stream=None):
        """Enqueue the links of the tracks of `batch`; unit_alpha (radians) and
        unit_side (+1 / -1) per unit, host or device."""
        from . import tpc_merge_tracks, tpc_merged_t
        ua = torch.as_tensor(np.ascontiguousarray(unit_alpha, np.float32)).to(self.device) \
            if not torch.is_tensor(unit_alpha) else unit_alpha
        us = torch.as_tensor(np.ascontiguousarray(unit_side, np.int32)).to(self.device) \
            if not torch.is_tensor(unit_side) else unit_side
        if ua.numel() != self.n_units or us.numel() != self.n_units:
            raise ValueError("unit_alpha and unit_side need %d entries" % self.n_units)
        self._keep = (ua, us)
        o = tpc_merged_t()
        o.next, o.prev, o.link_chi2 = _ptr(self.o_next), _ptr(self.o_prev), _ptr(self.o_chi2)
        o.counts, o.status = _ptr(self.o_counts), _ptr(self.o_status)
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = tpc_merge_tracks(batch.clusters_struct(), batch.geometry_struct(), f, self.tracker.tracks_struct(),
                              self.refitter.struct(), _ptr(ua), _ptr(us), self.n_units, self.params, o,
                              self.workspace.data_ptr(), self.ws_bytes, s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_merge_tracks: %s" % tpc_status_string(st))
        return st

    def struct(self):
        """The tpc_merged_t of this merger's outputs (the chain fit reads them)."""
        from . import tpc_merged_t
        o = tpc_merged_t()
        o.next, o.prev, o.link_chi2 = _ptr(self.o_next), _ptr(self.o_prev), _ptr(self.o_chi2)
        o.counts, o.status = _ptr(self.o_counts), _ptr(self.o_status)
        return o

    def result(self, n_tracks: int, sync=True):
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        counts = self.o_counts.cpu().numpy()
        if st != TPC_OK:
            raise TrackingError(st, "merging failed on the device: %s (counts %s)"
                                % (tpc_status_string(st), counts.tolist()))
        T = n_tracks
        return dict(next=self.o_next[:T], prev=self.o_prev[:T], link_chi2=self.o_chi2[:T],
                    n_pairs=int(counts[0]), n_candidates=int(counts[1]), n_links=int(counts[2]))


class ChainFitter:
    """Outputs of tpc_fit_chains: the fit of the merged chains of a Tracker's
    last batch (a Merger launched on it), indexed by each chain's head track."""

    def __init__(self, tracker):
        from . import tpc_refit_workspace_size
        self.tracker = tracker
        self.device = d = tracker.device
        T = max(1, tracker.cap_tracks)
        self.ws_bytes = tpc_refit_workspace_size(max(1, tracker.max_n), T, max(1, tracker.cap_hits))
        if self.ws_bytes == 0:
            raise ValueError("tpc_refit_workspace_size rejected the tracker's capacities")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d)
        self.o_params = torch.empty((T, 5), dtype=torch.float32, device=d)
        self.o_cov = torch.empty((T, 15), dtype=torch.float32, device=d)
        self.o_xref = torch.empty(T, dtype=torch.float32, device=d)
        self.o_chi2 = torch.empty(T, dtype=torch.float32, device=d)
        self.o_n = torch.empty(T, dtype=torch.int32, device=d)
        self.o_ok = torch.empty(T, dtype=torch.uint8, device=d)
        self.o_status = torch.zeros(1, dtype=torch.int32, device=d)

    def launch(self, batch: Batch, merged, unit_alpha, stream=None):
        """merged: a Merger (or anything with struct()) launched on `batch`;
        unit_alpha: the same angles, a device tensor."""
        from . import tpc_chain_fit_t, tpc_fit_chains
        o = tpc_chain_fit_t()
        o.params, o.cov, o.x_ref, o.chi2 = _ptr(self.o_params), _ptr(self.o_cov), _ptr(self.o_xref), _ptr(self.o_chi2)
        o.n_hits, o.ok, o.status = _ptr(self.o_n), _ptr(self.o_ok), _ptr(self.o_status)
        f = tpc_field_t()
        f.bz_tesla = batch.bz
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = tpc_fit_chains(batch.clusters_struct(), batch.geometry_struct(), f, self.tracker.params,
                            self.tracker.tracks_struct(), merged.struct(), _ptr(unit_alpha), int(unit_alpha.numel()),
                            o, self.workspace.data_ptr(), self.ws_bytes, s.cuda_stream)
        if st != TPC_OK:
            raise TrackingError(st, "tpc_fit_chains: %s" % tpc_status_string(st))
        return st

    def result(self, n_tracks: int, sync=True):
        if sync:
            torch.cuda.synchronize(self.device)
        st = int(self.o_status.item())
        if st != TPC_OK:
            raise TrackingError(st, "chain fit failed on the device: %s" % tpc_status_string(st))
        T = n_tracks
        return dict(params=self.o_params[:T], cov=self.o_cov[:T], x_ref=self.o_xref[:T], chi2=self.o_chi2[:T],
                    n_hits=self.o_n[:T], ok=self.o_ok[:T])

