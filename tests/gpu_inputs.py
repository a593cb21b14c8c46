"""Inputs for the GPU stages downstream of the tracker that do not come from
the GPU: track lists taken from the generator's truth or from the oracle's
own tracker, uploaded into a tpc_tracks_t, so that the GPU stage and the
oracle stage see identical inputs.  Used by the GPU tests only."""
from __future__ import annotations

import numpy as np


def truth_tracks(ev, min_hits=10):
    """Hit lists of the generated particles: per (unit, particle) the clusters
    in increasing row order, for the particles that cross every row of the
    unit at most once (no second leg of a looper in the unit) and leave at
    least min_hits clusters there.  Returns (first_hit, n_hits, hits, unit)."""
    n_units = len(ev.unit_offsets) - 1
    unit = np.repeat(np.arange(n_units, dtype=np.int64), np.diff(ev.unit_offsets))
    ids = np.nonzero(ev.label >= 0)[0]
    key = (unit[ids] << 40) | (ev.label[ids].astype(np.int64) << 8) | ev.row[ids].astype(np.int64)
    o = np.argsort(key, kind="stable")
    ids, key = ids[o], key[o]
    grp = key >> 8
    start = np.r_[0, np.nonzero(grp[1:] != grp[:-1])[0] + 1]
    end = np.r_[start[1:], len(grp)]
    dup = np.zeros(len(grp), bool)
    dup[1:] = key[1:] == key[:-1]  # same (unit, particle, row)
    has_dup = np.add.reduceat(dup.astype(np.int64), start) > 0 if len(start) else np.zeros(0, bool)
    keep = (~has_dup) & (end - start >= min_hits)
    s, e = start[keep], end[keep]
    n_hits = (e - s).astype(np.int32)
    first = np.r_[0, np.cumsum(n_hits)[:-1]].astype(np.int32) if len(n_hits) else np.zeros(0, np.int32)
    hits = np.concatenate([ids[a:b] for a, b in zip(s, e)]).astype(np.int32) if len(s) else np.zeros(0, np.int32)
    return first, n_hits, hits, (grp[s] >> 32).astype(np.int32)


class DeviceTracks:
    """A tpc_tracks_t over device copies of host arrays (a tracker's output
    as far as the downstream stages read it).  Fields not given are zero-
    filled arrays of the right size.  Stands in for a Tracker where the
    runtime's stage classes take one (cap_tracks, cap_hits, device, params,
    tracks_struct())."""

    def __init__(self, n_clusters, first_hit=None, n_hits=None, hits=None, params=None, x_ref=None, unit=None,
                 cluster_track=None, status=0, device="cuda"):
        import torch

        from paper_2106_03636_amd import make_params, tpc_tracks_t

        def dev(a, dtype, n, width=1):
            if a is None:
                a = np.zeros((n, width) if width > 1 else n, dtype)
            t = torch.from_numpy(np.ascontiguousarray(a, dtype).reshape(-1)).to(device)
            return t if t.numel() else torch.zeros(1, dtype=t.dtype, device=device)

        T = len(n_hits) if n_hits is not None else (len(x_ref) if x_ref is not None else 0)
        H = len(hits) if hits is not None else 0
        self.T, self.H = T, H
        self.cap_tracks, self.cap_hits, self.device, self.max_n = T, H, device, n_clusters
        self.params = make_params()  # tracking parameters (the refit reads sigma, cov0, sinphi_max)
        self.first_hit = dev(first_hit, np.int32, T)
        self.n_hits = dev(n_hits, np.int32, T)
        self.hits = dev(hits, np.int32, H)
        self.track_params = dev(params, np.float32, T, 5)
        self.cov = dev(None, np.float32, T, 15)
        self.x_ref = dev(x_ref, np.float32, T)
        self.chi2 = dev(None, np.float32, T)
        self.unit = dev(unit, np.int32, T)
        self.n_fit = dev(n_hits, np.int32, T)
        self.cluster_track = dev(cluster_track if cluster_track is not None else np.full(n_clusters, -1),
                                 np.int32, n_clusters)
        self.counts = dev(np.array([T, H, 0, 0, 0]), np.int64, 5)
        self.o_counts = self.counts  # the name a Tracker gives it
        self.status = dev(np.array([status]), np.int32, 1)
        s = tpc_tracks_t()
        s.cap_tracks, s.cap_hits = T, H
        for f in ("cluster_track", "cov", "x_ref", "chi2", "unit", "n_hits", "n_fit", "first_hit", "hits",
                  "counts", "status"):
            setattr(s, f, getattr(self, f).data_ptr())
        s.params = self.track_params.data_ptr()
        self.struct = s

    def tracks_struct(self):
        return self.struct

    @classmethod
    def from_oracle(cls, o, device="cuda"):
        """The output tracks of an oracle tracking run (oracle.run / run_event),
        their FP64 states rounded to FP32 as a tracking call stores them."""
        tl = o["track_tracklet"]
        return cls(int(o["n"]), o["track_first_hit"], o["track_n_hits"], o["track_hits"],
                   params=o["trk_params"][tl].astype(np.float32), x_ref=o["trk_xref"][tl].astype(np.float32),
                   unit=o["trk_unit"][tl], cluster_track=o["cluster_track"], device=device)


class DeviceRefit:
    """A tpc_refit_t over device copies of a refit's host arrays (the dict
    oracle.refit_tracks returns), rounded to FP32 as the refit call stores
    them.  Stands in for a Refitter where the merger takes one (tracker,
    struct())."""

    def __init__(self, tracks: DeviceTracks, r, status=0):
        import torch

        from paper_2106_03636_amd import tpc_refit_t
        d = tracks.device

        def dev(a, dtype):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype).reshape(-1)).to(d)
            return t if t.numel() else torch.zeros(1, dtype=t.dtype, device=d)

        self.tracker = tracks
        self.arrays = dict(params=dev(r["p"], np.float32), cov=dev(r["cov"], np.float32),
                           x_ref=dev(r["x_ref"], np.float32), chi2=dev(r["chi2"], np.float32),
                           params_out=dev(r["p_out"], np.float32), cov_out=dev(r["cov_out"], np.float32),
                           x_out=dev(r["x_out"], np.float32), ok=dev(r["ok"], np.uint8),
                           status=dev(np.array([status]), np.int32))
        s = tpc_refit_t()
        for f, v in self.arrays.items():
            setattr(s, f, v.data_ptr())
        self._s = s

    def struct(self):
        return self._s


class DeviceMerged:
    """A tpc_merged_t over device copies of links (next, prev) that do not
    come from the GPU (the oracle merger's)."""

    def __init__(self, next_, prev, status=0, device="cuda"):
        import torch

        from paper_2106_03636_amd import tpc_merged_t

        def dev(a, dtype):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype).reshape(-1)).to(device)
            return t if t.numel() else torch.zeros(1, dtype=t.dtype, device=device)

        self.next, self.prev = dev(next_, np.int32), dev(prev, np.int32)
        self.chi2 = dev(np.zeros(len(next_)), np.float64)
        self.counts = dev(np.zeros(3), np.int64)
        self.status = dev(np.array([status]), np.int32)
        s = tpc_merged_t()
        s.next, s.prev, s.link_chi2 = self.next.data_ptr(), self.prev.data_ptr(), self.chi2.data_ptr()
        s.counts, s.status = self.counts.data_ptr(), self.status.data_ptr()
        self._s = s

    def struct(self):
        return self._s

