"""Seeded synthetic TPC inputs shaped like the workloads of arXiv 2106.03636.

The paper's inputs are ALICE Pb-Pb / pp time frames (paper §2, §3.1.3, §3.2),
which are not available; these generators stand in for them.  They produce
TPC clusters of closed-form helices crossing the pad rows of 2 x 18 sectors,
smeared, plus uniform noise, and in continuous-readout form (collision times
spread over a slice and folded into z as the paper's §2 describes: a time
shift appears as a shift along the beam axis).

This module holds no step of the tracking method: it only draws random
numbers (numpy PCG64) and evaluates helix / pad-row intersections (in C, for
speed).  Both the HIP path and the CPU oracle consume its output.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_crossings.so")

# --- detector geometry -------------------------------------------------------
N_ROWS = 152
N_SECTORS = 36
ROW_X0, ROW_X1 = 85.0, 247.0
ROW_X_F32 = (ROW_X0 + np.arange(N_ROWS, dtype=np.float64) * (ROW_X1 - ROW_X0) / (N_ROWS - 1)).astype(np.float32)
ROW_X = ROW_X_F32.astype(np.float64)  # the row planes sit exactly at the float32 positions
HALF_OPEN_DEG = 10.0
TAN_HALF = math.tan(math.radians(HALF_OPEN_DEG))
Z_MAX = 250.0  # drift length, cm
V_DRIFT = 2.58  # cm / us
KAPPA = 0.00299792458  # GeV / (T cm)
SIGMA_Y, SIGMA_Z = 0.1, 0.15  # cm
VERTEX_SIGMA = (0.01, 0.01, 5.0)
NOISE_FRACTION = 0.05
ETA_MAX = 0.9
R_EXIT = ROW_X1 / math.cos(math.radians(HALF_OPEN_DEG))  # outer wall: the corner of the outermost row


def sector_alpha(sector: int) -> float:
    return math.radians((sector % 18) * 20.0 + 10.0)


def build(force: bool = False) -> str:
    """Compile the crossing and digit routines (gcc, OpenMP) next to this file."""
    srcs = [os.path.join(HERE, "crossings.c"), os.path.join(HERE, "digits.c")]
    newest = max(os.path.getmtime(f) for f in srcs)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()  # compiles when missing or older than its source
        lib = ctypes.CDLL(_LIB_PATH)
        d = ctypes.POINTER(ctypes.c_double)
        lib.synth_crossings.restype = ctypes.c_int64
        lib.synth_crossings.argtypes = [ctypes.c_int64, d, d, d, d, d, d, ctypes.c_int, d,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        vp = ctypes.c_void_p
        lib.synth_digits.restype = ctypes.c_int64
        lib.synth_digits.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32] + [ctypes.c_double] * 6 + [
            ctypes.c_int32, ctypes.c_uint64] + [vp] * 9
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Tracks:
    """Truth of generated primaries (global frame)."""
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    pt: np.ndarray
    phi0: np.ndarray
    tgl: np.ndarray
    q: np.ndarray
    t0: np.ndarray  # collision time, us

    def __len__(self):
        return len(self.pt)

    def curvature(self, bz: float) -> np.ndarray:
        return -KAPPA * bz * self.q / self.pt

    @staticmethod
    def concat(parts):
        return Tracks(*[np.concatenate([getattr(p, f) for p in parts]) for f in
                        ("vx", "vy", "vz", "pt", "phi0", "tgl", "q", "t0")])


def helix_crossings(tr: Tracks, bz: float, max_turns: float = 2.0, z_max: float = Z_MAX, r_exit: float = 0.0):
    """All (sector, row) crossings of the helices, noise-free, FP64, true z.
    With r_exit > 0 a helix ends where it first leaves the cylinder of that
    radius (R_EXIT: the outer wall); by default it is followed for max_turns.

    Returns a dict of arrays ordered by (track, sector, row, arc length).
    """
    lib = _load()
    n = len(tr)
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in
            (tr.vx, tr.vy, tr.vz, tr.curvature(bz), tr.phi0, tr.tgl)]
    counts = np.zeros(n, dtype=np.int64)
    lib.synth_crossings(n, *[_dptr(a) for a in args], N_ROWS, _dptr(ROW_X), TAN_HALF, z_max,
                        max_turns, float(r_exit), _ptr(counts), None, None, None, None, None, None, None, None)
    tot = int(counts.sum())
    out = dict(sector=np.empty(tot, np.int32), row=np.empty(tot, np.int32),
               track=np.empty(tot, np.int32), y=np.empty(tot), z=np.empty(tot),
               s=np.empty(tot), sinphi=np.empty(tot), cosphi=np.empty(tot))
    lib.synth_crossings(n, *[_dptr(a) for a in args], N_ROWS, _dptr(ROW_X), TAN_HALF, z_max,
                        max_turns, float(r_exit), _ptr(counts), _ptr(out["sector"]), _ptr(out["row"]),
                        _ptr(out["track"]), _ptr(out["y"]), _ptr(out["z"]), _ptr(out["s"]),
                        _ptr(out["sinphi"]), _ptr(out["cosphi"]))
    return out


# --- primaries ----------------------------------------------------------------

def _eta_to_tgl(eta):
    return np.sinh(eta)


def _vertex(rng, n):
    return (rng.normal(0, VERTEX_SIGMA[0], n), rng.normal(0, VERTEX_SIGMA[1], n),
            rng.normal(0, VERTEX_SIGMA[2], n))


def primaries_pp_sector(rng, n, sector=0, eta_range=(0.0, ETA_MAX), pt_range=(0.1, 10.0), vz=None):
    """pp-like tracks aimed into one sector; pT log-uniform."""
    vx, vy, vz_ = _vertex(rng, n)
    if vz is not None:
        vz_ = vz_ + vz
    a = sector_alpha(sector)
    half = math.radians(HALF_OPEN_DEG)
    phi0 = rng.uniform(a - half, a + half, n)
    lo, hi = np.log(pt_range[0]), np.log(pt_range[1])
    pt = np.exp(rng.uniform(lo, hi, n))
    eta = rng.uniform(eta_range[0], eta_range[1], n)
    q = rng.choice(np.array([-1.0, 1.0]), n)
    return Tracks(vx, vy, vz_, pt, phi0, _eta_to_tgl(eta), q, np.zeros(n))


def _pt_pbpb(rng, n):
    """90% exp(-pT / 0.3 GeV), 10% power-law tail p(pT) ~ (1 + pT/1 GeV)^-6."""
    soft = rng.random(n) < 0.9
    pt = np.empty(n)
    ns = int(soft.sum())
    pt[soft] = rng.exponential(0.3, ns)
    # inverse CDF of (1+x)^-6 on [0, inf): F = 1 - (1+x)^-5
    u = rng.random(n - ns)
    pt[~soft] = (1.0 - u) ** (-1.0 / 5.0) - 1.0
    return np.maximum(pt, 1e-3)


def primaries_pbpb(rng, n, t0=0.0, phi_range=None, vertex=None):
    """Soft Pb-Pb spectrum; a vertex per particle, or the given common one."""
    if vertex is None:
        vx, vy, vz = _vertex(rng, n)
    else:
        vx, vy, vz = (np.full(n, float(c)) for c in vertex)
    if phi_range is None:
        phi0 = rng.uniform(-math.pi, math.pi, n)
    else:
        phi0 = rng.uniform(phi_range[0], phi_range[1], n)
    eta = rng.uniform(-ETA_MAX, ETA_MAX, n)
    q = rng.choice(np.array([-1.0, 1.0]), n)
    return Tracks(vx, vy, vz, _pt_pbpb(rng, n), phi0, _eta_to_tgl(eta), q, np.full(n, float(t0)))


# --- events --------------------------------------------------------------------

@dataclass
class Event:
    """Clusters grouped by unit (one unit = one sector here), FP32 coordinates.

    Order inside a unit is random.  label = index of the generating track in
    `tracks`, or -1 for noise.  z is the continuous-readout coordinate z'.
    """
    y: np.ndarray
    z: np.ndarray
    row: np.ndarray
    unit_offsets: np.ndarray
    unit_sector: np.ndarray
    label: np.ndarray
    tracks: Tracks
    bz: float
    name: str = ""
    row_x: np.ndarray = field(default_factory=lambda: ROW_X_F32.copy())

    @property
    def n(self):
        return int(len(self.y))

    @property
    def n_units(self):
        return int(len(self.unit_offsets) - 1)

    def unit(self, u):
        a, b = int(self.unit_offsets[u]), int(self.unit_offsets[u + 1])
        return slice(a, b)

    def subset_units(self, units):
        """A new event made of the given units (clusters copied, order kept)."""
        parts = [self.unit(int(u)) for u in units]
        y = np.concatenate([self.y[s] for s in parts]) if parts else np.zeros(0, np.float32)
        z = np.concatenate([self.z[s] for s in parts]) if parts else np.zeros(0, np.float32)
        row = np.concatenate([self.row[s] for s in parts]) if parts else np.zeros(0, np.uint16)
        lab = np.concatenate([self.label[s] for s in parts]) if parts else np.zeros(0, np.int32)
        off = np.zeros(len(parts) + 1, np.int64)
        off[1:] = np.cumsum([s.stop - s.start for s in parts])
        return Event(y, z, row, off, self.unit_sector[np.asarray(units, dtype=np.int64)].copy(),
                     lab, self.tracks, self.bz, self.name + "[sub]", self.row_x)


def _assemble(rng, xs, tracks, bz, units_sectors, z_span_of_unit, shift_z, name):
    """Smear crossings, add noise per unit, group by unit, shuffle inside units."""
    sector = xs["sector"]
    keep_unit = np.full(N_SECTORS, -1, np.int64)
    for u, s in enumerate(units_sectors):
        keep_unit[s] = u
    unit = keep_unit[sector]
    m = unit >= 0
    unit = unit[m]
    row = xs["row"][m]
    trk = xs["track"][m]
    y = xs["y"][m] + rng.normal(0, SIGMA_Y, int(m.sum()))
    zt = xs["z"][m]
    side = np.where(sector[m] < 18, 1.0, -1.0)
    z = zt + shift_z(trk, side) + rng.normal(0, SIGMA_Z, int(m.sum()))
    n_units = len(units_sectors)
    ys, zs, rows, labs, units = [y], [z], [row], [trk], [unit]
    sig_per_unit = np.bincount(unit, minlength=n_units)
    for u in range(n_units):
        nn = int(round(NOISE_FRACTION * sig_per_unit[u]))
        if nn == 0:
            continue
        r = rng.integers(0, N_ROWS, nn)
        hw = ROW_X[r] * TAN_HALF
        ys.append(rng.uniform(-1.0, 1.0, nn) * hw)
        zlo, zhi = z_span_of_unit(u)
        zs.append(rng.uniform(zlo, zhi, nn))
        rows.append(r.astype(np.int32))
        labs.append(np.full(nn, -1, np.int32))
        units.append(np.full(nn, u, np.int64))
    y = np.concatenate(ys)
    z = np.concatenate(zs)
    row = np.concatenate(rows)
    lab = np.concatenate(labs)
    unit = np.concatenate(units)
    key = (unit.astype(np.uint64) << np.uint64(40)) | rng.integers(0, 1 << 40, len(unit), dtype=np.uint64)
    order = np.argsort(key, kind="stable")
    off = np.zeros(n_units + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(unit, minlength=n_units))
    return Event(y[order].astype(np.float32), z[order].astype(np.float32),
                 row[order].astype(np.uint16), off, np.asarray(units_sectors, np.int16),
                 lab[order].astype(np.int32), tracks, bz, name)


def _side_span(sector, t_max_us):
    shift = V_DRIFT * t_max_us
    return (0.0 - shift, Z_MAX) if sector < 18 else (-Z_MAX, 0.0 + shift)


def event_pp_sector(seed: int, n_tracks: int = 200, sector: int = 0, bz: float = 0.5) -> Event:
    """One TPC sector, one pp-like event: pT log-uniform 0.1-10 GeV, tracks aimed
    into the sector, |eta| < 0.9 on the sector's side."""
    rng = np.random.default_rng(seed)
    eta_range = (0.0, ETA_MAX) if sector < 18 else (-ETA_MAX, 0.0)
    tr = primaries_pp_sector(rng, n_tracks, sector, eta_range)
    xs = helix_crossings(tr, bz)
    return _assemble(rng, xs, tr, bz, [sector], lambda u: _side_span(sector, 0.0),
                     lambda trk, side: 0.0, "pp_sector")


def event_pbpb_central(seed: int, n_primaries: int = 15000, bz: float = 0.5) -> Event:
    """One central Pb-Pb collision, 36 sector units."""
    rng = np.random.default_rng(seed)
    tr = primaries_pbpb(rng, n_primaries)
    xs = helix_crossings(tr, bz)
    return _assemble(rng, xs, tr, bz, list(range(N_SECTORS)), lambda u: _side_span(u, 0.0),
                     lambda trk, side: 0.0, "pbpb_central")


def pbpb_multiplicity(rng, n):
    """Charged primaries of min-bias Pb-Pb: b with p(b) ~ b on [0, 15] fm,
    N_ch = 15000 (1 - b/15)^1.7 (mean ~3000)."""
    b = 15.0 * np.sqrt(rng.random(n))
    return np.round(15000.0 * (1.0 - b / 15.0) ** 1.7).astype(np.int64)


def event_pbpb_timeframe(seed: int, n_collisions: int = 50, slice_us: float = None,
                         bz: float = 0.5, physical: bool = False) -> Event:
    """Continuous-readout slice: n_collisions min-bias Pb-Pb collisions at times
    uniform over the slice (default n / 50 kHz); z' = z - side * v_drift * t0.

    By default every particle draws its own vertex and its helix is followed
    for two full turns (also after it has left through the outer wall): extra
    passes that load the tracker like loopers and secondaries do.  physical=True
    gives each collision one vertex and ends a helix at the outer wall
    (R_EXIT), as in a detector: the frame on which tracks are assigned to
    collisions."""
    rng = np.random.default_rng(seed)
    if slice_us is None:
        slice_us = n_collisions / 50e3 * 1e6
    mult = pbpb_multiplicity(rng, n_collisions)
    t0s = rng.uniform(0.0, slice_us, n_collisions)
    if physical:
        verts = np.stack(_vertex(rng, n_collisions), axis=1)
        parts = [primaries_pbpb(rng, int(m), t0=t, vertex=v) for m, t, v in zip(mult, t0s, verts)]
    else:
        parts = [primaries_pbpb(rng, int(m), t0=t) for m, t in zip(mult, t0s)]
    tr = Tracks.concat(parts)
    xs = helix_crossings(tr, bz, r_exit=R_EXIT if physical else 0.0)
    t0 = tr.t0

    def shift(trk, side):
        return -side * V_DRIFT * t0[trk]

    return _assemble(rng, xs, tr, bz, list(range(N_SECTORS)),
                     lambda u: _side_span(u, slice_us), shift, "pbpb_timeframe")


def event_uneven_chunks(seed: int, n_units: int = 512, n_lo: float = 1e3, n_hi: float = 1e5,
                        bz: float = 0.5) -> Event:
    """Batched workload: n_units sector chunks of log-uniform size [n_lo, n_hi]
    clusters, each from a pp-like (log-uniform pT) or a Pb-Pb-like (soft
    spectrum) generator, 50/50."""
    rng = np.random.default_rng(seed)
    target = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_units))
    kinds = rng.random(n_units) < 0.5
    ev_parts = []
    all_tracks = []
    trk_base = 0
    for u in range(n_units):
        sector = int(rng.integers(0, N_SECTORS))
        a = sector_alpha(sector)
        half = math.radians(HALF_OPEN_DEG)
        eta_range = (0.0, ETA_MAX) if sector < 18 else (-ETA_MAX, 0.0)
        want = target[u] / (1.0 + NOISE_FRACTION)
        est = max(4, int(want / 60.0))
        while True:
            if kinds[u]:
                tr = primaries_pp_sector(rng, est, sector, eta_range)
            else:
                tr = primaries_pbpb(rng, est, phi_range=(a - half, a + half))
                tr.tgl = np.abs(tr.tgl) * (1.0 if sector < 18 else -1.0)
            xs = helix_crossings(tr, bz)
            m = xs["sector"] == sector
            per_trk = np.bincount(xs["track"][m], minlength=est)
            cum = np.cumsum(per_trk)
            if cum[-1] >= want or est > 200000:
                k = int(np.searchsorted(cum, want)) + 1
                k = min(k, est)
                break
            est *= 2
        sel = m & (xs["track"] < k)
        sub = {key: v[sel] for key, v in xs.items()}
        sub["track"] = sub["track"] + trk_base
        trk_base += k
        all_tracks.append(Tracks(*[getattr(tr, f)[:k] for f in
                                   ("vx", "vy", "vz", "pt", "phi0", "tgl", "q", "t0")]))
        ev_parts.append((sector, sub))
    # assemble each unit separately (units may repeat a sector)
    ys, zs, rows, labs, offs, secs = [], [], [], [], [0], []
    tracks = Tracks.concat(all_tracks)
    for u, (sector, sub) in enumerate(ev_parts):
        sub = dict(sub)
        sub["sector"] = np.zeros_like(sub["sector"])  # unit-local: map the sector to slot 0
        e = _assemble(rng, sub, tracks, bz, [0], lambda _u, s=sector: _side_span(s, 0.0),
                      lambda trk, side: 0.0, "chunk")
        # _assemble used slot 0 (A side) for the side test only through sector ids; z kept
        ys.append(e.y); zs.append(e.z); rows.append(e.row); labs.append(e.label)
        offs.append(offs[-1] + e.n)
        secs.append(sector)
    return Event(np.concatenate(ys), np.concatenate(zs), np.concatenate(rows),
                 np.asarray(offs, np.int64), np.asarray(secs, np.int16), np.concatenate(labs),
                 tracks, bz, "uneven_chunks")


# --- serving: time frames composed from libraries of collisions ----------------

@dataclass
class CollisionLibrary:
    """Smeared clusters of collisions generated at t0 = 0, grouped by
    (collision, sector) and in random order inside each group."""
    y: np.ndarray
    z: np.ndarray
    row: np.ndarray
    label: np.ndarray
    offsets: np.ndarray  # [n_collisions * N_SECTORS + 1]
    n_collisions: int


def collision_library(rng, tracks_per_collision, bz: float = 0.5) -> CollisionLibrary:
    """Min-bias primaries (the soft Pb-Pb spectrum) of each collision."""
    counts = np.asarray(tracks_per_collision, np.int64)
    parts = [primaries_pbpb(rng, int(k)) for k in counts]
    tr = Tracks.concat(parts)
    coll = np.repeat(np.arange(len(counts)), counts)
    xs = helix_crossings(tr, bz)
    n = len(xs["y"])
    key = (coll[xs["track"]].astype(np.uint64) * np.uint64(N_SECTORS) + xs["sector"].astype(np.uint64))
    key = (key << np.uint64(32)) | rng.integers(0, 1 << 32, n, dtype=np.uint64)
    order = np.argsort(key)
    grp = (key[order] >> np.uint64(32)).astype(np.int64)
    off = np.zeros(len(counts) * N_SECTORS + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(grp, minlength=len(counts) * N_SECTORS))
    y = (xs["y"] + rng.normal(0, SIGMA_Y, n))[order].astype(np.float32)
    z = (xs["z"] + rng.normal(0, SIGMA_Z, n))[order].astype(np.float32)
    return CollisionLibrary(y, z, xs["row"][order].astype(np.uint16), xs["track"][order].astype(np.int32), off,
                            len(counts))


def compose_timeframe(rng, lib: CollisionLibrary, collisions, slice_us: float, bz: float = 0.5,
                      name: str = "tf") -> Event:
    """A continuous-readout frame of the given library collisions at times
    uniform over the slice (z' = z - side * v_drift * t0), 36 sector units,
    plus 5% uniform noise per unit.  Labels are library track ids."""
    collisions = np.asarray(collisions, np.int64)
    t0 = rng.uniform(0.0, slice_us, len(collisions))
    ys, zs, rows, labs, offs = [], [], [], [], [0]
    for u in range(N_SECTORS):
        side = 1.0 if u < 18 else -1.0
        a = lib.offsets[collisions * N_SECTORS + u]
        b = lib.offsets[collisions * N_SECTORS + u + 1]
        lens = b - a
        idx = np.concatenate([np.arange(x, y) for x, y in zip(a, b)]) if len(a) else np.zeros(0, np.int64)
        shift = np.repeat((-side * V_DRIFT * t0).astype(np.float32), lens)
        nn = int(round(NOISE_FRACTION * len(idx)))
        r = rng.integers(0, N_ROWS, nn)
        zlo, zhi = _side_span(u, slice_us)
        ys += [lib.y[idx], (rng.uniform(-1.0, 1.0, nn) * ROW_X[r] * TAN_HALF).astype(np.float32)]
        zs += [lib.z[idx] + shift, rng.uniform(zlo, zhi, nn).astype(np.float32)]
        rows += [lib.row[idx], r.astype(np.uint16)]
        labs += [lib.label[idx], np.full(nn, -1, np.int32)]
        offs.append(offs[-1] + len(idx) + nn)
    empty = Tracks(*[np.zeros(0) for _ in range(8)])
    return Event(np.concatenate(ys), np.concatenate(zs).astype(np.float32), np.concatenate(rows),
                 np.asarray(offs, np.int64), np.arange(N_SECTORS, dtype=np.int16), np.concatenate(labs),
                 empty, bz, name)


def serving_pool(seed: int = 5001, n_frames: int = 32, pbpb_fraction: float = 0.8, pbpb_collisions=(10, 50),
                 pp_collisions: int = 500, pp_tracks_mean: float = 10.0, pp_rate_khz: float = 1000.0,
                 lib_pbpb: int = 64, lib_pp: int = 2000, bz: float = 0.5):
    """Frames a request stream draws from: a pbpb_fraction share of Pb-Pb
    slices of U{pbpb_collisions} min-bias collisions (slice = n / 50 kHz), the
    rest pp frames of pp_collisions collisions of Poisson(pp_tracks_mean)
    tracks at pp_rate_khz.  Collisions come from libraries of lib_pbpb Pb-Pb
    and lib_pp pp collisions, each drawn at its own time, so frames share
    collisions but no two frames are alike.  Returns a list of Events."""
    rng = np.random.default_rng(seed)
    libA = collision_library(rng, pbpb_multiplicity(rng, lib_pbpb), bz)
    libP = collision_library(rng, rng.poisson(pp_tracks_mean, lib_pp), bz)
    frames = []
    for i in range(n_frames):
        if rng.random() < pbpb_fraction:
            k = int(rng.integers(pbpb_collisions[0], pbpb_collisions[1] + 1))
            coll = rng.choice(lib_pbpb, size=k, replace=k > lib_pbpb)
            frames.append(compose_timeframe(rng, libA, coll, k / 50e3 * 1e6, bz, "pbpb_slice_%d" % k))
        else:
            coll = rng.choice(lib_pp, size=pp_collisions, replace=pp_collisions > lib_pp)
            frames.append(compose_timeframe(rng, libP, coll, pp_collisions / pp_rate_khz * 1e3, bz, "pp_frame"))
    return frames


# --- raw ADC digits (clusterizer input) ---------------------------------------

PAD_W = 0.6                     # pad width, cm
TIME_BIN = 0.2 * V_DRIFT        # one 200 ns time bin, cm of drift
Z_OFF = 4096.0                  # time bin t is centred at z' = (t + 0.5) TIME_BIN - Z_OFF
SIG_PAD, SIG_TIME = 0.7, 0.7    # response widths, in pads and time bins
NOISE_ADC, THR_ADC = 1.0, 3     # noise (ADC rms) and zero-suppression threshold
PAD_HALF = np.ceil(ROW_X * TAN_HALF / PAD_W).astype(np.int32)  # row r has 2 * PAD_HALF[r] pads
PADS_TOTAL = int(2 * PAD_HALF.sum())
PAD_ROW_BASE = np.concatenate([[0], np.cumsum(2 * PAD_HALF)]).astype(np.int64)  # first pad of each row


@dataclass
class Digits:
    """Zero-suppressed ADC digits grouped by (unit, row, pad), times increasing
    inside a pad: digit k of pad (u, r, p) is at pad_offsets[u * PADS_TOTAL +
    PAD_ROW_BASE[r] + p] + k.  `clusters` is the event whose clusters made
    them (its labels are the truth)."""
    time: np.ndarray
    q: np.ndarray
    pad_offsets: np.ndarray
    n_units: int
    clusters: Event
    name: str = ""

    @property
    def n(self):
        return int(self.pad_offsets[-1])


def event_digits(ev: Event, seed: int, charge_mean: float = 60.0, charge_min: float = 40.0,
                 noise: float = NOISE_ADC) -> Digits:
    """Digits of every cluster of `ev` (signal and noise clusters alike): a
    charge of charge_min + Exp(charge_mean) ADC spread over +-2 pads and time
    bins by Gaussian responses (SIG_PAD, SIG_TIME), overlaps summed, noise of
    NOISE_ADC rms, rounded, kept from THR_ADC, clipped to 1023."""
    lib = _load()
    rng = np.random.default_rng(seed)
    n_units, n_rows = ev.n_units, N_ROWS
    unit = np.repeat(np.arange(n_units, dtype=np.int64), np.diff(ev.unit_offsets))
    key = unit * n_rows + ev.row.astype(np.int64)
    order = np.argsort(key, kind="stable").astype(np.int64)
    ur = np.zeros(n_units * n_rows + 1, np.int64)
    ur[1:] = np.cumsum(np.bincount(key, minlength=n_units * n_rows))
    q = charge_min + rng.exponential(charge_mean, ev.n)
    max_pads = int(2 * PAD_HALF.max())
    counts = np.zeros(n_units * n_rows * max_pads, np.int64)
    y = np.ascontiguousarray(ev.y, np.float32)
    z = np.ascontiguousarray(ev.z, np.float32)
    args = (n_units, n_rows, _ptr(PAD_HALF), max_pads, PAD_W, TIME_BIN, Z_OFF, SIG_PAD, SIG_TIME, float(noise),
            THR_ADC, int(seed) & ((1 << 64) - 1), _ptr(ur), _ptr(order), _ptr(y), _ptr(z), _ptr(q), _ptr(counts))
    lib.synth_digits(*args, None, None, None)
    # compact CSR over (unit, row, pad) from the padded [unit * row][max_pads] counts
    cm = counts.reshape(n_units, n_rows, max_pads)
    valid = np.arange(max_pads)[None, :] < (2 * PAD_HALF)[:, None]
    per_pad = cm[:, valid]  # [n_units, PADS_TOTAL] in (row, pad) order
    off = np.zeros(n_units * PADS_TOTAL + 1, np.int64)
    off[1:] = np.cumsum(per_pad.reshape(-1))
    starts = np.zeros_like(cm)
    starts[:, valid] = off[:-1].reshape(n_units, PADS_TOTAL)
    starts = np.ascontiguousarray(starts.reshape(-1))
    time = np.empty(int(off[-1]), np.uint16)
    qq = np.empty(int(off[-1]), np.uint16)
    lib.synth_digits(*args, _ptr(starts), _ptr(time), _ptr(qq))
    return Digits(time, qq, off, n_units, ev, ev.name + "_digits")


WORKLOADS = {
    "pp_sector": lambda seed=1001: event_pp_sector(seed),
    "pbpb_central": lambda seed=2001: event_pbpb_central(seed),
    "pbpb_timeframe_50": lambda seed=3001: event_pbpb_timeframe(seed),
    "uneven_chunks_512": lambda seed=4001: event_uneven_chunks(seed),
}
