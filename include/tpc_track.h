/*
 * tpc_track.h -- C ABI of the MI355X (gfx950) TPC sector track finder.
 *
 * The operation: find the tracks of charged particles in the clusters (hits)
 * of a TPC time frame.  Paper §2.1 states that TPC track finding over all
 * collisions of a time frame is the dominant synchronous GPU workload and that
 * it needs no other detector; paper §2.3 states that in continuous readout the
 * collisions overlap and hits carry no a-priori absolute z, which is why this
 * interface takes z' as measured (drift time times drift velocity) and never a
 * vertex z.  The clusters come from the clusterizer (paper §2.1); this library
 * consumes them and returns tracks plus a cluster-to-track map, per unit
 * (a TPC sector, or a chunk of one).  Units are independent.
 *
 * Steps, all on the GPU:
 *   1. ingest and validate;
 *   2. hit grid: per (unit, pad row) the clusters are binned in (y, z') and
 *      sorted by (row, bin, cluster id);
 *   3. neighbour finder: each cluster of rows 1..n_rows-2 keeps the best pair
 *      (one cluster in the row below, one in the row above) by an integer
 *      straight-line residual;
 *   4. cleaner: only mutual links survive; clusters with an upward link and no
 *      downward link start chains (a cellular automaton over pad rows);
 *   5. tracklet constructor: FP32 Kalman filter, two passes with pickup of
 *      further clusters; every cluster is owned by the tracklet with most hits;
 *   6. selector: tracklets that own enough of their hits become tracks.
 *
 * Conventions
 *   - Every pointer inside the structs is a DEVICE pointer (memory visible to
 *     the GPU), allocated and freed by the caller.  The library never
 *     allocates, frees or synchronizes.
 *   - Coordinates are in cm, in the local frame of the unit's sector: x along
 *     the sector's centre line (given per pad row), y across it, z' along the
 *     beam.  Decisions use coordinates rounded to 1/256 cm.
 *   - Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 *     void*; NULL = the default stream).  Results are valid once that stream
 *     has completed the work.
 *   - The return value reports errors the host can see (bad arguments, too
 *     small workspace, launch failures).  Errors that depend on the data
 *     (invalid clusters, capacities exceeded) are written to *out->status on
 *     the device; read it after the stream completes.  When it is not TPC_OK,
 *     no track output is valid; out->counts still reports required sizes for
 *     TPC_E_CAPACITY: counts[0] and [1] against cap_tracks and cap_hits,
 *     counts[4] (seeds) against the seed capacity n / tracklet_cap_div + 64
 *     (retry with a div of at most n / (counts[4] - 64), or l_min).
 */
#ifndef TPC_TRACK_H
#define TPC_TRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_PARAMS_VERSION 1

/* status codes */
#define TPC_OK 0
#define TPC_E_INVALID (-1)  /* malformed arguments or input data */
#define TPC_E_CAPACITY (-2) /* an output or internal capacity is too small */
#define TPC_E_NOMEM (-3)    /* the workspace is smaller than tpc_workspace_size() */
#define TPC_E_HIP (-4)      /* a HIP runtime call failed */
#define TPC_E_BUSY (-5)     /* reserved for callers that queue work */

/* Clusters of one batch.  Units are contiguous ranges of the arrays; the order
 * of clusters inside a unit is arbitrary.  A cluster's id is its index in the
 * arrays; ids break ties, so results do not depend on how the grid is binned. */
typedef struct tpc_clusters {
  int64_t n;                   /* number of clusters, 0 <= n < 2^30 */
  int32_t n_units;             /* >= 1 */
  int32_t reserved;
  const int64_t *unit_offsets; /* [n_units + 1], non-decreasing, [0] = 0, [n_units] = n;
                                  each unit holds fewer than 2^24 clusters */
  const float *y;              /* [n] local y, |y| <= 8192 */
  const float *z;              /* [n] z' (continuous readout), |z'| <= 8192 */
  const uint16_t *row;         /* [n] pad row, < n_rows */
} tpc_clusters_t;

/* Pad-row geometry shared by all units. */
typedef struct tpc_geometry {
  int32_t n_rows;              /* 3 <= n_rows <= 255 */
  int32_t reserved;
  const float *row_x;          /* [n_rows] row positions x_i (cm), increasing, 1 <= x < 8192 */
} tpc_geometry_t;

/* Solenoid field along z. */
typedef struct tpc_field {
  float bz_tesla;              /* 0 is allowed: straight tracks, q/pT not measured */
} tpc_field_t;

/* Tracking parameters.  Integer lengths are in quanta of 1/256 cm. */
typedef struct tpc_params {
  int32_t version;             /* TPC_PARAMS_VERSION */
  int32_t q_shift;             /* must be 8 */
  int32_t tan_half_q16;        /* tan(half sector opening) * 2^16; row half width
                                  H_i = (X_i * tan_half_q16) >> 16, X_i = rint(256 x_i) */
  int32_t bin_y_q;             /* grid: y bin width (at most 63 bins per row) */
  int32_t bin_occ;             /* grid: target clusters per bin (z bins adapt) */
  int32_t bin_zmin_q;          /* grid: shortest z bin */
  int32_t win_y_q, win_z_q;    /* neighbour windows: |Y_n X_i - Y_m X_j| <= win_y X_i,
                                  |Z_n - Z_m| <= win_z */
  int32_t w_y, w_z;            /* residual weights of the neighbour and pickup scores */
  int64_t smax_k;              /* neighbour cut: score <= smax_k (X_{i+1} - X_{i-1})^2 */
  int32_t l_min;               /* shortest chain that seeds a tracklet (>= 3) */
  int32_t ext_win_y_q;         /* pickup window around the rounded prediction */
  int32_t ext_win_z_q;
  int32_t ext_edge_q;          /* a walk stops once |Y_pred| > H_i + ext_edge_q */
  int32_t max_miss;            /* ... or after more than max_miss consecutive misses */
  int32_t n_min;               /* selector: at least n_min owned hits */
  int32_t f_min_q8;            /* selector: owned * 256 >= f_min_q8 * hits */
  int32_t tracklet_cap_div;    /* seed capacity = n / div + 64 (>= 2): tracklets with a chain
                                  of >= l_min hits that the constructor fits; the workspace
                                  holds a 152-row hit table per seed.  Seeds never exceed
                                  n / l_min, so div = l_min can never overflow; 16 holds the
                                  synthetic Pb-Pb time frames (about n / 27 seeds) */
  float sinphi_max;            /* walks stop when |sin(phi)| reaches this (0 < . < 1) */
  float sigma_y, sigma_z;      /* cluster resolution (cm), Kalman measurement errors */
  float cov0[5];               /* diagonal of the initial covariance */
  int32_t reserved;
} tpc_params_t;

/* Outputs.  Tracks are ordered by (unit, grid position of the chain's first
 * cluster); a track's hits are contiguous in `hits`, in increasing row order. */
typedef struct tpc_tracks {
  int64_t cap_tracks;          /* capacity of the per-track arrays */
  int64_t cap_hits;            /* capacity of `hits` */
  int32_t *cluster_track;      /* [n] track index of each cluster, -1 = none */
  float *params;               /* [cap_tracks][5] y, z, sin(phi), tan(lambda), q/pT at x_ref */
  float *cov;                  /* [cap_tracks][15] lower triangle, row-major */
  float *x_ref;                /* [cap_tracks] x of the innermost fitted hit */
  float *chi2;                 /* [cap_tracks] */
  int32_t *unit;               /* [cap_tracks] */
  int32_t *n_hits;             /* [cap_tracks] hits assigned to the track */
  int32_t *n_fit;              /* [cap_tracks] hits used by the fit (ndf = 2 n_fit - 5) */
  int32_t *first_hit;          /* [cap_tracks] offset into hits */
  int32_t *hits;               /* [cap_hits] cluster ids */
  int64_t *counts;             /* [5] n_tracks, n_track_hits, n_tracklets, n_grid_cells, n_seeds */
  int32_t *status;             /* [1] TPC_OK or a negative status (see above) */
} tpc_tracks_t;

/* Bytes of device workspace tpc_track_sectors needs for a batch of n_clusters
 * clusters in n_units units (an upper bound; host-only, pure).  0 on bad
 * arguments. */
size_t tpc_workspace_size(int64_t n_clusters, int32_t n_units, int32_t n_rows,
                          const tpc_params_t *params);

/* Track all units of a batch.  `workspace` is device memory of at least
 * tpc_workspace_size() bytes, aligned to 256 bytes, owned by the caller and
 * reused freely between calls (it holds no state across calls).  Calls that
 * share a workspace must be ordered on one stream.  Returns TPC_OK when the
 * work was enqueued. */
int tpc_track_sectors(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                      const tpc_field_t *field, const tpc_params_t *params, tpc_tracks_t *out,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Same as tpc_track_sectors, and records HIP events (hipEvent_t passed as
 * void*, created by the caller) on the stream around every kernel the call
 * launches: events[k] right before kernel k, events[tpc_kernel_count()] after
 * the last one.  n_events must be tpc_kernel_count() + 1.  For measurement;
 * results are those of tpc_track_sectors. */
int tpc_track_sectors_profiled(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                               const tpc_field_t *field, const tpc_params_t *params,
                               tpc_tracks_t *out, void *workspace, size_t workspace_bytes,
                               void *stream, void *const *events, int32_t n_events);

/* Bytes of the device scratch array tpc_track_sectors_noalloc uses as its
 * workspace (one array per GPU, held from the library's first use on that GPU
 * until the process ends). */
#define TPC_SCRATCH_BYTES (64u << 20)

/* Same as tpc_track_sectors, but allocates nothing and takes no workspace: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid allocation).  The workspace is the
 * library's own scratch array on the device that runs `stream`; its address is
 * looked up on the first call on each device.  Returns TPC_E_NOMEM when
 * tpc_workspace_size() of the batch exceeds TPC_SCRATCH_BYTES, TPC_E_HIP when
 * the array's address cannot be obtained; otherwise as tpc_track_sectors, with
 * the same results.  All calls on one GPU share that GPU's array, which keeps
 * the last call's contents (each call clears what it needs): calls that may
 * overlap in time on one GPU (several streams or host threads) race and must
 * be ordered by the caller, e.g. on one stream. */
int tpc_track_sectors_noalloc(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                              const tpc_field_t *field, const tpc_params_t *params,
                              tpc_tracks_t *out, void *stream);

/* Number of kernels one call launches, and the name of kernel i (host-only). */
int32_t tpc_kernel_count(void);
const char *tpc_kernel_name(int32_t i);

/* Human-readable text of a status code (static storage). */
const char *tpc_status_string(int status);

/* ------------------------------------------------------------------------- */
/* Clusterizer.  The producer of the clusters above: the paper states that a */
/* clusterizing algorithm turns the TPC's raw ADC values into hits (§2.1)    */
/* and that it runs much faster on GPUs than on CPUs (§3.2); it does not     */
/* describe it.  What this call computes:                                    */
/*   - input: zero-suppressed digits (time bin, ADC charge) grouped by       */
/*     (unit, row, pad), times strictly increasing inside a pad;             */
/*   - a digit of charge v at (pad p, time t) is a peak when v >= q_min and  */
/*     every digit among its eight neighbours (pads p-1..p+1 of the same     */
/*     row, times t-1..t+1) is smaller, or equal and later in (pad, time)    */
/*     order (so a plateau of equal charges yields one peak, its first       */
/*     digit);                                                               */
/*   - the cluster of a peak sums the digits of the 3x3 window around it:    */
/*     qtot = sum v, and the first moments in pad and time; its centre is    */
/*     pad = p + sum v (p' - p) / qtot, time = t + sum v (t' - t) / qtot     */
/*     (FP64), its position y = (pad + 0.5 - half[row]) pad_width and       */
/*     z' = (time + 0.5) time_bin - z_offset (FP64, rounded once to FP32);   */
/*   - clusters come in the order of their peaks: (unit, row, pad, time).    */
/* y, z, row and unit_offsets of the output form the tpc_clusters_t that     */
/* tpc_track_sectors takes.                                                  */
/* ------------------------------------------------------------------------- */

/* Pads: row r has 2 half[r] pads, pad p centred at y = (p + 0.5 - half[r]) *
 * pad_width; time bin t centred at z' = (t + 0.5) * time_bin - z_offset. */
typedef struct tpc_pad_geometry {
  int32_t n_rows;              /* 1..255 */
  int32_t pads_total;          /* sum over rows of 2 half[r] (pads per unit) */
  const int32_t *half;         /* [n_rows] device, >= 1 */
  float pad_width;             /* cm, > 0 */
  float time_bin;              /* cm of drift per time bin, > 0 */
  float z_offset;              /* cm */
  int32_t reserved;
} tpc_pad_geometry_t;

/* Digits (device pointers).  Digit k of pad (u, r, p) is at
 * pad_offsets[u * pads_total + (pads of rows < r) + p] + k. */
typedef struct tpc_digits {
  int64_t n;                   /* number of digits, 0 <= n < 2^31 */
  int32_t n_units;             /* >= 1 */
  int32_t reserved;
  const int64_t *pad_offsets;  /* [n_units * pads_total + 1], non-decreasing, [0] = 0, last = n */
  const uint16_t *time;        /* [n] time bin, strictly increasing inside a pad */
  const uint16_t *q;           /* [n] ADC charge */
} tpc_digits_t;

typedef struct tpc_clusterizer_params {
  int32_t q_min;               /* smallest peak charge, >= 1 */
  int32_t reserved;
} tpc_clusterizer_params_t;

/* Outputs (device pointers, allocated by the caller). */
typedef struct tpc_cluster_out {
  int64_t cap;                 /* capacity of the per-cluster arrays */
  float *y, *z;                /* [cap] position (cm) */
  uint16_t *row;               /* [cap] */
  int32_t *qtot;               /* [cap] charge of the 3x3 window */
  uint16_t *qmax;              /* [cap] peak charge */
  float *pad, *time;           /* [cap] centre in pads and time bins */
  int64_t *unit_offsets;       /* [n_units + 1] first cluster of each unit */
  int64_t *count;              /* [1] clusters found (also when it exceeds cap) */
  int32_t *status;             /* [1] TPC_OK, TPC_E_INVALID (malformed offsets or times),
                                  TPC_E_CAPACITY (count > cap); outputs valid only with TPC_OK */
} tpc_cluster_out_t;

/* Bytes of device workspace tpc_clusterize needs (host-only; 0 on bad shapes). */
size_t tpc_clusterize_workspace_size(int32_t n_units, const tpc_pad_geometry_t *geometry);

/* Clusters of all digits, enqueued on `stream`; the workspace (aligned to 256
 * bytes) holds no state across calls.  Returns TPC_OK when the work was
 * enqueued, TPC_E_INVALID / TPC_E_NOMEM on bad arguments or a small
 * workspace, TPC_E_HIP on a launch failure. */
int tpc_clusterize(const tpc_digits_t *digits, const tpc_pad_geometry_t *geometry,
                   const tpc_clusterizer_params_t *params, tpc_cluster_out_t *out, void *workspace,
                   size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------- */
/* Hit removal and track-model compression.  The consumer of the tracks: the */
/* paper states that hits of tracks not used for physics are removed and the */
/* remaining hits go through entropy-reduction steps such as the track model */
/* compression (§2.1); it does not give them.  What this call computes, per  */
/* cluster of a tracking call's input:                                       */
/*   - class 2 (removed): attached to a track with |q/pT| pt_remove > 1;     */
/*   - class 1 (residual): attached to another track whose helix, carried    */
/*     in FP64 from the track's state at x_ref to the cluster's row, stays   */
/*     within |sin(phi)| < sinphi_max: codes (y - y_track) / step and        */
/*     (z - z_track) / step, rounded half to even;                           */
/*   - class 0 (no track) and 3 (attached, helix does not reach the row):    */
/*     codes y / step and z / step, rounded half to even.                    */
/* Class-1 codes are also histogrammed, so the bits an entropy coder would   */
/* need follow from the histograms (the coder itself is not part of this     */
/* library).  Helix: C = -0.00299792458f * bz * q/pT as the tracker's fit    */
/* uses; sin(phi) grows by C dx, y by dx (sin1 + sin2) / (cos1 + cos2), z by */
/* tan(lambda) times the transverse arc length 2 asin(C L / 2) / C over the  */
/* chord L.                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct tpc_compress_params {
  float step;                  /* code unit (cm), > 0 */
  float pt_remove;             /* GeV, >= 0 (0 removes nothing) */
  float sinphi_max;            /* the helix model's limit, 0 < . < 1 */
  int32_t hist_half;           /* histograms cover codes [-hist_half, hist_half), 1..2048 */
} tpc_compress_params_t;

/* Outputs (device pointers, allocated by the caller). */
typedef struct tpc_compressed {
  uint8_t *cls;                /* [n] class of each cluster (0..3, above) */
  int32_t *code_y, *code_z;    /* [n] codes (0 for removed clusters) */
  int64_t *hist;               /* [4 hist_half]: class-1 y codes, then z codes; bin = code + hist_half */
  int64_t *counts;             /* [6]: clusters of classes 0..3, class-1 y and z codes outside the histograms */
  int32_t *status;             /* [1] TPC_OK, or the tracking call's own status when that is not TPC_OK */
} tpc_compressed_t;

/* Codes of the clusters of a tpc_track_sectors call (the same clusters and
 * geometry, and that call's output), enqueued on `stream` after it.  No
 * workspace.  Returns TPC_OK when the work was enqueued, TPC_E_INVALID on bad
 * arguments, TPC_E_HIP on a launch failure. */
int tpc_compress(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry, const tpc_field_t *field,
                 const tpc_tracks_t *tracks, const tpc_compress_params_t *params, tpc_compressed_t *out,
                 void *stream);

/* ------------------------------------------------------------------------- */
/* Collision assignment.  In continuous readout the collisions of a time     */
/* frame overlap in the drift volume, and tracks are assigned to them only   */
/* after tracking (paper §2, §2.3); the paper does not describe how.  What   */
/* this call computes:                                                       */
/*   - per track, z'_dca: z' at the transverse point of closest approach of  */
/*     its helix to the beam axis (FP64, from the FP32 state at x_ref, with  */
/*     curvature C = -0.00299792458f * bz * q/pT as the tracker's fit uses). */
/*     A track from a collision at time t0 and vertex z_v has                */
/*     z'_dca = z_v - side v_drift t0 (side +1 for A, -1 for C);             */
/*   - per side, a histogram of z'_dca over [-z_range, z_range) in bins of   */
/*     bin_width, of the "forming" tracks only: |C| < c_max.  A track whose  */
/*     circle fits inside the TPC (a looper) may be seen on a later leg or   */
/*     turn, where z'_dca is off by the z advance of a turn; c_max = 2 /     */
/*     (outer radius) keeps those out;                                       */
/*   - candidates: bins holding at least n_min forming tracks that are the  */
/*     largest within `reach` bins either side (a lower bin as large wins),  */
/*     numbered side A first, then by increasing bin;                        */
/*   - every track in the range (loopers too) joins the candidate whose bin  */
/*     is nearest to its own within `reach` bins (the lower one on a tie),   */
/*     else none (-1);                                                       */
/*   - per candidate: the tracks and forming tracks it holds, z = the mean   */
/*     z'_dca of its forming tracks (summed in fixed point, 2^-16 cm per     */
/*     track, so the result does not depend on the order of the sums), and   */
/*     t0 = -side z / v_drift (us), the vertex taken at z = 0.               */
/* ------------------------------------------------------------------------- */

typedef struct tpc_collision_params {
  float v_drift;               /* drift velocity (cm/us), > 0 */
  float bin_width;             /* histogram bin width (cm), > 0 */
  float z_range;               /* histogram range [-z_range, z_range), <= 2^20 cm;
                                  ceil(2 z_range / bin_width) <= 65536 bins per side */
  float c_max;                 /* forming tracks: |curvature| < c_max (1/cm), >= 0 */
  int32_t n_min;               /* forming tracks a candidate's bin holds at least, >= 1 */
  int32_t reach;               /* bins, 0 <= reach <= 64 */
} tpc_collision_params_t;

/* Outputs (device pointers, allocated by the caller). */
typedef struct tpc_collisions {
  int64_t cap;                 /* capacity of the per-candidate arrays */
  double *zdca;                /* [cap_tracks of the input] z'_dca per track */
  int32_t *collision;          /* [cap_tracks] candidate of each track, -1 none */
  int32_t *side;               /* [cap] +1 (A) or -1 (C) */
  int32_t *bin;                /* [cap] histogram bin on its side */
  int32_t *count;              /* [cap] tracks assigned */
  int32_t *n_form;             /* [cap] forming tracks assigned (>= n_min) */
  double *z;                   /* [cap] mean z'_dca of the forming tracks (cm) */
  double *t0;                  /* [cap] (us) */
  int64_t *n_collisions;       /* [1] number of candidates (also when it exceeds cap) */
  int32_t *status;             /* [1] TPC_OK, the tracker's own status when that is not TPC_OK,
                                  TPC_E_INVALID (a track's unit has no side +-1), or
                                  TPC_E_CAPACITY (n_collisions > cap); outputs are valid
                                  only with TPC_OK */
} tpc_collisions_t;

/* Bytes of device workspace tpc_assign_collisions needs (host-only, pure;
 * 0 on bad parameters). */
size_t tpc_collisions_workspace_size(const tpc_collision_params_t *params);

/* Assign the tracks of a tpc_track_sectors output to collisions.  `tracks` is
 * that call's output struct (params, x_ref, unit, counts, status are read on
 * the device, cap_tracks on the host); unit_side is a device array of n_units
 * entries, +1 or -1, the side of each unit's sector.  Enqueued on `stream`
 * after the tracking call (same stream, or ordered by the caller); the
 * workspace (aligned to 256 bytes) holds no state across calls.  Returns
 * TPC_OK when the work was enqueued, TPC_E_INVALID / TPC_E_NOMEM on bad
 * arguments or a small workspace, TPC_E_HIP on a launch failure. */
int tpc_assign_collisions(const tpc_tracks_t *tracks, const int32_t *unit_side, int32_t n_units,
                          const tpc_field_t *field, const tpc_collision_params_t *params,
                          tpc_collisions_t *out, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------- */
/* Track refit.  Synchronous processing needs full tracking (paper §2.1), at */
/* a track resolution that matches offline reconstruction (§2.3).  A track's */
/* parameters from tpc_track_sectors come from its tracklet's fit, over a    */
/* hit set the selector may since have shrunk (hits owned by other           */
/* tracklets leave the track).  This call fits every output track again     */
/* over exactly the hits it kept, in the order of its hit list (increasing   */
/* row):                                                                     */
/*   - measurements: y and z of each hit's cluster in quanta of 1/256 cm     */
/*     (rounded half to even), at x = row_x[row], errors sigma_y, sigma_z    */
/*     of the tracking parameters;                                           */
/*   - seed: the circle through the first, middle (index n/2) and last hit  */
/*     gives C and sin(phi) at the first hit, tan(lambda) follows from the   */
/*     z difference over the arc to the last hit;                            */
/*   - pass 1: covariance diag(cov0), update at the first hit, then          */
/*     transport and update at each later hit; its state at the last hit is  */
/*     the outer state;                                                      */
/*   - pass 2: covariance reset to diag(cov0), chi2 reset, update at the     */
/*     last hit, then transport and update back to the first hit; its state */
/*     there and its chi2 are the result;                                    */
/*   - FP32 throughout, the tracker's transport, Jacobian and update, with   */
/*     C = -0.00299792458f * bz * q/pT.                                      */
/* A track with fewer than 3 hits, whose seed fails (coincident points, no   */
/* circle through them, |sin(phi)| >= sinphi_max) or whose helix cannot      */
/* reach a hit's x within |sin(phi)| < sinphi_max in either pass is not      */
/* refitted: ok = 0 and all of its outputs are zero.                         */
/* ------------------------------------------------------------------------- */

/* Outputs (device pointers, allocated by the caller; the per-track arrays
 * hold at least the tracking output's cap_tracks entries, entry t refers to
 * track t). */
typedef struct tpc_refit {
  float *params;               /* [cap_tracks][5] y, z, sin(phi), tan(lambda), q/pT at x_ref */
  float *cov;                  /* [cap_tracks][15] lower triangle, row-major */
  float *x_ref;                /* [cap_tracks] x of the first (innermost) hit */
  float *chi2;                 /* [cap_tracks] chi2 of pass 2 (ndf = 2 n_hits - 5) */
  float *params_out;           /* [cap_tracks][5] outer state: pass 1 at x_out */
  float *cov_out;              /* [cap_tracks][15] */
  float *x_out;                /* [cap_tracks] x of the last (outermost) hit */
  uint8_t *ok;                 /* [cap_tracks] 1 refitted, 0 not (above) */
  int32_t *status;             /* [1] TPC_OK, the tracker's own status when that is not TPC_OK, or
                                  TPC_E_INVALID (a track hit names no cluster of the batch or a
                                  cluster outside |y|, |z| <= 8192, row < n_rows, or a track's hits
                                  first_hit .. first_hit + n_hits - 1 lie outside the first
                                  counts[1] entries of hits); outputs are valid only with TPC_OK */
} tpc_refit_t;

/* Bytes of device workspace tpc_refit_tracks needs for a batch of n_clusters
 * clusters and an output of these capacities (host-only, pure; 0 on bad
 * arguments). */
size_t tpc_refit_workspace_size(int64_t n_clusters, int64_t cap_tracks, int64_t cap_hits);

/* Refit the tracks of a tpc_track_sectors call: the same clusters, geometry,
 * field and tracking parameters (sigma_y, sigma_z, cov0, sinphi_max are
 * used), and that call's output (n_hits, first_hit, hits, counts and status
 * read on the device, the capacities on the host).  Enqueued on `stream`
 * after the tracking call; the workspace (aligned to 256 bytes) holds no
 * state across calls.  Returns TPC_OK when the work was enqueued,
 * TPC_E_INVALID on bad arguments (a null or misaligned workspace among them),
 * TPC_E_NOMEM when the workspace is smaller than tpc_refit_workspace_size(),
 * TPC_E_HIP on a launch failure. */
int tpc_refit_tracks(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry, const tpc_field_t *field,
                     const tpc_params_t *params, const tpc_tracks_t *tracks, tpc_refit_t *out, void *workspace,
                     size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------- */
/* Segment merging.  Full tracking (paper §2.1) joins the pieces of a track  */
/* that the sector tracking finds separately: in neighbouring sectors, or    */
/* split inside one; the paper does not describe how.  This call links the   */
/* refitted tracks of a tpc_track_sectors call (its tpc_refit_tracks output)  */
/* where one continues another.  Unit u's local frame is the global one      */
/* turned by unit_alpha[u] (x along the sector's centre line).  Segment b is */
/* a candidate continuation of segment a when                                */
/*   - both are refitted (ok), their units lie on the same side             */
/*     (unit_side) and |remainder(alpha_b - alpha_a, 2 pi)| <= max_dalpha    */
/*     (the same unit included);                                             */
/*   - b's first hit row follows a's last one by 1 .. max_gap rows;          */
/*   - |z_b,in - z_a,out| <= dz_max (b's inner state, a's outer state);      */
/*   - a's outer state, turned into b's frame (the point and the direction   */
/*     turn; z, tan(lambda), q/pT stay; the state moves to the turned        */
/*     point's x) and carried along the helix to b's x_ref, has              */
/*     |y_b,in - y| <= dy_max;                                               */
/*   - with both covariances carried along (the turn's and the transport's   */
/*     Jacobians), chi2 = r^T (C_a + C_b)^-1 r <= chi2_max over the five     */
/*     parameters, r = p_b,in - p_a carried (FP64).                          */
/* Each segment takes its best candidate in each direction (least chi2,      */
/* then the smaller track index); a and b are linked when each is the       */
/* other's best.  Links never form a cycle (rows increase along them).      */
/* ------------------------------------------------------------------------- */

typedef struct tpc_merge_params {
  int64_t cap_pairs;           /* capacity of the list of pairs that pass the row, side, angle, z and y rules */
  float max_dalpha;            /* radians, >= 0 */
  int32_t max_gap;             /* rows, 1..255 */
  float dz_max;                /* cm, >= 0 */
  float dy_max;                /* cm, >= 0 */
  float chi2_max;              /* > 0 */
  float sinphi_max;            /* the helix model's limit, 0 < . < 1 */
} tpc_merge_params_t;

/* Outputs (device pointers, allocated by the caller; per-track arrays of at
 * least the tracking output's cap_tracks entries). */
typedef struct tpc_merged {
  int32_t *next;               /* [cap_tracks] the segment continuing this one, -1 none */
  int32_t *prev;               /* [cap_tracks] the segment this one continues, -1 none */
  double *link_chi2;           /* [cap_tracks] chi2 of the link to next (0 without one) */
  int64_t *counts;             /* [3] pairs past the rules, candidates (chi2 <= chi2_max), links */
  int32_t *status;             /* [1] TPC_OK, the tracker's or the refit's own status when not TPC_OK,
                                  TPC_E_INVALID (a track's unit is out of range or has no side +-1,
                                  a hit names no cluster, or a track's hits first_hit ..
                                  first_hit + n_hits - 1 lie outside the first counts[1] entries of
                                  hits), TPC_E_CAPACITY (more pairs than cap_pairs; counts[0]
                                  holds the number); outputs are valid only with TPC_OK */
} tpc_merged_t;

/* Bytes of device workspace tpc_merge_tracks needs (host-only, pure; 0 on bad
 * arguments). */
size_t tpc_merge_workspace_size(int32_t n_units, int32_t n_rows, int64_t cap_tracks,
                                const tpc_merge_params_t *params);

/* Links between the tracks of a tpc_track_sectors call, from that call's
 * output (n_hits, first_hit, hits, unit, counts, status on the device) and
 * the tpc_refit_tracks output for it (both states, covariances, ok, status),
 * with the same clusters (their rows), geometry and field.  unit_alpha and
 * unit_side are device arrays of n_units entries.  Enqueued on `stream`
 * after those calls; the workspace (aligned to 256 bytes) holds no state
 * across calls.  Returns TPC_OK when the work was enqueued, TPC_E_INVALID /
 * TPC_E_NOMEM on bad arguments or a small workspace, TPC_E_HIP on a launch
 * failure. */
int tpc_merge_tracks(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry, const tpc_field_t *field,
                     const tpc_tracks_t *tracks, const tpc_refit_t *refit, const float *unit_alpha,
                     const int32_t *unit_side, int32_t n_units, const tpc_merge_params_t *params,
                     tpc_merged_t *out, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------- */
/* Fit of merged chains.  A chain is a run of linked segments (a            */
/* tpc_merge_tracks output): its head has no prev and a next.  Its hits are */
/* its segments' hit lists in link order, each measured in its own unit's   */
/* frame (quanta of 1/256 cm at the row's x).  The fit is the refit's       */
/* two-pass FP32 filter across frames:                                      */
/*   - seed: the circle through the first, middle (n/2) and last hit, their  */
/*     positions turned into the first hit's frame;                          */
/*   - pass 1 from the first hit: before a hit of another frame the state is */
/*     turned into that frame (the merger's turn; the covariance by its     */
/*     Jacobian), then carried to the hit and updated;                       */
/*   - pass 2 from the last hit back, covariance reset to diag(cov0),       */
/*     turning back at each change of frame;                                 */
/*   - the result is the state at the chain's first hit, in its frame.     */
/* A chain of fewer than 3 hits, or whose seed, a turn or a transport       */
/* fails, is not fitted (ok = 0, outputs zero).                              */
/* ------------------------------------------------------------------------- */

/* Outputs, indexed by the chain's head track (device pointers; per-track
 * arrays of at least the tracking output's cap_tracks entries). */
typedef struct tpc_chain_fit {
  float *params;               /* [cap_tracks][5] at x_ref, in the head segment's frame */
  float *cov;                  /* [cap_tracks][15] lower triangle, row-major */
  float *x_ref;                /* [cap_tracks] x of the chain's first hit */
  float *chi2;                 /* [cap_tracks] chi2 of pass 2 (ndf = 2 n_hits - 5) */
  int32_t *n_hits;             /* [cap_tracks] hits of the chain headed by this track, 0 if none */
  uint8_t *ok;                 /* [cap_tracks] 1 fitted, 0 not (or not a head) */
  int32_t *status;             /* [1] TPC_OK, the tracker's or the merger's own status when not TPC_OK,
                                  or TPC_E_INVALID (a hit names no cluster of the batch or one out of
                                  range; a track's hits lie outside the first counts[1] entries of
                                  hits; the links do not form chains of at most 64 segments: next
                                  and prev not mutual, a link to no track of the call, a closed
                                  loop; a chain segment without hits; a linked track's unit
                                  outside 0 .. n_units - 1); outputs are valid only with TPC_OK */
} tpc_chain_fit_t;

/* Fit the chains of a tpc_merge_tracks output: the tracking call's clusters,
 * geometry, field, tracking parameters (sigma_y, sigma_z, cov0, sinphi_max)
 * and output (n_hits, first_hit, hits, unit, counts, status), the merger's
 * next / prev / status, and the unit angles it used.  The workspace (aligned
 * to 256 bytes, at least tpc_refit_workspace_size(clusters->n,
 * tracks->cap_tracks, tracks->cap_hits) bytes) holds no state across calls.
 * Enqueued on `stream` after those calls.  Returns TPC_OK when the work was
 * enqueued, TPC_E_INVALID on bad arguments (a null or misaligned workspace
 * among them), TPC_E_NOMEM when the workspace is too small, TPC_E_HIP on a
 * launch failure. */
int tpc_fit_chains(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry, const tpc_field_t *field,
                   const tpc_params_t *params, const tpc_tracks_t *tracks, const tpc_merged_t *merged,
                   const float *unit_alpha, int32_t n_units, tpc_chain_fit_t *out, void *workspace,
                   size_t workspace_bytes, void *stream);

/* Intermediate arrays kept in the workspace after a call, for inspection and
 * tests.  Valid until the workspace is reused.  `what` selects the array:
 *   TPC_VIEW_PERM      int32 [n]  sorted position -> cluster id
 *   TPC_VIEW_CELL      int32 [cells+1] first sorted position of each grid cell
 *   TPC_VIEW_SEG       int32 [units*n_rows][12] per (unit,row): start, count,
 *                      zmin, zmax, H, by, ny, bz, nz, first cell, first neighbour-finder chunk, 0
 *   TPC_VIEW_UP/DN     int32 [n]  neighbour links (sorted positions, -1 none)
 *   TPC_VIEW_UPC/DNC   int32 [n]  links after cleaning
 *   TPC_VIEW_OWNER     uint32 [n] owner key per sorted position
 *   TPC_VIEW_TRK_START, _UNIT, _LEN  int32 per tracklet (capacity n/2 + 64, the
 *                      first counts[2] valid): start hit (sorted position), unit,
 *                      chain length.
 *   TPC_VIEW_TRK_*     the other tracklet fields, per SEED (seed capacity entries,
 *                      the first counts[4] valid; seed i is tracklet SEED_LIST[i];
 *                      tracklets that are not seeds have no fit, no hits, no key):
 *     NFIT int32, RLO int32, RHI int32, KEY uint32, OWNED int32, KEEP int32,
 *     PARAMS float[5], COV float[15], XREF float, CHI2 float, P1N int32.
 *   TPC_VIEW_SEED_LIST int32 [seed capacity] the seeds (tracklets with LEN >= l_min)
 *                      in tracklet order.
 *   TPC_VIEW_TRK_HITS  int32 [ceil(seed capacity/64)][n_rows][64] hit of each row
 *                      (-1 none) of seed i at [i/64][row][i%64], rows RLO..RHI
 *                      of the seed valid; bit 30 is set on the hits the
 *                      tracklet owns (the position is the low 30 bits).
 *   P1N is the number of hits (Kalman updates) of the constructor's first pass. */
enum {
  TPC_VIEW_PERM = 1, TPC_VIEW_CELL, TPC_VIEW_SEG, TPC_VIEW_UP, TPC_VIEW_DN, TPC_VIEW_UPC,
  TPC_VIEW_DNC, TPC_VIEW_OWNER, TPC_VIEW_TRK_START, TPC_VIEW_TRK_UNIT, TPC_VIEW_TRK_LEN,
  TPC_VIEW_TRK_NFIT, TPC_VIEW_TRK_RLO, TPC_VIEW_TRK_RHI, TPC_VIEW_TRK_KEY,
  TPC_VIEW_TRK_OWNED, TPC_VIEW_TRK_KEEP, TPC_VIEW_TRK_PARAMS, TPC_VIEW_TRK_COV,
  TPC_VIEW_TRK_XREF, TPC_VIEW_TRK_CHI2, TPC_VIEW_TRK_HITS, TPC_VIEW_SEED_LIST, TPC_VIEW_TRK_P1N
};

typedef struct tpc_view {
  void *ptr;                   /* device pointer into the workspace */
  int64_t count;               /* number of elements (capacity for tracklet arrays) */
  int32_t elem_bytes;
  int32_t reserved;
} tpc_view_t;

/* Locate an intermediate array.  The batch shape and params must be those of
 * the call that filled the workspace.  Host-only. */
int tpc_inspect(const tpc_clusters_t *clusters, int32_t n_rows, const tpc_params_t *params,
                const void *workspace, int what, tpc_view_t *view);

/* ------------------------------------------------------------------------
 * Serving: a request loop for time frames that arrive over time.
 *
 * The paper's EPNs take time frames as they arrive, one host core driving one
 * GPU with several queues, transfers overlapping processing (§3.1.1,
 * §3.1.2), memory for one time frame plus its scratch reused step by step
 * (§3.1.3), bounded input/output queues and back pressure when buffers fill
 * (§3.1.3, §3.3).  A tpc_server_t does that for this library: one host thread
 * per server admits submitted requests in arrival order while its device
 * arena has room, packs every admitted request into one batch (units are
 * independent, so a request's results do not depend on its batch-mates),
 * runs up to max_in_flight batches on their own streams so that copies and
 * kernels of different batches overlap, and returns each request's results
 * in host memory.  The arena and its streams are allocated once, at create.
 * ------------------------------------------------------------------------ */

typedef struct tpc_server tpc_server_t; /* opaque */

typedef struct tpc_server_config {
  size_t budget_bytes;         /* device memory the server allocates for batches */
  int32_t max_in_flight;       /* batches on the GPU at once (one stream each), 1..8 */
  int32_t queue_depth;         /* requests waiting for admission before submit says BUSY */
  int64_t max_batch_clusters;  /* clusters packed into one batch (0: no limit) */
  int32_t max_batch_requests;  /* requests packed into one batch (0: no limit) */
  int32_t n_rows;              /* geometry, as tpc_geometry_t */
  const float *row_x;          /* HOST pointer [n_rows]; copied at create */
  float bz_tesla;
  int32_t device;              /* HIP device ordinal */
  tpc_params_t params;
} tpc_server_config_t;

/* request flags: where the cluster arrays live and who keeps them alive */
#define TPC_REQ_COPY 0        /* host arrays, copied at submit (reusable at once) */
#define TPC_REQ_BORROW_HOST 1 /* host arrays (pinned for speed), read until the request is done */
#define TPC_REQ_DEVICE 2      /* device arrays, read until the request is done (not validated) */

/* One time frame (layout as tpc_clusters_t).  unit_offsets is always a HOST
 * pointer and is copied at submit; y, z and row follow `flags`. */
typedef struct tpc_request {
  int64_t n;
  int32_t n_units;
  int32_t flags;               /* TPC_REQ_* */
  const int64_t *unit_offsets; /* [n_units + 1] */
  const float *y;
  const float *z;
  const uint16_t *row;
} tpc_request_t;

/* Results of one request, in server-owned host memory (pinned) valid until
 * tpc_server_release(ticket).  Cluster ids and track indices are local to the
 * request (as if it had been tracked alone); for a request that shared its
 * batch they are made local by its first poll, on the polling thread.  Do not
 * release a ticket while another thread polls it. */
typedef struct tpc_result {
  int32_t status;              /* TPC_OK or the request's error */
  int32_t reserved;
  int64_t n, n_tracks, n_track_hits;
  const int32_t *cluster_track;  /* [n] */
  const float *params;           /* [n_tracks][5] */
  const float *cov;              /* [n_tracks][15] */
  const float *x_ref, *chi2;     /* [n_tracks] */
  const int32_t *unit, *n_hits, *n_fit, *first_hit; /* [n_tracks] */
  const int32_t *hits;           /* [n_track_hits] */
  double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
  int64_t batch_id;              /* batch the request ran in */
  int32_t batch_requests;        /* requests in that batch */
  int32_t reserved2;
} tpc_result_t;

typedef struct tpc_server_stats {
  int64_t submitted, completed, rejected_busy, rejected_nomem, rejected_invalid, batches;
  int32_t pending, in_flight;
  size_t arena_bytes, arena_used, arena_peak;
  double host_cpu_s;             /* CPU seconds the server's host thread has used (the paper
                                    measures the host cores a GPU needs, §3.1.1) */
} tpc_server_stats_t;

/* Create a server: allocates the arena (budget_bytes of device memory), the
 * streams and pinned host buffers, and starts its host thread. */
int tpc_server_create(const tpc_server_config_t *config, tpc_server_t **server);

/* Queue a request.  Returns TPC_OK and a ticket; TPC_E_BUSY when queue_depth
 * requests are already waiting (back pressure: retry later); TPC_E_NOMEM when
 * the request could never fit the arena; TPC_E_INVALID when its data are
 * malformed (host arrays are checked here; device arrays are checked by the
 * kernels).  A batch of several requests that fails on the device (invalid
 * data, capacity) is run again one request per batch, so a bad request fails
 * alone and the others still get the results they would get alone.  With
 * TPC_REQ_DEVICE the caller makes the arrays ready before submitting (the
 * server's streams do not wait on the caller's). */
int tpc_server_submit(tpc_server_t *server, const tpc_request_t *request, uint64_t *ticket);

/* Results of a ticket.  wait_us = 0: do not wait (TPC_E_BUSY if not done yet);
 * < 0: wait until done; > 0: wait up to that many microseconds.  Returns
 * TPC_OK when *result is filled (see result->status), TPC_E_BUSY if not done,
 * TPC_E_INVALID for an unknown ticket.  result->status is the tracking
 * status, or TPC_E_NOMEM when the server could not get pinned host memory
 * for the request's batch. */
int tpc_server_poll(tpc_server_t *server, uint64_t ticket, tpc_result_t *result, int64_t wait_us);

/* Free a completed request's results. */
int tpc_server_release(tpc_server_t *server, uint64_t ticket);

int tpc_server_stats(tpc_server_t *server, tpc_server_stats_t *stats);

/* Finish in-flight work, stop the thread, free everything. */
int tpc_server_destroy(tpc_server_t *server);

/* Device bytes one request of n clusters in n_units units occupies in the
 * arena while it runs (inputs, workspace, outputs).  Host-only, pure. */
size_t tpc_server_footprint(int64_t n, int32_t n_units, int32_t n_rows, const tpc_params_t *params);

#ifdef __cplusplus
}
#endif

#endif /* TPC_TRACK_H */
