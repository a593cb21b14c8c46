// Merging of track segments across sector boundaries: the segments the
// tracker found in neighbouring sectors (or split inside one) joined where
// one continues the other.  The paper's synchronous processing needs full
// tracking (§2.1) and does not describe this step; the operation is stated
// with tpc_merge_tracks in include/tpc_track.h.
//
// Launches on the caller's stream:
//   k_mg_init   status, counters, per-track outputs and best-match keys;
//   k_mg_rows   per track: first and last hit row; per (unit, z' cell)
//               counts of the refitted segments that start after row 0
//               (only those can continue another); cells are at least
//               dz_max wide, so a z' window meets at most three;
//   k_mg_scan   one block: bin offsets;
//   k_mg_fill   those segments filed by (unit, z' cell);
//   k_mg_sort   one wave per cell: its segments sorted by first row (bitonic
//               in LDS up to SORT_MAX; larger cells by one lane), with their
//               inner z', y, x and first row written in that order as one
//               16-byte record each (the scan below reads one record per
//               candidate, and neighbouring lanes share its cache lines);
//   k_mg_pairs  one lane per segment a: for each unit on its side within
//               max_dalpha, its outer state turned into that unit's frame
//               (parameters, FP64); in each cell its z' window meets, two
//               binary searches find the segments starting 1 .. max_gap rows
//               after a's last row, whose records are loaded a few at a time
//               and checked: z' window, then y carried along the helix
//               (parameters only); pairs that pass are buffered per lane in
//               LDS, and one atomic per wave reserves the list ranges of all
//               its lanes at the end (an atomic per pair, or per lane, on the
//               one counter would serialize them; a full buffer is flushed
//               by its lane alone);
//   k_mg_chi2   one lane per pair: the turn with its Jacobian, the helix
//               transport with its Jacobian, both covariances summed, chi2
//               by Cholesky (FP64); candidates take the least chi2 per
//               segment both ways (64-bit atomic minima on the chi2's bits:
//               non-negative doubles order like their bit patterns);
//   k_mg_pick   per candidate at its segment's least chi2: the least index;
//   k_mg_link   per segment: linked when its best outward match takes it as
//               its best inward match.
// FP64 with contraction off, so the decisions follow the exact arithmetic to
// about 1e-15 relative.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpc_track.h"

namespace {

constexpr int TPB = 256;
constexpr int SCAN_T = 1024;
constexpr int SORT_MAX = 1024;  // bins sorted in LDS up to this size
constexpr int PAIR_BUF = 16;   // pairs a lane of the scan buffers in LDS before it reserves list space
constexpr int MAX_BLOCKS = 4096;
constexpr double KAPPA = 0.00299792458;
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr unsigned long long NONE64 = ~0ull;

// a filed segment as the scan reads it
struct __align__(16) Filed {
  float z, y, x;  // inner z', y and x
  int32_t fr;     // first row
};
// and as the chi2 of a pair reads it: its inner state, unit and track index
struct __align__(16) Inner {
  float p[5], x;
  int32_t unit, b;
  float c[15], pad;
};
static_assert(sizeof(Inner) == 96, "six 16-byte loads");

struct MgArgs {
  // clusters, geometry
  const uint16_t *row;
  int64_t n_clusters;
  int32_t n_rows;
  // tracks
  const int32_t *trk_status, *n_hits, *first_hit, *hits, *unit;
  const int64_t *trk_counts;
  int64_t cap_tracks, cap_hits;
  // refit
  const float *p_in, *c_in, *x_in, *p_out, *c_out, *x_out;
  const uint8_t *ok;
  const int32_t *rf_status;
  // units
  const float *alpha;
  const int32_t *side;
  int32_t n_units;
  // parameters
  double k, smx, max_dalpha, dz_max, dy_max, chi2_max;
  int32_t max_gap;
  int32_t nzc;       // z' cells per unit
  double zlo, cw;    // first cell's lower edge, cell width
  int64_t cap_pairs;
  // outputs
  int32_t *next, *prev;
  double *link_chi2;
  int64_t *counts;
  int32_t *status;
  // workspace
  int32_t *bin;  // [nbins + 1] counts, then offsets
  int32_t *cursor;
  int32_t *idx;
  Filed *filed;   // the filed segments, in scan order
  Inner *inner;   // their inner states, in the same order
  int32_t *frs;    // their first rows, in filing order (the sort's key)
  int32_t *rows;  // first row | last row << 16
  unsigned long long *ob_chi, *ib_chi;
  int32_t *ob_idx, *ib_idx;
  int2 *pairs;
  double *pair_chi;
  unsigned long long *ctr;  // pairs, candidates, links
};

__device__ __forceinline__ int64_t n_tracks(const MgArgs &A) {
  const int64_t T = A.trk_counts[0];
  return T < A.cap_tracks ? T : A.cap_tracks;
}
__device__ __forceinline__ int64_t n_track_hits(const MgArgs &A) {
  const int64_t H = A.trk_counts[1];
  return H < A.cap_hits ? H : A.cap_hits;
}

// ---- FP64 track model --------------------------------------------------------

// asin(u)/u and (d/du asin(u)/u) / u, by their series below u = 1e-3
__device__ double asin_over(double u) {
#pragma clang fp contract(off)
  return u < 1e-3 ? 1.0 + u * u / 6.0 : asin(u) / u;
}
__device__ double asin_over_d(double u) {
#pragma clang fp contract(off)
  return u < 1e-3 ? 1.0 / 3.0 + 0.3 * u * u : (u / sqrt(1.0 - u * u) - asin(u)) / (u * u * u);
}

// The state (y, z, sin(phi), tan(lambda), q/pT) at plane x turned by d into
// another sector's frame: the point turns, so does the direction; the new
// state lives at the turned point's x.  J (optional): the Jacobian of the
// new state at the new plane against the old one (a shift of the track along
// the old y, taken back to the new plane along the track; a turn of the
// direction).  False when the direction reaches |sin| >= smx or cos <= 0.
__device__ __forceinline__ bool turn(const double p[5], double x, double d, double k, double smx, double q[5], double &xq,
                     double *J) {
#pragma clang fp contract(off)
  const double cd = cos(d), sd = sin(d);
  const double s = p[2];
  if (!(fabs(s) < 1.0)) return false;
  const double c = sqrt(1.0 - s * s);
  const double s2 = s * cd - c * sd, c2 = c * cd + s * sd;
  if (!(c2 > 0.0) || !(fabs(s2) < smx)) return false;
  xq = x * cd + p[0] * sd;
  q[0] = -x * sd + p[0] * cd;
  q[1] = p[1];
  q[2] = s2;
  q[3] = p[3];
  q[4] = p[4];
  if (J) {
#pragma unroll
    for (int i = 0; i < 25; ++i) J[i] = (i % 6 == 0) ? 1.0 : 0.0;
    J[0] = c / c2;
    J[5] = -sd * p[3] / c2;
    J[10] = -k * p[4] * sd;
    J[12] = c2 / c;
  }
  return true;
}

// Helix transport of the parameters from x1 to x2: sin(phi) grows by C dx,
// y by dx (sin1 + sin2) / (cos1 + cos2), z by tan(lambda) times the arc
// length sign(dx) L asin(u)/u (L the chord, u = |C| L / 2).  F (optional):
// its Jacobian.  False when |sin(phi)| reaches smx at either end or u >= 1.
__device__ __forceinline__ bool carry(const double p[5], double x1, double x2, double k, double smx, double q[5], double *F) {
#pragma clang fp contract(off)
  const double dx = x2 - x1;
  const double C = k * p[4];
  const double s1 = p[2], s2 = s1 + C * dx;
  if (!(fabs(s1) < smx) || !(fabs(s2) < smx)) return false;
  const double c1 = sqrt(1.0 - s1 * s1), c2 = sqrt(1.0 - s2 * s2);
  const double D = c1 + c2, N = s1 + s2;
  const double dy = dx * N / D;
  const double L = sqrt(dx * dx + dy * dy);
  const double u = fabs(C) * L * 0.5;
  if (!(u < 1.0)) return false;
  const double sg = dx < 0 ? -1.0 : 1.0;
  const double fu = asin_over(u);
  const double sT = sg * L * fu;
  q[0] = p[0] + dy;
  q[1] = p[1] + p[3] * sT;
  q[2] = s2;
  q[3] = p[3];
  q[4] = p[4];
  if (F) {
#pragma unroll
    for (int i = 0; i < 25; ++i) F[i] = (i % 6 == 0) ? 1.0 : 0.0;
    const double a = dx * ((2.0 * D + N * (s1 / c1 + s2 / c2)) / (D * D));
    const double b = dx * (k * dx * (D + N * s2 / c2) / (D * D));
    const double g = asin_over_d(u);
    const double dsdy = L > 0 ? sg * (dy / L) * (fu + u * u * g) : 0.0;
    const double dsdC = sg * C * L * L * L * g * 0.25;
    F[2] = a;
    F[4] = b;
    F[7] = p[3] * dsdy * a;
    F[8] = sT;
    F[9] = p[3] * (dsdy * b + dsdC * k);
    F[14] = k * dx;
  }
  return true;
}

// y of the parameters carried from x1 to x2 along the helix (the transport
// above without the arc length); false where the transport fails.
__device__ bool carry_y(const double p[5], double x1, double x2, double k, double smx, double &y) {
#pragma clang fp contract(off)
  const double dx = x2 - x1;
  const double C = k * p[4];
  const double s1 = p[2], s2 = s1 + C * dx;
  if (!(fabs(s1) < smx) || !(fabs(s2) < smx)) return false;
  const double c1 = sqrt(1.0 - s1 * s1), c2 = sqrt(1.0 - s2 * s2);
  const double dy = dx * (s1 + s2) / (c1 + c2);
  const double L = sqrt(dx * dx + dy * dy);
  if (!(fabs(C) * L * 0.5 < 1.0)) return false;
  y = p[0] + dy;
  return true;
}

// C <- M C M^T (5x5, full products)
__device__ __forceinline__ void sandwich(const double M[25], double C[25]) {
#pragma clang fp contract(off)
  double T[25];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 5; ++l) s += M[i * 5 + l] * C[l * 5 + j];
      T[i * 5 + j] = s;
    }
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 5; ++l) s += T[i * 5 + l] * M[j * 5 + l];
      C[i * 5 + j] = s;
    }
}

__device__ __forceinline__ void load_cov(const float *c15, double C[25]) {
  int m = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) C[i * 5 + j] = C[j * 5 + i] = double(c15[m++]);
}

// r^T S^-1 r by Cholesky; -1 when S is not positive definite
__device__ __forceinline__ double chi2_solve(const double S[25], const double r[5]) {
#pragma clang fp contract(off)
  double L[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) L[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = S[i * 5 + j];
#pragma unroll
      for (int m = 0; m < j; ++m) v -= L[i * 5 + m] * L[j * 5 + m];
      if (i == j) {
        if (!(v > 0.0)) return -1.0;
        L[i * 5 + i] = sqrt(v);
      } else {
        L[i * 5 + j] = v / L[j * 5 + j];
      }
    }
  double w[5], q = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double v = r[i];
#pragma unroll
    for (int m = 0; m < i; ++m) v -= L[i * 5 + m] * w[m];
    w[i] = v / L[i * 5 + i];
    q += w[i] * w[i];
  }
  return q;
}

__device__ __forceinline__ int zcell(const MgArgs &A, double z) {
  const double c = floor((z - A.zlo) / A.cw);
  return c < 0.0 ? 0 : (c >= double(A.nzc) ? A.nzc - 1 : int(c));
}

__device__ __forceinline__ double turn_angle(const MgArgs &A, int ua, int w) {
  return remainder(double(A.alpha[w]) - double(A.alpha[ua]), TWO_PI);
}

// ---- kernels -------------------------------------------------------------------

__global__ void __launch_bounds__(TPB) k_mg_init(MgArgs A) {
  const int64_t T = n_tracks(A);
  const int64_t nb = int64_t(A.n_units) * A.nzc + 1;
  const int64_t i0 = int64_t(blockIdx.x) * TPB + threadIdx.x, st = int64_t(gridDim.x) * TPB;
  if (i0 == 0) {
    *A.status = *A.trk_status != TPC_OK ? *A.trk_status : *A.rf_status;
    A.ctr[0] = A.ctr[1] = A.ctr[2] = 0ull;
  }
  for (int64_t i = i0; i < nb; i += st) A.bin[i] = 0;
  for (int64_t t = i0; t < T; t += st) {
    A.next[t] = A.prev[t] = -1;
    A.link_chi2[t] = 0.0;
    A.ob_chi[t] = A.ib_chi[t] = NONE64;
    A.ob_idx[t] = A.ib_idx[t] = INT32_MAX;
  }
}

__global__ void __launch_bounds__(TPB) k_mg_rows(MgArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t T = n_tracks(A), H = n_track_hits(A);
  bool bad = false;
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T; t += int64_t(gridDim.x) * TPB) {
    const int n = A.n_hits[t], f = A.first_hit[t], u = A.unit[t];
    if (n < 0 || f < 0 || int64_t(f) + n > H) {  // the track's hits lie outside the hit list
      bad = true;
      continue;
    }
    int fr = 0, lr = 0;
    if (n > 0) {
      const int32_t h0 = A.hits[f], h1 = A.hits[f + n - 1];
      if (h0 < 0 || h0 >= A.n_clusters || h1 < 0 || h1 >= A.n_clusters) {
        bad = true;
        continue;
      }
      fr = A.row[h0];
      lr = A.row[h1];
    }
    if (u < 0 || u >= A.n_units || (A.side[u] != 1 && A.side[u] != -1) || fr >= A.n_rows || lr >= A.n_rows) {
      bad = true;
      continue;
    }
    A.rows[t] = fr | (lr << 16);
    if (A.ok[t] && fr > 0) atomicAdd(&A.bin[u * A.nzc + zcell(A, double(A.p_in[t * 5 + 1]))], 1);
  }
  if (bad) *A.status = TPC_E_INVALID;
}

// exclusive scan of the bin counts (one block), and the fill cursors
__global__ void __launch_bounds__(SCAN_T) k_mg_scan(MgArgs A) {
  __shared__ int32_t s[SCAN_T];
  __shared__ int32_t carry_in;
  if (*A.status != TPC_OK) return;
  const int64_t nb = int64_t(A.n_units) * A.nzc;
  if (threadIdx.x == 0) carry_in = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 <= nb; b0 += SCAN_T) {
    const int64_t b = b0 + threadIdx.x;
    const int v = b < nb ? A.bin[b] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {
      const int a = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    const int ex = carry_in + s[threadIdx.x] - v;
    if (b <= nb) A.bin[b] = ex;
    if (b < nb) A.cursor[b] = ex;
    __syncthreads();
    if (threadIdx.x == SCAN_T - 1) carry_in += s[SCAN_T - 1];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(TPB) k_mg_fill(MgArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t T = n_tracks(A);
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T; t += int64_t(gridDim.x) * TPB) {
    const int fr = A.rows[t] & 0xFFFF;
    if (!A.ok[t] || fr == 0) continue;
    const int pos = atomicAdd(&A.cursor[A.unit[t] * A.nzc + zcell(A, double(A.p_in[t * 5 + 1]))], 1);
    A.idx[pos] = int32_t(t);
    A.frs[pos] = fr;
  }
}

// Adds the block's total of the threads' v to a counter with one atomic per
// block (the counter is shared by the whole grid: an atomic per wave on the
// one address serialized thousands of them).  Called by every thread of the
// block, after its loop.
__device__ __forceinline__ void block_count(unsigned long long &counter, unsigned v) {
  __shared__ unsigned s;
  if (threadIdx.x == 0) s = 0u;
  __syncthreads();
  if (v) atomicAdd(&s, v);
  __syncthreads();
  if (threadIdx.x == 0 && s) atomicAdd(&counter, (unsigned long long)s);
}

__device__ __forceinline__ void file_entry(const MgArgs &A, int32_t s, int32_t b, int32_t fr) {
  A.idx[s] = b;
  Filed f;
  f.z = A.p_in[int64_t(b) * 5 + 1];
  f.y = A.p_in[int64_t(b) * 5];
  f.x = A.x_in[b];
  f.fr = fr;
  A.filed[s] = f;
  Inner r;
  for (int j = 0; j < 5; ++j) r.p[j] = A.p_in[int64_t(b) * 5 + j];
  r.x = f.x;
  r.unit = A.unit[b];
  r.b = b;
  for (int j = 0; j < 15; ++j) r.c[j] = A.c_in[int64_t(b) * 15 + j];
  r.pad = 0.f;
  A.inner[s] = r;
}

__global__ void __launch_bounds__(64) k_mg_sort(MgArgs A) {
  __shared__ unsigned long long key[SORT_MAX];
  if (*A.status != TPC_OK) return;
  const int64_t nb = int64_t(A.n_units) * A.nzc;
  for (int64_t c = blockIdx.x; c < nb; c += gridDim.x) {  // block-uniform
    const int32_t s0 = A.bin[c], n = A.bin[c + 1] - s0;
    if (n == 0) continue;
    if (n > SORT_MAX) {  // rare: one lane, insertion sort by (first row, index) in place
      if (threadIdx.x == 0) {
        for (int32_t i = 1; i < n; ++i) {
          const int32_t b = A.idx[s0 + i], fr = A.frs[s0 + i];
          int32_t j = i - 1;
          for (; j >= 0 && (A.frs[s0 + j] > fr || (A.frs[s0 + j] == fr && A.idx[s0 + j] > b)); --j) {
            A.idx[s0 + j + 1] = A.idx[s0 + j];
            A.frs[s0 + j + 1] = A.frs[s0 + j];
          }
          A.idx[s0 + j + 1] = b;
          A.frs[s0 + j + 1] = fr;
        }
        for (int32_t i = 0; i < n; ++i) file_entry(A, s0 + i, A.idx[s0 + i], A.frs[s0 + i]);
      }
      continue;
    }
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += 64)
      key[i] = i < n ? (uint64_t(uint32_t(A.frs[s0 + i])) << 32) | uint32_t(A.idx[s0 + i]) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < np; i += 64) {
          const int l = i ^ j;
          if (l > i) {
            const unsigned long long x = key[i], y = key[l];
            if ((x > y) == ((i & k) == 0)) {
              key[i] = y;
              key[l] = x;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += 64)
      file_entry(A, s0 + i, int32_t(uint32_t(key[i])), int32_t(key[i] >> 32));
    __syncthreads();
  }
}

// The lane's buffered pairs (a, buf[0 .. n)) written to the list at a
// reserved range (one atomic per flush; past cap_pairs they are only counted).
__device__ __forceinline__ void flush(const MgArgs &A, int32_t a, const int32_t *buf, int n) {
  if (n == 0) return;
  const unsigned long long base = atomicAdd(&A.ctr[0], (unsigned long long)n);
  for (int i = 0; i < n; ++i)
    if (base + i < (unsigned long long)A.cap_pairs) A.pairs[base + i] = make_int2(a, buf[i * TPB]);
}

// first position in [lo, hi) of a cell (sorted by first row) whose first row is above r
__device__ __forceinline__ int32_t after_row(const MgArgs &A, int32_t lo, int32_t hi, int r) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (A.filed[mid].fr <= r) lo = mid + 1; else hi = mid;
  }
  return lo;
}

constexpr int SCAN_B = 4;  // candidate records loaded together

// The candidates of segment a (refitted, its last row below the last row):
// pairs into the lane's buffer, a full buffer flushed on its own.
__device__ __forceinline__ void scan_segment(const MgArgs &A, int64_t a, int lr, int32_t *buf, int &nbuf) {
  const int ua = A.unit[a];
  const int r1 = min(lr + A.max_gap, A.n_rows - 1);
  double pa[5];
  for (int i = 0; i < 5; ++i) pa[i] = double(A.p_out[a * 5 + i]);
  const double xa = double(A.x_out[a]);
  const double za = pa[1];
  for (int w = 0; w < A.n_units; ++w) {
    if (A.side[w] != A.side[ua]) continue;
    const double d = turn_angle(A, ua, w);
    if (!(fabs(d) <= A.max_dalpha)) continue;
    double q[5], xq = xa;
    if (w == ua) {
      for (int i = 0; i < 5; ++i) q[i] = pa[i];
    } else if (!turn(pa, xa, d, A.k, A.smx, q, xq, nullptr)) {
      continue;
    }
    const int c0 = zcell(A, za - A.dz_max), c1 = zcell(A, za + A.dz_max);
    for (int cz = c0; cz <= c1; ++cz) {
      const int32_t s0 = A.bin[w * A.nzc + cz], s1 = A.bin[w * A.nzc + cz + 1];
      if (s0 == s1) continue;
      // the cell is sorted by first row: the segments starting in rows lr+1 .. r1,
      // their records loaded SCAN_B at a time (the range is known, so no load
      // waits on the one before)
      const int32_t lo = after_row(A, s0, s1, lr), hi = after_row(A, lo, s1, r1);
      for (int32_t s = lo; s < hi; s += SCAN_B) {
        Filed f[SCAN_B];
#pragma unroll
        for (int e = 0; e < SCAN_B; ++e)
          if (s + e < hi) f[e] = A.filed[s + e];
#pragma unroll
        for (int e = 0; e < SCAN_B; ++e) {
          if (s + e >= hi) break;
          double y;
          if (!(fabs(double(f[e].z) - za) <= A.dz_max) || !carry_y(q, xq, double(f[e].x), A.k, A.smx, y) ||
              !(fabs(double(f[e].y) - y) <= A.dy_max))
            continue;
          if (nbuf == PAIR_BUF) {
            flush(A, int32_t(a), buf, nbuf);
            nbuf = 0;
          }
          buf[nbuf++ * TPB] = s + e;  // the filed slot; k_mg_chi2 puts the track index in its place
        }
      }
    }
  }
}

__global__ void __launch_bounds__(TPB) k_mg_pairs(MgArgs A) {
  // each lane's pair buffer: a column of a [PAIR_BUF][TPB] block (lanes side by side)
  __shared__ int32_t pbuf[PAIR_BUF * TPB];
  int32_t *buf = pbuf + threadIdx.x;
  if (*A.status != TPC_OK) return;
  const int64_t T = n_tracks(A);
  const int lane = __lane_id();
  for (int64_t a0 = int64_t(blockIdx.x) * TPB; a0 < T; a0 += int64_t(gridDim.x) * TPB) {
    const int64_t a = a0 + threadIdx.x;
    if ((a & ~int64_t(63)) >= T) break;  // whole wave past the tracks (wave-uniform)
    int nbuf = 0;
    const int lr = a < T ? A.rows[a] >> 16 : 0;
    if (a < T && A.ok[a] && lr + 1 < A.n_rows) scan_segment(A, a, lr, buf, nbuf);
    // the lanes' buffered pairs: one atomic per wave reserves all their ranges
    // (an atomic per lane on the one counter would serialize them)
    int incl = nbuf;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    long long base = 0;
    if (lane == 63 && total) base = (long long)atomicAdd(&A.ctr[0], (unsigned long long)total);
    base = __shfl(base, 63, 64);
    const unsigned long long mine = (unsigned long long)base + (unsigned long long)(incl - nbuf);
    for (int i = 0; i < nbuf; ++i)
      if (mine + i < (unsigned long long)A.cap_pairs) A.pairs[mine + i] = make_int2(int32_t(a), buf[i * TPB]);
  }
}


__global__ void __launch_bounds__(TPB) k_mg_chi2(MgArgs A) {
  if (*A.status != TPC_OK) return;
  const unsigned long long np = A.ctr[0];
  if (np > (unsigned long long)A.cap_pairs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.status = TPC_E_CAPACITY;
    return;
  }
  unsigned n_cand = 0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < int64_t(np); i += int64_t(gridDim.x) * TPB) {
    const int2 pr = A.pairs[i];
    const int a = pr.x;
    const Inner bi = A.inner[pr.y];  // b's inner state, filed next to the other candidates of a's cells
    const int b = bi.b, ub = bi.unit;
    A.pairs[i].y = b;                // k_mg_pick reads track indices
    const int ua = A.unit[a];
    double pa[5], C[25], q[5], c[5];
    for (int j = 0; j < 5; ++j) pa[j] = double(A.p_out[a * 5 + j]);
    load_cov(A.c_out + int64_t(a) * 15, C);
    double xq = double(A.x_out[a]);
    double chi = -1.0;
    bool ok = true;
    if (ua != ub) {
      double J[25];
      ok = turn(pa, double(A.x_out[a]), turn_angle(A, ua, ub), A.k, A.smx, q, xq, J);
      if (ok) sandwich(J, C);
    } else {
      for (int j = 0; j < 5; ++j) q[j] = pa[j];
    }
    double F[25];
    if (ok) ok = carry(q, xq, double(bi.x), A.k, A.smx, c, F);
    if (ok) {
#pragma clang fp contract(off)
      sandwich(F, C);
      double Cb[25], r[5];
      load_cov(bi.c, Cb);
      for (int j = 0; j < 25; ++j) C[j] += Cb[j];
      for (int j = 0; j < 5; ++j) r[j] = double(bi.p[j]) - c[j];
      chi = chi2_solve(C, r);
    }
    A.pair_chi[i] = chi;
    const bool cand = chi >= 0.0 && chi <= A.chi2_max;
    if (cand) {
      const unsigned long long bits = (unsigned long long)__double_as_longlong(chi);
      atomicMin(&A.ob_chi[a], bits);
      atomicMin(&A.ib_chi[b], bits);
    }
    n_cand += cand;
  }
  block_count(A.ctr[1], n_cand);
}

__global__ void __launch_bounds__(TPB) k_mg_pick(MgArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t np = int64_t(A.ctr[0]);
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < np; i += int64_t(gridDim.x) * TPB) {
    const double chi = A.pair_chi[i];
    if (!(chi >= 0.0 && chi <= A.chi2_max)) continue;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(chi);
    const int2 pr = A.pairs[i];
    if (A.ob_chi[pr.x] == bits) atomicMin(&A.ob_idx[pr.x], pr.y);
    if (A.ib_chi[pr.y] == bits) atomicMin(&A.ib_idx[pr.y], pr.x);
  }
}

__global__ void __launch_bounds__(TPB) k_mg_link(MgArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t T = n_tracks(A);
  unsigned n_link = 0;
  for (int64_t a = int64_t(blockIdx.x) * TPB + threadIdx.x; a < T; a += int64_t(gridDim.x) * TPB) {
    const int32_t b = A.ob_idx[a];
    const bool link = b != INT32_MAX && A.ib_idx[b] == int32_t(a);
    if (link) {
      A.next[a] = b;
      A.prev[b] = int32_t(a);
      A.link_chi2[a] = __longlong_as_double((long long)A.ob_chi[a]);
    }
    n_link += link;
  }
  block_count(A.ctr[2], n_link);
}

__global__ void k_mg_counts(MgArgs A) {
  A.counts[0] = int64_t(A.ctr[0]);
  A.counts[1] = int64_t(A.ctr[1]);
  A.counts[2] = int64_t(A.ctr[2]);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
  size_t bin, cursor, idx, filed, inner, frs, rows, ob_chi, ib_chi, ob_idx, ib_idx, pairs, pair_chi, ctr, total;
};

Layout layout(int64_t nbins, int64_t cap_tracks, int64_t cap_pairs) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.bin = take(size_t(nbins + 1) * 4);
  L.cursor = take(size_t(nbins) * 4);
  L.idx = take(size_t(cap_tracks) * 4);
  L.filed = take(size_t(cap_tracks) * sizeof(Filed));
  L.inner = take(size_t(cap_tracks) * sizeof(Inner));
  L.frs = take(size_t(cap_tracks) * 4);
  L.rows = take(size_t(cap_tracks) * 4);
  L.ob_chi = take(size_t(cap_tracks) * 8);
  L.ib_chi = take(size_t(cap_tracks) * 8);
  L.ob_idx = take(size_t(cap_tracks) * 4);
  L.ib_idx = take(size_t(cap_tracks) * 4);
  L.pairs = take(size_t(cap_pairs) * 8);
  L.pair_chi = take(size_t(cap_pairs) * 8);
  L.ctr = take(4 * 8);
  L.total = o;
  return L;
}

// z' cells of the candidate filing: at least dz_max wide where that keeps
// the bins below 2^18 (a window then meets at most three cells), over
// [-8256, 8256) cm (inputs lie within |z'| <= 8192; the rest is clamped).
struct Cells {
  int32_t nzc;
  double zlo, cw;
};
Cells cells(const tpc_merge_params_t *p, int32_t n_units) {
  constexpr double SPAN = 16512.0;
  const int64_t most = (int64_t(1) << 18) / (n_units > 0 ? n_units : 1);
  int64_t nz = p->dz_max > 0.f ? int64_t(SPAN / double(p->dz_max)) : most;
  if (nz > most) nz = most;
  if (nz > 65536) nz = 65536;
  if (nz < 1) nz = 1;
  Cells c;
  c.nzc = int32_t(nz);
  c.zlo = -SPAN / 2;
  c.cw = SPAN / double(nz);
  return c;
}

}  // namespace

extern "C" size_t tpc_merge_workspace_size(int32_t n_units, int32_t n_rows, int64_t cap_tracks,
                                           const tpc_merge_params_t *params) {
  if (!params || n_units < 1 || n_rows < 3 || n_rows > 255 || cap_tracks < 0 || cap_tracks >= (int64_t(1) << 31) ||
      params->cap_pairs < 0 || params->cap_pairs >= (int64_t(1) << 31) || n_units > (1 << 18))
    return 0;
  return layout(int64_t(n_units) * cells(params, n_units).nzc, cap_tracks, params->cap_pairs).total;
}

extern "C" int tpc_merge_tracks(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                                const tpc_field_t *field, const tpc_tracks_t *tracks, const tpc_refit_t *refit,
                                const float *unit_alpha, const int32_t *unit_side, int32_t n_units,
                                const tpc_merge_params_t *params, tpc_merged_t *out, void *workspace,
                                size_t workspace_bytes, void *stream) {
  if (!clusters || !geometry || !field || !tracks || !refit || !params || !out || !unit_alpha || !unit_side)
    return TPC_E_INVALID;
  if (clusters->n < 0 || (clusters->n > 0 && !clusters->row) || !geometry->row_x) return TPC_E_INVALID;
  if (!tracks->n_hits || !tracks->first_hit || !tracks->hits || !tracks->unit || !tracks->counts ||
      !tracks->status || tracks->cap_tracks < 0 || tracks->cap_hits < 0)
    return TPC_E_INVALID;
  if (!refit->params || !refit->cov || !refit->x_ref || !refit->params_out || !refit->cov_out ||
      !refit->x_out || !refit->ok || !refit->status)
    return TPC_E_INVALID;
  if (!out->next || !out->prev || !out->link_chi2 || !out->counts || !out->status) return TPC_E_INVALID;
  if (!(params->max_dalpha >= 0.f) || params->max_gap < 1 || params->max_gap > 255 || !(params->dz_max >= 0.f) ||
      !(params->dy_max >= 0.f) || !(params->chi2_max > 0.f) || !(params->sinphi_max > 0.f) ||
      !(params->sinphi_max < 1.f) || !isfinite(field->bz_tesla))
    return TPC_E_INVALID;
  const size_t need = tpc_merge_workspace_size(n_units, geometry->n_rows, tracks->cap_tracks, params);
  if (need == 0) return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  if (workspace_bytes < need) return TPC_E_NOMEM;
  MgArgs A;
  A.row = clusters->row;
  A.n_clusters = clusters->n;
  A.n_rows = geometry->n_rows;
  A.trk_status = tracks->status;
  A.n_hits = tracks->n_hits;
  A.first_hit = tracks->first_hit;
  A.hits = tracks->hits;
  A.unit = tracks->unit;
  A.trk_counts = tracks->counts;
  A.cap_tracks = tracks->cap_tracks;
  A.cap_hits = tracks->cap_hits;
  A.p_in = refit->params;
  A.c_in = refit->cov;
  A.x_in = refit->x_ref;
  A.p_out = refit->params_out;
  A.c_out = refit->cov_out;
  A.x_out = refit->x_out;
  A.ok = refit->ok;
  A.rf_status = refit->status;
  A.alpha = unit_alpha;
  A.side = unit_side;
  A.n_units = n_units;
  A.k = double(-float(KAPPA) * field->bz_tesla);  // the tracker's curvature constant, as its fit used it
  A.smx = params->sinphi_max;
  A.max_dalpha = params->max_dalpha;
  A.dz_max = params->dz_max;
  A.dy_max = params->dy_max;
  A.chi2_max = params->chi2_max;
  A.max_gap = params->max_gap;
  A.cap_pairs = params->cap_pairs;
  A.next = out->next;
  A.prev = out->prev;
  A.link_chi2 = out->link_chi2;
  A.counts = out->counts;
  A.status = out->status;
  const Cells cz = cells(params, n_units);
  A.nzc = cz.nzc;
  A.zlo = cz.zlo;
  A.cw = cz.cw;
  const int64_t nb = int64_t(n_units) * cz.nzc;
  const Layout L = layout(nb, tracks->cap_tracks, params->cap_pairs);
  char *w = static_cast<char *>(workspace);
  A.bin = reinterpret_cast<int32_t *>(w + L.bin);
  A.cursor = reinterpret_cast<int32_t *>(w + L.cursor);
  A.idx = reinterpret_cast<int32_t *>(w + L.idx);
  A.filed = reinterpret_cast<Filed *>(w + L.filed);
  A.inner = reinterpret_cast<Inner *>(w + L.inner);
  A.frs = reinterpret_cast<int32_t *>(w + L.frs);
  A.rows = reinterpret_cast<int32_t *>(w + L.rows);
  A.ob_chi = reinterpret_cast<unsigned long long *>(w + L.ob_chi);
  A.ib_chi = reinterpret_cast<unsigned long long *>(w + L.ib_chi);
  A.ob_idx = reinterpret_cast<int32_t *>(w + L.ob_idx);
  A.ib_idx = reinterpret_cast<int32_t *>(w + L.ib_idx);
  A.pairs = reinterpret_cast<int2 *>(w + L.pairs);
  A.pair_chi = reinterpret_cast<double *>(w + L.pair_chi);
  A.ctr = reinterpret_cast<unsigned long long *>(w + L.ctr);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto blocks = [](int64_t n) { return unsigned(n < TPB ? 1 : ((n + TPB - 1) / TPB > MAX_BLOCKS ? MAX_BLOCKS : (n + TPB - 1) / TPB)); };
  const int64_t T = tracks->cap_tracks;
  hipLaunchKernelGGL(k_mg_init, dim3(blocks(T > nb + 1 ? T : nb + 1)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_rows, dim3(blocks(T)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_scan, dim3(1), dim3(SCAN_T), 0, st, A);
  hipLaunchKernelGGL(k_mg_fill, dim3(blocks(T)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_sort, dim3(unsigned(nb < MAX_BLOCKS ? nb : MAX_BLOCKS)), dim3(64), 0, st, A);
  hipLaunchKernelGGL(k_mg_pairs, dim3(blocks(T)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_chi2, dim3(blocks(params->cap_pairs)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_pick, dim3(blocks(params->cap_pairs)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_link, dim3(blocks(T)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_mg_counts, dim3(1), dim3(1), 0, st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}
