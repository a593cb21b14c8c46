// Assignment of tracks to collisions in continuous readout (paper §2, §2.3:
// collisions overlap in the drift volume, and tracks are assigned to them only
// after tracking).  The operation and its arithmetic are stated with
// tpc_assign_collisions in include/tpc_track.h.
//
// Six small launches on the caller's stream, over data already in HBM:
//   k_col_clear   zero the histogram copies;
//   k_col_zdca    per track, z' at the closest approach to the beam axis (FP64)
//                 and the histogram of the forming tracks;
//   k_col_flags   per bin, the copies summed (with a halo of `reach` bins, in
//                 LDS) and the peak test; a count of peaks per block;
//   k_col_number  per bin, its candidate index: the peaks of earlier blocks
//                 plus a block scan (side A first, then by bin);
//   k_col_assign  per track, the nearest peak within reach; per-candidate
//                 counts and a fixed-point sum of z' (order-independent);
//   k_col_finish  per candidate, the copies summed: counts, mean z', t0.
// Design for CDNA4: a few bins take most tracks (a collision's tracks share
// one z'), so the per-bin atomics are spread over NCOPY private copies of
// every counter, copy = block index mod NCOPY; consecutive blocks go to the
// eight XCDs in turn, so each copy is updated from one XCD only.  Lanes of a
// wave that hit the same bin are first combined into one atomic.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpc_track.h"

namespace {

constexpr int TPB = 256;
constexpr int NCOPY = 16;
constexpr int MAX_BINS_PER_SIDE = 1 << 16;
constexpr int MAX_REACH = 64;
constexpr float MAX_Z_RANGE = 1048576.0f;  // keeps the fixed-point sums of z' far from overflow
constexpr int MAX_TRACK_BLOCKS = 2048;
constexpr double FIX_SCALE = 65536.0;  // z' sums in units of 2^-16 cm
constexpr float KAPPA = 0.00299792458f;

struct ColArgs {
  // tracks
  const float *par;
  const float *xref;
  const int32_t *unit;
  const int64_t *trk_counts;
  const int32_t *trk_status;
  const int32_t *unit_side;
  int32_t n_units;
  // parameters
  double k;     // curvature per unit q/pT (1/cm per c/GeV)
  double zr;    // histogram range [-zr, zr)
  double w;     // bin width
  double cmax;  // forming tracks: |curvature| < cmax
  double vd;    // drift velocity
  int32_t nb;   // bins per side
  int32_t n2;   // bins of both sides
  int32_t n_min, reach;
  int64_t cap;
  // outputs
  double *zdca;
  int32_t *col;
  int32_t *c_side, *c_bin, *c_count, *c_form;
  double *c_z, *c_t0;
  int64_t *n_col;
  int32_t *status;
  // workspace; [NCOPY][n2] arrays are indexed copy * n2 + bin
  int32_t *hist;            // [NCOPY][n2] forming tracks per bin
  unsigned long long *cf;   // [NCOPY][n2] tracks a peak bin's candidate holds << 32 | forming ones
  unsigned long long *sum;  // [NCOPY][n2] fixed-point sum of the forming tracks' z'
  int32_t *cand;            // [n2] candidate of a peak bin, else -1
  uint8_t *flag;            // [n2] peak bin
  int32_t *blk;             // [n2 / TPB] peaks per block of bins
};

__device__ __forceinline__ void fail(int32_t *status, int32_t code) { atomicCAS(status, TPC_OK, code); }

__device__ __forceinline__ bool bad(const ColArgs &A) { return *A.status != TPC_OK; }

// z' at the transverse point of closest approach to the beam axis (x = y = 0
// of the unit's sector frame).  With a = x cos(phi) + y sin(phi) and
// b = y cos(phi) - x sin(phi) (the point's components along its direction and
// along the left normal), the circle of curvature C through the point gives
//   |P(s)|^2 = |P0|^2 + (2/C) (a sin(Cs) + (b + 1/C) (1 - cos(Cs))),
// stationary where tan(Cs) = -aC / (1 + bC).  The root Cs = atan2(-aC, 1 + bC)
// is the minimum (the second derivative there is positive) and turns less
// than half a turn either way; atan2 keeps full relative accuracy as C -> 0,
// where s -> -a, the straight line.
__device__ __forceinline__ double zdca_of(const float *p, float xr, double k) {
  const double y = p[0], z = p[1], sp = p[2], tgl = p[3];
  const double C = k * double(p[4]);
  const double cp = sqrt(1.0 - sp * sp);
  const double x = xr;
  const double a = x * cp + y * sp;
  const double b = y * cp - x * sp;
  const double s = C == 0.0 ? -a : atan2(-a * C, 1.0 + b * C) / C;
  return z + tgl * s;
}

// Histogram bin of z' (range [-zr, zr) in bins of w), -1 outside; a value whose
// quotient rounds up to nb sits in the last bin.
__device__ __forceinline__ int32_t bin_of(double z, const ColArgs &A) {
  if (!(z >= -A.zr && z < A.zr)) return -1;
  const int32_t b = int32_t(floor((z + A.zr) / A.w));
  return b < A.nb ? b : A.nb - 1;
}

// Adds v to a[key] once per distinct key among the lanes with `on` (v is the
// same on every lane): each round takes the key of the lowest pending lane
// (v_readlane with a wave-uniform lane, no LDS traffic) and one lane adds v
// times the number of lanes holding it.  Every lane of the wave must call it.
__device__ __forceinline__ void wave_add_i32(int32_t *a, int32_t key, bool on, int32_t v) {
  uint64_t todo = __ballot(on);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int32_t lk = __builtin_amdgcn_readlane(key, leader);
    const uint64_t same = __ballot(on && key == lk) & todo;
    if (__lane_id() == leader) atomicAdd(&a[lk], v * __popcll(same));
    todo &= ~same;
  }
}

// As wave_add_i32 with per-lane values: the lanes holding the round's key
// are summed across the wave first (two's complement: signed values add as
// unsigned).
__device__ __forceinline__ void wave_add_u64(unsigned long long *a, int32_t key, bool on, unsigned long long v) {
  uint64_t todo = __ballot(on);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int32_t lk = __builtin_amdgcn_readlane(key, leader);
    const bool mine = on && key == lk;
    const uint64_t same = __ballot(mine) & todo;
    unsigned long long x = mine ? v : 0ull;
    if (__popcll(same) > 1)
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (__lane_id() == leader) atomicAdd(&a[lk], x);
    todo &= ~same;
  }
}

__global__ void __launch_bounds__(TPB) k_col_clear(ColArgs A) {
  const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (i == 0) {
    *A.status = *A.trk_status;  // no assignment of failed tracking
    *A.n_col = 0;
  }
  if (i < int64_t(NCOPY) * A.n2) A.hist[i] = 0;
}

__global__ void __launch_bounds__(TPB) k_col_zdca(ColArgs A) {
  if (bad(A)) return;
  const int64_t T = A.trk_counts[0];
  int32_t *hist = A.hist + int64_t(blockIdx.x % NCOPY) * A.n2;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  // whole waves iterate together (the aggregation needs every lane of the wave)
  const int64_t T_pad = (T + 63) & ~int64_t(63);
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T_pad; t += stride) {
    bool form = false;
    int32_t key = 0;
    if (t < T) {
      const int32_t u = A.unit[t];
      const int32_t side = (u >= 0 && u < A.n_units) ? A.unit_side[u] : 0;
      if (side != 1 && side != -1) {
        fail(A.status, TPC_E_INVALID);
      } else {
        const float *p = A.par + 5 * t;
        const double z = zdca_of(p, A.xref[t], A.k);
        A.zdca[t] = z;
        const int32_t b = bin_of(z, A);
        form = b >= 0 && fabs(A.k * double(p[4])) < A.cmax;
        key = (side > 0 ? 0 : A.nb) + b;
      }
    }
    wave_add_i32(hist, key, form, 1);
  }
}

// Bin i (both sides, side A first) is a candidate: at least n_min forming
// tracks, and the largest within reach on its own side (a lower bin as large
// wins).  h[j] holds the total of bin i.
__device__ __forceinline__ bool is_peak(const ColArgs &A, const int32_t *h, int32_t i, int32_t j) {
  const int32_t v = h[j];
  if (v < A.n_min) return false;
  const int32_t b = i < A.nb ? i : i - A.nb;
  for (int d = 1; d <= A.reach; ++d) {
    if (b - d >= 0 && h[j - d] >= v) return false;
    if (b + d < A.nb && h[j + d] > v) return false;
  }
  return true;
}

// Exclusive rank of a true `f` among the block's lanes, and the block total.
__device__ __forceinline__ int32_t block_rank(bool f, int32_t *wsum, int32_t *total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint64_t m = __ballot(f);
  const int32_t in_wave = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wave] = __popcll(m);
  __syncthreads();
  int32_t before = 0, all = 0;
  for (int w = 0; w < TPB / 64; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  *total = all;
  return before + in_wave;
}

__global__ void __launch_bounds__(TPB) k_col_flags(ColArgs A) {
  __shared__ int32_t h[TPB + 2 * MAX_REACH];
  __shared__ int32_t wsum[TPB / 64];
  if (bad(A)) return;
  const int32_t b0 = blockIdx.x * TPB;
  for (int32_t j = threadIdx.x; j < TPB + 2 * MAX_REACH; j += TPB) {  // h[j] = total of bin b0 - MAX_REACH + j
    const int32_t i = b0 - MAX_REACH + j;
    int32_t v = 0;
    if (i >= 0 && i < A.n2)
      for (int c = 0; c < NCOPY; ++c) v += A.hist[int64_t(c) * A.n2 + i];
    h[j] = v;
  }
  __syncthreads();
  const int32_t i = b0 + threadIdx.x;
  const bool f = i < A.n2 && is_peak(A, h, i, threadIdx.x + MAX_REACH);
  if (i < A.n2) A.flag[i] = f;
  int32_t total;
  block_rank(f, wsum, &total);
  if (threadIdx.x == 0) A.blk[blockIdx.x] = total;
}

__global__ void __launch_bounds__(TPB) k_col_number(ColArgs A) {
  __shared__ int32_t wsum[TPB / 64];
  __shared__ int32_t pre[2];
  if (bad(A)) return;
  const int32_t nblk = (A.n2 + TPB - 1) / TPB;
  if (threadIdx.x < 64) {  // peaks in the blocks before this one, and in all blocks
    int32_t before = 0, all = 0;
    for (int32_t b = threadIdx.x; b < nblk; b += 64) {
      const int32_t v = A.blk[b];
      all += v;
      if (b < int32_t(blockIdx.x)) before += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      before += __shfl_xor(before, o);
      all += __shfl_xor(all, o);
    }
    if (threadIdx.x == 0) {
      pre[0] = before;
      pre[1] = all;
    }
  }
  __syncthreads();
  const int32_t i = blockIdx.x * TPB + threadIdx.x;
  const bool f = i < A.n2 && A.flag[i];
  int32_t total;
  const int32_t c = pre[0] + block_rank(f, wsum, &total);
  if (i < A.n2) A.cand[i] = f ? c : -1;
  if (f) {
    for (int k = 0; k < NCOPY; ++k) {
      const int64_t o = int64_t(k) * A.n2 + i;
      A.cf[o] = 0ull;
      A.sum[o] = 0ull;
    }
    if (c < A.cap) {
      A.c_side[c] = i < A.nb ? 1 : -1;
      A.c_bin[c] = i < A.nb ? i : i - A.nb;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *A.n_col = pre[1];
    if (pre[1] > A.cap) fail(A.status, TPC_E_CAPACITY);
  }
}

__global__ void __launch_bounds__(TPB) k_col_assign(ColArgs A) {
  if (bad(A)) return;
  const int64_t T = A.trk_counts[0];
  const int64_t copy = int64_t(blockIdx.x % NCOPY) * A.n2;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  const int64_t T_pad = (T + 63) & ~int64_t(63);
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T_pad; t += stride) {
    int32_t c = -1, peak_bin = 0;
    bool form = false;
    unsigned long long fz = 0ull;
    if (t < T) {
      const int32_t side = A.unit_side[A.unit[t]];  // checked by k_col_zdca
      const double z = A.zdca[t];
      const int32_t b = bin_of(z, A);
      if (b >= 0) {
        const int32_t off = side > 0 ? 0 : A.nb;
        for (int d = 0; d <= A.reach && c < 0; ++d) {  // nearest peak, the lower bin first
          if (b - d >= 0 && A.cand[off + b - d] >= 0) {
            c = A.cand[off + b - d];
            peak_bin = off + b - d;
          } else if (b + d < A.nb && A.cand[off + b + d] >= 0) {
            c = A.cand[off + b + d];
            peak_bin = off + b + d;
          }
        }
        form = c >= 0 && fabs(A.k * double(A.par[5 * t + 4])) < A.cmax;
        fz = (unsigned long long)(long long)llrint(z * FIX_SCALE);
      }
      A.col[t] = c;
    }
    wave_add_u64(A.cf + copy, peak_bin, c >= 0, (1ull << 32) | (form ? 1ull : 0ull));
    wave_add_u64(A.sum + copy, peak_bin, form, fz);
  }
}

__global__ void __launch_bounds__(TPB) k_col_finish(ColArgs A) {
  if (bad(A)) return;
  const int64_t n = *A.n_col;
  for (int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x; c < n; c += int64_t(gridDim.x) * TPB) {
    const int32_t side = A.c_side[c];
    const int32_t i = (side > 0 ? 0 : A.nb) + A.c_bin[c];
    unsigned long long cf = 0ull, s = 0ull;
    for (int k = 0; k < NCOPY; ++k) {
      const int64_t o = int64_t(k) * A.n2 + i;
      cf += A.cf[o];
      s += A.sum[o];
    }
    const int32_t count = int32_t(cf >> 32), form = int32_t(cf & 0xffffffffull);
    const double z = double((long long)s) / FIX_SCALE / double(form);  // form >= n_min >= 1
    A.c_count[c] = count;
    A.c_form[c] = form;
    A.c_z[c] = z;
    A.c_t0[c] = -double(side) * z / A.vd;
  }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int32_t bins_per_side(const tpc_collision_params_t *cp) {
  if (!cp || !(cp->bin_width > 0.0f) || !(cp->z_range > 0.0f)) return 0;
  const double nb = ceil(2.0 * double(cp->z_range) / double(cp->bin_width));
  return nb >= 1.0 && nb <= double(MAX_BINS_PER_SIDE) && cp->z_range <= MAX_Z_RANGE ? int32_t(nb) : 0;
}

// Workspace layout for n2 bins (both sides); returns the total size.
size_t layout(int32_t n2, size_t off[6]) {
  const size_t n = size_t(n2), nc = size_t(NCOPY) * n;
  const size_t sz[6] = {4 * nc, 8 * nc, 8 * nc, 4 * n, n, 4 * ((n + TPB - 1) / TPB)};
  size_t o = 0;
  for (int k = 0; k < 6; ++k) {
    off[k] = o;
    o += align256(sz[k]);
  }
  return o;
}

}  // namespace

extern "C" size_t tpc_collisions_workspace_size(const tpc_collision_params_t *cp) {
  const int32_t nb = bins_per_side(cp);
  if (nb == 0) return 0;
  size_t off[6];
  return layout(2 * nb, off);
}

extern "C" int tpc_assign_collisions(const tpc_tracks_t *tracks, const int32_t *unit_side, int32_t n_units,
                                     const tpc_field_t *field, const tpc_collision_params_t *cp,
                                     tpc_collisions_t *out, void *workspace, size_t workspace_bytes,
                                     void *stream) {
  if (!tracks || !field || !cp || !out || !unit_side || n_units < 1) return TPC_E_INVALID;
  if (!tracks->params || !tracks->x_ref || !tracks->unit || !tracks->counts || !tracks->status ||
      tracks->cap_tracks < 0)
    return TPC_E_INVALID;
  if (!out->zdca || !out->collision || !out->n_collisions || !out->status || out->cap < 0) return TPC_E_INVALID;
  if (out->cap > 0 && (!out->side || !out->bin || !out->count || !out->n_form || !out->z || !out->t0))
    return TPC_E_INVALID;
  const int32_t nb = bins_per_side(cp);
  if (nb == 0 || !(cp->v_drift > 0.0f) || !(cp->c_max >= 0.0f) || cp->n_min < 1 || cp->reach < 0 ||
      cp->reach > MAX_REACH || !isfinite(field->bz_tesla))
    return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  size_t off[6];
  if (workspace_bytes < layout(2 * nb, off)) return TPC_E_NOMEM;

  ColArgs A;
  A.par = tracks->params;
  A.xref = tracks->x_ref;
  A.unit = tracks->unit;
  A.trk_counts = tracks->counts;
  A.trk_status = tracks->status;
  A.unit_side = unit_side;
  A.n_units = n_units;
  A.k = double(-KAPPA * field->bz_tesla);  // the tracker's curvature constant, as its fit used it
  A.zr = cp->z_range;
  A.w = cp->bin_width;
  A.cmax = cp->c_max;
  A.vd = cp->v_drift;
  A.nb = nb;
  A.n2 = 2 * nb;
  A.n_min = cp->n_min;
  A.reach = cp->reach;
  A.cap = out->cap;
  A.zdca = out->zdca;
  A.col = out->collision;
  A.c_side = out->side;
  A.c_bin = out->bin;
  A.c_count = out->count;
  A.c_form = out->n_form;
  A.c_z = out->z;
  A.c_t0 = out->t0;
  A.n_col = out->n_collisions;
  A.status = out->status;
  char *ws = static_cast<char *>(workspace);
  A.hist = reinterpret_cast<int32_t *>(ws + off[0]);
  A.cf = reinterpret_cast<unsigned long long *>(ws + off[1]);
  A.sum = reinterpret_cast<unsigned long long *>(ws + off[2]);
  A.cand = reinterpret_cast<int32_t *>(ws + off[3]);
  A.flag = reinterpret_cast<uint8_t *>(ws + off[4]);
  A.blk = reinterpret_cast<int32_t *>(ws + off[5]);

  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t tb = (tracks->cap_tracks + TPB - 1) / TPB;
  const unsigned track_blocks = unsigned(tb < 1 ? 1 : (tb > MAX_TRACK_BLOCKS ? MAX_TRACK_BLOCKS : tb));
  const unsigned bin_blocks = unsigned((A.n2 + TPB - 1) / TPB);
  const unsigned clear_blocks = unsigned((int64_t(NCOPY) * A.n2 + TPB - 1) / TPB);
  const int64_t cb = (out->cap + TPB - 1) / TPB;
  const unsigned cand_blocks = unsigned(cb < 1 ? 1 : (cb > 64 ? 64 : cb));
  hipLaunchKernelGGL(k_col_clear, dim3(clear_blocks), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_col_zdca, dim3(track_blocks), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_col_flags, dim3(bin_blocks), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_col_number, dim3(bin_blocks), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_col_assign, dim3(track_blocks), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_col_finish, dim3(cand_blocks), dim3(TPB), 0, st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}
