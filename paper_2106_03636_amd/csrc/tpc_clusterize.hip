// Clusterizer: zero-suppressed raw ADC digits to clusters, the producer of
// the tracker's input (paper §2.1: a clusterizing algorithm turns the raw
// ADC values into hits; §3.2: it runs much faster on GPUs than on CPUs).
// The operation is stated with tpc_clusterize in include/tpc_track.h.
//
// Four launches on the caller's stream:
//   k_clu_init   status and count;
//   k_clu_count  one wave per pad: the peaks among the pad's digits (their
//                neighbours in the pads either side found by binary search
//                over those pads' time-ordered digits), counted per pad and
//                per block of four pads; input checks;
//   k_clu_scan   one block: exclusive scan of the per-block counts, total,
//                capacity check;
//   k_clu_emit   one wave per pad again: each peak recomputed and written at
//                its block's base plus the counts of the pads and lanes
//                before it, so clusters come in (unit, row, pad, time) order.
// The digits are read twice (2 x 4 bytes each); everything else is small.
// Peaks and charge sums are integer; the centre and position are FP64
// expressions rounded once to FP32, so the result is exact.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpc_track.h"

namespace {

constexpr int TPB = 256;
constexpr int PADS_PER_BLOCK = TPB / 64;
constexpr int MAX_ROWS = 255;

struct CluArgs {
  const int64_t *off;  // [n_units * pads_total + 1]
  const uint16_t *time, *q;
  int64_t n;
  int64_t n_pads;      // n_units * pads_total
  int32_t n_units, n_rows, pads_total, q_min;
  const int32_t *half;  // [n_rows]
  double pw, tb, zoff;
  int64_t cap;
  // outputs
  float *y, *z, *padf, *timef;
  uint16_t *row, *qmax;
  int32_t *qtot;
  int64_t *unit_offsets, *count;
  int32_t *status;
  // workspace
  int32_t *pad_cnt;  // [n_pads]
  int32_t *blk;      // [n_pads / 4 + 1]
};

__device__ __forceinline__ void fail(int32_t *status, int32_t code) { atomicCAS(status, TPC_OK, code); }

// first digit in [lo, hi) with time >= t (times increasing)
__device__ __forceinline__ int64_t lower_time(const uint16_t *time, int64_t lo, int64_t hi, int32_t t) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int32_t(time[mid]) < t) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Row of pad index jr (0 <= jr < pads_total) from the rows' first pads.
__device__ __forceinline__ int row_of(const int32_t *rbase, int n_rows, int32_t jr) {
  int lo = 0, hi = n_rows - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rbase[mid] <= jr) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct PadCtx {
  int64_t j, a, b;         // pad index, its digits [a, b)
  int64_t am, bm, ap, bp;  // digits of the pads below and above (empty at a row's edge)
  int u, r, p;
};

__device__ __forceinline__ PadCtx pad_ctx(const CluArgs &A, const int32_t *rbase, int64_t j) {
  PadCtx c;
  c.j = j;
  c.u = int(j / A.pads_total);
  const int32_t jr = int32_t(j - int64_t(c.u) * A.pads_total);
  c.r = row_of(rbase, A.n_rows, jr);
  c.p = jr - rbase[c.r];
  const int np = 2 * A.half[c.r];
  c.a = A.off[j];
  c.b = A.off[j + 1];
  c.am = c.bm = c.ap = c.bp = 0;
  if (c.p > 0) {
    c.am = A.off[j - 1];
    c.bm = c.a;
  }
  if (c.p < np - 1) {
    c.ap = c.b;
    c.bp = A.off[j + 2];
  }
  return c;
}

struct Peak {
  bool is;
  int32_t t, v, Q, Sp, St;
};

// The peak test and 3x3 sums of digit d of pad c: neighbours in the same pad
// are the adjacent digits (times increase inside a pad); in the pads either
// side, the digits with time t-1..t+1.  A neighbour earlier in (pad, time)
// order must be smaller, a later one at most equal.
__device__ __forceinline__ Peak peak_at(const CluArgs &A, const PadCtx &c, int64_t d) {
  Peak k;
  k.t = A.time[d];
  k.v = A.q[d];
  k.Q = k.v;
  k.Sp = 0;
  k.St = 0;
  k.is = k.v >= A.q_min;
  if (!k.is) return k;
  // same pad: dp = 0, later digits win ties against the earlier ones
  if (d > c.a && int32_t(A.time[d - 1]) == k.t - 1) {
    const int32_t w = A.q[d - 1];
    if (!(w < k.v)) k.is = false;
    k.Q += w;
    k.St -= w;
  }
  if (d + 1 < c.b && int32_t(A.time[d + 1]) == k.t + 1) {
    const int32_t w = A.q[d + 1];
    if (!(w <= k.v)) k.is = false;
    k.Q += w;
    k.St += w;
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int dp = side ? 1 : -1;
    const int64_t lo = side ? c.ap : c.am, hi = side ? c.bp : c.bm;
    if (lo >= hi) continue;
    int64_t e = lower_time(A.time, lo, hi, k.t - 1);
    for (int m = 0; m < 3 && e < hi; ++m, ++e) {
      const int32_t te = A.time[e];
      if (te > k.t + 1) break;
      const int32_t w = A.q[e];
      // the pad above is later in (pad, time) order, the pad below earlier
      if (side ? !(w <= k.v) : !(w < k.v)) k.is = false;
      k.Q += w;
      k.Sp += dp * w;
      k.St += (te - k.t) * w;
    }
  }
  return k;
}

__device__ __forceinline__ void load_rbase(const CluArgs &A, int32_t *rbase) {
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int r = 0; r < A.n_rows; ++r) {
      rbase[r] = s;
      s += 2 * A.half[r];
    }
  }
  __syncthreads();
}

__global__ void k_clu_init(CluArgs A) {
  *A.status = TPC_OK;
  *A.count = 0;
}

// pad ranges that lie inside the digit arrays and do not decrease
__device__ __forceinline__ bool ranges_ok(const CluArgs &A, const PadCtx &c) {
  return c.a >= 0 && c.a <= c.b && c.b <= A.n && c.am >= 0 && c.am <= c.bm && c.bm <= A.n && c.ap >= 0 &&
         c.ap <= c.bp && c.bp <= A.n;
}

__global__ void __launch_bounds__(TPB) k_clu_count(CluArgs A) {
  __shared__ int32_t rbase[MAX_ROWS];
  __shared__ int32_t wcnt[PADS_PER_BLOCK];
  load_rbase(A, rbase);
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const int64_t j = int64_t(blockIdx.x) * PADS_PER_BLOCK + wave;
  int32_t cnt = 0;
  if (j < A.n_pads) {
    PadCtx c = pad_ctx(A, rbase, j);
    if (!ranges_ok(A, c) || (j == 0 && c.a != 0) || (j == A.n_pads - 1 && c.b != A.n)) {
      if (lane == 0) fail(A.status, TPC_E_INVALID);
      c.b = c.a;  // read none of its digits
    }
    for (int64_t d0 = c.a; d0 < c.b; d0 += 64) {
      const int64_t d = d0 + lane;
      bool pk = false;
      if (d < c.b) {
        if (d > c.a && A.time[d] <= A.time[d - 1]) fail(A.status, TPC_E_INVALID);  // times must increase
        pk = peak_at(A, c, d).is;
      }
      cnt += __popcll(__ballot(pk));
    }
    if (lane == 0) A.pad_cnt[j] = cnt;
  }
  if (lane == 0) wcnt[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < PADS_PER_BLOCK; ++w) s += wcnt[w];
    A.blk[blockIdx.x] = s;
  }
}

// one block: exclusive scan of the per-block counts, in place; each thread
// takes PER consecutive counts, so one block scan covers 1024 * PER of them
__global__ void __launch_bounds__(1024) k_clu_scan(CluArgs A, int64_t nblk) {
  constexpr int PER = 8;
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  for (int64_t base = 0; base < nblk; base += 1024 * PER) {
    const int64_t i0 = base + int64_t(threadIdx.x) * PER;
    int32_t v[PER];
    int64_t sum = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      v[e] = i0 + e < nblk ? A.blk[i0 + e] : 0;
      sum += v[e];
    }
    int64_t inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t x = __shfl_up(inc, o);
      if (lane >= o) inc += x;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int64_t ex = carry_s + inc - sum, all = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) ex += wsum[w];
      all += wsum[w];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      if (i0 + e < nblk) A.blk[i0 + e] = int32_t(ex);
      ex += v[e];
    }
    __syncthreads();  // every thread has read carry_s and wsum
    if (threadIdx.x == 0) carry_s += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *A.count = carry_s;
    A.unit_offsets[A.n_units] = carry_s;
    if (carry_s > A.cap) fail(A.status, TPC_E_CAPACITY);
  }
}

__global__ void __launch_bounds__(TPB) k_clu_emit(CluArgs A) {
  __shared__ int32_t rbase[MAX_ROWS];
  load_rbase(A, rbase);
  if (*A.status != TPC_OK) return;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const int64_t j = int64_t(blockIdx.x) * PADS_PER_BLOCK + wave;
  if (j >= A.n_pads) return;
  int64_t o = A.blk[blockIdx.x];
  for (int64_t k = int64_t(blockIdx.x) * PADS_PER_BLOCK; k < j; ++k) o += A.pad_cnt[k];
  const PadCtx c = pad_ctx(A, rbase, j);
  if (c.p == 0 && c.r == 0 && lane == 0) A.unit_offsets[c.u] = o;  // first pad of the unit
  const double half = double(A.half[c.r]);
  for (int64_t d0 = c.a; d0 < c.b; d0 += 64) {
    const int64_t d = d0 + lane;
    Peak k;
    k.is = false;
    if (d < c.b) k = peak_at(A, c, d);
    const uint64_t m = __ballot(k.is);
    if (k.is) {
      // the oracle's order of operations, each rounded (no fused multiply-add)
#pragma clang fp contract(off)
      const int64_t i = o + __popcll(m & ((1ull << lane) - 1ull));
      const double padf = double(c.p) + double(k.Sp) / double(k.Q);
      const double timef = double(k.t) + double(k.St) / double(k.Q);
      A.y[i] = float((padf + 0.5 - half) * A.pw);
      A.z[i] = float((timef + 0.5) * A.tb - A.zoff);
      A.padf[i] = float(padf);
      A.timef[i] = float(timef);
      A.row[i] = uint16_t(c.r);
      A.qmax[i] = uint16_t(k.v);
      A.qtot[i] = k.Q;
    }
    o += __popcll(m);
  }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" size_t tpc_clusterize_workspace_size(int32_t n_units, const tpc_pad_geometry_t *g) {
  if (!g || n_units < 1 || g->n_rows < 1 || g->n_rows > MAX_ROWS || g->pads_total < 1) return 0;
  const int64_t n_pads = int64_t(n_units) * g->pads_total;
  const int64_t nblk = (n_pads + PADS_PER_BLOCK - 1) / PADS_PER_BLOCK;
  return align256(sizeof(int32_t) * size_t(n_pads)) + align256(sizeof(int32_t) * size_t(nblk));
}

extern "C" int tpc_clusterize(const tpc_digits_t *digits, const tpc_pad_geometry_t *g,
                              const tpc_clusterizer_params_t *params, tpc_cluster_out_t *out, void *workspace,
                              size_t workspace_bytes, void *stream) {
  if (!digits || !g || !params || !out) return TPC_E_INVALID;
  if (digits->n < 0 || digits->n >= (int64_t(1) << 31) || digits->n_units < 1 || !digits->pad_offsets ||
      (digits->n > 0 && (!digits->time || !digits->q)))
    return TPC_E_INVALID;
  if (g->n_rows < 1 || g->n_rows > MAX_ROWS || !g->half || g->pads_total < 1 || !(g->pad_width > 0.0f) ||
      !(g->time_bin > 0.0f))
    return TPC_E_INVALID;
  if (params->q_min < 1) return TPC_E_INVALID;
  if (out->cap < 0 || !out->unit_offsets || !out->count || !out->status) return TPC_E_INVALID;
  if (out->cap > 0 && (!out->y || !out->z || !out->row || !out->qtot || !out->qmax || !out->pad || !out->time))
    return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  if (workspace_bytes < tpc_clusterize_workspace_size(digits->n_units, g)) return TPC_E_NOMEM;

  CluArgs A;
  A.off = digits->pad_offsets;
  A.time = digits->time;
  A.q = digits->q;
  A.n = digits->n;
  A.n_units = digits->n_units;
  A.n_rows = g->n_rows;
  A.pads_total = g->pads_total;
  A.n_pads = int64_t(digits->n_units) * g->pads_total;
  A.q_min = params->q_min;
  A.half = g->half;
  A.pw = g->pad_width;
  A.tb = g->time_bin;
  A.zoff = g->z_offset;
  A.cap = out->cap;
  A.y = out->y;
  A.z = out->z;
  A.padf = out->pad;
  A.timef = out->time;
  A.row = out->row;
  A.qmax = out->qmax;
  A.qtot = out->qtot;
  A.unit_offsets = out->unit_offsets;
  A.count = out->count;
  A.status = out->status;
  char *ws = static_cast<char *>(workspace);
  A.pad_cnt = reinterpret_cast<int32_t *>(ws);
  A.blk = reinterpret_cast<int32_t *>(ws + align256(sizeof(int32_t) * size_t(A.n_pads)));
  const int64_t nblk = (A.n_pads + PADS_PER_BLOCK - 1) / PADS_PER_BLOCK;

  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_clu_init, dim3(1), dim3(1), 0, st, A);
  hipLaunchKernelGGL(k_clu_count, dim3(unsigned(nblk)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_clu_scan, dim3(1), dim3(1024), 0, st, A, nblk);
  hipLaunchKernelGGL(k_clu_emit, dim3(unsigned(nblk)), dim3(TPB), 0, st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}
