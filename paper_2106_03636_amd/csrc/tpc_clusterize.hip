// Clusterizer: zero-suppressed raw ADC digits to clusters, the producer of
// the tracker's input (paper §2.1: a clusterizing algorithm turns the raw
// ADC values into hits; §3.2: it runs much faster on GPUs than on CPUs).
// The operation is stated with tpc_clusterize in include/tpc_track.h.
//
// Four launches on the caller's stream:
//   k_clu_init   status and count;
//   k_clu_count  one wave per pad: the peaks among the pad's digits (their
//                neighbours in the pads either side found by binary search
//                over those pads' time-ordered digits, staged in LDS with
//                the block's own pads), counted per pad and per block of
//                four pads; input checks;
//   k_clu_scan   one block: exclusive scan of the per-block counts, total,
//                capacity check;
//   k_clu_emit   one wave per pad again: each peak recomputed and written at
//                its block's base plus the counts of the pads and lanes
//                before it, so clusters come in (unit, row, pad, time) order.
// The digits are read twice (2 x 4 bytes each, once per pass into LDS, with
// the pads either side of a block's four pads); everything else is small.
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

// A pad's time-ordered digits: times and charges, n of them (LDS or global).
struct List {
  const uint16_t *t, *q;
  int32_t n;
};

struct Peak {
  bool is;
  int32_t t, v, Q, Sp, St;
};

// The peak test and 3x3 sums of digit i of `own`: neighbours in the same pad
// are the adjacent digits (times increase inside a pad); in the pads below
// and above (`lo`, `hi`: empty at a row's edge), the digits with time
// t-1..t+1, found by binary search.  A neighbour earlier in (pad, time) order
// must be smaller, a later one at most equal.
__device__ __forceinline__ Peak peak_at(int32_t q_min, const List &own, const List &lo, const List &hi, int32_t i) {
  Peak k;
  k.t = own.t[i];
  k.v = own.q[i];
  k.Q = k.v;
  k.Sp = 0;
  k.St = 0;
  k.is = k.v >= q_min;
  if (!k.is) return k;
  if (i > 0 && int32_t(own.t[i - 1]) == k.t - 1) {  // earlier in the same pad
    const int32_t w = own.q[i - 1];
    if (!(w < k.v)) k.is = false;
    k.Q += w;
    k.St -= w;
  }
  if (i + 1 < own.n && int32_t(own.t[i + 1]) == k.t + 1) {  // later in the same pad
    const int32_t w = own.q[i + 1];
    if (!(w <= k.v)) k.is = false;
    k.Q += w;
    k.St += w;
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const List &L = side ? hi : lo;
    const int dp = side ? 1 : -1;
    int32_t a = 0, b = L.n;  // first digit with time >= t - 1
    while (a < b) {
      const int32_t mid = (a + b) >> 1;
      if (int32_t(L.t[mid]) < k.t - 1) a = mid + 1; else b = mid;
    }
    for (int m = 0; m < 3 && a < L.n; ++m, ++a) {
      const int32_t te = L.t[a];
      if (te > k.t + 1) break;
      const int32_t w = L.q[a];
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
}

__global__ void k_clu_init(CluArgs A) {
  *A.status = TPC_OK;
  *A.count = 0;
}

// A block takes PADS_PER_BLOCK consecutive pads, one per wave.  The digits
// of those pads and of the pads just before and after (a contiguous range of
// the digit arrays) are staged in LDS when they fit, so every neighbour
// search runs in LDS; a block whose range does not fit reads the digit
// arrays directly.  Slot s holds pad j0 - 1 + s.
constexpr int SLOTS = PADS_PER_BLOCK + 2;
constexpr int STAGE_DIGITS = 6144;  // 24 KB of (time, charge)

struct Stage {
  int64_t a[SLOTS + 1];  // slot s: digits [a[s], a[s+1]) of the arrays
  int32_t rbase[MAX_ROWS];
  uint16_t t[STAGE_DIGITS], q[STAGE_DIGITS];
  int32_t cnt[PADS_PER_BLOCK];
  int ok, fits;
};

// Offsets of the staged pads, checked; the digits staged if they fit.
__device__ __forceinline__ void stage_block(const CluArgs &A, Stage &S, int64_t j0) {
  load_rbase(A, S.rbase);
  if (threadIdx.x <= SLOTS) {
    const int64_t j = j0 - 1 + threadIdx.x;  // the offset at the start of pad j
    S.a[threadIdx.x] = j < 0 ? -1 : (j > A.n_pads ? -2 : A.off[j]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // pads before the first and after the last are empty
    if (S.a[0] == -1) S.a[0] = S.a[1];
    for (int s = 1; s <= SLOTS; ++s)
      if (S.a[s] == -2) S.a[s] = S.a[s - 1];
    bool ok = true;
    for (int s = 0; s <= SLOTS; ++s) ok = ok && S.a[s] >= 0 && S.a[s] <= A.n && (s == 0 || S.a[s - 1] <= S.a[s]);
    if (j0 == 0) ok = ok && S.a[1] == 0;
    if (j0 + PADS_PER_BLOCK >= A.n_pads) ok = ok && A.off[A.n_pads] == A.n;
    if (!ok) fail(A.status, TPC_E_INVALID);
    S.ok = ok;
    S.fits = ok && S.a[SLOTS] - S.a[0] <= STAGE_DIGITS;
  }
  __syncthreads();
  if (S.fits) {
    const int32_t m = int32_t(S.a[SLOTS] - S.a[0]);
    for (int32_t e = threadIdx.x; e < m; e += TPB) {
      S.t[e] = A.time[S.a[0] + e];
      S.q[e] = A.q[S.a[0] + e];
    }
  }
  __syncthreads();
}

struct PadView {
  List own, lo, hi;
  int u, r, p;
  bool valid;
};

// pad j0 + w of the block, its lists in LDS (LDS) or in the arrays
template <bool LDS>
__device__ __forceinline__ PadView pad_view(const CluArgs &A, const Stage &S, int64_t j0, int w) {
  PadView v;
  const int64_t j = j0 + w;
  v.valid = j < A.n_pads;
  v.u = int(j / A.pads_total);
  const int32_t jr = int32_t(j - int64_t(v.u) * A.pads_total);
  v.r = row_of(S.rbase, A.n_rows, jr);
  v.p = jr - S.rbase[v.r];
  const int np = 2 * A.half[v.r];
  auto list = [&](int s) {
    List L;
    L.n = int32_t(S.a[s + 1] - S.a[s]);
    if (LDS) {
      L.t = S.t + (S.a[s] - S.a[0]);
      L.q = S.q + (S.a[s] - S.a[0]);
    } else {
      L.t = A.time + S.a[s];
      L.q = A.q + S.a[s];
    }
    return L;
  };
  v.own = list(w + 1);
  v.lo = list(w);
  v.hi = list(w + 2);
  if (v.p == 0) v.lo.n = 0;  // neighbours stay in the row
  if (v.p == np - 1) v.hi.n = 0;
  return v;
}

template <bool LDS>
__device__ __forceinline__ int32_t count_pad(const CluArgs &A, const Stage &S, int64_t j0, int w) {
  const PadView v = pad_view<LDS>(A, S, j0, w);
  int32_t cnt = 0;
  if (!v.valid) return 0;
  const int lane = __lane_id();
  for (int32_t i0 = 0; i0 < v.own.n; i0 += 64) {
    const int32_t i = i0 + lane;
    bool pk = false;
    if (i < v.own.n) {
      if (i > 0 && v.own.t[i] <= v.own.t[i - 1]) fail(A.status, TPC_E_INVALID);  // times must increase
      pk = peak_at(A.q_min, v.own, v.lo, v.hi, i).is;
    }
    cnt += __popcll(__ballot(pk));
  }
  return cnt;
}

__global__ void __launch_bounds__(TPB) k_clu_count(CluArgs A) {
  __shared__ Stage S;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const int64_t j0 = int64_t(blockIdx.x) * PADS_PER_BLOCK;
  stage_block(A, S, j0);
  int32_t cnt = 0;
  if (S.ok) cnt = S.fits ? count_pad<true>(A, S, j0, wave) : count_pad<false>(A, S, j0, wave);
  if (lane == 0) {
    S.cnt[wave] = cnt;
    if (j0 + wave < A.n_pads) A.pad_cnt[j0 + wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < PADS_PER_BLOCK; ++w) s += S.cnt[w];
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

template <bool LDS>
__device__ __forceinline__ void emit_pad(const CluArgs &A, const Stage &S, int64_t j0, int w) {
  const PadView v = pad_view<LDS>(A, S, j0, w);
  if (!v.valid) return;
  const int lane = __lane_id();
  const int64_t j = j0 + w;
  int64_t o = A.blk[blockIdx.x];
  for (int64_t k = j0; k < j; ++k) o += A.pad_cnt[k];
  if (v.p == 0 && v.r == 0 && lane == 0) A.unit_offsets[v.u] = o;  // first pad of the unit
  const double half = double(A.half[v.r]);
  for (int32_t i0 = 0; i0 < v.own.n; i0 += 64) {
    const int32_t i = i0 + lane;
    Peak k;
    k.is = false;
    if (i < v.own.n) k = peak_at(A.q_min, v.own, v.lo, v.hi, i);
    const uint64_t m = __ballot(k.is);
    if (k.is) {
      // the oracle's order of operations, each rounded (no fused multiply-add)
#pragma clang fp contract(off)
      const int64_t c = o + __popcll(m & ((1ull << lane) - 1ull));
      const double padf = double(v.p) + double(k.Sp) / double(k.Q);
      const double timef = double(k.t) + double(k.St) / double(k.Q);
      A.y[c] = float((padf + 0.5 - half) * A.pw);
      A.z[c] = float((timef + 0.5) * A.tb - A.zoff);
      A.padf[c] = float(padf);
      A.timef[c] = float(timef);
      A.row[c] = uint16_t(v.r);
      A.qmax[c] = uint16_t(k.v);
      A.qtot[c] = k.Q;
    }
    o += __popcll(m);
  }
}

__global__ void __launch_bounds__(TPB) k_clu_emit(CluArgs A) {
  __shared__ Stage S;
  if (*A.status != TPC_OK) return;
  const int wave = threadIdx.x >> 6;
  const int64_t j0 = int64_t(blockIdx.x) * PADS_PER_BLOCK;
  stage_block(A, S, j0);
  if (!S.ok) return;
  if (S.fits) emit_pad<true>(A, S, j0, wave);
  else emit_pad<false>(A, S, j0, wave);
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
