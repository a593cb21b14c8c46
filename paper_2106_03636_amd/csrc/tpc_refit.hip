// Track refit: every output track of a tracking call fitted again over
// exactly the hits it kept (the paper's synchronous processing needs full
// tracking, §2.1, at a resolution that matches offline reconstruction, §2.3).
// The operation is stated with tpc_refit_tracks in include/tpc_track.h.
//
// Seven launches on the caller's stream:
//   k_rf_init    clear the length histogram, take over the tracking status;
//   k_rf_pack    per cluster (coalesced): its row and its y, z in quanta,
//                packed into one 64-bit record;
//   k_rf_hist    histogram of the tracks' hit counts (LDS per block);
//   k_rf_scan    one block: bucket offsets, longest tracks first;
//   k_rf_order   each track's slot in the length order (one global atomic
//                per block and bucket, the slots inside a block from LDS);
//   k_rf_gather  per track hit: its cluster's record, in the order of the
//                track's hit list (one random 8-byte read per hit);
//   k_rf_fit     one lane per track, in length order (so the lanes of a wave
//                run loops of about the same length): seed, pass 1 forward,
//                pass 2 backward; state and covariance stay in registers.
// Clusters are in no particular order, so a track's hits are scattered over
// the cluster arrays: the pack turns three random reads per hit (y, z, row,
// each a cache line for 2 or 4 bytes) into one, and after the gather each
// lane of the fit reads a contiguous run of records.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpc_kalman.h"
#include "tpc_track.h"

namespace {

using namespace tpc_kf;

constexpr int TPB = 256;
constexpr int FTB = 128;  // threads per block of the fit
constexpr int NB = 256;   // length buckets (hit counts >= 255 share the last)
constexpr int GATHER_BLOCKS = 4096;
constexpr int FIT_BLOCKS = 4096;
constexpr float KAPPA = 0.00299792458f;
constexpr int QBIAS = 1 << 23;  // record fields hold Y + 2^23 and Z + 2^23 (24 bits each)

struct RfArgs {
  const float *y, *z;
  const uint16_t *row;
  int64_t n_clusters;
  const float *row_x;
  int32_t n_rows;
  const int32_t *trk_status, *n_hits, *first_hit, *hits;
  const int64_t *trk_counts;
  int64_t cap_tracks, cap_hits;
  float k, smx, sy2, sz2;
  float cov0[5];
  // outputs
  float *par, *cov, *xref, *chi2, *par_out, *cov_out, *xout;
  uint8_t *ok;
  int32_t *status;
  // workspace
  int32_t *bucket;   // [NB] histogram, then running offsets
  int32_t *order;    // [cap_tracks] slot -> track
  uint64_t *cl;      // [n_clusters] packed (row, Y, Z) per cluster, NO_REC when out of range
  uint64_t *rec;     // [cap_hits] packed (row, Y, Z) per track hit
  int32_t *bad;      // [1] a track hit names no cluster or one out of range, or a track's hits lie outside the list
};

constexpr uint64_t NO_REC = ~uint64_t(0);  // row field 0xFFFF: never a valid row

__device__ __forceinline__ int bucket_of(int n) {  // longest first
  return NB - 1 - (n < 0 ? 0 : n < NB - 1 ? n : NB - 1);
}
// tracks and track hits of the tracking call, within the output capacities
__device__ __forceinline__ int64_t n_tracks(const RfArgs &A) {
  const int64_t T = A.trk_counts[0];
  return T < A.cap_tracks ? T : A.cap_tracks;
}
__device__ __forceinline__ int64_t n_track_hits(const RfArgs &A) {
  const int64_t H = A.trk_counts[1];
  return H < A.cap_hits ? H : A.cap_hits;
}

__global__ void __launch_bounds__(TPB) k_rf_init(RfArgs A) {
  const int i = threadIdx.x;
  if (i == 0) {
    *A.status = *A.trk_status;
    *A.bad = 0;
  }
  if (i < NB) A.bucket[i] = 0;
}

__global__ void __launch_bounds__(TPB) k_rf_hist(RfArgs A) {
  __shared__ int32_t h[NB];
  if (*A.status != TPC_OK) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t T = n_tracks(A), H = n_track_hits(A);
  bool bad = false;
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T; t += int64_t(gridDim.x) * TPB) {
    const int n = A.n_hits[t];
    const int64_t f = A.first_hit[t];
    if (n < 0 || f < 0 || f + n > H) bad = true;  // the track's hits lie outside the hit list
    atomicAdd(&h[bucket_of(n)], 1);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&A.bucket[threadIdx.x], h[threadIdx.x]);
  if (bad) atomicOr(A.bad, 1);  // k_rf_fit reports it
}

// exclusive scan of the NB bucket counts (one block of NB threads)
__global__ void __launch_bounds__(NB) k_rf_scan(RfArgs A) {
  __shared__ int32_t s[NB];
  if (*A.status != TPC_OK) return;
  const int i = threadIdx.x;
  const int v = A.bucket[i];
  s[i] = v;
  __syncthreads();
  for (int d = 1; d < NB; d <<= 1) {
    const int a = i >= d ? s[i - d] : 0;
    __syncthreads();
    s[i] += a;
    __syncthreads();
  }
  A.bucket[i] = s[i] - v;
}

__global__ void __launch_bounds__(TPB) k_rf_pack(RfArgs A) {
  if (*A.status != TPC_OK) return;
  for (int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x; c < A.n_clusters; c += int64_t(gridDim.x) * TPB) {
    const int r = A.row[c];
    const float y = A.y[c], z = A.z[c];
    uint64_t v = NO_REC;
    if (r < A.n_rows && fabsf(y) <= 8192.f && fabsf(z) <= 8192.f) {  // |Y|, |Z| <= 2^21 fit the 24-bit fields
      const int Y = __float2int_rn(y * 256.0f), Z = __float2int_rn(z * 256.0f);
      v = (uint64_t(r) << 48) | (uint64_t(uint32_t(Y + QBIAS)) << 24) | uint64_t(uint32_t(Z + QBIAS));
    }
    A.cl[c] = v;
  }
}

// Slots of the length order: per block of TPB tracks, the tracks of each
// bucket count themselves in LDS, one thread per bucket reserves the block's
// range with one global atomic, and each track takes base + its LDS rank.
__global__ void __launch_bounds__(TPB) k_rf_order(RfArgs A) {
  static_assert(TPB == NB, "one thread per bucket");
  __shared__ int32_t cnt[NB], base[NB];
  if (*A.status != TPC_OK) return;
  const int64_t T = n_tracks(A);
  for (int64_t t0 = int64_t(blockIdx.x) * TPB; t0 < T; t0 += int64_t(gridDim.x) * TPB) {  // block-uniform
    const int64_t t = t0 + threadIdx.x;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int b = t < T ? bucket_of(A.n_hits[t]) : -1;
    const int rank = b >= 0 ? atomicAdd(&cnt[b], 1) : 0;
    __syncthreads();
    if (cnt[threadIdx.x]) base[threadIdx.x] = atomicAdd(&A.bucket[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) A.order[base[b] + rank] = int32_t(t);
    __syncthreads();  // cnt and base are reused by the next chunk
  }
}

__global__ void __launch_bounds__(TPB) k_rf_gather(RfArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t H = n_track_hits(A);
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < H; i += int64_t(gridDim.x) * TPB) {
    const int32_t h = A.hits[i];
    uint64_t r = h >= 0 && h < A.n_clusters ? A.cl[h] : NO_REC;
    if (r == NO_REC) {
      atomicOr(A.bad, 1);
      r = 0;
    }
    A.rec[i] = r;
  }
}

struct Hit {
  int row, Y, Z;
};
__device__ __forceinline__ Hit unpack(uint64_t r) {
  Hit h;
  h.row = int(r >> 48);
  h.Y = int((r >> 24) & 0xFFFFFFu) - QBIAS;
  h.Z = int(r & 0xFFFFFFu) - QBIAS;
  return h;
}

// The state in absolute coordinates (the filter runs relative to the first
// hit's quanta Yr, Zr), its covariance and x; zeros for a track not fitted.
__device__ __forceinline__ void store(KStateR &s, bool ok, int Yr, int Zr, float *p, float *c, float *x) {
  p[0] = ok ? s.p[0] + float(Yr) * (1.f / 256.f) : 0.f;
  p[1] = ok ? s.p[1] + float(Zr) * (1.f / 256.f) : 0.f;
#pragma unroll
  for (int q = 2; q < 5; ++q) p[q] = ok ? s.p[q] : 0.f;
#pragma unroll
  for (int q = 0; q < 15; ++q) c[q] = ok ? cv(s, q) : 0.f;
  *x = ok ? s.x : 0.f;
}

__global__ void __launch_bounds__(FTB) k_rf_fit(RfArgs A) {
  if (*A.status != TPC_OK) return;
  if (*A.bad) {  // every block sees the same flag; one writes the status
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.status = TPC_E_INVALID;
    return;
  }
  const int64_t T = n_tracks(A);
  KStateR s;  // the covariance in registers: no LDS round trip in the update chain
  const float k = A.k, smx = A.smx, sy2 = A.sy2, sz2 = A.sz2;
  for (int64_t i0 = int64_t(blockIdx.x) * FTB; i0 < T; i0 += int64_t(gridDim.x) * FTB) {
    const int64_t i = i0 + threadIdx.x;
    if ((i & ~int64_t(63)) >= T) break;  // whole wave past the tracks (wave-uniform)
    const bool valid = i < T;
    const int32_t t = valid ? A.order[i] : 0;
    const int n = valid ? A.n_hits[t] : 0;
    const uint64_t *R = A.rec + (valid ? A.first_hit[t] : 0);
    bool ok = valid && n >= 3;
    int Yr = 0, Zr = 0;
    if (ok) {
      const Hit a = unpack(R[0]), m = unpack(R[n / 2]), b = unpack(R[n - 1]);
      Yr = a.Y;
      Zr = a.Z;
      ok = seed3(s, A.row_x[a.row], A.row_x[m.row], A.row_x[b.row], float(m.Y - Yr) * (1.f / 256.f),
                 float(b.Y - Yr) * (1.f / 256.f), float(b.Z - Zr) * (1.f / 256.f), k, smx, A.cov0);
    }
    if (ok) kf_update(s, 0.f, 0.f, sy2, sz2);  // the first hit is the reference
    // pass 1: hits 1 .. n-1, the next record loaded ahead of the step
    int nmax = ok ? n : 0;
    for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, __shfl_xor(nmax, d));
    uint64_t nxt = ok ? R[1] : 0;
    for (int j = 1; j < nmax; ++j) {
      const uint64_t cur = nxt;
      if (ok && j + 1 < n) nxt = R[j + 1];
      if (!ok || j >= n) continue;
      const Hit h = unpack(cur);
      const float xr = A.row_x[h.row];
      Step st;
      if (!step_prepare(s, xr, k, smx, st)) {
        ok = false;
        continue;
      }
      step_apply(s, st, xr, k);
      upd_hit(s, make_int2(h.Y, h.Z), Yr, Zr, sy2, sz2);
    }
    // outer state: the end of pass 1
    if (valid) store(s, ok, Yr, Zr, A.par_out + int64_t(t) * 5, A.cov_out + int64_t(t) * 15, A.xout + t);
    // pass 2: hits n-2 .. 0, the covariance reset
    if (ok) {
      cov_reset(s, A.cov0);
      s.chi2 = 0.f;
      const Hit h = unpack(R[n - 1]);
      upd_hit(s, make_int2(h.Y, h.Z), Yr, Zr, sy2, sz2);
    }
    nxt = ok ? R[n - 2] : 0;
    for (int j = nmax - 2; j >= 0; --j) {
      const bool mine = ok && j <= n - 2;
      const uint64_t cur = nxt;
      if (mine && j >= 1) nxt = R[j - 1];
      if (!mine) continue;
      const Hit h = unpack(cur);
      const float xr = A.row_x[h.row];
      Step st;
      if (!step_prepare(s, xr, k, smx, st)) {
        ok = false;
        continue;
      }
      step_apply(s, st, xr, k);
      upd_hit(s, make_int2(h.Y, h.Z), Yr, Zr, sy2, sz2);
    }
    if (valid && !ok) store(s, false, 0, 0, A.par_out + int64_t(t) * 5, A.cov_out + int64_t(t) * 15, A.xout + t);
    if (valid) {
      A.ok[t] = ok ? 1 : 0;
      store(s, ok, Yr, Zr, A.par + int64_t(t) * 5, A.cov + int64_t(t) * 15, A.xref + t);
      A.chi2[t] = ok ? s.chi2 : 0.f;
    }
  }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" size_t tpc_refit_workspace_size(int64_t n_clusters, int64_t cap_tracks, int64_t cap_hits) {
  if (n_clusters < 0 || n_clusters >= (int64_t(1) << 30) || cap_tracks < 0 || cap_hits < 0 ||
      cap_tracks > (int64_t(1) << 31) || cap_hits > (int64_t(1) << 31))
    return 0;
  return align256(NB * 4 + 256) + align256(size_t(cap_tracks) * 4) + align256(size_t(n_clusters) * 8) +
         align256(size_t(cap_hits) * 8);
}

extern "C" int tpc_refit_tracks(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                                const tpc_field_t *field, const tpc_params_t *params, const tpc_tracks_t *tracks,
                                tpc_refit_t *out, void *workspace, size_t workspace_bytes, void *stream) {
  if (!clusters || !geometry || !field || !params || !tracks || !out) return TPC_E_INVALID;
  if (clusters->n < 0 || clusters->n >= (int64_t(1) << 30) ||
      (clusters->n > 0 && (!clusters->y || !clusters->z || !clusters->row)))
    return TPC_E_INVALID;
  if (geometry->n_rows < 3 || geometry->n_rows > 255 || !geometry->row_x) return TPC_E_INVALID;
  if (!tracks->n_hits || !tracks->first_hit || !tracks->hits || !tracks->counts || !tracks->status ||
      tracks->cap_tracks < 0 || tracks->cap_hits < 0)
    return TPC_E_INVALID;
  if (!isfinite(field->bz_tesla) || !(params->sinphi_max > 0.f) || !(params->sinphi_max < 1.f) ||
      !(params->sigma_y > 0.f) || !(params->sigma_z > 0.f))
    return TPC_E_INVALID;
  for (int q = 0; q < 5; ++q)
    if (!(params->cov0[q] > 0.f) || !isfinite(params->cov0[q])) return TPC_E_INVALID;
  if (!out->params || !out->cov || !out->x_ref || !out->chi2 || !out->params_out || !out->cov_out ||
      !out->x_out || !out->ok || !out->status)
    return TPC_E_INVALID;
  const size_t need = tpc_refit_workspace_size(clusters->n, tracks->cap_tracks, tracks->cap_hits);
  if (need == 0) return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  if (workspace_bytes < need) return TPC_E_NOMEM;
  RfArgs A;
  A.y = clusters->y;
  A.z = clusters->z;
  A.row = clusters->row;
  A.n_clusters = clusters->n;
  A.row_x = geometry->row_x;
  A.n_rows = geometry->n_rows;
  A.trk_status = tracks->status;
  A.n_hits = tracks->n_hits;
  A.first_hit = tracks->first_hit;
  A.hits = tracks->hits;
  A.trk_counts = tracks->counts;
  A.cap_tracks = tracks->cap_tracks;
  A.cap_hits = tracks->cap_hits;
  A.k = -KAPPA * field->bz_tesla;  // the tracker's curvature constant
  A.smx = params->sinphi_max;
  A.sy2 = params->sigma_y * params->sigma_y;
  A.sz2 = params->sigma_z * params->sigma_z;
  for (int q = 0; q < 5; ++q) A.cov0[q] = params->cov0[q];
  A.par = out->params;
  A.cov = out->cov;
  A.xref = out->x_ref;
  A.chi2 = out->chi2;
  A.par_out = out->params_out;
  A.cov_out = out->cov_out;
  A.xout = out->x_out;
  A.ok = out->ok;
  A.status = out->status;
  char *w = static_cast<char *>(workspace);
  A.bucket = reinterpret_cast<int32_t *>(w);
  A.bad = A.bucket + NB;
  w += align256(NB * 4 + 256);
  A.order = reinterpret_cast<int32_t *>(w);
  w += align256(size_t(tracks->cap_tracks) * 4);
  A.cl = reinterpret_cast<uint64_t *>(w);
  w += align256(size_t(clusters->n) * 8);
  A.rec = reinterpret_cast<uint64_t *>(w);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t tb = (tracks->cap_tracks + TPB - 1) / TPB;
  const int64_t hb = (tracks->cap_hits + TPB - 1) / TPB;
  const int64_t cb = (clusters->n + TPB - 1) / TPB;
  const int64_t fb = (tracks->cap_tracks + FTB - 1) / FTB;
  auto clamp = [](int64_t b, int64_t hi) { return unsigned(b < 1 ? 1 : (b > hi ? hi : b)); };
  hipLaunchKernelGGL(k_rf_init, dim3(1), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_pack, dim3(clamp(cb, GATHER_BLOCKS)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_hist, dim3(clamp(tb, 1024)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_scan, dim3(1), dim3(NB), 0, st, A);
  hipLaunchKernelGGL(k_rf_order, dim3(clamp(tb, 1024)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_gather, dim3(clamp(hb, GATHER_BLOCKS)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_fit, dim3(clamp(fb, FIT_BLOCKS)), dim3(FTB), 0, st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}

// ---------------------------------------------------------------------------
// Fit of merged chains: the hits of linked segments (a tpc_merge_tracks
// output) in chain order, across their sectors' frames.  Launches: status;
// the refit's k_rf_pack and k_rf_gather (every track hit as one packed
// record, in hit-list order); k_ch_len (each head's chain length, a length
// histogram); k_rf_scan; k_ch_order (heads in length order); k_ch_fit (one
// lane per head in that order, so the lanes of a wave walk chains of about
// one length): before a hit of another frame the state and its covariance
// are turned into that frame (the turn's Jacobian), then carried and updated
// as in the refit.  The state stays relative to the current frame's
// reference quanta (z: the chain's first hit; y: the first hit seen in the
// frame), re-based at each turn.  The operation is stated with
// tpc_fit_chains in include/tpc_track.h.

namespace {

constexpr int MAX_CHAIN = 64;  // segments a chain may hold
constexpr double CH_TWO_PI = 6.283185307179586476925286766559;

struct ChArgs {
  const float *y, *z;
  const uint16_t *row;
  int64_t n_clusters;
  const float *row_x;
  int32_t n_rows;
  const int32_t *trk_status, *n_hits, *first_hit, *hits, *unit;
  const int64_t *trk_counts;
  int64_t cap_tracks, cap_hits;
  const int32_t *next, *prev, *mg_status;
  const float *alpha;
  int32_t n_units;
  float k, smx, sy2, sz2;
  float cov0[5];
  float *par, *cov, *xref, *chi2;
  int32_t *n_chain;
  uint8_t *ok;
  int32_t *status;
  // workspace (the refit's layout)
  const uint64_t *rec;  // [cap_hits] packed (row, Y, Z) per track hit
  int32_t *order;       // [cap_tracks] slot -> chain head
  int32_t *bucket;      // [NB] length histogram, then offsets
  int32_t *bad;         // [0] a hit out of range (the gather's flag), [1] number of heads
};

struct CHit {
  float x;
  int Y, Z, u;
};

__device__ __forceinline__ CHit chain_hit(const ChArgs &A, int32_t seg, int j) {
  const Hit h = unpack(A.rec[A.first_hit[seg] + j]);
  CHit c;
  c.x = A.row_x[h.row];
  c.Y = h.Y;
  c.Z = h.Z;
  c.u = A.unit[seg];
  return c;
}

// the chain's hit j: its segment found by walking the links from the head
__device__ CHit chain_hit_at(const ChArgs &A, int32_t head, int j) {
  int32_t s = head;
  for (int g = 0; g < MAX_CHAIN && j >= A.n_hits[s]; ++g) {
    j -= A.n_hits[s];
    s = A.next[s];
  }
  return chain_hit(A, s, j);
}

__device__ __forceinline__ float frame_turn(const ChArgs &A, int from, int to) {
  return float(remainder(double(A.alpha[to]) - double(A.alpha[from]), CH_TWO_PI));
}

// Turn the state by d into another frame: the point (x, ya) and the
// direction turn, the state moves to the turned point's x; the covariance by
// the turn's Jacobian (rows y, z, sin(phi) change: dy'/dy = cos phi / cos
// phi', dz'/dy = -sin d tan(lambda) / cos phi', dsin'/dy = -C sin d,
// dsin'/dsin = cos phi' / cos phi).  ya: absolute y in, turned y out.
__device__ bool turn32(KStateR &s, float d, float &ya, float k, float smx) {
  const float cd = cosf(d), sd = sinf(d);
  const float sp = s.p[2];
  if (!(fabsf(sp) < 1.f)) return false;
  const float c = sqrtf(1.f - sp * sp);
  const float s2 = sp * cd - c * sd, c2 = c * cd + sp * sd;
  if (!(c2 > 0.f) || !(fabsf(s2) < smx)) return false;
  const float x2 = s.x * cd + ya * sd;
  const float y2 = -s.x * sd + ya * cd;
  const float j00 = c / c2, j10 = -sd * s.p[3] / c2, j20 = -k * s.p[4] * sd, j22 = c2 / c;
  float C[5][5];
  int m = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++m) C[i][j] = C[j][i] = s.c[m];
  // T = J C (rows 0..2 change), then C' = T J^T (columns 0..2 change)
  float T[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    T[0][j] = j00 * C[0][j];
    T[1][j] = C[1][j] + j10 * C[0][j];
    T[2][j] = j20 * C[0][j] + j22 * C[2][j];
    T[3][j] = C[3][j];
    T[4][j] = C[4][j];
  }
  m = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++m) {
      const float v = j == 0 ? j00 * T[i][0]
                    : j == 1 ? T[i][1] + j10 * T[i][0]
                    : j == 2 ? j20 * T[i][0] + j22 * T[i][2]
                             : T[i][j];
      s.c[m] = v;
    }
  s.p[2] = s2;
  s.x = x2;
  ya = y2;
  return true;
}

__global__ void __launch_bounds__(TPB) k_ch_init(ChArgs A) {
  const int i = threadIdx.x;
  if (i == 0) {
    *A.status = *A.trk_status != TPC_OK ? *A.trk_status : *A.mg_status;
    A.bad[0] = A.bad[1] = 0;
  }
  if (i < NB) A.bucket[i] = 0;
}

__device__ __forceinline__ int64_t ch_tracks(const ChArgs &A) {
  const int64_t T = A.trk_counts[0];
  return T < A.cap_tracks ? T : A.cap_tracks;
}

// per track: the checks of the input (its hits inside the hit list; links
// that are mutual, name tracks of the call and, followed back, reach a head
// within MAX_CHAIN segments, so that no closed loop is left; a linked track's
// unit in range), and the length of the chain it heads (0 for other tracks);
// heads counted and histogrammed by length (longest first)
__global__ void __launch_bounds__(TPB) k_ch_len(ChArgs A) {
  __shared__ int32_t h[NB];
  __shared__ int32_t heads;
  if (*A.status != TPC_OK) return;
  h[threadIdx.x] = 0;
  if (threadIdx.x == 0) heads = 0;
  __syncthreads();
  const int64_t T = ch_tracks(A);
  const int64_t H = A.trk_counts[1] < A.cap_hits ? A.trk_counts[1] : A.cap_hits;
  bool bad = false;
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T; t += int64_t(gridDim.x) * TPB) {
    const int nt = A.n_hits[t];
    const int64_t ft = A.first_hit[t];
    const int32_t nx = A.next[t], pv = A.prev[t];
    if (nt < 0 || ft < 0 || ft + nt > H) bad = true;
    if ((nx >= 0 && (nx >= T || A.prev[nx] != t)) || (pv >= 0 && (pv >= T || A.next[pv] != t))) bad = true;
    if ((nx >= 0 || pv >= 0) && (A.unit[t] < 0 || A.unit[t] >= A.n_units)) bad = true;
    if (pv >= 0 && !bad) {
      int32_t q = pv;
      for (int g = 1; q >= 0 && q < T && g < MAX_CHAIN; ++g) q = A.prev[q];
      if (q >= 0) bad = true;
    }
    int64_t n = 0;
    if (pv < 0 && nx >= 0) {
      int nseg = 0;
      for (int32_t q = int32_t(t); q >= 0; q = A.next[q], ++nseg) {
        if (q >= T || nseg >= MAX_CHAIN || A.n_hits[q] < 1) {
          bad = true;
          n = 0;
          break;
        }
        n += A.n_hits[q];
      }
      if (n > INT32_MAX) {
        bad = true;
        n = 0;
      }
      if (n > 0) {
        atomicAdd(&h[bucket_of(int(n))], 1);
        atomicAdd(&heads, 1);
      }
    }
    A.n_chain[t] = int32_t(n);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&A.bucket[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0 && heads) atomicAdd(&A.bad[1], heads);
  if (bad) *A.status = TPC_E_INVALID;
}

// slots of the heads in length order (one global atomic per block and bucket)
__global__ void __launch_bounds__(TPB) k_ch_order(ChArgs A) {
  __shared__ int32_t cnt[NB], base[NB];
  if (*A.status != TPC_OK) return;
  const int64_t T = ch_tracks(A);
  for (int64_t t0 = int64_t(blockIdx.x) * TPB; t0 < T; t0 += int64_t(gridDim.x) * TPB) {  // block-uniform
    const int64_t t = t0 + threadIdx.x;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int n = t < T ? A.n_chain[t] : 0;
    const int b = n > 0 ? bucket_of(n) : -1;
    const int rank = b >= 0 ? atomicAdd(&cnt[b], 1) : 0;
    __syncthreads();
    if (cnt[threadIdx.x]) base[threadIdx.x] = atomicAdd(&A.bucket[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) A.order[base[b] + rank] = int32_t(t);
    __syncthreads();
  }
}

// outputs of the tracks that head no fitted chain
__global__ void __launch_bounds__(TPB) k_ch_clear(ChArgs A) {
  if (*A.status != TPC_OK) return;
  const int64_t T = ch_tracks(A);
  for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x; t < T; t += int64_t(gridDim.x) * TPB) {
    if (A.n_chain[t] > 0) continue;
    A.ok[t] = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) A.par[t * 5 + q] = 0.f;
#pragma unroll
    for (int q = 0; q < 15; ++q) A.cov[t * 15 + q] = 0.f;
    A.xref[t] = 0.f;
    A.chi2[t] = 0.f;
  }
}

// A position in a chain: hit j of segment q (records R, nq hits, unit u).
// Segments have at least one hit (k_ch_len), and the steps below are taken
// only towards a hit of the chain, so every link they follow is checked.
struct Cursor {
  int32_t q;
  int j, nq, u;
  const uint64_t *R;
};
__device__ __forceinline__ void seg_at(const ChArgs &A, Cursor &c, int32_t q, int j) {
  c.q = q;
  c.nq = A.n_hits[q];
  c.u = A.unit[q];
  c.R = A.rec + A.first_hit[q];
  c.j = j;
}
__device__ __forceinline__ void step_fwd(const ChArgs &A, Cursor &c) {
  if (++c.j >= c.nq) seg_at(A, c, A.next[c.q], 0);
}
__device__ __forceinline__ void step_bwd(const ChArgs &A, Cursor &c) {
  if (--c.j < 0) {
    seg_at(A, c, A.prev[c.q], 0);
    c.j = c.nq - 1;
  }
}

// One hit of a chain: into its unit's frame when it changes (re-based on
// the hit), then the transport and the update.  False when the state
// cannot be carried there.
__device__ __forceinline__ bool chain_step(const ChArgs &A, KStateR &s, const Hit h, int u, int &cu, int &Yr,
                                           int Zr, float k, float smx, float sy2, float sz2) {
  const float x = A.row_x[h.row];
  if (u != cu) {
    float ya = s.p[0] + float(Yr) * (1.f / 256.f);
    if (!turn32(s, frame_turn(A, cu, u), ya, k, smx)) return false;
    cu = u;
    Yr = h.Y;
    s.p[0] = ya - float(Yr) * (1.f / 256.f);
  }
  Step st;
  if (!step_prepare(s, x, k, smx, st)) return false;
  step_apply(s, st, x, k);
  upd_hit(s, make_int2(h.Y, h.Z), Yr, Zr, sy2, sz2);
  return true;
}

__global__ void __launch_bounds__(FTB) k_ch_fit(ChArgs A) {
  if (*A.status != TPC_OK) return;
  if (A.bad[0]) {  // a track hit out of range (the gather's flag): every block sees it
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.status = TPC_E_INVALID;
    return;
  }
  const int64_t H = A.bad[1];
  const float k = A.k, smx = A.smx, sy2 = A.sy2, sz2 = A.sz2;
  for (int64_t i0 = int64_t(blockIdx.x) * FTB; i0 < H; i0 += int64_t(gridDim.x) * FTB) {
    const int64_t i = i0 + threadIdx.x;
    if ((i & ~int64_t(63)) >= H) break;  // whole wave past the heads (wave-uniform)
    const bool valid = i < H;            // the other lanes stay for the shuffles below
    KStateR s;
    const int64_t t = valid ? A.order[i] : 0;
    const int n = valid ? A.n_chain[t] : 0;
    bool ok = valid && n >= 3;
    int Yr = 0, Zr = 0, cu = 0;
    if (ok) {  // seed in the first hit's frame
      const CHit h0 = chain_hit(A, int32_t(t), 0), hm = chain_hit_at(A, int32_t(t), n / 2),
                 hl = chain_hit_at(A, int32_t(t), n - 1);
      cu = h0.u;
      Yr = h0.Y;
      Zr = h0.Z;
      const float y0 = float(Yr) * (1.f / 256.f);
      float xs[2], ys[2];
      const CHit hs[2] = {hm, hl};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float d = frame_turn(A, hs[e].u, cu);
        const float cd = cosf(d), sd = sinf(d), yy = float(hs[e].Y) * (1.f / 256.f);
        xs[e] = hs[e].u == cu ? hs[e].x : hs[e].x * cd + yy * sd;
        ys[e] = hs[e].u == cu ? float(hs[e].Y - Yr) * (1.f / 256.f) : (-hs[e].x * sd + yy * cd) - y0;
      }
      ok = seed3(s, h0.x, xs[0], xs[1], ys[0], ys[1], float(hl.Z - Zr) * (1.f / 256.f), k, smx, A.cov0);
    }
    // pass 1: hits 1 .. n-1 in chain order, the next record loaded ahead of the step
    int nmax = ok ? n : 0;
    for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, __shfl_xor(nmax, d));
    Cursor c;
    uint64_t nxt = 0;
    int nu = 0;
    if (ok) {
      kf_update(s, 0.f, 0.f, sy2, sz2);
      seg_at(A, c, int32_t(t), 0);
      step_fwd(A, c);
      nxt = c.R[c.j];
      nu = c.u;
    }
    for (int i = 1; i < nmax; ++i) {
      const uint64_t cur = nxt;
      const int u = nu;
      if (ok && i + 1 < n) {
        step_fwd(A, c);
        nxt = c.R[c.j];
        nu = c.u;
      }
      if (!ok || i >= n) continue;
      if (!chain_step(A, s, unpack(cur), u, cu, Yr, Zr, k, smx, sy2, sz2)) ok = false;
    }
    // pass 2: from the last hit back, covariance reset, turning back at each change of frame
    if (ok) {  // the cursor is on the last hit
      cov_reset(s, A.cov0);
      s.chi2 = 0.f;
      const Hit hl = unpack(nxt);
      upd_hit(s, make_int2(hl.Y, hl.Z), Yr, Zr, sy2, sz2);
      step_bwd(A, c);
      nxt = c.R[c.j];
      nu = c.u;
    }
    for (int i = nmax - 2; i >= 0; --i) {
      const bool mine = ok && i <= n - 2;
      const uint64_t cur = nxt;
      const int u = nu;
      if (mine && i >= 1) {
        step_bwd(A, c);
        nxt = c.R[c.j];
        nu = c.u;
      }
      if (!mine) continue;
      if (!chain_step(A, s, unpack(cur), u, cu, Yr, Zr, k, smx, sy2, sz2)) ok = false;
    }
    if (!valid) continue;
    A.ok[t] = ok ? 1 : 0;
    A.par[t * 5 + 0] = ok ? s.p[0] + float(Yr) * (1.f / 256.f) : 0.f;
    A.par[t * 5 + 1] = ok ? s.p[1] + float(Zr) * (1.f / 256.f) : 0.f;
#pragma unroll
    for (int q = 2; q < 5; ++q) A.par[t * 5 + q] = ok ? s.p[q] : 0.f;
#pragma unroll
    for (int q = 0; q < 15; ++q) A.cov[t * 15 + q] = ok ? s.c[q] : 0.f;
    A.xref[t] = ok ? s.x : 0.f;
    A.chi2[t] = ok ? s.chi2 : 0.f;
  }
}

}  // namespace

extern "C" int tpc_fit_chains(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry, const tpc_field_t *field,
                              const tpc_params_t *params, const tpc_tracks_t *tracks, const tpc_merged_t *merged,
                              const float *unit_alpha, int32_t n_units, tpc_chain_fit_t *out, void *workspace,
                              size_t workspace_bytes, void *stream) {
  if (!clusters || !geometry || !field || !params || !tracks || !merged || !unit_alpha || !out) return TPC_E_INVALID;
  if (clusters->n < 0 || clusters->n >= (int64_t(1) << 30) ||
      (clusters->n > 0 && (!clusters->y || !clusters->z || !clusters->row)))
    return TPC_E_INVALID;
  if (geometry->n_rows < 3 || geometry->n_rows > 255 || !geometry->row_x || n_units < 1) return TPC_E_INVALID;
  if (!tracks->n_hits || !tracks->first_hit || !tracks->hits || !tracks->unit || !tracks->counts ||
      !tracks->status || tracks->cap_tracks < 0 || tracks->cap_hits < 0)
    return TPC_E_INVALID;
  if (!merged->next || !merged->prev || !merged->status) return TPC_E_INVALID;
  if (!isfinite(field->bz_tesla) || !(params->sinphi_max > 0.f) || !(params->sinphi_max < 1.f) ||
      !(params->sigma_y > 0.f) || !(params->sigma_z > 0.f))
    return TPC_E_INVALID;
  for (int q = 0; q < 5; ++q)
    if (!(params->cov0[q] > 0.f) || !isfinite(params->cov0[q])) return TPC_E_INVALID;
  if (!out->params || !out->cov || !out->x_ref || !out->chi2 || !out->n_hits || !out->ok || !out->status)
    return TPC_E_INVALID;
  const size_t need = tpc_refit_workspace_size(clusters->n, tracks->cap_tracks, tracks->cap_hits);
  if (need == 0) return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  if (workspace_bytes < need) return TPC_E_NOMEM;
  // the refit's workspace layout; its pack and gather fill the hit records
  char *w = static_cast<char *>(workspace);
  RfArgs R{};
  R.y = clusters->y;
  R.z = clusters->z;
  R.row = clusters->row;
  R.n_clusters = clusters->n;
  R.row_x = geometry->row_x;
  R.n_rows = geometry->n_rows;
  R.trk_status = tracks->status;
  R.n_hits = tracks->n_hits;
  R.first_hit = tracks->first_hit;
  R.hits = tracks->hits;
  R.trk_counts = tracks->counts;
  R.cap_tracks = tracks->cap_tracks;
  R.cap_hits = tracks->cap_hits;
  R.status = out->status;
  R.bucket = reinterpret_cast<int32_t *>(w);
  R.bad = R.bucket + NB;
  w += align256(NB * 4 + 256);
  R.order = reinterpret_cast<int32_t *>(w);
  w += align256(size_t(tracks->cap_tracks) * 4);
  R.cl = reinterpret_cast<uint64_t *>(w);
  w += align256(size_t(clusters->n) * 8);
  R.rec = reinterpret_cast<uint64_t *>(w);
  ChArgs A;
  A.y = clusters->y;
  A.z = clusters->z;
  A.row = clusters->row;
  A.n_clusters = clusters->n;
  A.row_x = geometry->row_x;
  A.n_rows = geometry->n_rows;
  A.trk_status = tracks->status;
  A.n_hits = tracks->n_hits;
  A.first_hit = tracks->first_hit;
  A.hits = tracks->hits;
  A.unit = tracks->unit;
  A.trk_counts = tracks->counts;
  A.cap_tracks = tracks->cap_tracks;
  A.cap_hits = tracks->cap_hits;
  A.next = merged->next;
  A.prev = merged->prev;
  A.mg_status = merged->status;
  A.alpha = unit_alpha;
  A.n_units = n_units;
  A.k = -KAPPA * field->bz_tesla;
  A.smx = params->sinphi_max;
  A.sy2 = params->sigma_y * params->sigma_y;
  A.sz2 = params->sigma_z * params->sigma_z;
  for (int q = 0; q < 5; ++q) A.cov0[q] = params->cov0[q];
  A.par = out->params;
  A.cov = out->cov;
  A.xref = out->x_ref;
  A.chi2 = out->chi2;
  A.n_chain = out->n_hits;
  A.ok = out->ok;
  A.status = out->status;
  A.rec = R.rec;
  A.order = R.order;
  A.bucket = R.bucket;
  A.bad = R.bad;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto clamp = [](int64_t b, int64_t hi) { return unsigned(b < 1 ? 1 : (b > hi ? hi : b)); };
  const int64_t tb = (tracks->cap_tracks + TPB - 1) / TPB;
  const int64_t hb = (tracks->cap_hits + TPB - 1) / TPB;
  const int64_t cb = (clusters->n + TPB - 1) / TPB;
  const int64_t fb = (tracks->cap_tracks + FTB - 1) / FTB;
  hipLaunchKernelGGL(k_ch_init, dim3(1), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_pack, dim3(clamp(cb, GATHER_BLOCKS)), dim3(TPB), 0, st, R);
  hipLaunchKernelGGL(k_rf_gather, dim3(clamp(hb, GATHER_BLOCKS)), dim3(TPB), 0, st, R);
  hipLaunchKernelGGL(k_ch_len, dim3(clamp(tb, 1024)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_rf_scan, dim3(1), dim3(NB), 0, st, R);
  hipLaunchKernelGGL(k_ch_order, dim3(clamp(tb, 1024)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_ch_clear, dim3(clamp(tb, GATHER_BLOCKS)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_ch_fit, dim3(clamp(fb, FIT_BLOCKS)), dim3(FTB), 0, st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}
