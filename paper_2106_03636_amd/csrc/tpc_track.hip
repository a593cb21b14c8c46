// TPC sector track finding for MI355X (gfx950): kernels and the C ABI.
//
// The method (paper §2.1, §2.3): tracks of all collisions of a continuous-
// readout time frame, found per TPC sector without an a-priori z.  The steps
// and their integer / FP32 arithmetic are described in include/tpc_track.h;
// each kernel below restates the step it implements.
//
// Design for CDNA4: wave64 throughout.  The hit grid is a two-level stable
// counting sort (rows per 2048-hit tile, then bins per (unit,row) segment in
// LDS) using ballot-based peer matching for stable ranks; the neighbour finder
// and the cleaner are one-pass streaming kernels over the sorted hits; start
// hits are compacted with a reduce-then-scan; the Kalman tracklet constructor
// runs one tracklet per lane (the walk along the pad rows is sequential, so
// concurrency comes from tracklets); ownership is an order-independent 32-bit
// atomicMax of (hits << 24 | ~start id), which makes the result independent of
// scheduling.  No kernel allocates; every buffer lives in a caller workspace.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "tpc_track.h"
#include "tpc_kalman.h"

namespace {

using namespace tpc_kf;

constexpr int TPB = 256;          // threads per block of the streaming kernels
constexpr int TILE = 2048;        // hits per tile of the row pass
constexpr int ELEMS = 2048;       // elements per block of the start-flag scan
constexpr int SEGW = 12;          // int32 per (unit,row) record
constexpr int CTB = 128;          // threads per block of the constructor
constexpr int NCH = 256;          // hits per block of the neighbour finder (one per thread)
constexpr float KAPPA = 0.00299792458f;

// (unit,row) record fields
enum { S_START = 0, S_COUNT, S_ZMIN, S_ZMAX, S_H, S_BY, S_NY, S_BZ, S_NZ, S_CBASE, S_CHUNK };
// internal counters
enum { C_K = 0, C_CELLS = 1, C_TRACKS = 2, C_HITS = 3, C_TILES = 4, C_NCHUNK = 5, C_SEEDS = 6, C_NWIDE = 7,
       C_TICKET = 8, C_N = 9 };

struct Workspace {
  int64_t *ctr;
  int32_t *seg, *seg_cnt, *seg_zmin, *seg_zmax, *seg_nbins;
  float2 *seg_inv;  // per (unit,row): 1/by, 1/bz
  int32_t *unit_tiles, *tile_hist;
  int32_t *rs_idx;
  int2 *rs_yz;
  int32_t *perm;
  int2 *syz;
  int32_t *up, *dn, *upc, *dnc;
  uint8_t *flag;
  uint32_t *owner;
  int32_t *cell, *cursor;
  int32_t *chunk_seg, *wide;  // neighbour-finder chunk -> (unit,row); chunks too wide for LDS
  int32_t *blk, *blk_keep;
  uint64_t *lookback;  // per seed block: decoupled look-back word of the selector
  // per tracklet (chain start), capacity T_cap = n/2 + 64: a start hit has an
  // upward partner that starts nothing, so there are at most n/2
  int32_t *trk_start, *trk_unit, *trk_len;
  int32_t *tmp_r1, *tmp_hm, *tmp_hb;  // per tracklet, k_chains -> k_compact_seeds (aliases the hit table)
  // per seed (tracklet with a chain of >= l_min hits), capacity S_cap
  int32_t *seed_list, *sd_r1, *sd_hm, *sd_hb, *sd_nfit, *sd_rlo, *sd_rhi, *sd_owned, *sd_keep, *sd_p1n;
  uint32_t *sd_key;
  float *sd_par, *sd_cov, *sd_x, *sd_chi2;
  int32_t *trk_hits;  // seed hit table [S_cap / 64][n_rows][64]
  int64_t N, S, T_max, C_max, T_cap, S_cap, NB, KB, SB, KW, CH_max;
  size_t total;
};

struct Args {
  Workspace w;
  const int64_t *off;
  const float *y, *z;
  const uint16_t *row;
  const float *row_x;
  int64_t n;
  int32_t n_units, n_rows;
  float kcurv;  // -KAPPA * Bz: curvature per unit q/pT
  tpc_params_t p;
  tpc_tracks_t out;
};

// ---------------------------------------------------------------------------
// workspace layout (host and device agree through this one function)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool layout(int64_t n, int32_t n_units, int32_t n_rows, const tpc_params_t *p, char *base,
            Workspace *w) {
  if (n < 0 || n >= (int64_t(1) << 30) || n_units < 1 || n_rows < 3 || n_rows > 255 || !p ||
      p->bin_occ < 1 || p->tracklet_cap_div < 2)
    return false;
  Workspace L{};
  L.N = n;
  L.S = int64_t(n_units) * n_rows;
  L.T_max = n / TILE + n_units + 1;
  L.C_max = n / p->bin_occ + 65 * L.S + 1;
  L.T_cap = n / 2 + 64;
  L.S_cap = n / p->tracklet_cap_div + 64;
  L.NB = (n + ELEMS - 1) / ELEMS + 1;
  L.KB = (L.T_cap + TPB - 1) / TPB;
  L.SB = (L.S_cap + TPB - 1) / TPB;
  L.KW = (L.S_cap + 63) / 64;
  L.CH_max = n / NCH + L.S;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return base ? base + at : nullptr;
  };
  const size_t N = size_t(n), S = size_t(L.S), T = size_t(L.T_cap), K = size_t(L.S_cap);
  L.ctr = (int64_t *)take(sizeof(int64_t) * C_N);
  L.seg = (int32_t *)take(4 * S * SEGW);
  L.seg_cnt = (int32_t *)take(4 * S);
  L.seg_zmin = (int32_t *)take(4 * S);
  L.seg_zmax = (int32_t *)take(4 * S);
  L.seg_nbins = (int32_t *)take(4 * S);
  L.seg_inv = (float2 *)take(8 * S);
  L.unit_tiles = (int32_t *)take(4 * (size_t(n_units) + 1));
  L.tile_hist = (int32_t *)take(4 * size_t(n_rows) * size_t(L.T_max));
  L.perm = (int32_t *)take(4 * N);
  L.syz = (int2 *)take(8 * N);
  L.up = (int32_t *)take(4 * N);
  L.dn = (int32_t *)take(4 * N);
  L.upc = (int32_t *)take(4 * N);
  L.dnc = (int32_t *)take(4 * N);
  L.flag = (uint8_t *)take(N + 16);
  L.owner = (uint32_t *)take(4 * N);
  L.cell = (int32_t *)take(4 * (size_t(L.C_max) + 1));
  L.chunk_seg = (int32_t *)take(4 * size_t(L.CH_max));
  L.wide = (int32_t *)take(4 * size_t(L.CH_max));
  L.blk = (int32_t *)take(4 * size_t(L.NB));
  L.blk_keep = (int32_t *)take(4 * size_t(L.KB));
  L.lookback = (uint64_t *)take(8 * size_t(L.SB));
  L.trk_start = (int32_t *)take(4 * T);
  L.trk_unit = (int32_t *)take(4 * T);
  L.trk_len = (int32_t *)take(4 * T);
  L.seed_list = (int32_t *)take(4 * K);
  L.sd_r1 = (int32_t *)take(4 * K);
  L.sd_hm = (int32_t *)take(4 * K);
  L.sd_hb = (int32_t *)take(4 * K);
  L.sd_nfit = (int32_t *)take(4 * K);
  L.sd_rlo = (int32_t *)take(4 * K);
  L.sd_rhi = (int32_t *)take(4 * K);
  L.sd_owned = (int32_t *)take(4 * K);
  L.sd_keep = (int32_t *)take(4 * K);
  L.sd_p1n = (int32_t *)take(4 * K);
  L.sd_key = (uint32_t *)take(4 * K);
  L.sd_par = (float *)take(4 * 5 * K);
  L.sd_cov = (float *)take(4 * 15 * K);
  L.sd_x = (float *)take(4 * K);
  L.sd_chi2 = (float *)take(4 * K);
  // The seed hit table is written only by the tracklet constructor.  Before
  // it, the same memory holds arrays that are dead by then: the row-sorted
  // hits and the bin cursors of the grid build, and the per-tracklet seed
  // fields k_chains hands to k_compact_seeds.
  const size_t table = 4 * size_t(n_rows) * 64 * size_t(L.KW);
  const size_t grid_tmp = align256(4 * N) + align256(8 * N) + align256(4 * size_t(L.C_max));
  const size_t chain_tmp = 3 * align256(4 * T);
  const size_t region = table > grid_tmp ? (table > chain_tmp ? table : chain_tmp)
                                         : (grid_tmp > chain_tmp ? grid_tmp : chain_tmp);
  char *r = (char *)take(region);
  L.trk_hits = (int32_t *)r;
  L.rs_idx = (int32_t *)r;
  L.rs_yz = (int2 *)(r ? r + align256(4 * N) : nullptr);
  L.cursor = (int32_t *)(r ? r + align256(4 * N) + align256(8 * N) : nullptr);
  L.tmp_r1 = (int32_t *)r;
  L.tmp_hm = (int32_t *)(r ? r + align256(4 * T) : nullptr);
  L.tmp_hb = (int32_t *)(r ? r + 2 * align256(4 * T) : nullptr);
  L.total = o;
  *w = L;
  return true;
}

bool params_ok(const tpc_params_t *p) {
  return p && p->version == TPC_PARAMS_VERSION && p->q_shift == 8 && p->tan_half_q16 > 0 &&
         p->tan_half_q16 < (1 << 20) && p->bin_y_q > 0 && p->bin_occ > 0 && p->bin_zmin_q > 0 &&
         p->win_y_q >= 0 && p->win_y_q < (1 << 16) && p->win_z_q >= 0 && p->win_z_q < (1 << 16) &&
         p->w_y >= 0 && p->w_y <= 15 && p->w_z >= 0 && p->w_z <= 15 && p->smax_k >= 0 &&
         p->smax_k < (int64_t(1) << 30) && p->l_min >= 3 && p->ext_win_y_q >= 0 &&
         p->ext_win_y_q < (1 << 13) && p->ext_win_z_q >= 0 && p->ext_win_z_q < (1 << 13) &&
         p->ext_edge_q >= 0 && p->ext_edge_q < (1 << 20) && p->max_miss >= 0 && p->n_min >= 0 &&
         p->f_min_q8 >= 0 && p->f_min_q8 <= 256 * 256 && p->tracklet_cap_div >= 2 &&
         p->sinphi_max > 0.f && p->sinphi_max < 1.f && p->sigma_y > 0.f && p->sigma_z > 0.f &&
         p->cov0[0] > 0.f && p->cov0[1] > 0.f && p->cov0[2] > 0.f && p->cov0[3] > 0.f &&
         p->cov0[4] > 0.f;
}

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) {
  atomicCAS(st, 0, code);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << __lane_id()) - 1;
}

// Exclusive scan over the block (NT threads, NT/64 waves).  tmp: NT/64 ints of LDS.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int *tmp, int *total) {
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const int t = tmp[i];
    before += (i < wid) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

// Lanes of the wave holding the same key (bits of the key below 2^nbits).
__device__ __forceinline__ uint64_t peer_mask(uint32_t key, int nbits, bool active) {
  uint64_t m = __ballot(active);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (key >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ int quant(float v) { return __float2int_rn(v * 256.0f); }


__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// unit of tile b (largest u with unit_tiles[u] <= b)
__device__ __forceinline__ int unit_of_tile(const int32_t *ut, int n_units, int b) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ut[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// step 1: clear what must start at zero, validate geometry and offsets

// Blocks are dealt to the 8 XCDs in turn.  Renumber the first n_work
// (rounded up to 8) blocks so that each XCD runs one contiguous range of work
// chunks: neighbouring chunks read the same rows, which then stay in that
// XCD's L2.  Blocks past them keep their number.  A bijection on [0, grid)
// when the grid is a multiple of 8.
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t n_work) {
  const int64_t n8 = (n_work + 7) & ~int64_t(7);
  if (b >= n8) return b;
  return (b & 7) * (n8 >> 3) + (b >> 3);
}

// Minimum and maximum over the 64 lanes (all lanes active).  The result is
// moved to a scalar register, so loops bounded by it are uniform: their
// counter, exit test and row-indexed loads stay scalar.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

constexpr int RB = 32;  // rows of the hit table read per round trip in the row loops
constexpr int OWNED = 1 << 30;  // hit table entries (< 2^30) of hits their tracklet owns, once selected

// Hit table of the seeds: [seed / 64][row][seed % 64], so the 64 lanes of a
// wave (64 consecutive seeds) at one row touch one contiguous 256-byte run.
// Returns the column of seed i; its row r is at col[r * 64].
__device__ __forceinline__ int32_t *seed_column(const Workspace &w, int64_t i, int nr) {
  return w.trk_hits + ((i >> 6) * nr) * 64 + (i & 63);
}

__global__ void k_init(Args A) {
  const Workspace &w = A.w;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < w.S) {
    w.seg_cnt[i] = 0;
    w.seg_zmin[i] = INT32_MAX;
    w.seg_zmax[i] = INT32_MIN;
  }
  if (i < A.n) {
    w.owner[i] = 0u;
    A.out.cluster_track[i] = -1;
  }
  if (i < C_N) w.ctr[i] = 0;
  if (i < w.SB) w.lookback[i] = 0;
  if (i < w.KB) w.blk_keep[i] = 0;
  if (i < 5) A.out.counts[i] = 0;
  if (i == 0) *A.out.status = TPC_OK;
}

__global__ void __launch_bounds__(1024) k_units(Args A) {
  __shared__ int tmp[16];
  const Workspace &w = A.w;
  bool bad = false;
  for (int r = threadIdx.x; r < A.n_rows; r += blockDim.x) {
    const float x = A.row_x[r];
    if (!(x >= 1.f && x < 8192.f)) bad = true;  // 1 cm .. 8192 cm: X is at least 256 quanta
    if (r > 0 && !(x > A.row_x[r - 1])) bad = true;
    // rows two apart at most 32 cm apart: keeps the neighbour cut below 2^56
    if (r > 0 && r + 1 < A.n_rows && x >= 1.f && x < 8192.f &&
        __float2ll_rn(A.row_x[r + 1] * 256.f) - __float2ll_rn(A.row_x[r - 1] * 256.f) >= 8192)
      bad = true;
  }
  if (threadIdx.x == 0 && (A.off[0] != 0 || A.off[A.n_units] != A.n)) bad = true;
  int carry = 0;
  for (int base = 0; base < A.n_units; base += blockDim.x) {
    const int u = base + threadIdx.x;
    int tiles = 0;
    if (u < A.n_units) {
      const int64_t a = A.off[u], b = A.off[u + 1];
      if (b < a || b - a >= (int64_t(1) << 24) || a < 0 || b > A.n) bad = true;
      else tiles = int((b - a + TILE - 1) / TILE);
    }
    int tot;
    const int ex = block_exclusive_scan<1024>(tiles, tmp, &tot);
    if (u < A.n_units) w.unit_tiles[u] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    w.unit_tiles[A.n_units] = carry;
    w.ctr[C_TILES] = carry;
  }
  if (bad) set_status(A.out.status, TPC_E_INVALID);
}

// ---------------------------------------------------------------------------
// step 2a: per tile, row histogram and z extent (also validates the clusters)

__global__ void __launch_bounds__(TPB) k_tile_hist(Args A) {
  __shared__ int cnt[256], zmn[256], zmx[256];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int b = blockIdx.x;
  if (b >= w.ctr[C_TILES]) return;
  const int u = unit_of_tile(w.unit_tiles, A.n_units, b);
  const int64_t beg = A.off[u] + int64_t(b - w.unit_tiles[u]) * TILE;
  const int64_t end = min(beg + TILE, A.off[u + 1]);
  for (int r = threadIdx.x; r < 256; r += TPB) {
    cnt[r] = 0;
    zmn[r] = INT32_MAX;
    zmx[r] = INT32_MIN;
  }
  __syncthreads();
  bool bad = false;
  for (int64_t i = beg + threadIdx.x; i < end; i += TPB) {
    const int r = A.row[i];
    const float yf = A.y[i], zf = A.z[i];
    if (r >= A.n_rows || !(fabsf(yf) <= 8192.f) || !(fabsf(zf) <= 8192.f)) {
      bad = true;
      continue;
    }
    const int Z = quant(zf);
    atomicAdd(&cnt[r], 1);
    atomicMin(&zmn[r], Z);
    atomicMax(&zmx[r], Z);
  }
  if (bad) set_status(A.out.status, TPC_E_INVALID);
  __syncthreads();
  for (int r = threadIdx.x; r < A.n_rows; r += TPB) {
    const int c = cnt[r];
    w.tile_hist[int64_t(r) * w.T_max + b] = c;
    if (c) {
      const int64_t s = int64_t(u) * A.n_rows + r;
      atomicAdd(&w.seg_cnt[s], c);
      atomicMin(&w.seg_zmin[s], zmn[r]);
      atomicMax(&w.seg_zmax[s], zmx[r]);
    }
  }
}

// step 2b: per unit, row starts and the grid shape of every (unit,row).
// y: [-H, H] in bins of by (at most 63); z: data-driven [zmin, zmax] (no
// a-priori z in continuous readout, paper §2.3), cut into as many bins as
// give about bin_occ hits per bin, none shorter than bin_zmin.
__global__ void __launch_bounds__(256) k_seg_plan(Args A) {
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int u = blockIdx.x, r = threadIdx.x;
  const int64_t s = int64_t(u) * A.n_rows + r;
  const int cnt = r < A.n_rows ? w.seg_cnt[s] : 0;
  int tot;
  const int pre = block_exclusive_scan<256>(cnt, tmp, &tot);
  if (r >= A.n_rows) return;
  const tpc_params_t &P = A.p;
  const int64_t X = __float2ll_rn(A.row_x[r] * 256.0f);
  const int64_t H = (X * P.tan_half_q16) >> 16;
  int64_t by = P.bin_y_q;
  if (by < 2 * H / 63 + 1) by = 2 * H / 63 + 1;
  const int64_t ny = 2 * H / by + 1;
  const int64_t zmin = cnt ? w.seg_zmin[s] : 0, zmax = cnt ? w.seg_zmax[s] : 0;
  const int64_t span = zmax - zmin;
  const int64_t per = int64_t(P.bin_occ) * ny;
  int64_t nz_occ = (cnt + per - 1) / per;
  if (nz_occ < 1) nz_occ = 1;
  const int64_t nz_span = span / P.bin_zmin_q + 1;
  int64_t nz = nz_occ < nz_span ? nz_occ : nz_span;
  if (nz < 1) nz = 1;
  const int64_t bz = span / nz + 1;
  int32_t *rec = w.seg + s * SEGW;
  rec[S_START] = int32_t(A.off[u] + pre);
  rec[S_COUNT] = cnt;
  rec[S_ZMIN] = int32_t(zmin);
  rec[S_ZMAX] = int32_t(zmax);
  rec[S_H] = int32_t(H);
  rec[S_BY] = int32_t(by);
  rec[S_NY] = int32_t(ny);
  rec[S_BZ] = int32_t(bz);
  rec[S_NZ] = int32_t(nz);
  rec[10] = 0;
  rec[11] = 0;
  w.seg_nbins[s] = int32_t(ny * nz);
  w.seg_inv[s] = make_float2(1.f / float(by), 1.f / float(bz));
}

// step 2c: first cell of every (unit,row), and the end sentinel
__global__ void __launch_bounds__(1024) k_cell_base(Args A) {
  __shared__ int tmp[16];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  int carry = 0, ccarry = 0;
  for (int64_t base = 0; base < w.S; base += 1024) {
    const int64_t s = base + threadIdx.x;
    const int v = s < w.S ? w.seg_nbins[s] : 0;
    const int nch = s < w.S ? (w.seg[s * SEGW + S_COUNT] + NCH - 1) / NCH : 0;
    int tot, ctot;
    const int ex = block_exclusive_scan<1024>(v, tmp, &tot);
    const int cex = block_exclusive_scan<1024>(nch, tmp, &ctot);
    if (s < w.S) {
      w.seg[s * SEGW + S_CBASE] = carry + ex;
      w.seg[s * SEGW + S_CHUNK] = ccarry + cex;
    }
    carry += tot;
    ccarry += ctot;
  }
  if (threadIdx.x == 0) {
    w.ctr[C_CELLS] = carry;
    w.ctr[C_NCHUNK] = ccarry;
    A.out.counts[3] = carry;
    w.cell[carry] = int32_t(A.n);
  }
}

// step 2d: output position of each tile's first hit of each row; the
// (unit,row) of every neighbour-finder chunk
__global__ void __launch_bounds__(64) k_tile_offsets(Args A) {
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t s = blockIdx.x;
  const int u = int(s / A.n_rows), r = int(s % A.n_rows);
  const int t0 = w.unit_tiles[u], t1 = w.unit_tiles[u + 1];
  int carry = w.seg[s * SEGW + S_START];
  int32_t *h = w.tile_hist + int64_t(r) * w.T_max;
  const int lane = __lane_id();
  // neighbour-finder chunks of this (unit,row) point back to it
  const int c0 = w.seg[s * SEGW + S_CHUNK], nch = (w.seg[s * SEGW + S_COUNT] + NCH - 1) / NCH;
  for (int j = lane; j < nch; j += 64) w.chunk_seg[c0 + j] = int32_t(s);
  for (int t = t0; t < t1; t += 64) {
    const int i = t + lane;
    const int v = i < t1 ? h[i] : 0;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (i < t1) h[i] = carry + x - v;
    carry += __shfl(x, 63);
  }
}

// step 2e: stable scatter of every tile's hits to row order.  Each wave owns a
// contiguous quarter of the tile, holds its rows in registers, and ranks equal
// rows with ballots, so hits of one row keep the order of their ids.  The
// tile is first put in row order in LDS, so that each row's run of hits is
// written to HBM as one contiguous piece.
__global__ void __launch_bounds__(TPB) k_tile_scatter(Args A) {
  constexpr int CH = TILE / 4 / 64;  // 64-hit chunks per wave
  __shared__ int wcnt[4][256];
  __shared__ int tbase[256], tloc[256];  // per row: first output position, first staged slot
  __shared__ int2 s_yz[TILE];
  __shared__ int s_id[TILE];
  __shared__ uint8_t s_row[TILE];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int b = blockIdx.x;
  if (b >= w.ctr[C_TILES]) return;
  const int u = unit_of_tile(w.unit_tiles, A.n_units, b);
  const int64_t beg = A.off[u] + int64_t(b - w.unit_tiles[u]) * TILE;
  const int64_t end = min(beg + TILE, A.off[u + 1]);
  const int wid = threadIdx.x >> 6, lane = __lane_id();
  const int64_t sub_beg = beg + int64_t(wid) * (TILE / 4);
  const int64_t sub_end = min(sub_beg + TILE / 4, end);
  int rr[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t i = sub_beg + c * 64 + lane;
    rr[c] = i < sub_end ? int(A.row[i]) : -1;
  }
  for (int r = threadIdx.x; r < 4 * 256; r += TPB) (&wcnt[0][0])[r] = 0;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (rr[c] >= 0) atomicAdd(&wcnt[wid][rr[c]], 1);
  __syncthreads();
  if (threadIdx.x < 64) {  // staged slots: rows in order (exclusive scan of the tile's row counts)
    int run = 0;
    for (int r0 = 0; r0 < 256; r0 += 64) {
      const int r = r0 + lane;
      const int v = r < A.n_rows ? wcnt[0][r] + wcnt[1][r] + wcnt[2][r] + wcnt[3][r] : 0;
      int x = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
      }
      tloc[r] = run + x - v;
      run += __shfl(x, 63);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < A.n_rows; r += TPB) {
    int base = w.tile_hist[int64_t(r) * w.T_max + b];
    tbase[r] = base;
    int loc = tloc[r];
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // per wave: first staged slot of its hits of the row
      const int t = wcnt[k][r];
      wcnt[k][r] = loc;
      loc += t;
    }
  }
  __syncthreads();
  int pos[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const bool act = rr[c] >= 0;
    const int r = act ? rr[c] : 0;
    const uint64_t peers = peer_mask(uint32_t(r), 8, act);
    pos[c] = act ? wcnt[wid][r] + __popcll(peers & lanemask_lt()) : 0;
    __builtin_amdgcn_wave_barrier();
    if (act && (63 - __clzll(peers)) == lane) wcnt[wid][r] += __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (rr[c] >= 0) {
      const int64_t i = sub_beg + c * 64 + lane;
      s_id[pos[c]] = int32_t(i);
      s_yz[pos[c]] = make_int2(quant(A.y[i]), quant(A.z[i]));
      s_row[pos[c]] = uint8_t(rr[c]);
    }
  }
  __syncthreads();
  const int n_tile = int(end - beg);
  for (int j = threadIdx.x; j < n_tile; j += TPB) {  // each row's run to consecutive positions
    const int r = s_row[j];
    const int gp = tbase[r] + (j - tloc[r]);
    w.rs_idx[gp] = s_id[j];
    w.rs_yz[gp] = s_yz[j];
  }
}

__device__ __forceinline__ int bin_of(const int32_t *rec, int Y, int Z) {
  const int H = rec[S_H];
  const int iy = clampi(Y + H, 0, 2 * H) / rec[S_BY];
  const int iz = (Z - rec[S_ZMIN]) / rec[S_BZ];
  return iz * rec[S_NY] + iy;
}

// step 2f: per (unit,row), counting sort by bin, stable (hits arrive in id
// order and one wave ranks them chunk by chunk with ballots), and the cell
// table.  Fast path: bins and per-hit ranks in LDS, data moved by all threads
// afterwards; rows too large for LDS take the same steps with global cursors.
constexpr int BIN_POOL = 12288;  // LDS ints shared by the bin counters and the per-hit slots
constexpr int KREG = 24;         // hits per thread kept in registers by the bin sort (rows <= 6144)

__device__ __forceinline__ void scan_bins(int *hist, int nbins, int32_t *cell_out, int start, int *tmp) {
  const int per = (nbins + TPB - 1) / TPB;
  const int b0 = min(nbins, int(threadIdx.x) * per), b1 = min(nbins, b0 + per);
  int run = 0;
  for (int b = b0; b < b1; ++b) run += hist[b];
  int tot;
  int pre = block_exclusive_scan<TPB>(run, tmp, &tot);
  for (int b = b0; b < b1; ++b) {
    const int v = hist[b];
    hist[b] = pre;
    cell_out[b] = start + pre;
    pre += v;
  }
}

__global__ void __launch_bounds__(TPB) k_bin_sort(Args A) {
  __shared__ int pool[BIN_POOL];
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t s = blockIdx.x;
  const int32_t *rec = w.seg + s * SEGW;
  const int start = rec[S_START], count = rec[S_COUNT], cbase = rec[S_CBASE];
  const int nbins = rec[S_NY] * rec[S_NZ];
  int nbits = 1;
  while ((1 << nbits) < nbins) ++nbits;
  const int lane = __lane_id();
  if (nbins + count <= BIN_POOL) {
    int *hist_lds = pool, *slot = pool + nbins;
    for (int b = threadIdx.x; b < nbins; b += TPB) hist_lds[b] = 0;
    // the thread's first KREG hits stay in registers from here to the scatter
    int2 ryz[KREG];
    int rid[KREG];
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      const int p = int(threadIdx.x) + k * TPB;
      if (p < count) {
        ryz[k] = w.rs_yz[start + p];
        rid[k] = w.rs_idx[start + p];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      const int p = int(threadIdx.x) + k * TPB;
      if (p < count) {
        const int bn = bin_of(rec, ryz[k].x, ryz[k].y);
        slot[p] = bn;
        atomicAdd(&hist_lds[bn], 1);
      }
    }
    for (int p = int(threadIdx.x) + KREG * TPB; p < count; p += TPB) {
      const int2 yz = w.rs_yz[start + p];
      const int bn = bin_of(rec, yz.x, yz.y);
      slot[p] = bn;
      atomicAdd(&hist_lds[bn], 1);
    }
    __syncthreads();
    scan_bins(hist_lds, nbins, w.cell + cbase, start, tmp);
    __syncthreads();
    if (threadIdx.x < 64) {  // stable ranks, one wave, chunk by chunk; the next chunk's bins load early
      int nb = lane < count ? slot[lane] : 0;
      for (int c = 0; c < count; c += 64) {
        const int p = c + lane;
        const bool act = p < count;
        const int bn = nb;
        nb = p + 64 < count ? slot[p + 64] : 0;
        const uint64_t peers = peer_mask(uint32_t(bn), nbits, act);
        const int lp = act ? hist_lds[bn] + __popcll(peers & lanemask_lt()) : 0;
        __builtin_amdgcn_wave_barrier();
        if (act && (63 - __clzll(peers)) == lane) hist_lds[bn] += __popcll(peers);
        if (act) slot[p] = lp;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      const int p = int(threadIdx.x) + k * TPB;
      if (p < count) {
        const int lp = slot[p];
        w.perm[start + lp] = rid[k];
        w.syz[start + lp] = ryz[k];
      }
    }
    for (int p = int(threadIdx.x) + KREG * TPB; p < count; p += TPB) {
      const int lp = slot[p];
      w.perm[start + lp] = w.rs_idx[start + p];
      w.syz[start + lp] = w.rs_yz[start + p];
    }
    return;
  }
  // large rows: cursors in the workspace
  int *hist = w.cursor + cbase;
  for (int b = threadIdx.x; b < nbins; b += TPB) hist[b] = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < count; p += TPB) {
    const int2 yz = w.rs_yz[start + p];
    atomicAdd(&hist[bin_of(rec, yz.x, yz.y)], 1);
  }
  __syncthreads();
  scan_bins(hist, nbins, w.cell + cbase, start, tmp);
  __syncthreads();
  if (threadIdx.x >= 64) return;
  for (int c = 0; c < count; c += 64) {
    const int p = c + lane;
    const bool act = p < count;
    int2 yz = make_int2(0, 0);
    int idx = 0, bn = 0;
    if (act) {
      yz = w.rs_yz[start + p];
      idx = w.rs_idx[start + p];
      bn = bin_of(rec, yz.x, yz.y);
    }
    const uint64_t peers = peer_mask(uint32_t(bn), nbits, act);
    int pos = 0;
    if (act) pos = start + hist[bn] + __popcll(peers & lanemask_lt());
    __builtin_amdgcn_wave_barrier();
    if (act && (63 - __clzll(peers)) == lane) hist[bn] += __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    if (act) {
      w.perm[pos] = idx;
      w.syz[pos] = yz;
    }
  }
}

// ---------------------------------------------------------------------------
// step 3: neighbour finder.  For hit m of row i (0 < i < n_rows-1): candidates
// n of rows j = i-1, i+1 with |Y_n X_i - Y_m X_j| <= win_y X_i (origin-pointing
// in the bending plane) and |Z_n - Z_m| <= win_z (no vertex pointing in z).  Of
// all pairs (d below, u above), the least (score, id_d, id_u) with
// score = w_y R_y^2 + w_z R_z^2, R = (V_d - V_m)(X_u - X_i) + (V_u - V_m)(X_i - X_d),
// is kept when score <= smax_k (X_{i+1} - X_{i-1})^2.

// a / b for 0 <= a < 2^24 and 0 < b < 2^24: a float quotient is within one
// of the result, then corrected with integer products.
__device__ __forceinline__ int div_small(int a, int b, float inv_b) {
  int q = int(float(a) * inv_b);
  if (q * b > a) --q;
  else if ((q + 1) * b <= a) ++q;
  return q;
}

struct Win {
  int iy0, iy1, iz0, iz1, ny, cbase;
  bool empty;
};

// The fields of a (unit,row) record that the window search reads.
struct Rec {
  int count, zmin, zmax, H, by, ny, bz, cbase;
};

// loaded with three 16-byte loads (records are 48 bytes, 16-byte aligned)
__device__ __forceinline__ Rec rec_fields_v(const int32_t *rec) {
  const int4 a = reinterpret_cast<const int4 *>(rec)[0], b = reinterpret_cast<const int4 *>(rec)[1],
             c = reinterpret_cast<const int4 *>(rec)[2];
  static_assert(S_COUNT == 1 && S_ZMIN == 2 && S_ZMAX == 3 && S_H == 4 && S_BY == 5 && S_NY == 6 && S_BZ == 7 &&
                    S_CBASE == 9 && SEGW == 12,
                "record layout");
  Rec f;
  f.count = a.y;
  f.zmin = a.z;
  f.zmax = a.w;
  f.H = b.x;
  f.by = b.y;
  f.ny = b.z;
  f.bz = b.w;
  f.cbase = c.y;
  return f;
}

// Window bounds are within +-2^30 and coordinates within +-2^21 (every
// cluster is checked), so the sums below stay exact in int32.
__device__ __forceinline__ Win window_cells(const int32_t *rec, float2 inv, int ylo, int yhi, int zlo, int zhi) {
  Win c;
  const int count = rec[S_COUNT];
  const int zmin = rec[S_ZMIN], zmax = rec[S_ZMAX];
  c.empty = count == 0 || zhi < zmin || zlo > zmax || yhi < ylo;
  if (c.empty) return c;
  const int H = rec[S_H], span = zmax - zmin;
  const int by = rec[S_BY], bz = rec[S_BZ];
  c.iy0 = div_small(clampi(ylo + H, 0, 2 * H), by, inv.x);
  c.iy1 = div_small(clampi(yhi + H, 0, 2 * H), by, inv.x);
  c.iz0 = div_small(clampi(zlo - zmin, 0, span), bz, inv.y);
  c.iz1 = div_small(clampi(zhi - zmin, 0, span), bz, inv.y);
  c.ny = rec[S_NY];
  c.cbase = rec[S_CBASE];
  return c;
}

// The same window from a record already in registers.
__device__ __forceinline__ Win window_cells(const Rec &r, float2 inv, int ylo, int yhi, int zlo, int zhi) {
  Win c;
  const int count = r.count;
  const int zmin = r.zmin, zmax = r.zmax;
  c.empty = count == 0 || zhi < zmin || zlo > zmax || yhi < ylo;
  if (c.empty) return c;
  const int H = r.H, span = zmax - zmin;
  const int by = r.by, bz = r.bz;
  c.iy0 = div_small(clampi(ylo + H, 0, 2 * H), by, inv.x);
  c.iy1 = div_small(clampi(yhi + H, 0, 2 * H), by, inv.x);
  c.iz0 = div_small(clampi(zlo - zmin, 0, span), bz, inv.y);
  c.iz1 = div_small(clampi(zhi - zmin, 0, span), bz, inv.y);
  c.ny = r.ny;
  c.cbase = r.cbase;
  return c;
}

// A z-slab of a neighbour row staged in LDS: hits at positions [q0, q0 + nq)
// (int2, first) and the cell table entries [c0, c0 + nc] (after them), in one
// pool of STAGE_INTS ints per row.
constexpr int STAGE_INTS = 2560;
constexpr int STAGE_KH = 5;   // hit loads per thread (nq <= 1280)
constexpr int STAGE_KC = 10;  // cell loads per thread (nc < 2560)

struct Slab {
  int q0, nq, c0, nc;
  bool lds;  // false: read the workspace directly
};

template <bool LDS>
__device__ __forceinline__ int cell_at(const Workspace &w, const Slab &sl, const int *lc, int c) {
  return LDS ? lc[2 * sl.nq + c - sl.c0] : w.cell[c];
}
template <bool LDS>
__device__ __forceinline__ int2 hit_at(const Workspace &w, const Slab &sl, const int2 *lh, int q) {
  return LDS ? lh[q - sl.q0] : w.syz[q];
}

// Candidate rows: the exact y interval of the window in row j and its cells.
struct Cand {
  int ylo, yhi;  // Y_n in [ylo, yhi]  <=>  |Y_n X_i - Y_m X_j| <= W X_i
  Win c;
};

// The window is ceil(Y_m X_j / X_i) - W <= Y_n <= floor(Y_m X_j / X_i) + W
// (W is an integer, so it moves out of the floor and the ceiling).
// In FP64, exactly: |Y_m| <= 2^21 and X < 2^22, so every product and sum is
// an integer below 2^53; the quotient from the reciprocal is within one of
// the floor and corrected by exact products.
__device__ __forceinline__ Cand cand_window(const int32_t *rec, float2 inv, int Ym, int Zm, double xi,
                                            double inv_xi, double xj, int WY, int WZ) {
  Cand k;
  const double a = double(Ym) * xj;
  double q = floor(a * inv_xi);
  if (q * xi > a) q -= 1.0;
  else if ((q + 1.0) * xi <= a) q += 1.0;
  const double lo = q + (q * xi != a ? 1.0 : 0.0) - double(WY), hi = q + double(WY);
  // |Y| <= 2^21 for every cluster: clamping keeps the compares exact in int32
  k.ylo = int(fmin(fmax(lo, -1073741824.0), 1073741824.0));
  k.yhi = int(fmin(fmax(hi, -1073741824.0), 1073741824.0));
  k.c = window_cells(rec, inv, k.ylo, k.yhi, Zm - WZ, Zm + WZ);
  return k;
}

constexpr int MAXU = 8;  // row-above candidates kept in registers
constexpr int MAXD = 8;  // row-below candidates kept in registers

// Scores of rows whose S_max is below 2^48 are evaluated in FP64 exactly:
// a residual of 2^24 or more (with a nonzero weight) puts the score at 2^48
// or above, past S_max, and below that every product and sum is an integer
// under 2^53.  Other rows take the int64 path.
constexpr double SMAX_F64 = 281474976710656.0;  // 2^48
constexpr double RES_F64 = 16777216.0;          // 2^24

// Positions of the candidates of one neighbour row that pass the exact
// window, in grid order; at most N are kept (more set `overflow`).
template <bool LDS, int N>
__device__ __forceinline__ int collect(const Workspace &w, const Cand &k, const Slab &sl, const int *lc,
                                       const int2 *lh, int zlo, int zhi, int (&q)[N], bool &overflow) {
  int n = 0;
  for (int iz = k.c.iz0; iz <= k.c.iz1; ++iz) {
    const int cb = k.c.cbase + iz * k.c.ny;
    const int v0 = cell_at<LDS>(w, sl, lc, cb + k.c.iy0), v1 = cell_at<LDS>(w, sl, lc, cb + k.c.iy1 + 1);
    for (int p = v0; p < v1; ++p) {
      const int2 hp = hit_at<LDS>(w, sl, lh, p);
      if (hp.x < k.ylo || hp.x > k.yhi || hp.y < zlo || hp.y > zhi) continue;
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j == n) q[j] = p;
      if (n < N) ++n;
      else overflow = true;
    }
  }
  return n;
}

// Best (d, u) pair of hit m; see the step description above.  F64: scores in
// FP64 (S_max < 2^48), else in int64.  Both windows' candidates are gathered
// first (a few per side), then every pair is scored; a hit with more
// candidates than the registers hold scans the windows again pair by pair.
template <bool LDS, bool F64>
__device__ __forceinline__ void best_pair(const Args &A, int m, const int32_t *recd, const int32_t *recu,
                                          float2 invd, float2 invu,
                                          const Slab &sd, const Slab &su, const int *lcd, const int *lcu,
                                          const int2 *lhd, const int2 *lhu, int64_t Xi, double inv_xi,
                                          int64_t Xd, int64_t Xu, int64_t smax, int &best_d, int &best_u) {
  const Workspace &w = A.w;
  const int64_t WY = A.p.win_y_q, WZ = A.p.win_z_q, wy = A.p.w_y, wz = A.p.w_z;
  const int dxd = int(Xi - Xd), dxu = int(Xu - Xi);
  const int2 hm = w.syz[m];
  const int Ym = hm.x, Zm = hm.y;
  const Cand kd = cand_window(recd, invd, Ym, Zm, double(Xi), inv_xi, double(Xd), int(WY), int(WZ));
  const Cand ku = cand_window(recu, invu, Ym, Zm, double(Xi), inv_xi, double(Xu), int(WY), int(WZ));
  best_d = -1;
  best_u = -1;
  if (kd.c.empty || ku.c.empty) return;
  const int zlo = Zm - int(WZ), zhi = Zm + int(WZ);
  int uq[MAXU], dq[MAXD];
  bool overflow = false;
  const int nu = collect<LDS, MAXU>(w, ku, su, lcu, lhu, zlo, zhi, uq, overflow);
  if (nu == 0) return;
  const int nd = collect<LDS, MAXD>(w, kd, sd, lcd, lhd, zlo, zhi, dq, overflow);
  if (nd == 0) return;
  int64_t best_s = INT64_MAX;
  double best_f = 1e300;
  const double dxu_f = double(dxu), dxd_f = double(dxd), wy_f = double(wy), wz_f = double(wz);
  const double smax_f = double(smax);
  auto consider = [&](int d, int2 hd, int uu, int2 hu) {
    bool take;
    if (F64) {
      const double ry = fma(double(hu.x - Ym), dxd_f, double(hd.x - Ym) * dxu_f);
      const double rz = fma(double(hu.y - Zm), dxd_f, double(hd.y - Zm) * dxu_f);
      if ((wy && fabs(ry) >= RES_F64) || (wz && fabs(rz) >= RES_F64)) return;
      const double sc = fma(wy_f * ry, ry, wz_f * (rz * rz));
      if (sc > smax_f || sc > best_f) return;
      take = sc < best_f;
      if (take) best_f = sc;
    } else {
      const int64_t ry = int64_t(hd.x - Ym) * dxu + int64_t(hu.x - Ym) * dxd;
      const int64_t rz = int64_t(hd.y - Zm) * dxu + int64_t(hu.y - Zm) * dxd;
      // a residual of 2^28 or more puts the score above 2^56 > smax
      if ((wy && llabs(ry) >= (int64_t(1) << 28)) || (wz && llabs(rz) >= (int64_t(1) << 28))) return;
      const int64_t sc = wy * ry * ry + wz * rz * rz;
      if (sc > smax || sc > best_s) return;
      take = sc < best_s;
      if (take) best_s = sc;
    }
    if (!take) {  // equal score: smaller ids win
      const int idd = w.perm[d], idb = w.perm[best_d];
      take = idd < idb || (idd == idb && w.perm[uu] < w.perm[best_u]);
    }
    if (take) {
      best_d = d;
      best_u = uu;
    }
  };
  if (!overflow) {
#pragma unroll
    for (int a = 0; a < MAXD; ++a) {
      if (a < nd) {
        const int2 hd = hit_at<LDS>(w, sd, lhd, dq[a]);
#pragma unroll
        for (int b = 0; b < MAXU; ++b)
          if (b < nu) consider(dq[a], hd, uq[b], hit_at<LDS>(w, su, lhu, uq[b]));
      }
    }
    return;
  }
  // more candidates than the registers hold: every pair from the windows
  for (int izd = kd.c.iz0; izd <= kd.c.iz1; ++izd) {
    const int cd = kd.c.cbase + izd * kd.c.ny;
    const int q0 = cell_at<LDS>(w, sd, lcd, cd + kd.c.iy0), q1 = cell_at<LDS>(w, sd, lcd, cd + kd.c.iy1 + 1);
    for (int d = q0; d < q1; ++d) {
      const int2 hd = hit_at<LDS>(w, sd, lhd, d);
      if (hd.x < kd.ylo || hd.x > kd.yhi || hd.y < zlo || hd.y > zhi) continue;
      for (int izu = ku.c.iz0; izu <= ku.c.iz1; ++izu) {
        const int cu = ku.c.cbase + izu * ku.c.ny;
        const int v0 = cell_at<LDS>(w, su, lcu, cu + ku.c.iy0), v1 = cell_at<LDS>(w, su, lcu, cu + ku.c.iy1 + 1);
        for (int q = v0; q < v1; ++q) {
          const int2 h = hit_at<LDS>(w, su, lhu, q);
          if (h.x < ku.ylo || h.x > ku.yhi || h.y < zlo || h.y > zhi) continue;
          consider(d, hd, q, h);
        }
      }
    }
  }
}

// Slab of row record `rec` covering z in [zlo, zhi] (all y); stage it when it fits.
__device__ __forceinline__ Slab make_slab(const Workspace &w, const int32_t *rec, int64_t zlo, int64_t zhi) {
  Slab sl;
  sl.q0 = sl.nq = sl.c0 = sl.nc = 0;
  sl.lds = true;
  const int count = rec[S_COUNT];
  const int64_t zmin = rec[S_ZMIN], zmax = rec[S_ZMAX];
  if (count == 0 || zhi < zmin || zlo > zmax) return sl;  // no candidate will be visited
  const int64_t span = zmax - zmin;
  const int bz = rec[S_BZ], ny = rec[S_NY];
  auto cl = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
  const int iz0 = int(cl(zlo - zmin, 0, span)) / bz, iz1 = int(cl(zhi - zmin, 0, span)) / bz;
  sl.c0 = rec[S_CBASE] + iz0 * ny;
  sl.nc = (iz1 - iz0 + 1) * ny;  // entries c0 .. c0 + nc (inclusive end)
  sl.q0 = w.cell[sl.c0];
  sl.nq = w.cell[sl.c0 + sl.nc] - sl.q0;
  sl.lds = 2 * sl.nq + sl.nc + 1 <= STAGE_INTS;
  return sl;
}

// One chunk of NCH hits of one (unit,row): which hits, and the z slabs of
// the two neighbour rows that hold every candidate of every hit of the chunk.
// The z range comes from the z bins of the chunk's first and last hits (hits
// are in (z bin, y bin) order and bins are exact floors), widened by the
// window.
struct Chunk {
  int64_t s;
  int r, m, n_here;
  const int32_t *rec;
  Slab sd, su;
};

__device__ __forceinline__ Chunk chunk_setup(const Args &A, int b) {
  const Workspace &w = A.w;
  Chunk c;
  c.s = w.chunk_seg[b];
  c.r = int(c.s % A.n_rows);
  c.rec = w.seg + c.s * SEGW;
  const int start = c.rec[S_START], count = c.rec[S_COUNT];
  const int p0 = (b - c.rec[S_CHUNK]) * NCH;
  c.n_here = min(NCH, count - p0);
  c.m = start + p0 + int(threadIdx.x);
  c.sd.lds = c.su.lds = true;
  c.sd.nq = c.su.nq = 0;
  if (c.r == 0 || c.r == A.n_rows - 1) return c;
  const int zmin = c.rec[S_ZMIN], bz = c.rec[S_BZ];
  const int za = w.syz[start + p0].y, zb = w.syz[start + p0 + c.n_here - 1].y;
  const int64_t WZ = A.p.win_z_q;
  const int64_t zlo = int64_t(zmin) + int64_t((za - zmin) / bz) * bz - WZ;
  const int64_t zhi = int64_t(zmin) + int64_t((zb - zmin) / bz + 1) * bz - 1 + WZ;
  c.sd = make_slab(w, c.rec - SEGW, zlo, zhi);
  c.su = make_slab(w, c.rec + SEGW, zlo, zhi);
  return c;
}

template <bool LDS, bool F64>
__device__ __forceinline__ void chunk_links(const Args &A, const Chunk &c, const int *lcd, const int *lcu,
                                            const int2 *lhd, const int2 *lhu) {
  const Workspace &w = A.w;
  const int r = c.r;
  const int64_t Xi = __float2ll_rn(A.row_x[r] * 256.0f);
  const int64_t Xd = __float2ll_rn(A.row_x[r - 1] * 256.0f);
  const int64_t Xu = __float2ll_rn(A.row_x[r + 1] * 256.0f);
  const int64_t smax = A.p.smax_k * (Xu - Xd) * (Xu - Xd);
  int bd, bu;
  best_pair<LDS, F64>(A, c.m, c.rec - SEGW, c.rec + SEGW, w.seg_inv[c.s - 1], w.seg_inv[c.s + 1], c.sd, c.su, lcd, lcu, lhd, lhu, Xi, 1.0 / double(Xi), Xd,
                 Xu, smax, bd, bu);
  w.dn[c.m] = bd;
  w.up[c.m] = bu;
}

// Chunks whose slabs fit in LDS (and whose rows allow FP64 scores); the others
// are listed for k_neighbours_wide.
// 6 waves per SIMD (80 registers, a few spilled): measured faster than the
// 4 that 98 registers would allow and than 7 or 8 with more spills.
__global__ void __launch_bounds__(NCH) __attribute__((amdgpu_waves_per_eu(6, 8))) k_neighbours(Args A) {
  __shared__ __align__(16) int pool[2][STAGE_INTS];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_chunks = w.ctr[C_NCHUNK];
  const int b = int(xcd_chunk(blockIdx.x, n_chunks));
  if (b >= n_chunks) return;
  const Chunk c = chunk_setup(A, b);
  const bool act = int(threadIdx.x) < c.n_here;
  if (c.r == 0 || c.r == A.n_rows - 1) {
    if (act) {
      w.up[c.m] = -1;
      w.dn[c.m] = -1;
    }
    return;
  }
  const int64_t Xd = __float2ll_rn(A.row_x[c.r - 1] * 256.0f), Xu = __float2ll_rn(A.row_x[c.r + 1] * 256.0f);
  const bool f64 = double(A.p.smax_k * (Xu - Xd) * (Xu - Xd)) < SMAX_F64;
  if (!(c.sd.lds && c.su.lds && f64)) {
    if (threadIdx.x == 0) w.wide[atomicAdd(reinterpret_cast<unsigned long long *>(&w.ctr[C_NWIDE]), 1ull)] = b;
    return;
  }
  {  // stage both slabs: hits, then cells, each with all loads issued before the stores
    int2 *lhd = reinterpret_cast<int2 *>(pool[0]), *lhu = reinterpret_cast<int2 *>(pool[1]);
    int2 vd[STAGE_KH], vu[STAGE_KH];
#pragma unroll
    for (int k = 0; k < STAGE_KH; ++k) {
      const int i = int(threadIdx.x) + k * NCH;
      if (i < c.sd.nq) vd[k] = w.syz[c.sd.q0 + i];
      if (i < c.su.nq) vu[k] = w.syz[c.su.q0 + i];
    }
#pragma unroll
    for (int k = 0; k < STAGE_KH; ++k) {
      const int i = int(threadIdx.x) + k * NCH;
      if (i < c.sd.nq) lhd[i] = vd[k];
      if (i < c.su.nq) lhu[i] = vu[k];
    }
    int cd[STAGE_KC], cu[STAGE_KC];
    const bool cdo = c.sd.nq + c.sd.nc > 0, cuo = c.su.nq + c.su.nc > 0;
#pragma unroll
    for (int k = 0; k < STAGE_KC; ++k) {
      const int i = int(threadIdx.x) + k * NCH;
      if (cdo && i <= c.sd.nc) cd[k] = w.cell[c.sd.c0 + i];
      if (cuo && i <= c.su.nc) cu[k] = w.cell[c.su.c0 + i];
    }
#pragma unroll
    for (int k = 0; k < STAGE_KC; ++k) {
      const int i = int(threadIdx.x) + k * NCH;
      if (cdo && i <= c.sd.nc) pool[0][2 * c.sd.nq + i] = cd[k];
      if (cuo && i <= c.su.nc) pool[1][2 * c.su.nq + i] = cu[k];
    }
  }
  __syncthreads();
  if (act)
    chunk_links<true, true>(A, c, pool[0], pool[1], reinterpret_cast<const int2 *>(pool[0]),
                      reinterpret_cast<const int2 *>(pool[1]));
}

// The listed chunks, reading the neighbour rows from the workspace, int64 scores.
__global__ void __launch_bounds__(NCH) k_neighbours_wide(Args A) {
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_wide = w.ctr[C_NWIDE];
  for (int64_t j = blockIdx.x; j < n_wide; j += gridDim.x) {
    const Chunk c = chunk_setup(A, w.wide[j]);
    if (int(threadIdx.x) < c.n_here) chunk_links<false, false>(A, c, nullptr, nullptr, nullptr, nullptr);
  }
}

// ---------------------------------------------------------------------------
// step 4: cleaner (only mutual links survive), start flags and their count per
// block of ELEMS positions.

__global__ void __launch_bounds__(TPB) k_clean(Args A) {
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t base = int64_t(blockIdx.x) * ELEMS;
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < ELEMS / TPB; ++e) {
    const int64_t p = base + e * TPB + threadIdx.x;
    if (p < A.n) {
      const int u = w.up[p], d = w.dn[p];
      const int uc = (u >= 0 && w.dn[u] == p) ? u : -1;
      const int dc = (d >= 0 && w.up[d] == p) ? d : -1;
      w.upc[p] = uc;
      w.dnc[p] = dc;
      const int f = (uc >= 0 && dc < 0) ? 1 : 0;
      w.flag[p] = uint8_t(f);
      cnt += f;
    }
  }
  int tot;
  block_exclusive_scan<TPB>(cnt, tmp, &tot);
  if (threadIdx.x == 0) w.blk[blockIdx.x] = tot;
}

// one-block exclusive scan of per-block counts; total into counters, capacity check
__global__ void __launch_bounds__(1024) k_scan_blocks(int32_t *blk, int64_t nb, int64_t *ctr_total,
                                                      int64_t *out_total, int64_t cap,
                                                      int32_t *status, int32_t *blk2,
                                                      int64_t *ctr_total2, int64_t *out_total2,
                                                      int64_t cap2) {
  __shared__ int tmp[16];
  if (*status != TPC_OK) return;
  for (int which = 0; which < (blk2 ? 2 : 1); ++which) {
    int32_t *b = which ? blk2 : blk;
    int carry = 0;
    constexpr int PER = 8;  // consecutive entries per thread, one block scan per 8192
    for (int64_t base = 0; base < nb; base += 1024 * PER) {
      const int64_t i0 = base + int64_t(threadIdx.x) * PER;
      int v[PER], sum = 0;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        v[e] = i0 + e < nb ? b[i0 + e] : 0;
        sum += v[e];
      }
      int tot;
      int ex = carry + block_exclusive_scan<1024>(sum, tmp, &tot);
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        if (i0 + e < nb) b[i0 + e] = ex;
        ex += v[e];
      }
      carry += tot;
    }
    if (threadIdx.x == 0) {
      int64_t *ct = which ? ctr_total2 : ctr_total;
      int64_t *ot = which ? out_total2 : out_total;
      const int64_t c = which ? cap2 : cap;
      *ct = carry;
      if (ot) *ot = carry;
      if (carry > c) set_status(status, TPC_E_CAPACITY);
    }
  }
}

// step 4b: compaction of start hits in position order -> tracklet list
__global__ void __launch_bounds__(TPB) k_compact_starts(Args A) {
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  // each thread takes ELEMS / TPB consecutive flags (one 8-byte load), so one
  // block scan numbers the block's starts in position order
  constexpr int PER = ELEMS / TPB;
  static_assert(PER == 8, "one 64-bit load of flags per thread");
  const int64_t p0 = int64_t(blockIdx.x) * ELEMS + int64_t(threadIdx.x) * PER;
  uint64_t f8 = 0;
  if (p0 + PER <= A.n) {
    f8 = *reinterpret_cast<const uint64_t *>(w.flag + p0);  // flags are 256-byte aligned
  } else {
    for (int e = 0; e < PER; ++e)
      if (p0 + e < A.n) f8 |= uint64_t(w.flag[p0 + e]) << (8 * e);
  }
  const int cnt = __popcll(f8 & 0x0101010101010101ull);
  int tot;
  int t = w.blk[blockIdx.x] + block_exclusive_scan<TPB>(cnt, tmp, &tot);
  if (cnt) {
    int lo = 0, hi = A.n_units - 1;  // unit of the first flag: largest u with off[u] <= p0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.off[mid] <= p0) lo = mid; else hi = mid - 1;
    }
    for (int e = 0; e < PER; ++e) {
      if ((f8 >> (8 * e)) & 1) {
        const int64_t p = p0 + e;
        while (A.off[lo + 1] <= p) ++lo;
        w.trk_start[t] = int32_t(p);
        w.trk_unit[t] = lo;
        ++t;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// step 5: tracklet constructor (FP32 Kalman filter, one tracklet per lane);
// the filter itself is in tpc_kalman.h.

// round(v + ref) to the nearest integer, halves to even, for a float v and an
// integer ref, without forming the (less precise) float sum.
__device__ __forceinline__ int round_offset(float v, int ref) {
  const float t = floorf(v);
  const float fr = v - t;  // exact for |v| < 2^23
  int r = int(t);
  if (fr > 0.5f || (fr == 0.5f && ((r + ref) & 1))) ++r;
  return r + ref;
}

// Least (w_y dY^2 + w_z dZ^2, id) inside the pickup window of the rounded
// prediction, from the row's record rf (already loaded) and its bin-size
// reciprocals inv.  The state is relative to the integer reference (Yr, Zr).
// stop = 1 when the prediction has left the sector.
__device__ int pick(const Args &A, const Rec &rf, float2 inv, float yp, float zp, int Yr, int Zr,
                    bool &stop, int2 &best_yz) {
  const Workspace &w = A.w;
  const float vy = yp * 256.f, vz = zp * 256.f;
  // a prediction that is not finite (or beyond 4e15 quanta) ends the walk;
  // one beyond every cluster (|v| >= 1e9 quanta) is outside the sector in y
  // (a stop) and outside every window in z (a miss)
  if (!(fabsf(vy) < 1.0e9f) || !(fabsf(vz) < 4.0e15f)) {
    stop = true;
    return -1;
  }
  const int Yp = round_offset(vy, Yr);
  if (abs(Yp) > rf.H + A.p.ext_edge_q) {
    stop = true;
    return -1;
  }
  if (!(fabsf(vz) < 1.0e9f)) return -1;
  const int Zp = round_offset(vz, Zr);
  const int WY = A.p.ext_win_y_q, WZ = A.p.ext_win_z_q;
  const Win c = window_cells(rf, inv, Yp - WY, Yp + WY, Zp - WZ, Zp + WZ);
  if (c.empty) return -1;
  // windows < 2^13 and weights <= 15 keep the score below 2^31
  int best_s = INT32_MAX;
  int best = -1;
  // The cell bounds of up to ZB z bins are loaded together; their hits are
  // taken as one list, HB at a time, so that a lane's batches follow its
  // number of hits rather than its number of bins, and one pickup waits for
  // few round trips.
  constexpr int ZB = 4, HB = 4;
  for (int izb = c.iz0; izb <= c.iz1; izb += ZB) {
    int qa[ZB], e[ZB];  // first hit of each bin; end of each bin in the joint list
    int tot = 0;
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const bool v = izb + k <= c.iz1;
      const int cb = c.cbase + (izb + k) * c.ny;
      qa[k] = v ? w.cell[cb + c.iy0] : 0;
      const int qb = v ? w.cell[cb + c.iy1 + 1] : 0;
      tot += qb - qa[k];
      e[k] = tot;
    }
    for (int j0 = 0; j0 < tot; j0 += HB) {
      int qq[HB];
      int2 hh[HB];
#pragma unroll
      for (int j = 0; j < HB; ++j) {
        const int t = j0 + j;
        qq[j] = t < e[0] ? qa[0] + t : t < e[1] ? qa[1] + (t - e[0]) : t < e[2] ? qa[2] + (t - e[1])
                                                                               : qa[3] + (t - e[2]);
        hh[j] = t < tot ? w.syz[qq[j]] : make_int2(0, 0);
      }
#pragma unroll
      for (int j = 0; j < HB; ++j) {
        if (j0 + j >= tot) break;
        const int2 h = hh[j];
        const int dY = h.x - Yp, dZ = h.y - Zp;
        if (abs(dY) > WY || abs(dZ) > WZ) continue;
        const int sc = A.p.w_y * dY * dY + A.p.w_z * dZ * dZ;
        if (sc < best_s || (sc == best_s && w.perm[qq[j]] < w.perm[best])) {
          best_s = sc;
          best = qq[j];
          best_yz = h;
        }
      }
    }
  }
  return best;
}

// step 5a: chains.  Per tracklet: the row of its start hit and the length of
// the chain along the cleaned upward links (a cellular automaton over pad
// rows); chains of >= l_min hits become seeds, and their start row, middle
// and last hits are kept for the seed fit.
constexpr int CHAIN_BLOCKS = 2048;  // grid of the per-tracklet kernels (blocks loop over 256-tracklet chunks)

__global__ void __launch_bounds__(TPB) k_chains(Args A) {
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_trk = w.ctr[C_K];
  const int64_t n_chunks = (n_trk + TPB - 1) / TPB;
  for (int64_t b = blockIdx.x; b < n_chunks; b += gridDim.x) {
    const int64_t t = b * TPB + threadIdx.x;
    int seed = 0;
    if (t < n_trk) {
      const int nr = A.n_rows;
      const int h0 = w.trk_start[t], u = w.trk_unit[t];
      const int32_t *segu = w.seg + int64_t(u) * nr * SEGW;
      int lo = 0, hi = nr - 1;  // row of the start hit: last row whose start <= h0
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segu[mid * SEGW + S_START] <= h0) lo = mid; else hi = mid - 1;
      }
      const int r1 = lo;
      // one walk; hm trails at half speed, so it ends on the chain's hit L/2
      int L = 0, hb = h0, hm = h0;
      for (int h = h0; h >= 0 && r1 + L < nr; h = w.upc[h]) {
        hb = h;
        ++L;
        if ((L & 1) == 0) hm = w.upc[hm];
      }
      w.trk_len[t] = L;
      seed = L >= A.p.l_min;
      if (seed) {  // handed to k_compact_seeds, which files them by seed
        w.tmp_r1[t] = r1;
        w.tmp_hm[t] = hm;
        w.tmp_hb[t] = hb;
      }
    }
    int tot;
    block_exclusive_scan<TPB>(seed, tmp, &tot);
    if (threadIdx.x == 0) w.blk_keep[b] = tot;  // chunks past the tracklets keep k_init's 0
  }
}

// step 5b: list of seeds in tracklet order, with their seed-fit inputs
__global__ void __launch_bounds__(TPB) k_compact_seeds(Args A) {
  __shared__ int tmp[4];
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_trk = w.ctr[C_K];
  const int64_t n_chunks = (n_trk + TPB - 1) / TPB;
  for (int64_t b = blockIdx.x; b < n_chunks; b += gridDim.x) {
    const int64_t t = b * TPB + threadIdx.x;
    const int seed = (t < n_trk && w.trk_len[t] >= A.p.l_min) ? 1 : 0;
    int tot;
    const int ex = block_exclusive_scan<TPB>(seed, tmp, &tot);
    if (seed) {
      const int64_t i = w.blk_keep[b] + ex;
      if (i < w.S_cap) {  // beyond: the scan has already reported TPC_E_CAPACITY
        w.seed_list[i] = int32_t(t);
        w.sd_r1[i] = w.tmp_r1[t];
        w.sd_hm[i] = w.tmp_hm[t];
        w.sd_hb[i] = w.tmp_hb[t];
      }
    }
  }
}

// step 5c: Kalman fit of every seed, one seed per lane.
// Seed: circle through the first, middle and last chain hits.  Pass 1 fits
// the chain inner to outer (following the cleaned links) and extends it to
// the last row; pass 2 restarts from the outermost hit with the covariance
// reset and walks down to row 0, reusing pass-1 hits and picking hits in the
// other rows.  The filter keeps one committed state (at its last update);
// each row is predicted by a parameter-only transport from it, and the
// covariance is transported only when a hit is picked (helix transports
// compose exactly).  The lanes of a wave step through the rows together (a
// lane idles on rows outside its walk), so their hit-table accesses and
// (unit,row) records coalesce; each lane's own sequence of operations is that
// of its walk alone.
// 5 waves per SIMD (96 registers): the walk waits on dependent gathers, so
// each pickup loads its cell bounds and hits in batches (and the row's record
// before the transport), and each lane keeps its covariance in LDS rather
// than in 15 registers, which frees the registers for the batches at 5
// waves; measured faster than 4 waves with the covariance in registers and
// than 6 waves (spills)
__global__ void __launch_bounds__(CTB) __attribute__((amdgpu_waves_per_eu(5, 8))) k_fit(Args A) {
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_seeds = w.ctr[C_SEEDS];
  const int64_t i = xcd_chunk(blockIdx.x, (n_seeds + CTB - 1) / CTB) * CTB + threadIdx.x;
  if ((i & ~int64_t(63)) >= n_seeds) return;  // whole wave past the seeds
  const bool valid = i < n_seeds;
  const int64_t t = valid ? w.seed_list[i] : 0;
  const tpc_params_t &P = A.p;
  const int nr = A.n_rows;
  int32_t *col = seed_column(w, i, nr);
  const float sy2 = P.sigma_y * P.sigma_y, sz2 = P.sigma_z * P.sigma_z;
  const float k = A.kcurv, smx = P.sinphi_max;
  int nfit = 0, rlo = -1, rhi = -1;
  int h0 = 0, u = 0, L = 0, r1 = 0, Yr = 0, Zr = 0;
  const int32_t *segu = w.seg;
  const float2 *invs = w.seg_inv;
  __shared__ float cov_lds[CTB * 15];  // per wave [15][64]: lanes side by side, no bank conflicts
  KState s;
  s.c = cov_lds + (threadIdx.x >> 6) * (15 * 64) + (threadIdx.x & 63);
  bool ok = false;
  if (valid) {
    h0 = w.trk_start[t];
    u = w.trk_unit[t];
    L = w.trk_len[t];
    r1 = w.sd_r1[i];
    segu = w.seg + int64_t(u) * nr * SEGW;
    invs = w.seg_inv + int64_t(u) * nr;
    // seed, in coordinates relative to the first chain hit: small numbers
    // keep FP32 precise even at |z'| of metres (continuous readout)
    const int2 ya = w.syz[h0], ym = w.syz[w.sd_hm[i]], yb = w.syz[w.sd_hb[i]];
    Yr = ya.x;
    Zr = ya.y;
    const float y1 = float(ym.x - Yr) * (1.f / 256.f), y2 = float(yb.x - Yr) * (1.f / 256.f);
    const float z2 = float(yb.y - Zr) * (1.f / 256.f);
    ok = seed3(s, A.row_x[r1], A.row_x[r1 + L / 2], A.row_x[r1 + L - 1], y1, y2, z2, k, smx, P.cov0);
  }
  // pass 1: the chain rows, then extension rows, in one walk up the rows;
  // one propagate/update site serves both kinds of row.
  int r_out = r1, misses = 0, hc = h0, p1n = ok ? 1 : 0;
  bool act = ok;
  if (ok) {
    col[r1 * 64] = h0;
    upd_hit(s, w.syz[h0], Yr, Zr, sy2, sz2);
  }
  for (int r = wave_min(ok ? r1 : nr) + 1; r < nr; ++r) {
    if (!__any(act)) break;
    if (!act || r <= r1) continue;
    int h = -1;
    int2 yz = make_int2(0, 0);
    const bool chain = r < r1 + L;
    // the row's record for a pickup, loaded before the transport it waits on
    Rec rf{};
    float2 inv = make_float2(0.f, 0.f);
    if (!chain) {
      rf = rec_fields_v(segu + r * SEGW);
      inv = invs[r];
    }
    Step st;
    const float xr = A.row_x[r];
    if (!step_prepare(s, xr, k, smx, st)) {
      act = false;
      continue;
    }
    if (chain) {
      hc = w.upc[hc];
      h = hc;
      yz = w.syz[h];
    } else {
      bool stop = false;
      h = pick(A, rf, inv, s.p[0] + st.dy, s.p[1] + s.p[3] * st.sT, Yr, Zr, stop, yz);
      if (stop) {
        act = false;
        continue;
      }
    }
    col[r * 64] = h;
    if (h >= 0) {
      step_apply(s, st, xr, k);
      upd_hit(s, yz, Yr, Zr, sy2, sz2);
      r_out = r;
      ++p1n;
      misses = 0;
    } else if (++misses > P.max_miss) {
      act = false;
    }
  }
  // pass 2: from the outermost hit down to row 0, covariance reset
  act = ok;
  if (ok) {
    cov_reset(s, P.cov0);
    s.chi2 = 0.f;
    upd_hit(s, w.syz[col[r_out * 64]], Yr, Zr, sy2, sz2);
    nfit = 1;
    rhi = r_out;
    rlo = r_out;
    misses = 0;
  }
  for (int r = wave_max(ok ? r_out - 1 : -1); r >= 0; --r) {
    if (!__any(act)) break;
    if (!act || r >= r_out) continue;
    int h = r >= r1 ? col[r * 64] : -1;  // pass-1 hit of this row, if any
    int2 yz = make_int2(0, 0);
    const Rec rf = rec_fields_v(segu + r * SEGW);
    const float2 inv = invs[r];
    Step st;
    const float xr = A.row_x[r];
    if (!step_prepare(s, xr, k, smx, st)) {
      act = false;
      continue;
    }
    bool upd = true;
    if (h >= 0) {
      yz = w.syz[h];
    } else {
      bool stop = false;
      h = pick(A, rf, inv, s.p[0] + st.dy, s.p[1] + s.p[3] * st.sT, Yr, Zr, stop, yz);
      if (stop) {
        act = false;
        continue;
      }
      col[r * 64] = h;
      if (h < 0) {
        rlo = r;
        if (r < r1 && ++misses > P.max_miss) act = false;
        upd = false;
      } else {
        misses = 0;
      }
    }
    if (upd) {
      step_apply(s, st, xr, k);
      upd_hit(s, yz, Yr, Zr, sy2, sz2);
      ++nfit;
      rlo = r;
    }
  }
  uint32_t key = 0;
  if (nfit > 0) {
    const uint32_t local = uint32_t(w.perm[h0] - A.off[u]);
    key = (uint32_t(nfit) << 24) | (0xFFFFFFu - local);
    s.p[0] += float(Yr) * (1.f / 256.f);  // back to absolute coordinates
    s.p[1] += float(Zr) * (1.f / 256.f);
  } else {
#pragma unroll
    for (int j = 0; j < 5; ++j) s.p[j] = 0.f;
#pragma unroll
    for (int j = 0; j < 15; ++j) s.c[j * 64] = 0.f;
    s.x = 0.f;
    s.chi2 = 0.f;
  }
  if (valid) {
    w.sd_nfit[i] = nfit;
    w.sd_p1n[i] = p1n;
    w.sd_rlo[i] = rlo;
    w.sd_rhi[i] = rhi;
    w.sd_key[i] = key;
#pragma unroll
    for (int j = 0; j < 5; ++j) w.sd_par[i * 5 + j] = s.p[j];
#pragma unroll
    for (int j = 0; j < 15; ++j) w.sd_cov[i * 15 + j] = s.c[j * 64];
    w.sd_x[i] = s.x;
    w.sd_chi2[i] = s.chi2;
  }
  // ownership: every hit goes to the tracklet with the largest key
  const bool has = nfit > 0;
  const int rb = wave_max(has ? rhi : -1);
  for (int r0 = wave_min(has ? rlo : nr); r0 <= rb; r0 += RB) {
    int h[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) h[k] = (has && r0 + k >= rlo && r0 + k <= rhi) ? col[(r0 + k) * 64] : -1;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (h[k] >= 0) atomicMax(&w.owner[h[k]], key);
  }
}

// ---------------------------------------------------------------------------
// step 6: selector and output.  Keep a tracklet that owns >= n_min of its
// hits and at least f_min of them; tracks keep the tracklet order; no refit.
//
// One pass over the seed list (tracklets that are not seeds own nothing and
// are never kept; k_chains set their owned = keep = 0).  Seeds are in
// tracklet order, so an exclusive scan over seed order numbers the tracks in
// tracklet order.  The scan is a single-pass decoupled look-back: a block
// takes the next 256 seeds by ticket (so every seed block it waits on has
// already started), counts and marks its tracklets' owned hits, publishes its
// (tracks, hits) aggregate, adds up its predecessors' aggregates until it
// meets an inclusive prefix, publishes its own inclusive prefix, and writes
// its tracks.  The grid is a fixed number of blocks that loop over tickets,
// so the launch does not depend on the tracklet capacity.

// look-back word: flag (bits 62-63: 1 aggregate, 2 inclusive prefix),
// tracks (bits 31-61), hits (bits 0-30).  The counts travel in the same
// 64-bit word as their flag, so relaxed device-scope atomics suffice: no
// other memory is published with it (release/acquire would write back and
// invalidate the caches at every step).
constexpr uint64_t LB_AGG = uint64_t(1) << 62, LB_INC = uint64_t(2) << 62;
__device__ __forceinline__ uint64_t lb_word(uint64_t flag, int tracks, int hits) {
  return flag | (uint64_t(uint32_t(tracks)) << 31) | uint64_t(uint32_t(hits));
}
constexpr int SELECT_BLOCKS = 2048;
constexpr int LB_SPIN_MAX = 1 << 26;

__global__ void __launch_bounds__(TPB) k_select_emit(Args A) {
  __shared__ int tmp[4];
  __shared__ int64_t s_vb;
  __shared__ int s_bt, s_bh;  // tracks and hits of the blocks before this one
  const Workspace &w = A.w;
  if (*A.out.status != TPC_OK) return;
  const int64_t n_seeds = w.ctr[C_SEEDS];
  const int64_t nvb = (n_seeds + TPB - 1) / TPB;
  const int nr = A.n_rows;
  const tpc_tracks_t &O = A.out;
  for (;;) {
    if (threadIdx.x == 0)
      s_vb = int64_t(atomicAdd(reinterpret_cast<unsigned long long *>(&w.ctr[C_TICKET]), 1ull));
    __syncthreads();
    const int64_t vb = s_vb;
    if (vb >= nvb) return;
    const int64_t i = vb * TPB + threadIdx.x;
    const bool valid = i < n_seeds;
    const int64_t t = valid ? w.seed_list[i] : 0;
    const int nfit = valid ? w.sd_nfit[i] : 0;
    const bool has = nfit > 0;
    const uint32_t key = has ? w.sd_key[i] : 0u;
    const int rlo = has ? w.sd_rlo[i] : 0, rhi = has ? w.sd_rhi[i] : -1;
    int32_t *col = seed_column(w, i, nr);
    // owned hits: those whose owner key is this tracklet's, marked for the output
    int owned = 0;
    {
      const int rb = wave_max(has ? rhi : -1);
      for (int r0 = wave_min(has ? rlo : nr); r0 <= rb; r0 += RB) {  // RB rows per round trip
        int h[RB];
        uint32_t o[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) h[k] = (r0 + k >= rlo && r0 + k <= rhi) ? col[(r0 + k) * 64] : -1;
#pragma unroll
        for (int k = 0; k < RB; ++k) o[k] = h[k] >= 0 ? w.owner[h[k]] : 0u;
#pragma unroll
        for (int k = 0; k < RB; ++k)
          if (h[k] >= 0 && o[k] == key) {
            ++owned;
            col[(r0 + k) * 64] = h[k] | OWNED;
          }
      }
    }
    const int keep = has && owned >= A.p.n_min && int64_t(owned) * 256 >= int64_t(A.p.f_min_q8) * nfit;
    if (valid) {
      w.sd_owned[i] = owned;
      w.sd_keep[i] = keep;
    }
    int tk, to;
    const int ek = block_exclusive_scan<TPB>(keep, tmp, &tk);
    const int eo = block_exclusive_scan<TPB>(keep ? owned : 0, tmp, &to);
    if (threadIdx.x < 64) {  // wave 0: publish, then look back 64 predecessors at a time
      uint64_t *lb = w.lookback;
      const int lane = threadIdx.x;
      int bt = 0, bh = 0;
      if (vb == 0) {
        if (lane == 0)
          __hip_atomic_store(&lb[0], lb_word(LB_INC, tk, to), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (lane == 0)
          __hip_atomic_store(&lb[vb], lb_word(LB_AGG, tk, to), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t top = vb - 1;  // lane k reads block top - k
        int spins = 0;
        for (;;) {
          const int64_t j = top - lane;
          // before block 0 counts as an inclusive prefix of nothing
          const uint64_t v =
              j >= 0 ? __hip_atomic_load(&lb[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_INC;
          const uint64_t inc = __ballot((v >> 62) == 2), empty = __ballot((v >> 62) == 0);
          const int first = inc ? __ffsll(static_cast<unsigned long long>(inc)) - 1 : 64;  // nearest prefix
          const uint64_t before = first < 64 ? ((uint64_t(1) << first) << 1) - 1 : ~uint64_t(0);
          if (empty & before) {  // a block between us and that prefix has not published yet
            // the blocks looked at hold earlier tickets, so they are running or done
            if (++spins > LB_SPIN_MAX) {
              if (lane == 0) set_status(A.out.status, TPC_E_HIP);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          int vt = lane <= first ? int((v >> 31) & 0x7FFFFFFF) : 0;
          int vh = lane <= first ? int(v & 0x7FFFFFFF) : 0;
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            vt += __shfl_xor(vt, o, 64);
            vh += __shfl_xor(vh, o, 64);
          }
          bt += vt;
          bh += vh;
          if (first < 64) break;
          top -= 64;
        }
        if (lane == 0)
          __hip_atomic_store(&lb[vb], lb_word(LB_INC, bt + tk, bh + to), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      if (lane == 0) {
        s_bt = bt;
        s_bh = bh;
        if (vb == nvb - 1) {  // the last block knows the totals
          const int64_t nt = int64_t(bt) + tk, nh = int64_t(bh) + to;
          w.ctr[C_TRACKS] = nt;
          w.ctr[C_HITS] = nh;
          O.counts[0] = nt;
          O.counts[1] = nh;
          if (nt > O.cap_tracks || nh > O.cap_hits) set_status(A.out.status, TPC_E_CAPACITY);
        }
      }
    }
    __syncthreads();
    const int tr = s_bt + ek;
    int64_t off = int64_t(s_bh) + eo;
    const bool fits = keep && tr < O.cap_tracks && off + owned <= O.cap_hits;
    int elo = 0, ehi = -1;
    if (fits) {
#pragma unroll
      for (int j = 0; j < 5; ++j) O.params[int64_t(tr) * 5 + j] = w.sd_par[i * 5 + j];
#pragma unroll
      for (int j = 0; j < 15; ++j) O.cov[int64_t(tr) * 15 + j] = w.sd_cov[i * 15 + j];
      O.x_ref[tr] = w.sd_x[i];
      O.chi2[tr] = w.sd_chi2[i];
      O.unit[tr] = w.trk_unit[t];
      O.n_hits[tr] = owned;
      O.n_fit[tr] = nfit;
      O.first_hit[tr] = int32_t(off);
      elo = rlo;
      ehi = rhi;
    }
    {
      const int rb = wave_max(fits ? ehi : -1);
      for (int r0 = wave_min(fits ? elo : nr); r0 <= rb; r0 += RB) {  // RB rows per round trip
        int h[RB], id[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) h[k] = (r0 + k >= elo && r0 + k <= ehi) ? col[(r0 + k) * 64] : -1;
#pragma unroll
        for (int k = 0; k < RB; ++k) id[k] = (h[k] >= 0 && (h[k] & OWNED)) ? w.perm[h[k] & (OWNED - 1)] : -1;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          if (id[k] >= 0) {
            O.hits[off++] = id[k];
            O.cluster_track[id[k]] = tr;
          }
        }
      }
    }
    __syncthreads();  // s_vb, s_bt, s_bh are rewritten by the next ticket
  }
}

inline unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }
inline unsigned round8(int64_t b) { return unsigned((b + 7) & ~int64_t(7)); }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" size_t tpc_workspace_size(int64_t n_clusters, int32_t n_units, int32_t n_rows,
                                     const tpc_params_t *params) {
  if (!params_ok(params)) return 0;
  Workspace w;
  if (!layout(n_clusters, n_units, n_rows, params, nullptr, &w)) return 0;
  return w.total;
}

extern "C" const char *tpc_status_string(int status) {
  switch (status) {
    case TPC_OK: return "ok";
    case TPC_E_INVALID: return "invalid argument or input data";
    case TPC_E_CAPACITY: return "capacity exceeded (see counts for the required sizes)";
    case TPC_E_NOMEM: return "workspace too small";
    case TPC_E_HIP: return "HIP runtime error";
    case TPC_E_BUSY: return "busy";
    default: return "unknown status";
  }
}

namespace {

const char *const kKernelNames[] = {
    "k_init",        "k_units",      "k_tile_hist",  "k_seg_plan",      "k_cell_base",
    "k_tile_offsets", "k_tile_scatter", "k_bin_sort",  "k_neighbours",    "k_neighbours_wide", "k_clean",
    "k_scan_blocks", "k_compact_starts", "k_chains", "k_scan_blocks", "k_compact_seeds",
    "k_fit",         "k_select_emit"};
constexpr int kNumKernels = int(sizeof(kKernelNames) / sizeof(kKernelNames[0]));

int track_impl(const tpc_clusters_t *c, const tpc_geometry_t *g, const tpc_field_t *f,
               const tpc_params_t *p, tpc_tracks_t *out, void *workspace, size_t ws_bytes,
               void *stream, void *const *events, int n_events) {
  if (!c || !g || !f || !p || !out || !params_ok(p)) return TPC_E_INVALID;
  if (c->n < 0 || c->n >= (int64_t(1) << 30) || c->n_units < 1 || !c->unit_offsets) return TPC_E_INVALID;
  if (c->n > 0 && (!c->y || !c->z || !c->row)) return TPC_E_INVALID;
  if (g->n_rows < 3 || g->n_rows > 255 || !g->row_x) return TPC_E_INVALID;
  if (!(f->bz_tesla == f->bz_tesla) || fabsf(f->bz_tesla) > 100.f) return TPC_E_INVALID;
  if (!out->counts || !out->status || out->cap_tracks < 0 || out->cap_hits < 0) return TPC_E_INVALID;
  if (c->n > 0 && !out->cluster_track) return TPC_E_INVALID;
  if (out->cap_tracks > 0 && (!out->params || !out->cov || !out->x_ref || !out->chi2 || !out->unit ||
                              !out->n_hits || !out->n_fit || !out->first_hit))
    return TPC_E_INVALID;
  if (out->cap_hits > 0 && !out->hits) return TPC_E_INVALID;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TPC_E_INVALID;
  if (events && n_events != kNumKernels + 1) return TPC_E_INVALID;
  Args A;
  memset(&A, 0, sizeof(A));
  if (!layout(c->n, c->n_units, g->n_rows, p, static_cast<char *>(workspace), &A.w)) return TPC_E_INVALID;
  if (A.w.total > ws_bytes) return TPC_E_NOMEM;
  A.off = c->unit_offsets;
  A.y = c->y;
  A.z = c->z;
  A.row = c->row;
  A.row_x = g->row_x;
  A.n = c->n;
  A.n_units = c->n_units;
  A.n_rows = g->n_rows;
  A.kcurv = -KAPPA * f->bz_tesla;
  A.p = *p;
  A.out = *out;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Workspace &w = A.w;
  (void)hipGetLastError();
  int ki = 0;
  // profiling: event k is recorded right before kernel k, the last one after the last kernel
  auto mark = [&]() {
    if (events) (void)hipEventRecord(static_cast<hipEvent_t>(events[ki]), st);
    ++ki;
  };
  int64_t init_n = w.S > c->n ? w.S : (c->n > C_N ? c->n : int64_t(C_N));
  if (init_n < w.SB) init_n = w.SB;
  if (init_n < w.KB) init_n = w.KB;
  mark();
  hipLaunchKernelGGL(k_init, dim3(blocks_for(init_n, TPB)), dim3(TPB), 0, st, A);
  mark();
  hipLaunchKernelGGL(k_units, dim3(1), dim3(1024), 0, st, A);
  if (c->n > 0) {
    mark();
    hipLaunchKernelGGL(k_tile_hist, dim3(unsigned(w.T_max)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_seg_plan, dim3(unsigned(c->n_units)), dim3(256), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_cell_base, dim3(1), dim3(1024), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_tile_offsets, dim3(unsigned(w.S)), dim3(64), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_tile_scatter, dim3(unsigned(w.T_max)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_bin_sort, dim3(unsigned(w.S)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_neighbours, dim3(round8(w.CH_max)), dim3(NCH), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_neighbours_wide, dim3(1024), dim3(NCH), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_clean, dim3(unsigned(w.NB)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, w.blk, w.NB, w.ctr + C_K,
                       out->counts + 2, w.T_cap, out->status, (int32_t *)nullptr, (int64_t *)nullptr,
                       (int64_t *)nullptr, int64_t(0));
    mark();
    hipLaunchKernelGGL(k_compact_starts, dim3(unsigned(w.NB)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_chains, dim3(unsigned(w.KB < CHAIN_BLOCKS ? w.KB : CHAIN_BLOCKS)), dim3(TPB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, w.blk_keep, w.KB, w.ctr + C_SEEDS,
                       out->counts + 4, w.S_cap, out->status, (int32_t *)nullptr, (int64_t *)nullptr,
                       (int64_t *)nullptr, int64_t(0));
    mark();
    hipLaunchKernelGGL(k_compact_seeds, dim3(unsigned(w.KB < CHAIN_BLOCKS ? w.KB : CHAIN_BLOCKS)), dim3(TPB), 0,
                       st, A);
    mark();
    hipLaunchKernelGGL(k_fit, dim3(round8(blocks_for(w.S_cap, CTB))), dim3(CTB), 0, st, A);
    mark();
    hipLaunchKernelGGL(k_select_emit, dim3(unsigned(w.SB < SELECT_BLOCKS ? w.SB : SELECT_BLOCKS)), dim3(TPB), 0,
                       st, A);
  }
  while (ki <= kNumKernels) mark();  // empty batch: the remaining events mark the same point
  if (hipGetLastError() != hipSuccess) return TPC_E_HIP;
  return TPC_OK;
}

}  // namespace

extern "C" int tpc_track_sectors(const tpc_clusters_t *c, const tpc_geometry_t *g,
                                 const tpc_field_t *f, const tpc_params_t *p, tpc_tracks_t *out,
                                 void *workspace, size_t ws_bytes, void *stream) {
  return track_impl(c, g, f, p, out, workspace, ws_bytes, stream, nullptr, 0);
}

extern "C" int tpc_track_sectors_profiled(const tpc_clusters_t *c, const tpc_geometry_t *g,
                                          const tpc_field_t *f, const tpc_params_t *p,
                                          tpc_tracks_t *out, void *workspace, size_t ws_bytes,
                                          void *stream, void *const *events, int32_t n_events) {
  if (!events) return TPC_E_INVALID;
  return track_impl(c, g, f, p, out, workspace, ws_bytes, stream, events, n_events);
}

// ---------------------------------------------------------------------------
// Workspace for callers that cannot allocate: one file-scope device array per
// GPU (the loader places a copy on every device the library runs on, and it
// stays until the process ends).  Host code never passes the array's name to
// a kernel: the name is a host-side stand-in.  Its device address is looked up
// once per device with that device current and kept in scratch_ptr.

__device__ __align__(256) unsigned char scratch[TPC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices];

// Address of the scratch array on the device that runs `stream` (the current
// device for the null stream), or nullptr when it cannot be obtained.
void *scratch_for(hipStream_t stream) {
  int dev = -1;
  if (stream) {
    if (hipStreamGetDevice(stream, &dev) != hipSuccess) return nullptr;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" int tpc_track_sectors_noalloc(const tpc_clusters_t *c, const tpc_geometry_t *g,
                                         const tpc_field_t *f, const tpc_params_t *p,
                                         tpc_tracks_t *out, void *stream) {
  if (!c || !g || !p || !params_ok(p)) return TPC_E_INVALID;
  const size_t need = tpc_workspace_size(c->n, c->n_units, g->n_rows, p);
  if (need == 0) return TPC_E_INVALID;
  if (need > size_t(TPC_SCRATCH_BYTES)) return TPC_E_NOMEM;
  void *ws = scratch_for(static_cast<hipStream_t>(stream));
  if (!ws) return TPC_E_HIP;
  return track_impl(c, g, f, p, out, ws, size_t(TPC_SCRATCH_BYTES), stream, nullptr, 0);
}

extern "C" int32_t tpc_kernel_count(void) { return kNumKernels; }

extern "C" const char *tpc_kernel_name(int32_t i) {
  return (i >= 0 && i < kNumKernels) ? kKernelNames[i] : "";
}

extern "C" int tpc_inspect(const tpc_clusters_t *c, int32_t n_rows, const tpc_params_t *p,
                           const void *workspace, int what, tpc_view_t *v) {
  if (!c || !p || !v || !workspace || !params_ok(p)) return TPC_E_INVALID;
  Workspace w;
  if (!layout(c->n, c->n_units, n_rows, p, (char *)workspace, &w)) return TPC_E_INVALID;
  const int64_t N = c->n, T = w.T_cap, K = w.S_cap;
  void *ptr = nullptr;
  int64_t cnt = 0;
  int eb = 4;
  switch (what) {
    case TPC_VIEW_PERM: ptr = w.perm; cnt = N; break;
    case TPC_VIEW_CELL: ptr = w.cell; cnt = w.C_max + 1; break;
    case TPC_VIEW_SEG: ptr = w.seg; cnt = w.S * SEGW; break;
    case TPC_VIEW_UP: ptr = w.up; cnt = N; break;
    case TPC_VIEW_DN: ptr = w.dn; cnt = N; break;
    case TPC_VIEW_UPC: ptr = w.upc; cnt = N; break;
    case TPC_VIEW_DNC: ptr = w.dnc; cnt = N; break;
    case TPC_VIEW_OWNER: ptr = w.owner; cnt = N; break;
    case TPC_VIEW_TRK_START: ptr = w.trk_start; cnt = T; break;
    case TPC_VIEW_TRK_UNIT: ptr = w.trk_unit; cnt = T; break;
    case TPC_VIEW_TRK_LEN: ptr = w.trk_len; cnt = T; break;
    case TPC_VIEW_TRK_NFIT: ptr = w.sd_nfit; cnt = K; break;
    case TPC_VIEW_TRK_RLO: ptr = w.sd_rlo; cnt = K; break;
    case TPC_VIEW_TRK_RHI: ptr = w.sd_rhi; cnt = K; break;
    case TPC_VIEW_TRK_KEY: ptr = w.sd_key; cnt = K; break;
    case TPC_VIEW_TRK_OWNED: ptr = w.sd_owned; cnt = K; break;
    case TPC_VIEW_TRK_KEEP: ptr = w.sd_keep; cnt = K; break;
    case TPC_VIEW_TRK_PARAMS: ptr = w.sd_par; cnt = K * 5; break;
    case TPC_VIEW_TRK_COV: ptr = w.sd_cov; cnt = K * 15; break;
    case TPC_VIEW_TRK_XREF: ptr = w.sd_x; cnt = K; break;
    case TPC_VIEW_TRK_CHI2: ptr = w.sd_chi2; cnt = K; break;
    case TPC_VIEW_TRK_HITS: ptr = w.trk_hits; cnt = w.KW * 64 * n_rows; break;
    case TPC_VIEW_SEED_LIST: ptr = w.seed_list; cnt = K; break;
    case TPC_VIEW_TRK_P1N: ptr = w.sd_p1n; cnt = K; break;
    default: return TPC_E_INVALID;
  }
  v->ptr = ptr;
  v->count = cnt;
  v->elem_bytes = eb;
  v->reserved = 0;
  return TPC_OK;
}
