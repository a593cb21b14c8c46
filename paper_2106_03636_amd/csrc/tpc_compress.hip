// Hit removal and track-model compression, the consumer of the tracks (paper
// §2.1: hits of tracks not used for physics are removed, the remaining hits
// go through entropy-reduction steps such as the track model compression).
// The operation is stated with tpc_compress in include/tpc_track.h.
//
// Two launches on the caller's stream:
//   k_cmp_init   clear the histograms and counts, take over the tracking
//                call's status;
//   k_cmp_codes  per cluster (grid-stride): its class and codes; each block
//                counts its classes and builds its residual histograms in
//                LDS, then adds the non-zero bins to the global ones.
// One cluster reads its position and row (10 bytes), its track index (4)
// and, when attached, its track's state (24, shared by the track's clusters
// and mostly served by the cache); it writes its class and codes (9 bytes).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpc_track.h"

namespace {

constexpr int TPB = 256;
constexpr int MAX_HIST_HALF = 2048;
constexpr int CMP_BLOCKS = 1024;
constexpr float KAPPA = 0.00299792458f;

struct CmpArgs {
  const float *y, *z;
  const uint16_t *row;
  int64_t n;
  const float *row_x;
  int32_t n_rows;
  const int32_t *cluster_track, *trk_status;
  const int64_t *trk_counts;
  const float *par, *xref;
  double k, step, pt_remove, sinphi_max;
  int32_t hh;  // hist_half
  uint8_t *cls;
  int32_t *code_y, *code_z;
  unsigned long long *hist, *counts;
  int32_t *status;
};

__global__ void __launch_bounds__(TPB) k_cmp_init(CmpArgs A) {
  const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (i == 0) *A.status = *A.trk_status;  // no codes for a failed tracking call
  if (i < 4 * int64_t(A.hh)) A.hist[i] = 0ull;
  if (i < 6) A.counts[i] = 0ull;
}

// The track's state (y, z, sin(phi), tan(lambda), q/pT at x1) carried along
// its helix to the plane x2 in FP64: sin(phi) changes by C dx (C = k q/pT),
// y by dx (sin1 + sin2) / (cos1 + cos2), z by tan(lambda) times the
// transverse arc length, 2 asin(C L / 2) / C over the chord L.  False when
// |sin(phi)| reaches sinphi_max or the chord is longer than a diameter.
__device__ __forceinline__ bool carry(const float *p, double x1, double x2, double k, double smax, double &yo,
                                      double &zo) {
#pragma clang fp contract(off)
  const double dx = x2 - x1;
  const double C = k * double(p[4]);
  const double s1 = p[2];
  const double s2 = s1 + C * dx;
  if (!(fabs(s1) < smax) || !(fabs(s2) < smax)) return false;
  const double c1 = sqrt(1.0 - s1 * s1), c2 = sqrt(1.0 - s2 * s2);
  const double dy = dx * (s1 + s2) / (c1 + c2);
  const double L = sqrt(dx * dx + dy * dy);
  const double u = fabs(C) * L * 0.5;
  if (!(u < 1.0)) return false;
  const double f = u < 1e-3 ? 1.0 + u * u / 6.0 : asin(u) / u;  // asin(u) / u
  const double sT = (dx < 0 ? -1.0 : 1.0) * L * f;
  yo = double(p[0]) + dy;
  zo = double(p[1]) + double(p[3]) * sT;
  return true;
}

__global__ void __launch_bounds__(TPB) k_cmp_codes(CmpArgs A) {
  __shared__ int32_t hy[2 * MAX_HIST_HALF], hz[2 * MAX_HIST_HALF];
  __shared__ int32_t cnt[6];
  if (*A.status != TPC_OK) return;
  const int32_t nb = 2 * A.hh;
  for (int32_t b = threadIdx.x; b < nb; b += TPB) hy[b] = hz[b] = 0;
  if (threadIdx.x < 6) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t T = A.trk_counts[0];
  for (int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x; c < A.n; c += int64_t(gridDim.x) * TPB) {
    const int32_t t = A.cluster_track[c];
    const int r = A.row[c];
    double vy = double(A.y[c]) / A.step, vz = double(A.z[c]) / A.step;
    int cl = 0;
    if (t >= 0 && t < T && r < A.n_rows) {
      const float *p = A.par + int64_t(t) * 5;
      double yp, zp;
      if (fabs(double(p[4])) * A.pt_remove > 1.0) {
        cl = 2;
      } else if (carry(p, double(A.xref[t]), double(A.row_x[r]), A.k, A.sinphi_max, yp, zp)) {
        cl = 1;
        vy = (double(A.y[c]) - yp) / A.step;  // a difference and a quotient: nothing to fuse
        vz = (double(A.z[c]) - zp) / A.step;
      } else {
        cl = 3;
      }
    }
    int32_t cy = 0, cz = 0;
    if (cl != 2) {
      cy = int32_t(rint(vy));
      cz = int32_t(rint(vz));
    }
    A.cls[c] = uint8_t(cl);
    A.code_y[c] = cy;
    A.code_z[c] = cz;
    const int first = __ffsll((unsigned long long)__ballot(1)) - 1;  // lowest active lane
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // class counts: one LDS atomic per wave and class
      const uint64_t m = __ballot(cl == k);
      if (__lane_id() == first && m) atomicAdd(&cnt[k], __popcll(m));
    }
    if (cl == 1) {
      if (cy >= -A.hh && cy < A.hh) atomicAdd(&hy[cy + A.hh], 1); else atomicAdd(&cnt[4], 1);
      if (cz >= -A.hh && cz < A.hh) atomicAdd(&hz[cz + A.hh], 1); else atomicAdd(&cnt[5], 1);
    }
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < nb; b += TPB) {
    if (hy[b]) atomicAdd(&A.hist[b], (unsigned long long)hy[b]);
    if (hz[b]) atomicAdd(&A.hist[nb + b], (unsigned long long)hz[b]);
  }
  if (threadIdx.x < 6 && cnt[threadIdx.x]) atomicAdd(&A.counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

}  // namespace

extern "C" int tpc_compress(const tpc_clusters_t *clusters, const tpc_geometry_t *geometry,
                            const tpc_field_t *field, const tpc_tracks_t *tracks,
                            const tpc_compress_params_t *params, tpc_compressed_t *out, void *stream) {
  if (!clusters || !geometry || !field || !tracks || !params || !out) return TPC_E_INVALID;
  if (clusters->n < 0 || (clusters->n > 0 && (!clusters->y || !clusters->z || !clusters->row))) return TPC_E_INVALID;
  if (geometry->n_rows < 1 || geometry->n_rows > 255 || !geometry->row_x) return TPC_E_INVALID;
  if (!tracks->cluster_track || !tracks->params || !tracks->x_ref || !tracks->counts || !tracks->status)
    return TPC_E_INVALID;
  if (!(params->step > 0.0f) || !(params->pt_remove >= 0.0f) || !(params->sinphi_max > 0.0f) ||
      !(params->sinphi_max < 1.0f) || params->hist_half < 1 || params->hist_half > MAX_HIST_HALF ||
      !isfinite(field->bz_tesla))
    return TPC_E_INVALID;
  if (!out->cls || !out->code_y || !out->code_z || !out->hist || !out->counts || !out->status) return TPC_E_INVALID;
  CmpArgs A;
  A.y = clusters->y;
  A.z = clusters->z;
  A.row = clusters->row;
  A.n = clusters->n;
  A.row_x = geometry->row_x;
  A.n_rows = geometry->n_rows;
  A.cluster_track = tracks->cluster_track;
  A.trk_status = tracks->status;
  A.trk_counts = tracks->counts;
  A.par = tracks->params;
  A.xref = tracks->x_ref;
  A.k = double(-KAPPA * field->bz_tesla);  // the tracker's curvature constant, as its fit used it
  A.step = params->step;
  A.pt_remove = params->pt_remove;
  A.sinphi_max = params->sinphi_max;
  A.hh = params->hist_half;
  A.cls = out->cls;
  A.code_y = out->code_y;
  A.code_z = out->code_z;
  A.hist = reinterpret_cast<unsigned long long *>(out->hist);
  A.counts = reinterpret_cast<unsigned long long *>(out->counts);
  A.status = out->status;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ib = (4 * int64_t(A.hh) + TPB - 1) / TPB;
  const int64_t cb = (A.n + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_cmp_init, dim3(unsigned(ib)), dim3(TPB), 0, st, A);
  hipLaunchKernelGGL(k_cmp_codes, dim3(unsigned(cb < 1 ? 1 : (cb > CMP_BLOCKS ? CMP_BLOCKS : cb))), dim3(TPB), 0,
                     st, A);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}
