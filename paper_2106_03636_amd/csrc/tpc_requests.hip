// Request-local outputs of a batch that packs several requests (the serving
// loop's batches): tpc_internal::rebase_requests, declared in tpc_internal.h.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpc_internal.h"
#include "tpc_track.h"

namespace {

__device__ __forceinline__ int upper_index(const int64_t *a, int32_t n, int64_t v) {
  // last r in [0, n) with a[r] <= v (a ascending, a[0] <= v)
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_req_bases(const int64_t *unit_base, int32_t R, tpc_tracks_t O,
                                                   int64_t *req) {
  if (*O.status != TPC_OK) return;  // counts may then exceed the capacities
  const int64_t T = O.counts[0], H = O.counts[1];
  for (int r = threadIdx.x; r <= R; r += blockDim.x) {
    int64_t t0 = T, h0 = H;
    if (r < R) {  // first track of the request's units (tracks are in unit order)
      int64_t lo = 0, hi = T;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (O.unit[mid] < unit_base[r]) lo = mid + 1; else hi = mid;
      }
      t0 = lo;
      h0 = t0 < T ? O.first_hit[t0] : H;
    }
    req[2 * r] = t0;
    req[2 * r + 1] = h0;
  }
}

__global__ void __launch_bounds__(256) k_req_apply(const int64_t *cluster_base, const int64_t *unit_base,
                                                   int32_t R, tpc_tracks_t O, int64_t n, const int64_t *req) {
  if (*O.status != TPC_OK) return;
  const int64_t T = O.counts[0], H = O.counts[1];
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t v = O.cluster_track[i];
    if (v >= 0) O.cluster_track[i] = int32_t(v - req[2 * upper_index(cluster_base, R, i)]);
  }
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < T; t += stride) {
    const int r = upper_index(unit_base, R, O.unit[t]);
    O.unit[t] = int32_t(O.unit[t] - unit_base[r]);
    O.first_hit[t] = int32_t(O.first_hit[t] - req[2 * r + 1]);
  }
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < H; k += stride) {
    int lo = 0, hi = R - 1;  // request whose hits hold position k
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (req[2 * mid + 1] <= k) lo = mid; else hi = mid - 1;
    }
    O.hits[k] = int32_t(O.hits[k] - cluster_base[lo]);
  }
}

}  // namespace

namespace tpc_internal {

int rebase_requests(const int64_t *cluster_base, const int64_t *unit_base, int32_t R, const tpc_tracks_t *out,
                    int64_t n, int64_t *req, void *stream) {
  if (!cluster_base || !unit_base || R < 1 || !out || !req || n < 0) return TPC_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_req_bases, dim3(1), dim3(256), 0, st, unit_base, R, *out, req);
  hipLaunchKernelGGL(k_req_apply, dim3(2048), dim3(256), 0, st, cluster_base, unit_base, R, *out, n,
                     static_cast<const int64_t *>(req));
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_E_HIP;
}

}  // namespace tpc_internal
