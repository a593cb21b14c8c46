// Library-internal calls shared by tpc_track.hip and tpc_server.cpp (C++
// linkage, hidden: not part of the C ABI in include/tpc_track.h).
#pragma once

#include <stdint.h>

#include "tpc_track.h"

namespace tpc_internal {

// Outputs of one tpc_track_sectors call over R requests packed one after
// the other (request r owns clusters [cluster_base[r], cluster_base[r+1]) and
// units [unit_base[r], unit_base[r+1])), made request-local in place on
// `stream`: cluster_track, first_hit, unit and hits of each request count
// from its own first track, hit, unit and cluster.  req[2r], req[2r+1] get
// the request's first track and first hit in the packed outputs; req[2R],
// req[2R+1] the totals.  cluster_base, unit_base and req are device arrays
// of R+1, R+1 and 2(R+1) entries; R >= 1.  Enqueues kernels only.
int rebase_requests(const int64_t *cluster_base, const int64_t *unit_base, int32_t R,
                    const tpc_tracks_t *out, int64_t n, int64_t *req, void *stream);

}  // namespace tpc_internal
