// Request loop for time frames arriving over time (tpc_server_* in tpc_track.h).
//
// One host thread per server drives the GPU (paper §3.1.1): it admits queued
// requests in arrival order while the device arena has room (memory-based
// admission with back pressure, §3.1.3 / §3.3), packs all admitted requests
// into one batch -- units are independent, so each request's results are
// those it would get alone -- and keeps up to max_in_flight batches on their
// own streams, so that the copies of one batch overlap the kernels of another
// (§3.1.2).  Every device buffer is carved out of one arena allocated at
// create; pinned host staging is pooled and reused.

#include <hip/hip_runtime.h>
#include <pthread.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tpc_internal.h"
#include "tpc_track.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t al(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// device arena: first-fit over one allocation, blocks coalesce on release

class Arena {
 public:
  void init(size_t bytes) {
    size_ = bytes;
    free_.clear();
    free_[0] = bytes;
    used_ = peak_ = 0;
  }
  // offset of a block of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = al(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

// ---------------------------------------------------------------------------
// pinned host blocks, pooled by power-of-two size class (hipHostFree would
// synchronize the device, so blocks are kept until the server ends)

class PinnedPool {
 public:
  void *get(size_t bytes) {
    size_t cls = 4096;
    while (cls < bytes) cls <<= 1;
    std::lock_guard<std::mutex> g(mu_);
    auto &lst = free_[cls];
    if (!lst.empty()) {
      void *p = lst.back();
      lst.pop_back();
      return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    size_of_[p] = cls;
    return p;
  }
  void put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    free_[size_of_[p]].push_back(p);
  }
  void clear() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto &kv : size_of_) (void)hipHostFree(kv.first);
    size_of_.clear();
    free_.clear();
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void *>> free_;
  std::unordered_map<void *, size_t> size_of_;
};

// ---------------------------------------------------------------------------

// Pinned result blocks of one batch; shared by its requests until the last
// of them is released.
struct BatchOut {
  PinnedPool *pool = nullptr;
  void *h_head = nullptr;  // counts[4] + status
  void *h_out = nullptr;   // the batch's results, packed
  ~BatchOut() {
    pool->put(h_head);
    pool->put(h_out);
  }
};

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  int32_t n_units = 0;
  std::vector<int64_t> offsets;
  int32_t flags = TPC_REQ_COPY;
  void *staging = nullptr;  // TPC_REQ_COPY: pinned y [n] f32, z [n] f32, row [n] u16
  const float *src_y = nullptr, *src_z = nullptr;  // where the arrays are read from
  const uint16_t *src_row = nullptr;
  enum { PENDING, RUNNING, DONE } state = PENDING;
  int32_t status = TPC_OK;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t batch_id = -1;
  int32_t batch_requests = 0;
  size_t footprint = 0;
  bool solo = false;  // runs in a batch of its own (after its batch failed)
  // results: the request's slice of its batch's packed results, made
  // request-local on the device before they were copied back
  std::shared_ptr<BatchOut> out;
  int64_t n_tracks = 0, n_track_hits = 0;
  const int32_t *b_ct = nullptr, *b_unit = nullptr, *b_nhits = nullptr, *b_nfit = nullptr,
                *b_first = nullptr, *b_hits = nullptr;
  const float *b_params = nullptr, *b_cov = nullptr, *b_xref = nullptr, *b_chi2 = nullptr;
};

struct OutLayout {  // device buffers of a batch, offsets inside its arena block
  size_t off_in_offsets, off_y, off_z, off_row, off_ws, ws_bytes, off_ct, off_params, off_cov,
      off_xref, off_chi2, off_unit, off_nhits, off_nfit, off_first, off_hits, off_counts, off_status,
      off_cbase, off_ubase, off_req, total;
  int64_t cap_tracks, cap_hits;
};

// a batch of R requests with n clusters in n_units units in all
bool batch_layout(int64_t n, int32_t n_units, int32_t R, int32_t n_rows, const tpc_params_t &p,
                  OutLayout *L) {
  const size_t ws = tpc_workspace_size(n, n_units, n_rows, &p);
  if (ws == 0) return false;
  const int64_t nmin = p.n_min > 0 ? p.n_min : 1;
  L->cap_tracks = n / nmin + 1;
  L->cap_hits = n > 0 ? n : 1;
  const size_t N = size_t(n > 0 ? n : 1), T = size_t(L->cap_tracks);
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = al(o + b);
    return at;
  };
  L->off_in_offsets = take(8 * (size_t(n_units) + 1));
  L->off_y = take(4 * N);
  L->off_z = take(4 * N);
  L->off_row = take(2 * N);
  L->off_ws = take(ws);
  L->ws_bytes = ws;
  L->off_ct = take(4 * N);
  L->off_params = take(4 * 5 * T);
  L->off_cov = take(4 * 15 * T);
  L->off_xref = take(4 * T);
  L->off_chi2 = take(4 * T);
  L->off_unit = take(4 * T);
  L->off_nhits = take(4 * T);
  L->off_nfit = take(4 * T);
  L->off_first = take(4 * T);
  L->off_hits = take(4 * size_t(L->cap_hits));
  L->off_counts = take(5 * 8);
  L->off_status = take(8);
  L->off_cbase = take(8 * (size_t(R) + 1));
  L->off_ubase = take(8 * (size_t(R) + 1));
  L->off_req = take(16 * (size_t(R) + 1));
  L->total = o;
  return true;
}

struct Batch {
  int64_t id = 0;
  std::vector<Request *> reqs;
  std::vector<int64_t> cluster_base, unit_base;
  int64_t n = 0;
  int32_t n_units = 0;
  size_t arena_off = 0;
  OutLayout L{};
  int slot = -1;
  int phase = 0;              // 0: kernels queued, 1: result copies queued
  int32_t host_status = TPC_OK;  // set when the batch could not be launched (pinned memory)
  void *h_offsets = nullptr;  // pinned: unit offsets [n_units + 1], cluster and unit bases [R + 1] each
  std::shared_ptr<BatchOut> out;
  size_t out_bytes = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_kernel = nullptr, ev_copy = nullptr;
  Batch *batch = nullptr;
};

}  // namespace

struct tpc_server {
  tpc_server_config_t cfg{};
  std::vector<float> row_x;
  float *d_row_x = nullptr;
  char *d_arena = nullptr;
  Arena arena;
  PinnedPool pinned;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int64_t next_batch = 0;
  bool stop = false;
  std::thread th;
  tpc_server_stats_t st{};

  void loop();
  bool form_and_launch();  // called with mu held
  void launch(Batch *b);   // without mu
  bool progress_slot(Slot &s);
  void finish(Batch *b);
  void requeue_solo(Batch *b);
};

namespace {

bool validate_request(const tpc_request_t *r, int32_t n_rows) {
  if (!r || r->n < 0 || r->n >= (int64_t(1) << 30) || r->n_units < 1 || !r->unit_offsets) return false;
  if (r->flags != TPC_REQ_COPY && r->flags != TPC_REQ_BORROW_HOST && r->flags != TPC_REQ_DEVICE) return false;
  if (r->n > 0 && (!r->y || !r->z || !r->row)) return false;
  if (r->unit_offsets[0] != 0 || r->unit_offsets[r->n_units] != r->n) return false;
  for (int32_t u = 0; u < r->n_units; ++u) {
    const int64_t a = r->unit_offsets[u], b = r->unit_offsets[u + 1];
    if (b < a || b - a >= (int64_t(1) << 24)) return false;
  }
  if (r->flags == TPC_REQ_DEVICE) return true;  // device arrays: checked by the kernels
  for (int64_t i = 0; i < r->n; ++i)
    if (r->row[i] >= n_rows || !(std::fabs(r->y[i]) <= 8192.f) || !(std::fabs(r->z[i]) <= 8192.f))
      return false;
  return true;
}

}  // namespace

bool tpc_server::form_and_launch() {
  int free_slot = -1;
  for (size_t i = 0; i < slots.size(); ++i)
    if (!slots[i].batch) {
      free_slot = int(i);
      break;
    }
  if (free_slot < 0 || pending.empty()) return false;
  // take requests in arrival order while the batch still fits
  std::unique_ptr<Batch> b(new Batch);
  int64_t n = 0;
  int32_t units = 0;
  OutLayout L{};
  size_t take = 0;
  for (size_t i = 0; i < pending.size(); ++i) {
    Request *r = pending[i];
    if (i > 0 && (r->solo || pending[0]->solo)) break;
    if (cfg.max_batch_requests > 0 && int32_t(i) >= cfg.max_batch_requests) break;
    if (i > 0 && cfg.max_batch_clusters > 0 && n + r->n > cfg.max_batch_clusters) break;
    OutLayout L2{};
    if (!batch_layout(n + r->n, units + r->n_units, int32_t(i + 1), cfg.n_rows, cfg.params, &L2)) break;
    if (L2.total > arena.largest_free()) break;
    n += r->n;
    units += r->n_units;
    L = L2;
    take = i + 1;
  }
  if (take == 0) return false;  // the head does not fit yet: wait for memory (back pressure)
  const size_t off = arena.alloc(L.total);
  if (off == SIZE_MAX) return false;
  b->id = next_batch++;
  b->n = n;
  b->n_units = units;
  b->L = L;
  b->arena_off = off;
  b->slot = free_slot;
  int64_t cb = 0, ub = 0;
  const double t = now_s();
  for (size_t i = 0; i < take; ++i) {
    Request *r = pending.front();
    pending.pop_front();
    r->state = Request::RUNNING;
    r->t_admit = t;
    r->batch_id = b->id;
    r->batch_requests = int32_t(take);
    b->reqs.push_back(r);
    b->cluster_base.push_back(cb);
    b->unit_base.push_back(ub);
    cb += r->n;
    ub += r->n_units;
  }
  slots[free_slot].batch = b.get();
  ++st.batches;
  Batch *raw = b.release();
  mu.unlock();
  launch(raw);
  mu.lock();
  return true;
}

void tpc_server::launch(Batch *b) {
  Slot &s = slots[b->slot];
  char *base = d_arena + b->arena_off;
  const OutLayout &L = b->L;
  // concatenated unit offsets, then the requests' cluster and unit bases
  const size_t R = b->reqs.size(), nu1 = size_t(b->n_units) + 1;
  b->h_offsets = pinned.get(8 * (nu1 + 2 * (R + 1)));
  b->out = std::make_shared<BatchOut>();
  b->out->pool = &pinned;
  // head: counts[4], status, pad[3], then per request its first track and hit
  b->out->h_head = pinned.get(64 + 16 * (R + 1));
  b->phase = 0;
  if (!b->h_offsets || !b->out->h_head) {  // no pinned memory: the batch fails as a whole
    b->host_status = TPC_E_NOMEM;
    (void)hipEventRecord(s.ev_kernel, s.stream);
    return;
  }
  int64_t *ho = static_cast<int64_t *>(b->h_offsets);
  int64_t u = 0;
  ho[0] = 0;
  for (size_t i = 0; i < R; ++i) {
    const Request *r = b->reqs[i];
    for (int32_t k = 1; k <= r->n_units; ++k) ho[++u] = b->cluster_base[i] + r->offsets[k];
  }
  int64_t *hcb = ho + nu1, *hub = hcb + (R + 1);
  for (size_t i = 0; i < R; ++i) {
    hcb[i] = b->cluster_base[i];
    hub[i] = b->unit_base[i];
  }
  hcb[R] = b->n;
  hub[R] = b->n_units;
  (void)hipMemcpyAsync(base + L.off_in_offsets, ho, 8 * nu1, hipMemcpyHostToDevice, s.stream);
  if (R > 1) {
    (void)hipMemcpyAsync(base + L.off_cbase, hcb, 8 * (R + 1), hipMemcpyHostToDevice, s.stream);
    (void)hipMemcpyAsync(base + L.off_ubase, hub, 8 * (R + 1), hipMemcpyHostToDevice, s.stream);
  }
  for (size_t i = 0; i < b->reqs.size(); ++i) {
    const Request *r = b->reqs[i];
    if (r->n == 0) continue;
    const size_t cb = size_t(b->cluster_base[i]);
    const hipMemcpyKind kind = r->flags == TPC_REQ_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    (void)hipMemcpyAsync(base + L.off_y + 4 * cb, r->src_y, 4 * size_t(r->n), kind, s.stream);
    (void)hipMemcpyAsync(base + L.off_z + 4 * cb, r->src_z, 4 * size_t(r->n), kind, s.stream);
    (void)hipMemcpyAsync(base + L.off_row + 2 * cb, r->src_row, 2 * size_t(r->n), kind, s.stream);
  }
  tpc_clusters_t c{};
  c.n = b->n;
  c.n_units = b->n_units;
  c.unit_offsets = reinterpret_cast<const int64_t *>(base + L.off_in_offsets);
  c.y = reinterpret_cast<const float *>(base + L.off_y);
  c.z = reinterpret_cast<const float *>(base + L.off_z);
  c.row = reinterpret_cast<const uint16_t *>(base + L.off_row);
  tpc_geometry_t g{};
  g.n_rows = cfg.n_rows;
  g.row_x = d_row_x;
  tpc_field_t f{};
  f.bz_tesla = cfg.bz_tesla;
  tpc_tracks_t o{};
  o.cap_tracks = L.cap_tracks;
  o.cap_hits = L.cap_hits;
  o.cluster_track = reinterpret_cast<int32_t *>(base + L.off_ct);
  o.params = reinterpret_cast<float *>(base + L.off_params);
  o.cov = reinterpret_cast<float *>(base + L.off_cov);
  o.x_ref = reinterpret_cast<float *>(base + L.off_xref);
  o.chi2 = reinterpret_cast<float *>(base + L.off_chi2);
  o.unit = reinterpret_cast<int32_t *>(base + L.off_unit);
  o.n_hits = reinterpret_cast<int32_t *>(base + L.off_nhits);
  o.n_fit = reinterpret_cast<int32_t *>(base + L.off_nfit);
  o.first_hit = reinterpret_cast<int32_t *>(base + L.off_first);
  o.hits = reinterpret_cast<int32_t *>(base + L.off_hits);
  o.counts = reinterpret_cast<int64_t *>(base + L.off_counts);
  o.status = reinterpret_cast<int32_t *>(base + L.off_status);
  int rc = tpc_track_sectors(&c, &g, &f, &cfg.params, &o, base + L.off_ws, L.ws_bytes, s.stream);
  if (rc == TPC_OK && R > 1)  // indices of each request counted from its own first track, hit, cluster
    rc = tpc_internal::rebase_requests(reinterpret_cast<const int64_t *>(base + L.off_cbase),
                                       reinterpret_cast<const int64_t *>(base + L.off_ubase), int32_t(R), &o,
                                       b->n, reinterpret_cast<int64_t *>(base + L.off_req), s.stream);
  int64_t *hh = static_cast<int64_t *>(b->out->h_head);
  hh[0] = hh[1] = hh[2] = hh[3] = 0;
  hh[4] = rc;  // launch status if the call failed on the host
  if (rc == TPC_OK) {
    (void)hipMemcpyAsync(hh, base + L.off_counts, 32, hipMemcpyDeviceToHost, s.stream);
    (void)hipMemcpyAsync(hh + 4, base + L.off_status, 4, hipMemcpyDeviceToHost, s.stream);
    if (R > 1) (void)hipMemcpyAsync(hh + 8, base + L.off_req, 16 * (R + 1), hipMemcpyDeviceToHost, s.stream);
  }
  (void)hipEventRecord(s.ev_kernel, s.stream);
}

// Advance the batch of a slot; true when something changed.
bool tpc_server::progress_slot(Slot &s) {
  Batch *b = s.batch;
  if (!b) return false;
  if (b->phase == 0) {
    if (hipEventQuery(s.ev_kernel) != hipSuccess) return false;
    if (b->host_status != TPC_OK) {
      for (Request *r : b->reqs) r->status = b->host_status;
      finish(b);
      return true;
    }
    const int64_t *hh = static_cast<const int64_t *>(b->out->h_head);
    const int32_t status = int32_t(reinterpret_cast<const int32_t *>(hh + 4)[0]);
    if (status != TPC_OK) {
      if (b->reqs.size() > 1 && (status == TPC_E_INVALID || status == TPC_E_CAPACITY)) {
        requeue_solo(b);  // find which request it was: each runs again alone
        return true;
      }
      for (Request *r : b->reqs) r->status = status;
      finish(b);
      return true;
    }
    const int64_t T = hh[0], H = hh[1];
    const OutLayout &L = b->L;
    const size_t N = size_t(b->n);
    b->out_bytes = 4 * N + 4 * size_t(T) * (5 + 15 + 1 + 1 + 4) + 4 * size_t(H) + 64;
    b->out->h_out = pinned.get(b->out_bytes);
    if (!b->out->h_out) {
      for (Request *r : b->reqs) r->status = TPC_E_NOMEM;
      finish(b);
      return true;
    }
    char *ho = static_cast<char *>(b->out->h_out);
    char *base = d_arena + b->arena_off;
    size_t o = 0;
    auto cp = [&](size_t dev_off, size_t bytes) {
      if (bytes) (void)hipMemcpyAsync(ho + o, base + dev_off, bytes, hipMemcpyDeviceToHost, s.stream);
      o += bytes;
    };
    cp(L.off_ct, 4 * N);
    cp(L.off_params, 20 * size_t(T));
    cp(L.off_cov, 60 * size_t(T));
    cp(L.off_xref, 4 * size_t(T));
    cp(L.off_chi2, 4 * size_t(T));
    cp(L.off_unit, 4 * size_t(T));
    cp(L.off_nhits, 4 * size_t(T));
    cp(L.off_nfit, 4 * size_t(T));
    cp(L.off_first, 4 * size_t(T));
    cp(L.off_hits, 4 * size_t(H));
    (void)hipEventRecord(s.ev_copy, s.stream);
    b->phase = 1;
    return true;
  }
  if (hipEventQuery(s.ev_copy) != hipSuccess) return false;
  // each request's slice of the packed results (tracks are in unit order)
  const int64_t *hh = static_cast<const int64_t *>(b->out->h_head);
  const int64_t T = hh[0], H = hh[1];
  const char *ho = static_cast<const char *>(b->out->h_out);
  const size_t N = size_t(b->n);
  const int32_t *ct = reinterpret_cast<const int32_t *>(ho);
  const float *par = reinterpret_cast<const float *>(ho + 4 * N);
  const float *cov = par + 5 * T;
  const float *xr = cov + 15 * T;
  const float *c2 = xr + T;
  const int32_t *un = reinterpret_cast<const int32_t *>(c2 + T);
  const int32_t *nh = un + T;
  const int32_t *nf = nh + T;
  const int32_t *fh = nf + T;
  const int32_t *hits = fh + T;
  const size_t R = b->reqs.size();
  for (size_t i = 0; i < R; ++i) {
    Request *r = b->reqs[i];
    const int64_t t0 = R > 1 ? hh[8 + 2 * i] : 0, t1 = R > 1 ? hh[8 + 2 * i + 2] : T;
    const int64_t h0 = R > 1 ? hh[8 + 2 * i + 1] : 0, h1 = R > 1 ? hh[8 + 2 * i + 3] : H;
    r->n_tracks = t1 - t0;
    r->n_track_hits = h1 - h0;
    r->b_ct = ct + b->cluster_base[i];
    r->b_params = par + 5 * t0;
    r->b_cov = cov + 15 * t0;
    r->b_xref = xr + t0;
    r->b_chi2 = c2 + t0;
    r->b_unit = un + t0;
    r->b_nhits = nh + t0;
    r->b_nfit = nf + t0;
    r->b_first = fh + t0;
    r->b_hits = hits + h0;
    r->out = b->out;
    r->status = TPC_OK;
  }
  finish(b);
  return true;
}

void tpc_server::finish(Batch *b) {
  const double t = now_s();
  pinned.put(b->h_offsets);
  b->out.reset();
  std::lock_guard<std::mutex> g(mu);
  for (Request *r : b->reqs) {
    pinned.put(r->staging);
    r->staging = nullptr;
    r->t_done = t;
    r->state = Request::DONE;
    ++st.completed;
  }
  arena.release(b->arena_off, b->L.total);
  slots[b->slot].batch = nullptr;
  delete b;
  cv_done.notify_all();
}

void tpc_server::requeue_solo(Batch *b) {
  pinned.put(b->h_offsets);
  b->out.reset();
  std::lock_guard<std::mutex> g(mu);
  for (auto it = b->reqs.rbegin(); it != b->reqs.rend(); ++it) {
    Request *r = *it;
    r->solo = true;
    r->state = Request::PENDING;
    r->batch_id = -1;
    pending.push_front(r);
  }
  arena.release(b->arena_off, b->L.total);
  slots[b->slot].batch = nullptr;
  delete b;
}

void tpc_server::loop() {
  (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool did = false;
    // progress in-flight batches (HIP queries and copies without the lock)
    lk.unlock();
    for (Slot &s : slots) did |= progress_slot(s);
    lk.lock();
    while (form_and_launch()) did = true;
    bool busy = !pending.empty();
    for (Slot &s : slots) busy |= s.batch != nullptr;
    if (stop && !busy) break;
    if (!did) cv_work.wait_for(lk, std::chrono::microseconds(busy ? 20 : 2000));
  }
}

extern "C" size_t tpc_server_footprint(int64_t n, int32_t n_units, int32_t n_rows, const tpc_params_t *p) {
  if (!p) return 0;
  OutLayout L{};
  if (!batch_layout(n, n_units, 1, n_rows, *p, &L)) return 0;
  return L.total;
}

extern "C" int tpc_server_create(const tpc_server_config_t *cfg, tpc_server_t **out) {
  if (!cfg || !out || cfg->budget_bytes == 0 || cfg->max_in_flight < 1 || cfg->max_in_flight > 8 ||
      cfg->queue_depth < 1 || cfg->n_rows < 3 || cfg->n_rows > 255 || !cfg->row_x)
    return TPC_E_INVALID;
  if (tpc_workspace_size(1, 1, cfg->n_rows, &cfg->params) == 0) return TPC_E_INVALID;
  std::unique_ptr<tpc_server> s(new tpc_server);
  s->cfg = *cfg;
  s->row_x.assign(cfg->row_x, cfg->row_x + cfg->n_rows);
  s->cfg.row_x = s->row_x.data();
  if (hipSetDevice(cfg->device) != hipSuccess) return TPC_E_HIP;
  if (hipMalloc(&s->d_arena, cfg->budget_bytes) != hipSuccess) return TPC_E_NOMEM;
  if (hipMalloc(&s->d_row_x, sizeof(float) * cfg->n_rows) != hipSuccess) {
    (void)hipFree(s->d_arena);
    return TPC_E_NOMEM;
  }
  (void)hipMemcpy(s->d_row_x, s->row_x.data(), sizeof(float) * cfg->n_rows, hipMemcpyHostToDevice);
  s->arena.init(cfg->budget_bytes);
  s->slots.resize(size_t(cfg->max_in_flight));
  for (Slot &sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev_kernel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev_copy, hipEventDisableTiming) != hipSuccess) {
      for (Slot &q : s->slots) {  // undo what was made
        if (q.ev_copy) (void)hipEventDestroy(q.ev_copy);
        if (q.ev_kernel) (void)hipEventDestroy(q.ev_kernel);
        if (q.stream) (void)hipStreamDestroy(q.stream);
      }
      (void)hipFree(s->d_row_x);
      (void)hipFree(s->d_arena);
      return TPC_E_HIP;
    }
  }
  s->st.arena_bytes = cfg->budget_bytes;
  tpc_server *raw = s.release();
  raw->th = std::thread([raw] { raw->loop(); });
  *out = raw;
  return TPC_OK;
}

extern "C" int tpc_server_submit(tpc_server_t *s, const tpc_request_t *r, uint64_t *ticket) {
  if (!s || !r || !ticket) return TPC_E_INVALID;
  if (!validate_request(r, s->cfg.n_rows)) {
    std::lock_guard<std::mutex> g(s->mu);
    ++s->st.rejected_invalid;
    return TPC_E_INVALID;
  }
  OutLayout L{};
  if (!batch_layout(r->n, r->n_units, 1, s->cfg.n_rows, s->cfg.params, &L) || L.total > s->arena.size()) {
    std::lock_guard<std::mutex> g(s->mu);
    ++s->st.rejected_nomem;
    return TPC_E_NOMEM;
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (int32_t(s->pending.size()) >= s->cfg.queue_depth) {
      ++s->st.rejected_busy;
      return TPC_E_BUSY;
    }
  }
  std::unique_ptr<Request> q(new Request);
  q->n = r->n;
  q->n_units = r->n_units;
  q->offsets.assign(r->unit_offsets, r->unit_offsets + r->n_units + 1);
  q->footprint = L.total;
  q->flags = r->flags;
  if (r->flags == TPC_REQ_COPY) {
    q->staging = s->pinned.get(10 * size_t(r->n) + 16);
    if (!q->staging) return TPC_E_NOMEM;
    char *st = static_cast<char *>(q->staging);
    if (r->n) {
      memcpy(st, r->y, 4 * size_t(r->n));
      memcpy(st + 4 * size_t(r->n), r->z, 4 * size_t(r->n));
      memcpy(st + 8 * size_t(r->n), r->row, 2 * size_t(r->n));
    }
    q->src_y = reinterpret_cast<const float *>(st);
    q->src_z = reinterpret_cast<const float *>(st + 4 * size_t(r->n));
    q->src_row = reinterpret_cast<const uint16_t *>(st + 8 * size_t(r->n));
  } else {
    q->src_y = r->y;
    q->src_z = r->z;
    q->src_row = r->row;
  }
  std::lock_guard<std::mutex> g(s->mu);
  q->ticket = s->next_ticket++;
  q->t_submit = now_s();
  *ticket = q->ticket;
  s->pending.push_back(q.get());
  s->reqs[q->ticket] = std::move(q);
  ++s->st.submitted;
  s->cv_work.notify_one();
  return TPC_OK;
}

extern "C" int tpc_server_poll(tpc_server_t *s, uint64_t ticket, tpc_result_t *res, int64_t wait_us) {
  if (!s || !res) return TPC_E_INVALID;
  Request *r = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return TPC_E_INVALID;
    r = it->second.get();
    if (r->state != Request::DONE) {
      if (wait_us == 0) return TPC_E_BUSY;
      auto done = [r] { return r->state == Request::DONE; };
      if (wait_us < 0) s->cv_done.wait(lk, done);
      else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), done)) return TPC_E_BUSY;
    }
  }
  // a done request is only erased by tpc_server_release, which the caller
  // does not run concurrently with a poll of the same ticket
  memset(res, 0, sizeof(*res));
  res->status = r->status;
  res->n = r->n;
  res->t_submit = r->t_submit;
  res->t_admit = r->t_admit;
  res->t_done = r->t_done;
  res->batch_id = r->batch_id;
  res->batch_requests = r->batch_requests;
  if (r->status != TPC_OK) return TPC_OK;
  res->n_tracks = r->n_tracks;
  res->n_track_hits = r->n_track_hits;
  res->params = r->b_params;
  res->cov = r->b_cov;
  res->x_ref = r->b_xref;
  res->chi2 = r->b_chi2;
  res->n_hits = r->b_nhits;
  res->n_fit = r->b_nfit;
  res->cluster_track = r->b_ct;
  res->unit = r->b_unit;
  res->first_hit = r->b_first;
  res->hits = r->b_hits;
  return TPC_OK;
}

extern "C" int tpc_server_release(tpc_server_t *s, uint64_t ticket) {
  if (!s) return TPC_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state != Request::DONE) return TPC_E_INVALID;
  s->reqs.erase(it);
  return TPC_OK;
}

extern "C" int tpc_server_stats(tpc_server_t *s, tpc_server_stats_t *out) {
  if (!s || !out) return TPC_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  out->pending = int32_t(s->pending.size());
  int32_t fl = 0;
  for (Slot &sl : s->slots) fl += sl.batch != nullptr;
  out->in_flight = fl;
  out->arena_used = s->arena.used();
  out->arena_peak = s->arena.peak();
  out->host_cpu_s = 0.0;
  clockid_t cid;
  struct timespec ts;
  if (pthread_getcpuclockid(s->th.native_handle(), &cid) == 0 && clock_gettime(cid, &ts) == 0)
    out->host_cpu_s = double(ts.tv_sec) + 1e-9 * double(ts.tv_nsec);
  return TPC_OK;
}

extern "C" int tpc_server_destroy(tpc_server_t *s) {
  if (!s) return TPC_E_INVALID;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ev_kernel) (void)hipEventDestroy(sl.ev_kernel);
    if (sl.ev_copy) (void)hipEventDestroy(sl.ev_copy);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto &kv : s->reqs)
    if (kv.second->staging) s->pinned.put(kv.second->staging);
  s->reqs.clear();
  s->pinned.clear();
  (void)hipFree(s->d_arena);
  (void)hipFree(s->d_row_x);
  delete s;
  return TPC_OK;
}
