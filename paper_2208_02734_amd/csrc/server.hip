// Serving loop: continuous batching of k-NN requests against a resident
// index.
//
// Requests (host query rows + their k and r) are queued by mask_server_submit.
// One scheduler thread admits them in arrival order into ragged batches: a
// batch takes requests while they fit both the batch-size limit and a free
// block of the device arena (memory admission), packs their rows, per-query
// k, r and output offsets into pinned staging memory at the same offset as
// the arena block, copies them to the device, runs the ragged descent and
// copies the results back, all on one of n_streams streams.  Up to n_streams
// batches are in flight at once; requests that arrive meanwhile wait for a
// stream and for arena space.  With a batching window, a batch that is not
// full waits until its oldest request has been queued for the window, so
// that requests arriving close together share one launch.  A finished batch (its event completed) hands
// every request its rows and the completion time and returns its arena block.
// Each query's result is the same alone or in any batch (the descent runs one
// query per workgroup).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace mask {
namespace {

double now_seconds() {
  using clock = std::chrono::steady_clock;
  return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing of freed blocks.
class RangeAllocator {
 public:
  explicit RangeAllocator(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  int n_q = 0, k = 0, r = 0;
  std::vector<float> q;  // n_q x dim
  std::vector<int32_t> ids;
  std::vector<float> dist;
  double t_arrival = 0, t_done = 0;
  double t_submit = 0;  // steady clock at submission (batching window)
  int state = 0;  // 0 queued, 1 on the device, 2 done
};

// Layout of one batch inside its arena block (device) and the same offsets of
// the pinned staging buffer (host).
struct BatchLayout {
  size_t q_off, k_off, r_off, o_off, id_off, d_off, bytes;
};

BatchLayout layout_for(int64_t n_q, int64_t n_out, int ld) {
  BatchLayout L{};
  size_t p = 0;
  L.q_off = p; p = align256(p + (size_t)n_q * ld * sizeof(float));
  L.k_off = p; p = align256(p + (size_t)n_q * sizeof(int32_t));
  L.r_off = p; p = align256(p + (size_t)n_q * sizeof(int32_t));
  L.o_off = p; p = align256(p + (size_t)n_q * sizeof(int64_t));
  L.id_off = p; p = align256(p + (size_t)n_out * sizeof(int32_t));
  L.d_off = p; p = align256(p + (size_t)n_out * sizeof(float));
  L.bytes = p;
  return L;
}

struct Batch {
  std::vector<Request*> reqs;
  size_t off = 0;
  BatchLayout L{};
  int64_t n_q = 0, n_out = 0;
  int stream = 0;
  hipEvent_t done = nullptr;
};

}  // namespace
}  // namespace mask

struct mask_server {
  const mask_index* ix = nullptr;
  mask_server_params p{};
  bool profile = false;  // p.beam_eighths sets per-level beams
  mask::Arena mem;
  char* dev = nullptr;   // device arena
  char* host = nullptr;  // pinned staging, same offsets
  mask::RangeAllocator* ranges = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<bool> stream_busy;
  std::vector<hipEvent_t> events;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<mask::Request*> queue;
  int64_t queued_queries = 0;
  std::unordered_map<uint64_t, mask::Request*> reqs;
  std::vector<mask::Batch> inflight;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string error;
  mask_server_stats st{};
  std::thread worker;
  explicit mask_server(const mask_allocator* a) : mem(a, nullptr) {}
};

namespace mask {
namespace {

// Everything below runs with s->mu held.
bool retire(mask_server* s) {
  bool any = false;
  for (size_t b = 0; b < s->inflight.size();) {
    Batch& B = s->inflight[b];
    const hipError_t e = hipEventQuery(B.done);
    if (e == hipErrorNotReady) { ++b; continue; }
    if (e != hipSuccess) s->error = std::string("batch failed: ") + hipGetErrorString(e);
    const double t = now_seconds();
    const int32_t* ids = reinterpret_cast<const int32_t*>(s->host + B.off + B.L.id_off);
    const float* dist = reinterpret_cast<const float*>(s->host + B.off + B.L.d_off);
    int64_t o = 0;
    for (Request* r : B.reqs) {
      const size_t n = (size_t)r->n_q * r->k;
      r->ids.assign(ids + o, ids + o + n);
      r->dist.assign(dist + o, dist + o + n);
      o += n;
      r->t_done = t;
      r->state = 2;
      s->st.completed_requests += 1;
      s->st.completed_queries += r->n_q;
    }
    s->ranges->release(B.off, B.L.bytes);
    s->stream_busy[B.stream] = false;
    s->inflight.erase(s->inflight.begin() + b);
    any = true;
  }
  return any;
}

// Seconds until the queued partial batch may launch (0: now).
double hold_time(const mask_server* s) {
  if (s->p.batch_window_us <= 0 || s->stop || s->queue.empty()) return 0.0;
  if (s->queued_queries >= s->p.max_batch_queries) return 0.0;
  const double ready = s->queue.front()->t_submit + 1e-6 * s->p.batch_window_us;
  const double now = now_seconds();
  return ready > now ? ready - now : 0.0;
}

bool launch_one(mask_server* s) {
  if (s->queue.empty()) return false;
  if (hold_time(s) > 0.0) return false;
  int stream = -1;
  for (size_t i = 0; i < s->stream_busy.size(); ++i)
    if (!s->stream_busy[i]) { stream = (int)i; break; }
  if (stream < 0) return false;
  const int ld = s->ix->ld, dim = s->ix->dim;
  // admit requests in arrival order while they fit the batch and the arena
  Batch B;
  int64_t nq = 0, nout = 0;
  size_t count = 0;
  for (Request* r : s->queue) {
    if (count > 0 && nq + r->n_q > s->p.max_batch_queries) break;
    const BatchLayout L = layout_for(nq + r->n_q, nout + (int64_t)r->n_q * r->k, ld);
    if (L.bytes > s->ranges->size() - s->ranges->used()) break;
    nq += r->n_q;
    nout += (int64_t)r->n_q * r->k;
    ++count;
  }
  if (count == 0) return false;
  B.L = layout_for(nq, nout, ld);
  size_t off = 0;
  while (!s->ranges->alloc(B.L.bytes, &off)) {
    // fragmentation: shrink the batch until its block fits
    if (count == 1) return false;
    Request* last = s->queue[count - 1];
    nq -= last->n_q;
    nout -= (int64_t)last->n_q * last->k;
    --count;
    B.L = layout_for(nq, nout, ld);
  }
  B.off = off;
  B.n_q = nq;
  B.n_out = nout;
  B.stream = stream;
  B.done = s->events[stream];
  char* h = s->host + off;
  float* hq = reinterpret_cast<float*>(h + B.L.q_off);
  int32_t* hk = reinterpret_cast<int32_t*>(h + B.L.k_off);
  int32_t* hr = reinterpret_cast<int32_t*>(h + B.L.r_off);
  int64_t* ho = reinterpret_cast<int64_t*>(h + B.L.o_off);
  int64_t qi = 0, o = 0;
  int32_t k_max = 1, r_max = 1;
  for (size_t i = 0; i < count; ++i) {
    Request* r = s->queue.front();
    s->queue.pop_front();
    s->queued_queries -= r->n_q;
    r->state = 1;
    B.reqs.push_back(r);
    for (int j = 0; j < r->n_q; ++j, ++qi) {
      std::memcpy(hq + qi * ld, r->q.data() + (size_t)j * dim, dim * sizeof(float));
      if (ld > dim) std::memset(hq + qi * ld + dim, 0, (ld - dim) * sizeof(float));
      hk[qi] = r->k;
      hr[qi] = r->r;
      ho[qi] = o;
      o += r->k;
    }
    k_max = std::max(k_max, r->k);
    r_max = std::max(r_max, r->r);
  }
  hipStream_t st = s->streams[stream];
  char* d = s->dev + off;
  MASK_HIP(hipMemcpyAsync(d, h, B.L.id_off, hipMemcpyHostToDevice, st));
  mask_matrix m{};
  m.layout = MASK_DENSE;
  m.n = nq;
  m.dim = dim;
  m.ld = ld;
  m.x = reinterpret_cast<const float*>(d + B.L.q_off);
  const mask_status rc = mask_query_ragged(
      s->ix, &m, reinterpret_cast<const int32_t*>(d + B.L.k_off),
      reinterpret_cast<const int32_t*>(d + B.L.r_off), reinterpret_cast<const int64_t*>(d + B.L.o_off),
      k_max, r_max, s->profile ? s->p.beam_eighths : nullptr,
      reinterpret_cast<int32_t*>(d + B.L.id_off),
      reinterpret_cast<float*>(d + B.L.d_off), st);
  if (rc != MASK_OK) throw Error{rc, std::string("ragged query: ") + mask_last_error()};
  MASK_HIP(hipMemcpyAsync(h + B.L.id_off, d + B.L.id_off, B.L.bytes - B.L.id_off,
                          hipMemcpyDeviceToHost, st));
  MASK_HIP(hipEventRecord(B.done, st));
  s->stream_busy[stream] = true;
  s->st.batches += 1;
  s->st.batched_queries += nq;
  s->st.peak_arena_bytes = (int64_t)s->ranges->peak();
  s->inflight.push_back(std::move(B));
  return true;
}

void worker_loop(mask_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = false;
    try {
      progress |= retire(s);
      while (launch_one(s)) progress = true;
    } catch (const Error& e) {
      s->error = e.msg;
    }
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (!progress) {
      double wait = s->inflight.empty() ? 2e-3 : 20e-6;
      const double hold = hold_time(s);
      if (hold > 0.0 && hold < wait) wait = hold;
      s->cv.wait_for(lk, std::chrono::duration<double>(wait));
    }
  }
}

mask_status fail_server(const Error& e) {
  set_error(e.msg);
  return e.status;
}

}  // namespace
}  // namespace mask

using namespace mask;

extern "C" {

double mask_clock(void) { return now_seconds(); }

mask_status mask_server_create(const mask_index* ix, const mask_server_params* p,
                               const mask_allocator* a, mask_server** out) {
  try {
    MASK_CHECK(ix && p && out, "NULL argument");
    if (ix->sparse) throw Error{MASK_ERR_UNSUPPORTED, "serving a CSR index"};
    MASK_CHECK(p->arena_bytes >= 4096, "arena_bytes too small");
    MASK_CHECK(p->max_batch_queries >= 1, "max_batch_queries < 1");
    MASK_CHECK(p->n_streams >= 1 && p->n_streams <= 16, "n_streams must be in [1, 16]");
    MASK_CHECK(p->batch_window_us >= 0 && p->batch_window_us <= 1000000,
               "batch_window_us must be in [0, 1e6]");
    *out = nullptr;
    auto s = std::make_unique<mask_server>(a);
    s->ix = ix;
    s->p = *p;
    for (int d = 0; d < MASK_MAX_LEVELS; ++d) {
      MASK_CHECK(p->beam_eighths[d] >= 0 && p->beam_eighths[d] <= 8 * kMaxBeam,
                 "beam_eighths out of range");
      s->profile = s->profile || (d < ix->n_levels && p->beam_eighths[d] > 0);
    }
    s->dev = static_cast<char*>(s->mem.alloc_bytes((size_t)p->arena_bytes));
    void* h = nullptr;
    MASK_HIP(hipHostMalloc(&h, (size_t)p->arena_bytes, hipHostMallocDefault));
    s->host = static_cast<char*>(h);
    s->ranges = new RangeAllocator((size_t)p->arena_bytes);
    for (int i = 0; i < p->n_streams; ++i) {
      hipStream_t st;
      MASK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->streams.push_back(st);
      hipEvent_t ev;
      MASK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      s->events.push_back(ev);
    }
    s->stream_busy.assign(p->n_streams, false);
    s->worker = std::thread(worker_loop, s.get());
    *out = s.release();
    return MASK_OK;
  } catch (const Error& e) {
    return fail_server(e);
  }
}

mask_status mask_server_submit(mask_server* s, const float* q_host, int32_t n_q, int32_t k,
                               int32_t r, double t_arrival, uint64_t* ticket) {
  try {
    MASK_CHECK(s && q_host && ticket, "NULL argument");
    MASK_CHECK(n_q >= 1, "n_q < 1");
    MASK_CHECK(k >= 1 && k <= kMaxBeam && r >= 1 && r <= kMaxBeam, "k or r out of range");
    if (s->profile)
      for (int d = 0; d < s->ix->n_levels; ++d)
        MASK_CHECK(((int64_t)r * s->p.beam_eighths[d] + 7) / 8 <= kMaxBeam,
                   "r too large for the server's beam profile");
    const BatchLayout L = layout_for(n_q, (int64_t)n_q * k, s->ix->ld);
    if (L.bytes > (size_t)s->p.arena_bytes || n_q > s->p.max_batch_queries)
      throw Error{MASK_ERR_BUSY, "request can never fit the arena or the batch limit"};
    auto* rq = new Request();
    rq->n_q = n_q;
    rq->k = k;
    rq->r = r;
    rq->t_arrival = t_arrival;
    rq->t_submit = now_seconds();
    rq->q.assign(q_host, q_host + (size_t)n_q * s->ix->dim);
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->stop) {
        delete rq;
        throw Error{MASK_ERR_SHUTDOWN, "server is shutting down"};
      }
      rq->ticket = s->next_ticket++;
      s->reqs[rq->ticket] = rq;
      s->queue.push_back(rq);
      s->queued_queries += n_q;
      s->st.submitted_requests += 1;
      s->st.submitted_queries += n_q;
      *ticket = rq->ticket;
    }
    s->cv.notify_one();
    return MASK_OK;
  } catch (const Error& e) {
    return fail_server(e);
  }
}

mask_status mask_server_poll(mask_server* s, uint64_t ticket, int32_t* done, int32_t* ids_host,
                             float* dist_host, double* t_done) {
  try {
    MASK_CHECK(s && done, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->error.empty()) throw Error{MASK_ERR_DEVICE, s->error};
    auto it = s->reqs.find(ticket);
    MASK_CHECK(it != s->reqs.end(), "unknown ticket");
    Request* r = it->second;
    *done = r->state == 2;
    if (!*done) return MASK_OK;
    if (ids_host) std::memcpy(ids_host, r->ids.data(), r->ids.size() * sizeof(int32_t));
    if (dist_host) std::memcpy(dist_host, r->dist.data(), r->dist.size() * sizeof(float));
    if (t_done) *t_done = r->t_done;
    s->reqs.erase(it);
    delete r;
    return MASK_OK;
  } catch (const Error& e) {
    return fail_server(e);
  }
}

mask_status mask_server_stats_get(mask_server* s, mask_server_stats* out) {
  if (!s || !out) {
    set_error("NULL argument");
    return MASK_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  out->queued_requests = (int64_t)s->queue.size();
  out->inflight_batches = (int64_t)s->inflight.size();
  out->arena_used_bytes = (int64_t)s->ranges->used();
  return MASK_OK;
}

mask_status mask_server_replay(mask_server* s, const float* pool_host, int64_t pool_rows,
                               int64_t n_req, const double* t_offset, const int32_t* n_q,
                               const int64_t* pool_off, const int32_t* k, const int32_t* r,
                               double* latency, double* span) {
  try {
    MASK_CHECK(s && pool_host && t_offset && n_q && pool_off && k && r && latency,
               "NULL argument");
    MASK_CHECK(n_req >= 0 && pool_rows >= 1, "bad sizes");
    const int dim = s->ix->dim;
    for (int64_t i = 0; i < n_req; ++i) {
      MASK_CHECK(n_q[i] >= 1 && pool_off[i] >= 0 && pool_off[i] + n_q[i] <= pool_rows,
                 "request rows outside the pool");
      MASK_CHECK(i == 0 || t_offset[i] >= t_offset[i - 1], "arrival times must not decrease");
    }
    struct Out { uint64_t ticket; int64_t i; double t_arr; };
    std::deque<Out> outstanding;
    const double t0 = now_seconds() + 1e-3;
    double t_last = t0;
    int64_t next = 0;
    auto drain = [&](bool all) {
      while (!outstanding.empty()) {
        const Out o = outstanding.front();
        int32_t done = 0;
        double td = 0;
        const mask_status st = mask_server_poll(s, o.ticket, &done, nullptr, nullptr, &td);
        if (st != MASK_OK) throw Error{st, mask_last_error()};
        if (!done) {
          if (!all) return;
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          continue;
        }
        latency[o.i] = td - o.t_arr;
        t_last = std::max(t_last, td);
        outstanding.pop_front();
      }
    };
    while (next < n_req) {
      const double ta = t0 + t_offset[next];
      if (now_seconds() < ta) {
        drain(false);
        if (now_seconds() + 50e-6 < ta) std::this_thread::sleep_for(std::chrono::microseconds(20));
        continue;
      }
      uint64_t ticket = 0;
      const mask_status st = mask_server_submit(
          s, pool_host + pool_off[next] * (int64_t)dim, n_q[next], k[next], r[next], ta, &ticket);
      if (st != MASK_OK) throw Error{st, mask_last_error()};
      outstanding.push_back({ticket, next, ta});
      ++next;
    }
    drain(true);
    if (span) *span = t_last - t0;
    return MASK_OK;
  } catch (const Error& e) {
    return fail_server(e);
  }
}

mask_status mask_server_destroy(mask_server* s) {
  if (!s) return MASK_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_one();
  if (s->worker.joinable()) s->worker.join();
  for (auto st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& kv : s->reqs) delete kv.second;
  for (auto ev : s->events) (void)hipEventDestroy(ev);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->host) (void)hipHostFree(s->host);
  delete s->ranges;
  delete s;
  return MASK_OK;
}

}  // extern "C"
