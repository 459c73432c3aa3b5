// Serving form: a stream of solve requests with continuous admission, on one
// GPU, entirely in the library.
//
// A request (N, d, seed, target, step cap) is queued on submission.  Slot
// threads (one per concurrent solve, each with a HIP stream of its own)
// take the request at the head of the queue as soon as its device
// footprint (workspace, frame, state scalars) fits in the caller's pool,
// run the Haar start and the solve (graph-captured chunks of steps, one done
// flag poll per chunk) on their stream, read μ and the step count back and
// release the range.  First in line is served first: a request that does
// not fit yet holds the ones behind it, so none is overtaken forever.  A
// request larger than the whole pool is rejected at submission.  Every
// result is a pure function of the request (its own seed and stream id), the
// same alone and in any mix.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/trstmi.h"
#include "launch.h"
#include "pool_alloc.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Record {
  trstmi_params params{};
  uint64_t size = 0;      // footprint in the pool
  uint64_t offset = 0;
  int32_t status = TRSTMI_REQ_QUEUED;
  double mu = NAN;
  int64_t steps = 0;
  Clock::time_point t_submit, t_admit, t_finish;
  std::string error;
};

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

uint64_t footprint_of(const trstmi_params* p) {
  const size_t ws = trstmi_workspace_bytes(p);
  if (ws == 0) return 0;
  return trstmi::PoolAllocator::round(ws) + trstmi::PoolAllocator::round((uint64_t)16 * p->n * p->d) + 256;
}

trstmi_status server_fail(trstmi_status st, const std::string& msg) { return trstmi::set_last_error(st, msg); }

// What a slot thread hands back for a finished request.
struct Outcome {
  int32_t status;
  double mu;
  int64_t steps;
  std::string error;
};

}  // namespace

struct trstmi_server {
  trstmi_server_params p{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<int64_t> queue;
  std::map<int64_t, Record> recs;
  trstmi::PoolAllocator pool;
  std::vector<std::thread> workers;
  int64_t next_id = 0;
  int32_t active = 0;

  void work();
  Outcome run_one(const Record& r, hipStream_t s);
};

// The Haar start and the solve of one admitted request in its pool range
// [workspace | frame | mu, radius, step, flags], on the slot's stream.  The
// record is only read here; the caller stores the outcome under the lock.
Outcome trstmi_server::run_one(const Record& r, hipStream_t s) {
  char* base = (char*)p.pool + r.offset;
  const size_t ws_bytes = trstmi::PoolAllocator::round(trstmi_workspace_bytes(&r.params));
  const size_t fr_bytes = trstmi::PoolAllocator::round((uint64_t)16 * r.params.n * r.params.d);
  char* sc = base + ws_bytes + fr_bytes;
  trstmi_state st{(double*)(base + ws_bytes), (double*)sc, (double*)(sc + 8), (int64_t*)(sc + 16),
                  (int32_t*)(sc + 24)};
  Outcome o{TRSTMI_REQ_DONE, NAN, 0, ""};
  trstmi_status e = trstmi_init_haar(&r.params, &st, base, ws_bytes, s);
  if (e == TRSTMI_OK) e = trstmi_solve(&r.params, &st, base, ws_bytes, p.chunk, s);
  if (e != TRSTMI_OK) {
    o.status = TRSTMI_REQ_ERROR;
    o.error = trstmi_last_error();
    return o;
  }
  hipError_t he = hipMemcpyAsync(&o.mu, st.mu, sizeof(double), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&o.steps, st.step, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    o.status = TRSTMI_REQ_ERROR;
    o.error = std::string("read result: ") + hipGetErrorString(he);
  }
  return o;
}

void trstmi_server::work() {
  hipStream_t s = nullptr;
  hipError_t he = hipSetDevice(device);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  for (;;) {
    int64_t id = -1;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stop) break;
        if (!queue.empty()) {
          Record& head = recs[queue.front()];
          uint64_t off = 0;
          if (pool.alloc(head.size, &off)) {
            id = queue.front();
            queue.pop_front();
            head.offset = off;
            head.status = TRSTMI_REQ_RUNNING;
            head.t_admit = Clock::now();
            ++active;
            break;
          }
        }
        cv.wait(lk);
      }
      if (id < 0) break;
    }
    const Record* r;
    {
      std::lock_guard<std::mutex> lk(mu);
      r = &recs[id];  // map nodes are stable, and nobody else writes a running record
    }
    Outcome o = he == hipSuccess ? run_one(*r, s)
                                 : Outcome{TRSTMI_REQ_ERROR, NAN, 0, std::string("slot stream: ") + hipGetErrorString(he)};
    {
      std::lock_guard<std::mutex> lk(mu);
      Record& w = recs[id];
      w.status = o.status;
      w.mu = o.mu;
      w.steps = o.steps;
      w.error = std::move(o.error);
      w.t_finish = Clock::now();
      pool.release(w.offset, w.size);
      --active;
    }
    cv.notify_all();
  }
  if (s) (void)hipStreamDestroy(s);
}

extern "C" {

size_t trstmi_request_footprint(const trstmi_params* p) { return p ? footprint_of(p) : 0; }

trstmi_status trstmi_server_create(const trstmi_server_params* p, trstmi_server** out) {
  if (!p || !out) return server_fail(TRSTMI_E_INVALID_ARG, "params and out must be host pointers");
  if (!p->pool || ((uintptr_t)p->pool & 255) || p->pool_bytes < 256)
    return server_fail(TRSTMI_E_INVALID_ARG, "pool: null, not 256-byte aligned, or smaller than 256 bytes");
  if (p->slots < 1 || p->slots > 64) return server_fail(TRSTMI_E_INVALID_ARG, "slots must be in [1, 64]");
  if (p->chunk < 1) return server_fail(TRSTMI_E_INVALID_ARG, "chunk must be >= 1");
  if (p->candidates < 1 || p->recheck_topk < 1 || !(p->radius0 > 0.0) || !(p->target_factor >= 0.0))
    return server_fail(TRSTMI_E_INVALID_ARG, "candidates, recheck_topk, radius0 or target_factor out of range");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return server_fail(TRSTMI_E_HIP, std::string("device: ") + hipGetErrorString(e));
  trstmi_server* s = new trstmi_server;
  s->p = *p;
  s->device = dev;
  s->pool.reset(p->pool_bytes);
  for (int32_t k = 0; k < p->slots; ++k) s->workers.emplace_back([s]() { s->work(); });
  *out = s;
  return TRSTMI_OK;
}

trstmi_status trstmi_server_submit(trstmi_server* s, const trstmi_request* rq, int64_t* id) {
  if (!s || !rq || !id) return server_fail(TRSTMI_E_INVALID_ARG, "server, request and id must be host pointers");
  Record r;
  trstmi_default_params(&r.params, rq->n, rq->d);
  r.params.candidates = s->p.candidates;
  r.params.mode = s->p.mode;
  r.params.recheck_topk = s->p.recheck_topk;
  r.params.seed = rq->seed;
  r.params.radius0 = s->p.radius0;
  r.params.max_steps = rq->max_steps;
  const double n = (double)rq->n, d = (double)rq->d;
  const double welch = rq->n > rq->d ? std::sqrt((n - d) / (d * (n - 1.0))) : 0.0;
  r.params.target_mu = std::isnan(rq->target_mu) ? s->p.target_factor * welch : rq->target_mu;
  r.t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return server_fail(TRSTMI_E_INVALID_ARG, "the server is shutting down");
  const int64_t k = s->next_id++;
  r.params.stream_id = rq->stream_id;
  r.size = footprint_of(&r.params);
  if (r.size == 0) {
    r.status = TRSTMI_REQ_REJECTED;
    r.error = "invalid request: need 2 <= n <= 262144, 1 <= d <= 512 (the BF16 screen: d <= 128), seed and "
              "stream_id below 2^32";
    r.t_admit = r.t_finish = r.t_submit;
  } else if (r.size > s->pool.capacity()) {
    r.status = TRSTMI_REQ_REJECTED;
    r.error = "footprint " + std::to_string(r.size) + " B exceeds the pool (" + std::to_string(s->pool.capacity()) +
              " B)";
    r.t_admit = r.t_finish = r.t_submit;
  }
  const bool queued = r.status == TRSTMI_REQ_QUEUED;
  s->recs.emplace(k, std::move(r));
  if (queued) s->queue.push_back(k);
  *id = k;
  s->cv.notify_all();
  return TRSTMI_OK;
}

static trstmi_status fill_result(trstmi_server* s, int64_t id, trstmi_request_result* out) {
  auto it = s->recs.find(id);
  if (it == s->recs.end()) return server_fail(TRSTMI_E_INVALID_ARG, "unknown request id");
  const Record& r = it->second;
  out->status = r.status;
  out->mu = r.mu;
  out->steps = r.steps;
  out->target_mu = r.params.target_mu;
  out->reached = r.status == TRSTMI_REQ_DONE && r.mu <= r.params.target_mu;
  const bool admitted = r.status == TRSTMI_REQ_RUNNING || r.status == TRSTMI_REQ_DONE || r.status == TRSTMI_REQ_ERROR;
  const bool finished = r.status >= TRSTMI_REQ_DONE;
  out->queue_s = admitted ? seconds(r.t_submit, r.t_admit) : NAN;
  out->run_s = (admitted && finished) ? seconds(r.t_admit, r.t_finish) : NAN;
  out->footprint = r.size;
  if (!r.error.empty()) trstmi::set_last_error(TRSTMI_OK, r.error);
  return TRSTMI_OK;
}

trstmi_status trstmi_server_poll(trstmi_server* s, int64_t id, trstmi_request_result* out) {
  if (!s || !out) return server_fail(TRSTMI_E_INVALID_ARG, "server and out must be host pointers");
  std::lock_guard<std::mutex> lk(s->mu);
  return fill_result(s, id, out);
}

trstmi_status trstmi_server_wait(trstmi_server* s, int64_t id, double timeout_s, trstmi_request_result* out) {
  if (!s || !out) return server_fail(TRSTMI_E_INVALID_ARG, "server and out must be host pointers");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->recs.find(id);
  if (it == s->recs.end()) return server_fail(TRSTMI_E_INVALID_ARG, "unknown request id");
  const bool forever = timeout_s < 0 || timeout_s > 1e9;  // (a deadline that far out would overflow)
  const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                        std::chrono::duration<double>(!forever && timeout_s > 0 ? timeout_s : 0.0));
  while (it->second.status < TRSTMI_REQ_DONE && (forever || Clock::now() < until)) {
    if (forever)
      s->cv.wait(lk);
    else
      s->cv.wait_until(lk, until);
    // another thread may have forgotten the record meanwhile: look it up again
    it = s->recs.find(id);
    if (it == s->recs.end()) return server_fail(TRSTMI_E_INVALID_ARG, "the request was forgotten while waiting");
  }
  return fill_result(s, id, out);
}

trstmi_status trstmi_server_cancel(trstmi_server* s, int64_t id) {
  if (!s) return server_fail(TRSTMI_E_INVALID_ARG, "server must be a host pointer");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->recs.find(id);
  if (it == s->recs.end()) return server_fail(TRSTMI_E_INVALID_ARG, "unknown request id");
  if (it->second.status != TRSTMI_REQ_QUEUED)
    return server_fail(TRSTMI_E_INVALID_ARG, "only a queued request can be cancelled");
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == id) {
      s->queue.erase(q);
      break;
    }
  it->second.status = TRSTMI_REQ_CANCELLED;
  it->second.t_admit = it->second.t_finish = Clock::now();
  s->cv.notify_all();
  return TRSTMI_OK;
}

trstmi_status trstmi_server_forget(trstmi_server* s, int64_t id) {
  if (!s) return server_fail(TRSTMI_E_INVALID_ARG, "server must be a host pointer");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->recs.find(id);
  if (it == s->recs.end()) return server_fail(TRSTMI_E_INVALID_ARG, "unknown request id");
  if (it->second.status < TRSTMI_REQ_DONE)
    return server_fail(TRSTMI_E_INVALID_ARG, "only a finished request can be forgotten");
  s->recs.erase(it);
  return TRSTMI_OK;
}

trstmi_status trstmi_server_get_stats(trstmi_server* s, trstmi_server_stats* out) {
  if (!s || !out) return server_fail(TRSTMI_E_INVALID_ARG, "server and out must be host pointers");
  std::lock_guard<std::mutex> lk(s->mu);
  out->pool_capacity = s->pool.capacity();
  out->pool_used = s->pool.used();
  out->pool_peak = s->pool.peak();
  out->active = s->active;
  out->queued = (int32_t)s->queue.size();
  out->submitted = s->next_id;
  return TRSTMI_OK;
}

trstmi_status trstmi_server_destroy(trstmi_server* s) {
  if (!s) return TRSTMI_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (int64_t id : s->queue) {
      s->recs[id].status = TRSTMI_REQ_CANCELLED;
      s->recs[id].t_admit = s->recs[id].t_finish = Clock::now();
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
  return TRSTMI_OK;
}

}  // extern "C"
