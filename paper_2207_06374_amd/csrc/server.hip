// Serving form: a stream of solve requests served by continuous batching on
// one GPU, entirely in the library.
//
// A request (N, d, seed, target, step cap) is queued on submission.  One
// engine thread owns a HIP stream and a table of admitted requests in device
// memory: each admitted request has a row holding every argument record of
// its step (frame, radius, step counter and workspace live in its range of
// the caller's pool).  Per step the engine launches each kernel of the
// BF16-screen step once per group of admitted requests with the same d and
// screen tile form (the request is a grid dimension; each block reads its
// request's record), so one launch sequence advances every request in
// flight, each with exactly the arithmetic of its own single-search step;
// the groups run on streams of their own (forked from the engine's stream
// and joined back), so their launches overlap.  After every `chunk` steps
// one small kernel gathers every request's flags, step and coherence for a
// single read-back; finished requests leave the table, and the queue's head
// requests are admitted into the free rows as long as their footprint
// (workspace, frame, state scalars) fits in the pool.  First in line is
// served first: a request that does not fit yet holds the ones behind it, so
// none is overtaken forever.  A request larger than the whole pool is
// rejected at submission.  While the admitted set stays the same, a chunk of
// steps is captured once into a HIP graph and replayed.
//
// Every result is a pure function of the request (its own seed and stream
// id): the same alone, in any mix, and as trstmi_solve gives it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
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

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

// Device table at the start of the caller's pool: [rows][StepArgs] | lists
// (the groups' rows back to back, then every admitted row) | poll records.
uint64_t table_bytes(int32_t rows) {
  return align256((uint64_t)rows * sizeof(trstmi::StepArgs)) + align256((uint64_t)2 * rows * sizeof(int32_t)) +
         align256((uint64_t)rows * sizeof(trstmi::PollRecord));
}

// An admitted request in the engine.
struct Running {
  int64_t id;
  trstmi_params params;
  trstmi_state st;
  int32_t row;
};

constexpr int kGroupStreams = 4;  // streams the groups' launches are spread over

// Admitted requests of one d and one screen form, launched together.
struct Group {
  int32_t d;
  int32_t form;
  int32_t lane;               // group stream it runs on
  double work;                // algorithmic screen flops per step (for the stream assignment)
  int32_t first, count;       // their rows in the list region
  trstmi::PerturbArgs shape_pa, shape_pr, shape_pc;  // launch shapes (largest n)
  int32_t ldk16;
  int32_t gram_grid, recheck_grid;
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
  trstmi::PoolAllocator pool;  // over the pool past the table
  char* pool_base = nullptr;   // first byte past the table
  std::thread engine;
  int32_t active = 0;
  int64_t next_id = 0;

  // engine thread only
  hipStream_t stream = nullptr;
  hipStream_t gstream[kGroupStreams] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kGroupStreams] = {};
  char* tab_dev = nullptr;
  int32_t* list_dev = nullptr;
  trstmi::PollRecord* poll_dev = nullptr;
  std::vector<trstmi::StepArgs> tab_host;
  std::vector<int32_t> list_host;
  std::vector<trstmi::PollRecord> poll_host;
  std::vector<int32_t> free_rows;
  std::map<int32_t, Running> running;  // by row
  std::vector<Group> groups;
  hipGraphExec_t graph = nullptr;
  int stable_chunks = 0;

  void work();
  trstmi_status admit(Running& r);
  trstmi_status rebuild();
  trstmi_status launch_steps(int steps);
  trstmi_status run_chunk();
  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    stable_chunks = 0;
  }
};

// The Haar start of a newly admitted request and its row of the table.
trstmi_status trstmi_server::admit(Running& r) {
  const size_t ws_bytes = trstmi::PoolAllocator::round(trstmi_workspace_bytes(&r.params));
  char* base = (char*)r.st.frame - ws_bytes;
  trstmi_status e = trstmi_init_haar(&r.params, &r.st, base, ws_bytes, stream);
  if (e != TRSTMI_OK) return e;
  tab_host[r.row] = trstmi::bf16_step_args(&r.params, &r.st, base, nullptr, nullptr);
  return TRSTMI_OK;
}

// Groups by d, the list region and the table rows, uploaded in stream order.
trstmi_status trstmi_server::rebuild() {
  drop_graph();
  groups.clear();
  std::map<std::pair<int32_t, int32_t>, std::vector<int32_t>> by_d;
  for (auto& kv : running) by_d[{(int32_t)kv.second.params.d, tab_host[kv.first].g.form}].push_back(kv.first);
  list_host.clear();
  for (auto& kv : by_d) {
    Group g{};
    g.d = kv.first.first;
    g.form = kv.first.second;
    g.first = (int32_t)list_host.size();
    g.count = (int32_t)kv.second.size();
    int64_t n_max = 0;
    for (int32_t row : kv.second) {
      const trstmi::StepArgs& A = tab_host[row];
      list_host.push_back(row);
      if (A.pa.n > n_max) {
        n_max = A.pa.n;
        g.shape_pa = A.pa;
        g.shape_pr = A.pr;
        g.shape_pc = A.pc;
      }
      const int gg = (int)((long)A.g.nseg * ((A.g.slots + 7) / 8 * 8));
      g.gram_grid = std::max(g.gram_grid, gg);
      g.recheck_grid = std::max(g.recheck_grid, trstmi::recheck_grid(A.ra.list_cap));
      g.ldk16 = A.ra.ldk16;
    }
    // one step's recheck items of a request are few (its listed tiles); the
    // grid-stride loop covers them with fewer blocks per request in a group
    g.recheck_grid = std::min(g.recheck_grid, std::max(256, 8192 / g.count));
    for (int32_t row : kv.second) {
      const double n = (double)tab_host[row].pa.n;
      g.work += 4.0 * g.d * n * (n - 1.0) * p.candidates;
    }
    groups.push_back(g);
  }
  // largest groups first, each to the stream with the least work so far
  std::vector<int> order(groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return groups[x].work > groups[y].work; });
  double load[kGroupStreams] = {};
  for (int i : order) {
    int best = 0;
    for (int q = 1; q < kGroupStreams; ++q)
      if (load[q] < load[best]) best = q;
    groups[i].lane = best;
    load[best] += groups[i].work;
  }
  const int32_t nall = (int32_t)list_host.size();
  for (auto& kv : running) list_host.push_back(kv.first);  // every admitted row, for the poll
  (void)nall;
  hipError_t e = hipMemcpyAsync(tab_dev, tab_host.data(), tab_host.size() * sizeof(trstmi::StepArgs),
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && !list_host.empty())
    e = hipMemcpyAsync(list_dev, list_host.data(), list_host.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host copies may change after this
  if (e != hipSuccess) return server_fail(TRSTMI_E_HIP, std::string("engine table: ") + hipGetErrorString(e));
  return TRSTMI_OK;
}

// One chunk of steps of every admitted request.  Each group of requests runs
// on one of the group streams (forked from the engine stream and joined back
// to it), its steps in each request's own kernel order: candidates, screen,
// top-k, regeneration, recheck, selection, commit.  Groups are independent,
// so the small groups' launches overlap the large ones' instead of waiting
// behind them.
trstmi_status trstmi_server::launch_steps(int steps) {
  const size_t S = sizeof(trstmi::StepArgs);
  bool used[kGroupStreams] = {};
  for (const Group& g : groups) used[g.lane] = true;
  hipError_t e = hipEventRecord(fork_ev, stream);
  for (int q = 0; q < kGroupStreams && e == hipSuccess; ++q)
    if (used[q]) e = hipStreamWaitEvent(gstream[q], fork_ev, 0);
  for (int i = 0; i < steps && e == hipSuccess; ++i)
    for (const Group& g : groups) {
      hipStream_t gs = gstream[g.lane];
      auto ref = [&](size_t member) {
        return trstmi::TabRef{tab_dev + member, S, list_dev + g.first, g.count};
      };
      if (e == hipSuccess) e = trstmi::launch_perturb_tab(ref(offsetof(trstmi::StepArgs, pa)), g.shape_pa, p.candidates, gs);
      if (e == hipSuccess)
        e = trstmi::launch_gram_bf16_tab(ref(offsetof(trstmi::StepArgs, g)), g.ldk16, g.form, g.gram_grid, gs);
      if (e == hipSuccess) e = trstmi::launch_topk_tab(ref(offsetof(trstmi::StepArgs, ta)), gs);
      if (e == hipSuccess) e = trstmi::launch_perturb_tab(ref(offsetof(trstmi::StepArgs, pr)), g.shape_pr, p.recheck_topk, gs);
      if (e == hipSuccess) e = trstmi::launch_recheck_tab(ref(offsetof(trstmi::StepArgs, ra)), g.ldk16, g.recheck_grid, gs);
      if (e == hipSuccess) e = trstmi::launch_select_tab(ref(offsetof(trstmi::StepArgs, sa)), gs);
      if (e == hipSuccess) e = trstmi::launch_perturb_tab(ref(offsetof(trstmi::StepArgs, pc)), g.shape_pc, 1, gs);
    }
  for (int q = 0; q < kGroupStreams && e == hipSuccess; ++q)
    if (used[q]) {
      e = hipEventRecord(join_ev[q], gstream[q]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, join_ev[q], 0);
    }
  if (e != hipSuccess) return server_fail(TRSTMI_E_HIP, std::string("engine step: ") + hipGetErrorString(e));
  return TRSTMI_OK;
}

// One chunk of steps for every admitted request: replayed from a captured
// graph once the admitted set has been stable for a chunk, else launched
// directly (capture failure falls back to direct launches).
trstmi_status trstmi_server::run_chunk() {
  if (!graph && stable_chunks >= 1) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
      const trstmi_status cst = launch_steps(p.chunk);
      const hipError_t e2 = hipStreamEndCapture(stream, &g);
      if (cst != TRSTMI_OK || e2 != hipSuccess || !g || hipGraphInstantiate(&graph, g, nullptr, nullptr, 0) != hipSuccess)
        graph = nullptr;
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
    }
  }
  if (graph) {
    const hipError_t e = hipGraphLaunch(graph, stream);
    if (e != hipSuccess) return server_fail(TRSTMI_E_HIP, std::string("engine graph: ") + hipGetErrorString(e));
  } else {
    const trstmi_status st = launch_steps(p.chunk);
    if (st != TRSTMI_OK) return st;
  }
  ++stable_chunks;
  return TRSTMI_OK;
}

void trstmi_server::work() {
  hipError_t he = hipSetDevice(device);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  for (int q = 0; q < kGroupStreams && he == hipSuccess; ++q) {
    he = hipStreamCreateWithFlags(&gstream[q], hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&join_ev[q], hipEventDisableTiming);
  }
  if (he == hipSuccess) he = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming);
  std::string engine_error = he == hipSuccess ? "" : std::string("engine stream: ") + hipGetErrorString(he);
  for (;;) {
    // admission: the queue's head while a row is free and its footprint fits
    std::vector<Running> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        while (!queue.empty() && !free_rows.empty()) {
          Record& head = recs[queue.front()];
          uint64_t off = 0;
          if (!engine_error.empty()) {
            head.status = TRSTMI_REQ_ERROR;
            head.error = engine_error;
            head.t_admit = head.t_finish = Clock::now();
            queue.pop_front();
            continue;
          }
          if (!pool.alloc(head.size, &off)) break;
          head.offset = off;
          head.status = TRSTMI_REQ_RUNNING;
          head.t_admit = Clock::now();
          ++active;
          Running r{};
          r.id = queue.front();
          r.params = head.params;
          char* base = pool_base + off;
          const size_t ws_bytes = trstmi::PoolAllocator::round(trstmi_workspace_bytes(&head.params));
          const size_t fr_bytes = trstmi::PoolAllocator::round((uint64_t)16 * head.params.n * head.params.d);
          char* sc = base + ws_bytes + fr_bytes;
          r.st = trstmi_state{(double*)(base + ws_bytes), (double*)sc, (double*)(sc + 8), (int64_t*)(sc + 16),
                              (int32_t*)(sc + 24)};
          r.row = free_rows.back();
          free_rows.pop_back();
          queue.pop_front();
          admitted.push_back(r);
        }
        if (!admitted.empty() || !running.empty()) break;
        if (stop && queue.empty()) break;
        cv.wait(lk);
      }
      if (admitted.empty() && running.empty()) break;  // stopping, nothing left
    }
    cv.notify_all();

    // Haar starts and table rows of the new requests
    std::vector<std::pair<int64_t, std::string>> failed;
    for (Running& r : admitted) {
      const trstmi_status e = engine_error.empty() ? admit(r) : TRSTMI_E_HIP;
      if (e != TRSTMI_OK) {
        failed.emplace_back(r.id, engine_error.empty() ? std::string(trstmi_last_error()) : engine_error);
        std::lock_guard<std::mutex> lk(mu);
        free_rows.push_back(r.row);
        continue;
      }
      running[r.row] = r;
    }
    trstmi_status st = TRSTMI_OK;
    if (!admitted.empty()) st = rebuild();
    if (st == TRSTMI_OK && !running.empty()) st = run_chunk();
    // one read-back of every admitted request's state
    const int32_t nrun = (int32_t)running.size();
    if (st == TRSTMI_OK && nrun > 0) {
      const trstmi::TabRef all{tab_dev + offsetof(trstmi::StepArgs, sa), sizeof(trstmi::StepArgs),
                               list_dev + (list_host.size() - nrun), nrun};
      hipError_t e = trstmi::launch_poll_tab(all, poll_dev, stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(poll_host.data(), poll_dev, nrun * sizeof(trstmi::PollRecord), hipMemcpyDeviceToHost,
                           stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) st = server_fail(TRSTMI_E_HIP, std::string("engine poll: ") + hipGetErrorString(e));
    }
    if (st != TRSTMI_OK && engine_error.empty()) engine_error = trstmi_last_error();

    // finished (or, after an engine error, every) request leaves the table
    std::vector<int32_t> leaving;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto& f : failed) {
        Record& w = recs[f.first];
        w.status = TRSTMI_REQ_ERROR;
        w.error = f.second;
        w.t_finish = Clock::now();
        pool.release(w.offset, w.size);
        --active;
      }
      int32_t i = 0;
      for (auto& kv : running) {
        const trstmi::PollRecord& pr = poll_host[i++];
        const bool done = st == TRSTMI_OK && (pr.flags & TRSTMI_FLAG_DONE);
        if (!done && st == TRSTMI_OK) continue;
        Record& w = recs[kv.second.id];
        if (done) {
          w.status = TRSTMI_REQ_DONE;
          w.mu = pr.mu;
          w.steps = pr.step;
        } else {
          w.status = TRSTMI_REQ_ERROR;
          w.error = engine_error;
        }
        w.t_finish = Clock::now();
        pool.release(w.offset, w.size);
        --active;
        leaving.push_back(kv.first);
      }
      for (int32_t row : leaving) free_rows.push_back(row);
    }
    if (!leaving.empty()) {
      for (int32_t row : leaving) running.erase(row);
      drop_graph();
      if (!running.empty() && rebuild() != TRSTMI_OK && engine_error.empty()) engine_error = trstmi_last_error();
    }
    if (!failed.empty() || !leaving.empty()) cv.notify_all();
  }
  drop_graph();
  for (int q = 0; q < kGroupStreams; ++q) {
    if (gstream[q]) (void)hipStreamDestroy(gstream[q]);
    if (join_ev[q]) (void)hipEventDestroy(join_ev[q]);
  }
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  if (stream) (void)hipStreamDestroy(stream);
}

extern "C" {

size_t trstmi_request_footprint(const trstmi_params* p) { return p ? footprint_of(p) : 0; }

size_t trstmi_server_table_bytes(int32_t slots) { return slots >= 1 && slots <= 1024 ? table_bytes(slots) : 0; }

double trstmi_welch_bound(int64_t n, int64_t d) {
  if (n < 2 || d < 1) return NAN;
  return n > d ? std::sqrt(((double)n - (double)d) / ((double)d * ((double)n - 1.0))) : 0.0;
}

trstmi_status trstmi_server_create(const trstmi_server_params* p, trstmi_server** out) {
  if (!p || !out) return server_fail(TRSTMI_E_INVALID_ARG, "params and out must be host pointers");
  if (p->slots < 1 || p->slots > 1024) return server_fail(TRSTMI_E_INVALID_ARG, "slots must be in [1, 1024]");
  if (!p->pool || ((uintptr_t)p->pool & 255) || p->pool_bytes < table_bytes(p->slots) + 256)
    return server_fail(TRSTMI_E_INVALID_ARG, "pool: null, not 256-byte aligned, or not larger than the engine table (" +
                                                 std::to_string(table_bytes(p->slots)) + " bytes for these slots)");
  if (p->chunk < 1) return server_fail(TRSTMI_E_INVALID_ARG, "chunk must be >= 1");
  if (p->candidates < 1 || p->recheck_topk < 1 || !(p->radius0 > 0.0) || !(p->target_factor >= 0.0))
    return server_fail(TRSTMI_E_INVALID_ARG, "candidates, recheck_topk, radius0 or target_factor out of range");
  if (p->mode != TRSTMI_MODE_BF16_SCREEN)
    return server_fail(TRSTMI_E_UNSUPPORTED, "the serving engine runs the BF16-screen form (TRSTMI_MODE_BF16_SCREEN)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return server_fail(TRSTMI_E_HIP, std::string("device: ") + hipGetErrorString(e));
  trstmi_server* s = new trstmi_server;
  s->p = *p;
  s->device = dev;
  const uint64_t tb = table_bytes(p->slots);
  char* base = (char*)p->pool;
  s->tab_dev = base;
  s->list_dev = (int32_t*)(base + align256((uint64_t)p->slots * sizeof(trstmi::StepArgs)));
  s->poll_dev = (trstmi::PollRecord*)((char*)s->list_dev + align256((uint64_t)2 * p->slots * sizeof(int32_t)));
  s->pool_base = base + tb;
  s->pool.reset(p->pool_bytes - tb);
  s->tab_host.assign(p->slots, trstmi::StepArgs{});
  s->poll_host.assign(p->slots, trstmi::PollRecord{});
  for (int32_t r = p->slots - 1; r >= 0; --r) s->free_rows.push_back(r);
  s->engine = std::thread([s]() { s->work(); });
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
  const double welch = trstmi_welch_bound(rq->n, rq->d);
  r.params.target_mu = std::isnan(rq->target_mu) ? s->p.target_factor * (std::isnan(welch) ? 0.0 : welch)
                                                 : rq->target_mu;
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
  s->engine.join();
  delete s;
  return TRSTMI_OK;
}

}  // extern "C"
