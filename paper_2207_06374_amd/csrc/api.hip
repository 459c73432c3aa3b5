// C ABI of the candidate-coherence library: argument validation, workspace
// layout, and the launch sequences of the random start, one step, and a solve.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/trstmi.h"
#include "launch.h"

using namespace trstmi;

namespace {

thread_local std::string g_last_error;

trstmi_status fail(trstmi_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

trstmi_status hip_fail(hipError_t e, const char* where) {
  return fail(TRSTMI_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define TRY_HIP(expr, where)                  \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// ---------------------------------------------------------------------------
// Kernel timing.  When enabled, every kernel launch of the library is
// bracketed by two HIP events recorded on the launch's own stream; reading
// the totals waits for those events and sums the elapsed times per kernel
// name.  Timing can be limited to one kernel name (each timed launch adds two
// event records to its stream).  Launches made while a stream is being
// captured into a graph are not timed.
// ---------------------------------------------------------------------------
struct TimingRecord {
  const char* name;
  hipEvent_t start, stop;
};

struct Timing {
  std::mutex mu;
  bool on = false;
  std::string only;  // empty: every kernel
  std::vector<TimingRecord> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, int64_t>> totals;  // name -> (ms, launches)

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Timing& timing() {
  static Timing t;
  return t;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Records a start event now and a stop event when finish() is called.
class TimedLaunch {
 public:
  TimedLaunch(const char* name, hipStream_t s) : name_(name), s_(s) {
    Timing& T = timing();
    std::lock_guard<std::mutex> g(T.mu);
    if (!T.on || (!T.only.empty() && T.only != name) || capturing(s)) return;
    start_ = T.get();
    stop_ = T.get();
    if (start_ && stop_ && hipEventRecord(start_, s) == hipSuccess) active_ = true;
  }
  hipError_t finish(hipError_t launch_status) {
    if (!active_) return launch_status;
    Timing& T = timing();
    std::lock_guard<std::mutex> g(T.mu);
    if (hipEventRecord(stop_, s_) == hipSuccess) T.pending.push_back({name_, start_, stop_});
    return launch_status;
  }

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
  bool active_ = false;
};

#define TIMED(name, stream, expr) \
  [&]() { TimedLaunch tl_(name, stream); return tl_.finish(expr); }()

trstmi_status drain_timing() {
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  for (auto& r : T.pending) {
    hipError_t e = hipEventSynchronize(r.stop);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return hip_fail(e, "timing");
    auto& acc = T.totals[r.name];
    acc.first += ms;
    acc.second += 1;
    T.pool.push_back(r.start);
    T.pool.push_back(r.stop);
  }
  T.pending.clear();
  return TRSTMI_OK;
}

constexpr int64_t kMaxN = 1 << 18;
constexpr int64_t kMaxSteps = 0xFFFFFFFFLL;  // steps are counted in one 32-bit Philox counter word
constexpr int64_t kMaxChannels = 2147483647;  // channels per quantiser call (int32 indices)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Elements per column of an internal candidate buffer: 2d rounded up to a
// multiple of 8 (FP64 / FP32) or of 32 (BF16: one MFMA K step), zero padded.
int32_t ld_of(int64_t d) { return (int32_t)((2 * d + 7) / 8 * 8); }
int32_t ld16_of(int64_t d) { return (int32_t)((2 * d + 31) / 32 * 32); }
int32_t ld_mode(int64_t d, int32_t mode) { return mode == TRSTMI_MODE_BF16_SCREEN ? ld16_of(d) : ld_of(d); }

int nt_of(int64_t n, int tile) { return (int)((n + tile - 1) / tile); }

int64_t ntiles_of(int64_t n, int tile) {
  const int64_t nt = nt_of(n, tile);
  return nt * (nt + 1) / 2;
}

size_t elem_of_mode(int32_t mode) { return mode == TRSTMI_MODE_FP64 ? 8 : (mode == TRSTMI_MODE_FP32 ? 4 : 2); }

// Offsets of the step workspace.
struct Layout {
  int64_t n, d;
  int32_t C, k, ld, ldc;  // ld: FP64/FP32 buffers; ldc: the mode's candidate buffer
  size_t cand, cand_max, dec, tile_max, rechecked, thr, recheck, recheck_max, list, list_count, total;
};

Layout layout_of(const trstmi_params* p) {
  Layout L{};
  L.n = p->n;
  L.d = p->d;
  L.C = p->candidates;
  L.k = p->mode == TRSTMI_MODE_BF16_SCREEN ? p->recheck_topk : 0;
  L.ld = ld_of(p->d);
  L.ldc = ld_mode(p->d, p->mode);
  size_t off = 0;
  L.cand = off;
  off = align256(off + (size_t)L.C * L.n * L.ldc * elem_of_mode(p->mode));
  L.cand_max = off;
  off = align256(off + (size_t)L.C * 8);
  L.dec = off;
  off = align256(off + sizeof(Decision));
  if (p->mode == TRSTMI_MODE_BF16_SCREEN) {
    L.tile_max = off;
    off = align256(off + (size_t)L.C * ntiles_of(L.n, kTileBF16) * 16);  // 4 waves per tile
    L.rechecked = off;
    off = align256(off + (size_t)L.k * 4);
    L.thr = off;
    off = align256(off + (size_t)L.k * 8);
    L.recheck = off;
    off = align256(off + (size_t)L.k * L.n * L.ld * 8);
    L.recheck_max = off;
    off = align256(off + (size_t)L.k * 8);
    L.list = off;
    off = align256(off + (size_t)L.k * ntiles_of(L.n, kTileBF16) * 8);
    L.list_count = off;
    off = align256(off + 8);
  }
  L.total = off;
  return L;
}

trstmi_status check_size(int64_t n, int64_t d) {
  if (n < 2 || n > kMaxN) return fail(TRSTMI_E_INVALID_ARG, "n must be in [2, 262144]");
  if (d < 1 || d > TRSTMI_MAX_D) return fail(TRSTMI_E_INVALID_ARG, "d must be in [1, 512]");
  if (n * ((d + 1) / 2) >= (int64_t)1 << 32) return fail(TRSTMI_E_INVALID_ARG, "n * ceil(d/2) must be < 2^32");
  return TRSTMI_OK;
}

trstmi_status check_mode(int32_t mode) {
  if (mode != TRSTMI_MODE_FP64 && mode != TRSTMI_MODE_FP32 && mode != TRSTMI_MODE_BF16_SCREEN)
    return fail(TRSTMI_E_INVALID_ARG, "unknown mode");
  return TRSTMI_OK;
}

trstmi_status check_params(const trstmi_params* p) {
  if (!p) return fail(TRSTMI_E_INVALID_ARG, "params is NULL");
  trstmi_status st = check_size(p->n, p->d);
  if (st) return st;
  if ((st = check_mode(p->mode))) return st;
  if (p->candidates < 1 || p->candidates > TRSTMI_MAX_CANDIDATES)
    return fail(TRSTMI_E_INVALID_ARG, "candidates must be in [1, 32768]");
  if (p->mode == TRSTMI_MODE_BF16_SCREEN &&
      (p->recheck_topk < 1 || p->recheck_topk > p->candidates || p->recheck_topk > TRSTMI_MAX_TOPK))
    return fail(TRSTMI_E_INVALID_ARG, "recheck_topk must be in [1, min(candidates, 64)]");
  if (p->mode == TRSTMI_MODE_BF16_SCREEN && p->d > 128)
    return fail(TRSTMI_E_UNSUPPORTED, "the BF16 screen form supports d <= 128");
  if (p->seed >> 32 || p->stream_id >> 32) return fail(TRSTMI_E_INVALID_ARG, "seed and stream_id must be < 2^32");
  const bool ok_r = std::isfinite(p->radius0) && std::isfinite(p->radius_min) && std::isfinite(p->radius_max) &&
                    p->radius_min > 0 && p->radius_min <= p->radius0 && p->radius0 <= p->radius_max;
  if (!ok_r) return fail(TRSTMI_E_INVALID_ARG, "need finite 0 < radius_min <= radius0 <= radius_max");
  if (!(std::isfinite(p->grow) && p->grow >= 1.0) || !(std::isfinite(p->shrink) && p->shrink > 0 && p->shrink <= 1.0))
    return fail(TRSTMI_E_INVALID_ARG, "need grow >= 1 and 0 < shrink <= 1");
  // the step index is one 32-bit word of the Philox counter: steps 0 .. 2^32 - 2
  if (p->max_steps < 0 || p->max_steps > kMaxSteps) return fail(TRSTMI_E_INVALID_ARG, "max_steps must be in [0, 2^32 - 1]");
  if (std::isnan(p->target_mu) || std::isnan(p->near_tie)) return fail(TRSTMI_E_INVALID_ARG, "NaN parameter");
  return TRSTMI_OK;
}

trstmi_status check_state(const trstmi_state* s) {
  if (!s || !s->frame || !s->mu || !s->radius || !s->step || !s->flags)
    return fail(TRSTMI_E_INVALID_ARG, "state or one of its pointers is NULL");
  if (((uintptr_t)s->frame & 15) || ((uintptr_t)s->mu & 7) || ((uintptr_t)s->radius & 7) ||
      ((uintptr_t)s->step & 7) || ((uintptr_t)s->flags & 3))
    return fail(TRSTMI_E_INVALID_ARG, "state pointer misaligned (frame needs 16 bytes)");
  return TRSTMI_OK;
}

trstmi_status check_ws(void* ws, size_t have, size_t need) {
  if (need == 0) return TRSTMI_OK;
  if (!ws) return fail(TRSTMI_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws & 255) return fail(TRSTMI_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (have < need) return fail(TRSTMI_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return TRSTMI_OK;
}

double tau_of(const trstmi_params* p) {
  if (p->near_tie > 0) return p->near_tie;
  return p->mode == TRSTMI_MODE_FP32 ? 4e-6 : 2e-12;
}

// Certified bound on |screened - exact| coherence for unit columns in C^d.
// Input: rounding the real and imaginary parts of an entry to bfloat16
// (relative error <= u = 2^-8 each) moves the complex entry by at most u
// times its modulus, so the complex inner product of two unit columns moves
// by at most 2u + u^2 (triangle and Cauchy-Schwarz inequalities).
// Accumulation: bf16 x bf16 products are exact in FP32 and the MFMA adds 2d
// of them per real part, with |terms| summing to <= (1 + u)^2.  The only
// assumption made about v_mfma_f32_16x16x32_bf16 is that each addition is
// faithful (error below one ulp of its result, any rounding direction), so
// each part is off by <= gamma_{2d} (1 + u)^2 with gamma_n = n w / (1 - n w),
// w = 2^-23; sqrt(2) for Re and Im together.  The last terms cover the FP32
// epilogue (8 v, v = 2^-24) and the FP64 value's rounding.
double screen_eps(int64_t d) {
  const double u = std::ldexp(1.0, -8), w = std::ldexp(1.0, -23), v = std::ldexp(1.0, -24);
  const double nw = 2.0 * d * w;
  const double gamma = nw / (1.0 - nw);
  return (2 * u + u * u) + std::sqrt(2.0) * gamma * (1 + u) * (1 + u) + 8 * v + 1e-12;
}

PerturbArgs perturb_base(const trstmi_params* p) {
  PerturbArgs a{};
  a.n = p->n;
  a.d = (int32_t)p->d;
  a.seed = (uint32_t)p->seed;
  a.stream_id = (uint32_t)p->stream_id;
  a.tag = 0;
  a.have_z = 1;
  return a;
}

GramArgs gram_base(int64_t n, int64_t d, const void* cand, int64_t stride, int32_t ld, int tile, uint64_t* mx,
                   const int32_t* flags) {
  GramArgs g{};
  g.cand = cand;
  g.slot_stride = stride;
  g.ldk = ld;
  g.n = (int32_t)n;
  g.d = (int32_t)d;
  g.nt = nt_of(n, tile);
  g.cand_max = mx;
  g.flags = flags;
  return g;
}

PerturbArgs candidate_args(const trstmi_params* p, const trstmi_state* st, const Layout& L, char* ws,
                           const double* z) {
  PerturbArgs pa = perturb_base(p);
  pa.base = st->frame;
  pa.radius = st->radius;
  pa.tstep = st->step;
  pa.gate = st->flags;
  pa.gate_mask = TRSTMI_FLAG_DONE;
  pa.gate_want = 0;
  pa.z_explicit = z;
  pa.out = ws + L.cand;
  pa.out_kind = p->mode == TRSTMI_MODE_FP64 ? kOutF64 : (p->mode == TRSTMI_MODE_FP32 ? kOutF32 : kOutBF16);
  pa.out_ld = L.ldc;
  pa.out_slot_stride = L.n * L.ldc;
  pa.zero_max = (uint64_t*)(ws + L.cand_max);
  return pa;
}

SelectArgs select_args(const trstmi_params* p, const trstmi_state* st, const Layout& L, char* ws,
                       const trstmi_report* rep) {
  SelectArgs sa{};
  sa.tau = tau_of(p);
  sa.mu = st->mu;
  sa.radius = st->radius;
  sa.step = st->step;
  sa.flags = st->flags;
  sa.grow = p->grow;
  sa.shrink = p->shrink;
  sa.radius_min = p->radius_min;
  sa.radius_max = p->radius_max;
  sa.max_steps = p->max_steps;
  sa.target_mu = p->target_mu;
  sa.dec = (Decision*)(ws + L.dec);
  sa.rep_best = rep ? rep->best : nullptr;
  return sa;
}

// commit: regenerate the accepted candidate in FP64 into the frame, in place
PerturbArgs commit_args(const trstmi_params* p, const trstmi_state* st, const Layout& L, char* ws, const double* z) {
  Decision* dec = (Decision*)(ws + L.dec);
  PerturbArgs pc = perturb_base(p);
  pc.base = st->frame;
  pc.radius = &dec->radius_old;
  pc.tstep = &dec->t_old;
  pc.cand_idx = &dec->best;
  pc.gate = &dec->commit;
  pc.gate_mask = 1;
  pc.gate_want = 1;
  pc.z_explicit = z;
  pc.out = st->frame;
  pc.out_kind = kOutF64;
  pc.out_ld = (int32_t)(2 * L.d);
  pc.out_slot_stride = 2 * L.d * L.n;
  return pc;
}

}  // namespace

namespace trstmi {

// Every record of one BF16-screen step (parameters already validated, mode
// TRSTMI_MODE_BF16_SCREEN).
StepArgs bf16_step_args(const trstmi_params* p, const trstmi_state* st, char* ws, const double* z,
                        const trstmi_report* rep) {
  const Layout L = layout_of(p);
  const int C = p->candidates;
  const int64_t slot_stride = L.n * L.ldc;
  const int64_t slot_stride64 = L.n * L.ld;
  uint64_t* cand_max = (uint64_t*)(ws + L.cand_max);
  StepArgs A{};
  A.pa = candidate_args(p, st, L, ws, z);
  A.sa = select_args(p, st, L, ws, rep);

  uint32_t* tile_max = (uint32_t*)(ws + L.tile_max);
  int32_t* rechecked = (int32_t*)(ws + L.rechecked);
  double* thr = (double*)(ws + L.thr);
  uint64_t* recheck_max = (uint64_t*)(ws + L.recheck_max);
  A.g = gram_base(L.n, L.d, ws + L.cand, slot_stride, L.ldc, kTileBF16, cand_max, st->flags);
  A.g.tile_max = tile_max;
  gram_bf16_prepare(A.g, C);

  TopkArgs& ta = A.ta;
  ta.cand_max = cand_max;
  ta.C = C;
  ta.k = L.k;
  ta.eps = screen_eps(L.d);
  ta.screen_tie = 2e-5;
  ta.flags = st->flags;
  ta.rechecked = rechecked;
  ta.thr = thr;
  ta.dec = (Decision*)(ws + L.dec);
  ta.rep_cand_mu = rep ? rep->cand_mu : nullptr;
  ta.rep_rechecked = rep ? rep->rechecked : nullptr;
  ta.tile_max = tile_max;
  ta.screen_nt = nt_of(L.n, kTileBF16);
  ta.list = (int2*)(ws + L.list);
  ta.list_count = (int32_t*)(ws + L.list_count);
  ta.list_cap = (int32_t)(L.k * ntiles_of(L.n, kTileBF16));

  A.pr = A.pa;
  A.pr.cand_idx = rechecked;
  A.pr.out = ws + L.recheck;
  A.pr.out_kind = kOutF64;
  A.pr.out_ld = L.ld;
  A.pr.out_slot_stride = slot_stride64;
  A.pr.zero_max = recheck_max;

  RecheckArgs& ra = A.ra;
  ra.screen = (const uint16_t*)(ws + L.cand);
  ra.screen_stride = slot_stride;
  ra.ldk16 = L.ldc;
  ra.cand64 = (const double*)(ws + L.recheck);
  ra.stride64 = slot_stride64;
  ra.ld64 = L.ld;
  ra.n = (int32_t)L.n;
  ra.d = (int32_t)L.d;
  ra.nt = nt_of(L.n, kTileBF16);
  ra.k = L.k;
  ra.list = (const int2*)(ws + L.list);
  ra.count = (const int32_t*)(ws + L.list_count);
  ra.list_cap = ta.list_cap;
  ra.rechecked = rechecked;
  ra.thr = thr;
  ra.recheck_max = recheck_max;
  ra.flags = st->flags;

  A.sa.cand_max = recheck_max;
  A.sa.count = L.k;
  A.sa.is_f32 = 0;
  A.sa.slot_cand = rechecked;
  A.sa.use_screen_near = 1;
  A.sa.rep_cand_mu = rep ? rep->recheck_mu : nullptr;

  A.pc = commit_args(p, st, L, ws, z);
  return A;
}

}  // namespace trstmi

namespace {

trstmi_status enqueue_step(const trstmi_params* p, const trstmi_state* st, char* ws, const double* z,
                           const trstmi_report* rep, hipStream_t s) {
  const Layout L = layout_of(p);
  const int C = p->candidates;
  if (p->mode == TRSTMI_MODE_BF16_SCREEN) {
    const StepArgs A = bf16_step_args(p, st, ws, z, rep);
    TRY_HIP(TIMED("perturb", s, launch_perturb(A.pa, C, s)), "perturb");
    TRY_HIP(TIMED("gram_bf16", s, launch_gram_bf16(A.g, C, s)), "gram_bf16");
    TRY_HIP(TIMED("topk", s, launch_topk(A.ta, s)), "topk");
    TRY_HIP(TIMED("perturb_recheck", s, launch_perturb(A.pr, L.k, s)), "perturb_recheck");
    TRY_HIP(TIMED("recheck", s, launch_recheck_pairs(A.ra, s)), "recheck");
    TRY_HIP(TIMED("select", s, launch_select(A.sa, s)), "select");
    CommitCopyArgs cc{};
    cc.dec = (const Decision*)(ws + L.dec);
    cc.slot_cand = (const int32_t*)(ws + L.rechecked);
    cc.k = L.k;
    cc.src = (const double*)(ws + L.recheck);
    cc.src_slot_stride = L.n * L.ld;
    cc.src_ld = L.ld;
    cc.frame = st->frame;
    cc.n = L.n;
    cc.d = (int32_t)L.d;
    TRY_HIP(TIMED("commit", s, launch_commit_copy(cc, s)), "commit");
    return TRSTMI_OK;
  }
  const PerturbArgs pa = candidate_args(p, st, L, ws, z);
  TRY_HIP(TIMED("perturb", s, launch_perturb(pa, C, s)), "perturb");
  const bool f32 = p->mode == TRSTMI_MODE_FP32;
  uint64_t* cand_max = (uint64_t*)(ws + L.cand_max);
  GramArgs g = gram_base(L.n, L.d, ws + L.cand, L.n * L.ldc, L.ldc, f32 ? kTileF32 : kTileF64, cand_max, st->flags);
  TRY_HIP(TIMED(f32 ? "gram_f32" : "gram_f64", s, f32 ? launch_gram_f32(g, C, s) : launch_gram_f64(g, C, s)), "gram");
  SelectArgs sa = select_args(p, st, L, ws, rep);
  sa.cand_max = cand_max;
  sa.count = C;
  sa.is_f32 = f32 ? 1 : 0;
  sa.rep_cand_mu = rep ? rep->cand_mu : nullptr;
  TRY_HIP(TIMED("select", s, launch_select(sa, s)), "select");
  if (f32) {
    TRY_HIP(TIMED("commit", s, launch_perturb(commit_args(p, st, L, ws, z), 1, s)), "commit");
  } else {
    CommitCopyArgs cc{};
    cc.dec = (const Decision*)(ws + L.dec);
    cc.src = (const double*)(ws + L.cand);
    cc.src_slot_stride = L.n * L.ldc;
    cc.src_ld = L.ldc;
    cc.frame = st->frame;
    cc.n = L.n;
    cc.d = (int32_t)L.d;
    TRY_HIP(TIMED("commit", s, launch_commit_copy(cc, s)), "commit");
  }
  return TRSTMI_OK;
}

// ---------------------------------------------------------------------------
// Batched form: layout of the workspace (computed on the host from the
// parameters on every call).
// ---------------------------------------------------------------------------
constexpr int kBatchGridCap = 1024;   // persistent blocks (4 per CU)
constexpr int kBatchMaxN = 256;
constexpr int kBatchMaxD = 16;
constexpr int kBatchMaxC = 256;

struct BatchLayout {
  size_t hdr = 0, tab = 0, inst = 0, state = 0, units = 0, frames = 0, cand = 0, scratch = 0, total = 0;
  int nunits = 0;
  int grid = 0;
  int64_t scratch_stride = 0;
  std::vector<int64_t> frame_off;
  std::vector<int32_t> wpi;
  std::vector<int2> unit_list;
};

trstmi_status batch_layout(const trstmi_batch_params* p, const trstmi_batch_instance* inst, BatchLayout& L) {
  if (!p || !inst) return fail(TRSTMI_E_INVALID_ARG, "batch params or instances NULL");
  if (p->count < 1 || p->count > (1 << 20)) return fail(TRSTMI_E_INVALID_ARG, "batch count must be in [1, 2^20]");
  if (p->candidates < 1 || p->candidates > kBatchMaxC)
    return fail(TRSTMI_E_INVALID_ARG, "batch candidates must be in [1, 256]");
  const bool ok_r = std::isfinite(p->radius0) && std::isfinite(p->radius_min) && std::isfinite(p->radius_max) &&
                    p->radius_min > 0 && p->radius_min <= p->radius0 && p->radius0 <= p->radius_max;
  if (!ok_r) return fail(TRSTMI_E_INVALID_ARG, "need finite 0 < radius_min <= radius0 <= radius_max");
  if (!(std::isfinite(p->grow) && p->grow >= 1.0) || !(std::isfinite(p->shrink) && p->shrink > 0 && p->shrink <= 1.0))
    return fail(TRSTMI_E_INVALID_ARG, "need grow >= 1 and 0 < shrink <= 1");
  const int lds = batch_lds_words();
  L.frame_off.resize(p->count);
  L.wpi.resize(p->count);
  int64_t off = 0, max_frame = 0;
  std::vector<std::pair<int64_t, int32_t>> order;
  for (int32_t i = 0; i < p->count; ++i) {
    const trstmi_batch_instance& I = inst[i];
    if (I.n < 2 || I.n > kBatchMaxN || I.d < 1 || I.d > kBatchMaxD)
      return fail(TRSTMI_E_INVALID_ARG, "batch instance " + std::to_string(i) + ": need 2 <= n <= 256, 1 <= d <= 16");
    if (I.max_steps < 0 || I.max_steps > kMaxSteps || std::isnan(I.target_mu))
      return fail(TRSTMI_E_INVALID_ARG, "batch instance " + std::to_string(i) + ": bad max_steps or target");
    const int64_t need = (int64_t)I.n * batch_row_words(I.d);
    int32_t w = I.waves_per_item;
    if (w == 0) w = need * 4 <= lds ? 1 : (need * 2 <= lds ? 2 : 4);
    if (w != 1 && w != 2 && w != 4)
      return fail(TRSTMI_E_INVALID_ARG, "batch instance " + std::to_string(i) + ": waves_per_item must be 0, 1, 2 or 4");
    if (need * (4 / w) > lds)
      return fail(TRSTMI_E_INVALID_ARG, "batch instance " + std::to_string(i) + ": too large for waves_per_item");
    L.wpi[i] = w;
    L.frame_off[i] = off;
    const int64_t fl = 2 * (int64_t)I.d * I.n;
    off += (fl + 31) / 32 * 32;
    max_frame = fl > max_frame ? fl : max_frame;
    order.push_back({-(int64_t)I.n * I.n * I.d, i});
  }
  std::stable_sort(order.begin(), order.end());
  L.unit_list.clear();
  for (auto& o : order) {
    const int32_t i = o.second;
    const int per = 4 / L.wpi[i];
    for (int c0 = 0; c0 < p->candidates; c0 += per) L.unit_list.push_back(make_int2(i, c0));
  }
  L.nunits = (int)L.unit_list.size();
  L.grid = L.nunits < kBatchGridCap ? L.nunits : kBatchGridCap;  // scratch is sized for kBatchGridCap blocks
  L.scratch_stride = (max_frame + 31) / 32 * 32;
  size_t o = 0;
  L.hdr = o;
  o = align256(o + 256);
  L.tab = o;
  o = align256(o + batch_tab_bytes());
  L.inst = o;
  o = align256(o + (size_t)p->count * batch_inst_bytes());
  L.state = o;
  o = align256(o + (size_t)p->count * batch_state_bytes());
  L.units = o;
  o = align256(o + (size_t)L.nunits * sizeof(int2));
  L.frames = o;
  o = align256(o + (size_t)off * 8);
  L.cand = o;
  o = align256(o + (size_t)p->count * p->candidates * 8);
  L.scratch = o;
  o = align256(o + (size_t)kBatchGridCap * 4 * L.scratch_stride * 8);
  L.total = o;
  return TRSTMI_OK;
}

// Blocks of a step launch: the resident capacity of the device (queried once),
// at most the number of units and the scratch slots of the workspace.
int batch_grid(const BatchLayout& L) {
  static int cap = 0;
  if (cap == 0) {
    const int m = batch_step_max_blocks();
    cap = m > 0 ? m : 1;
  }
  int g = L.grid < cap ? L.grid : cap;
  return g > 0 ? g : 1;
}

BatchArgs batch_args(const trstmi_batch_params* p, const BatchLayout& L, char* ws) {
  BatchArgs b{};
  b.inst = ws + L.inst;
  b.state = ws + L.state;
  b.units = (const int2*)(ws + L.units);
  b.nunits = L.nunits;
  b.C = p->candidates;
  b.frames = (double*)(ws + L.frames);
  b.cand_max = (uint64_t*)(ws + L.cand);
  b.scratch = (double*)(ws + L.scratch);
  b.scratch_stride = L.scratch_stride;
  b.count = p->count;
  b.done_instances = (int32_t*)(ws + L.hdr) + 2;
  b.tab = ws + L.tab;
  b.tau = p->near_tie > 0 ? p->near_tie : 2e-12;
  b.grow = p->grow;
  b.shrink = p->shrink;
  b.radius_min = p->radius_min;
  b.radius_max = p->radius_max;
  return b;
}

trstmi_status batch_prepare(const trstmi_batch_params* p, const trstmi_batch_instance* inst, const void* ws,
                            size_t ws_bytes, BatchLayout& L) {
  trstmi_status st = batch_layout(p, inst, L);
  if (st) return st;
  return check_ws(const_cast<void*>(ws), ws_bytes, L.total);
}

}  // namespace

namespace trstmi {
// The calling thread's error message, for other parts of the library.
trstmi_status set_last_error(trstmi_status code, const std::string& msg) { return fail(code, msg); }

void lse_grad_scalars(int64_t n, int64_t d, char* ws, const uint64_t** s_bits, const double** log_sum) {
  const size_t frame_bytes = align256((size_t)n * ld_mode(d, TRSTMI_MODE_FP64) * 8);
  *s_bits = (const uint64_t*)(ws + frame_bytes);
  *log_sum = (const double*)(ws + trstmi_lse_workspace_bytes(n, d));
}
}  // namespace trstmi

extern "C" {

void trstmi_default_params(trstmi_params* p, int64_t n, int64_t d) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = n;
  p->d = d;
  p->candidates = 64;
  p->mode = TRSTMI_MODE_FP64;
  p->recheck_topk = 8;
  p->seed = 0;
  p->stream_id = 0;
  p->radius0 = 0.1;
  p->grow = 2.0;
  p->shrink = 0.5;
  p->radius_min = 1e-12;
  p->radius_max = 1.0;
  p->max_steps = 1000;
  p->target_mu = 0.0;
  p->near_tie = 0.0;
}

size_t trstmi_workspace_bytes(const trstmi_params* p) {
  if (check_params(p)) return 0;
  return layout_of(p).total;
}

size_t trstmi_coherence_workspace_bytes(int64_t n, int64_t d, int32_t mode) {
  if (check_size(n, d) || check_mode(mode)) return 0;
  return align256((size_t)n * ld_mode(d, mode) * elem_of_mode(mode)) + 256;
}

trstmi_status trstmi_round_bf16(const double* x, int64_t count, uint16_t* out, hipStream_t stream) {
  if (count < 0) return fail(TRSTMI_E_INVALID_ARG, "count must be >= 0");
  if (count == 0) return TRSTMI_OK;
  if (!x || !out) return fail(TRSTMI_E_INVALID_ARG, "x and out must be device pointers");
  if (((uintptr_t)x & 7) || ((uintptr_t)out & 1)) return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  TRY_HIP(launch_round_bf16(x, count, out, stream), "round_bf16");
  return TRSTMI_OK;
}

trstmi_status trstmi_coherence(int64_t n, int64_t d, int32_t mode, const double* frame, double* mu_out,
                               void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if ((st = check_mode(mode))) return st;
  if (!frame || !mu_out) return fail(TRSTMI_E_INVALID_ARG, "frame and mu_out must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)mu_out & 7)) return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_coherence_workspace_bytes(n, d, mode);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  char* ws = (char*)workspace;
  const int32_t ld = ld_mode(d, mode);
  uint64_t* mx = (uint64_t*)(ws + align256((size_t)n * ld * elem_of_mode(mode)));

  PerturbArgs pa{};
  pa.base = frame;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = mode == TRSTMI_MODE_FP64 ? kOutF64 : (mode == TRSTMI_MODE_FP32 ? kOutF32 : kOutBF16);
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise");
  const int tile = mode == TRSTMI_MODE_FP64 ? kTileF64 : (mode == TRSTMI_MODE_FP32 ? kTileF32 : kTileBF16);
  GramArgs g = gram_base(n, d, ws, n * ld, ld, tile, mx, nullptr);
  if (mode == TRSTMI_MODE_FP64) TRY_HIP(launch_gram_f64(g, 1, stream), "gram_f64");
  else if (mode == TRSTMI_MODE_FP32) TRY_HIP(launch_gram_f32(g, 1, stream), "gram_f32");
  else TRY_HIP(launch_gram_bf16(g, 1, stream), "gram_bf16");
  InitFinishArgs f{};
  f.max_bits = mx;
  f.is_f32 = mode == TRSTMI_MODE_FP64 ? 0 : 1;
  f.mu_out = mu_out;
  TRY_HIP(launch_init_finish(f, stream), "finish");
  return TRSTMI_OK;
}

trstmi_status trstmi_coherence_pair(int64_t n, int64_t d, const double* frame, double* mu_out, int64_t* pair_out,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (!frame || !mu_out || !pair_out) return fail(TRSTMI_E_INVALID_ARG, "frame, mu_out and pair_out must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)mu_out & 7) || ((uintptr_t)pair_out & 7))
    return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_coherence_workspace_bytes(n, d, TRSTMI_MODE_FP64);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  char* ws = (char*)workspace;
  const int32_t ld = ld_mode(d, TRSTMI_MODE_FP64);
  uint64_t* mx = (uint64_t*)(ws + align256((size_t)n * ld * 8));
  PerturbArgs pa{};
  pa.base = frame;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = kOutF64;
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise");
  GramArgs g = gram_base(n, d, ws, n * ld, ld, kTileF64, mx, nullptr);
  TRY_HIP(launch_gram_f64(g, 1, stream), "gram_f64");
  TRY_HIP(launch_gram_f64_pair(g, mx + 1, mu_out, pair_out, stream), "gram_f64_pair");
  return TRSTMI_OK;
}

size_t trstmi_lse_workspace_bytes(int64_t n, int64_t d) {
  if (check_size(n, d)) return 0;
  const int64_t nt = (n + kTileF64 - 1) / kTileF64;
  return align256((size_t)n * ld_mode(d, TRSTMI_MODE_FP64) * 8) + 256 + align256((size_t)(nt * (nt + 1) / 2) * 16);
}

trstmi_status trstmi_lse(int64_t n, int64_t d, const double* frame, double delta, int32_t squared, double* out,
                         void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(TRSTMI_E_INVALID_ARG, "delta must be finite and > 0");
  if (squared != 0 && squared != 1) return fail(TRSTMI_E_INVALID_ARG, "squared must be 0 or 1");
  if (!frame || !out) return fail(TRSTMI_E_INVALID_ARG, "frame and out must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)out & 7)) return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_lse_workspace_bytes(n, d);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  char* ws = (char*)workspace;
  const int32_t ld = ld_mode(d, TRSTMI_MODE_FP64);
  const size_t frame_bytes = align256((size_t)n * ld * 8);
  uint64_t* mx = (uint64_t*)(ws + frame_bytes);
  double* partial = (double*)(ws + frame_bytes + 256);
  const int64_t nt = (n + kTileF64 - 1) / kTileF64;

  PerturbArgs pa{};
  pa.base = frame;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = kOutF64;
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise");
  GramArgs g = gram_base(n, d, ws, n * ld, ld, kTileF64, mx, nullptr);
  TRY_HIP(TIMED("lse_pass", stream, launch_lse_pass(g, delta, squared, partial, stream)), "lse_pass");
  TRY_HIP(launch_lse_finish(mx, partial, nt * (nt + 1) / 2, delta, squared, out, nullptr, stream), "lse_finish");
  return TRSTMI_OK;
}

size_t trstmi_miso_workspace_bytes(int64_t n, int64_t d, int64_t m) {
  if (n < 1 || n > kMaxN || d < 1 || d > TRSTMI_MAX_D || m < 0 || m > kMaxChannels) return 0;
  return align256((size_t)n * ld_of(d) * 8) + align256((size_t)(miso_blocks(m) > 0 ? miso_blocks(m) : 1) * 16);
}

trstmi_status trstmi_miso_quantize(const double* codebook, int64_t n, int64_t d, const double* channels, int64_t m,
                                   int32_t* index, double* gain, double* dist, double* summary, void* workspace,
                                   size_t workspace_bytes, hipStream_t stream) {
  if (n < 1 || n > kMaxN) return fail(TRSTMI_E_INVALID_ARG, "n must be in [1, 262144]");
  if (d < 1 || d > TRSTMI_MAX_D) return fail(TRSTMI_E_INVALID_ARG, "d must be in [1, 512]");
  if (m < 0 || m > kMaxChannels) return fail(TRSTMI_E_INVALID_ARG, "m must be in [0, 2^31 - 1]");
  if (!codebook) return fail(TRSTMI_E_INVALID_ARG, "codebook must be a device pointer");
  if (m > 0 && !channels) return fail(TRSTMI_E_INVALID_ARG, "channels must be a device pointer");
  if (((uintptr_t)codebook & 15) || ((uintptr_t)channels & 15) || ((uintptr_t)index & 3) ||
      ((uintptr_t)gain & 7) || ((uintptr_t)dist & 7) || ((uintptr_t)summary & 7))
    return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_miso_workspace_bytes(n, d, m);
  trstmi_status st = check_ws(workspace, workspace_bytes, need);
  if (st) return st;
  char* ws = (char*)workspace;
  const int32_t ld = ld_of(d);
  PerturbArgs pa{};
  pa.base = codebook;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = kOutF64;
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise codebook");
  MisoArgs a{};
  a.codebook = (const double*)ws;
  a.ldk = ld;
  a.n = (int32_t)n;
  a.d = (int32_t)d;
  a.channels = channels;
  a.m = m;
  a.index = index;
  a.gain = gain;
  a.dist = dist;
  a.partial = (double*)(ws + align256((size_t)n * ld * 8));
  TRY_HIP(TIMED("miso", stream, launch_miso(a, summary, stream)), "miso_quantize");
  return TRSTMI_OK;
}

size_t trstmi_lse_grad_workspace_bytes(int64_t n, int64_t d) {
  if (check_size(n, d) || d > 64) return 0;
  const int64_t nkb = (n + kTileF64 - 1) / kTileF64;
  const int64_t nch = lse_grad_chunks((int)nkb);
  return trstmi_lse_workspace_bytes(n, d) + 256 + align256((size_t)nkb * nch * 2 * 2 * kTileF64 * 2 * d * 8);
}

trstmi_status trstmi_lse_grad(int64_t n, int64_t d, const double* frame, double delta, double* out, double* grad,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (d > 64) return fail(TRSTMI_E_UNSUPPORTED, "the smooth-maximum gradient supports d <= 64");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(TRSTMI_E_INVALID_ARG, "delta must be finite and > 0");
  if (!frame || !out || !grad) return fail(TRSTMI_E_INVALID_ARG, "frame, out and grad must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)out & 7) || ((uintptr_t)grad & 15))
    return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_lse_grad_workspace_bytes(n, d);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  const size_t lse_bytes = trstmi_lse_workspace_bytes(n, d);
  char* ws = (char*)workspace;
  const int32_t ld = ld_mode(d, TRSTMI_MODE_FP64);
  const size_t frame_bytes = align256((size_t)n * ld * 8);
  uint64_t* mx = (uint64_t*)(ws + frame_bytes);
  double* partial = (double*)(ws + frame_bytes + 256);
  double* log_sum = (double*)(ws + lse_bytes);
  double* gpart = (double*)(ws + lse_bytes + 256);
  const int64_t nt = (n + kTileF64 - 1) / kTileF64;

  PerturbArgs pa{};
  pa.base = frame;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = kOutF64;
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise");
  GramArgs g = gram_base(n, d, ws, n * ld, ld, kTileF64, mx, nullptr);
  TRY_HIP(TIMED("lse_pass", stream, launch_lse_pass(g, delta, 1, partial, stream)), "lse_pass");
  TRY_HIP(launch_lse_finish(mx, partial, nt * (nt + 1) / 2, delta, 1, out, log_sum, stream), "lse_finish");
  GradArgs ga{};
  ga.frame = (const double*)ws;
  ga.raw = frame;
  ga.ld = ld;
  int32_t L = 16;  // LDS column: 2d rounded up to a power of two >= 16, plus one
  while (L < 2 * d) L *= 2;
  ga.ldp = L + 1;
  ga.n = (int32_t)n;
  ga.d = (int32_t)d;
  ga.s_bits = mx;
  ga.log_sum = log_sum;
  ga.inv_delta = 1.0 / delta;
  ga.partial = gpart;
  ga.grad = grad;
  TRY_HIP(TIMED("lse_grad", stream, launch_lse_grad(ga, stream)), "lse_grad");
  return TRSTMI_OK;
}

trstmi_status trstmi_screen_tiles_set(const trstmi_screen_tile* entries, int32_t count) {
  if (count < 0 || count > 4096 || (count > 0 && !entries))
    return fail(TRSTMI_E_INVALID_ARG, "count must be in [0, 4096] with a host array of that many entries");
  std::vector<ScreenTile> t(count);
  for (int32_t i = 0; i < count; ++i) {
    const trstmi_screen_tile& e = entries[i];
    if (e.ks < 1 || e.ks > 8 || e.n_max < 2 || (e.form != 0 && e.form != 1) || (e.form == 0 && e.ks > 4) ||
        e.seg < 1 || e.seg > 64)
      return fail(TRSTMI_E_INVALID_ARG, "screen tile entry " + std::to_string(i) +
                                            ": need 1 <= ks <= 8, n_max >= 2, form 0 (ks <= 4) or 1, 1 <= seg <= 64");
    t[i] = ScreenTile{e.ks, e.n_max, e.form, e.seg};
  }
  screen_tiles_set(t.data(), count);
  return TRSTMI_OK;
}

size_t trstmi_lse_hvp_workspace_bytes(int64_t n, int64_t d) {
  if (check_size(n, d) || d > 64) return 0;
  return trstmi_lse_workspace_bytes(n, d) + 256 + hv_scratch_bytes(n, d);
}

trstmi_status trstmi_lse_hvp(int64_t n, int64_t d, const double* frame, const double* v, double delta, double* out,
                             double* hv, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (d > 64) return fail(TRSTMI_E_UNSUPPORTED, "the Hessian-vector product supports d <= 64");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(TRSTMI_E_INVALID_ARG, "delta must be finite and > 0");
  if (!frame || !v || !out || !hv) return fail(TRSTMI_E_INVALID_ARG, "frame, v, out and hv must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)v & 15) || ((uintptr_t)out & 7) || ((uintptr_t)hv & 15))
    return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_lse_hvp_workspace_bytes(n, d);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  const size_t lse_bytes = trstmi_lse_workspace_bytes(n, d);
  char* ws = (char*)workspace;
  const int32_t ld = ld_mode(d, TRSTMI_MODE_FP64);
  const size_t frame_bytes = align256((size_t)n * ld * 8);
  uint64_t* mx = (uint64_t*)(ws + frame_bytes);
  double* partial = (double*)(ws + frame_bytes + 256);
  double* log_sum = (double*)(ws + lse_bytes);
  const int64_t nt = (n + kTileF64 - 1) / kTileF64;
  PerturbArgs pa{};
  pa.base = frame;
  pa.have_z = 0;
  pa.n = n;
  pa.d = (int32_t)d;
  pa.out = ws;
  pa.out_kind = kOutF64;
  pa.out_ld = ld;
  pa.out_slot_stride = n * ld;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "normalise");
  GramArgs g = gram_base(n, d, ws, n * ld, ld, kTileF64, mx, nullptr);
  TRY_HIP(launch_lse_pass(g, delta, 1, partial, stream), "lse_pass");
  TRY_HIP(launch_lse_finish(mx, partial, nt * (nt + 1) / 2, delta, 1, out, log_sum, stream), "lse_finish");
  HvArgs h{};
  hv_layout(h, ws + lse_bytes + 256, n, d);
  h.raw = frame;
  h.v = v;
  h.s_bits = mx;
  h.inv_delta = 1.0 / delta;
  h.out = hv;
  TRY_HIP(TIMED("lse_hv", stream, launch_lse_hv(h, stream)), "lse_hv");
  return TRSTMI_OK;
}

size_t trstmi_tr_workspace_bytes(int64_t n, int64_t d) {
  const size_t g = trstmi_lse_grad_workspace_bytes(n, d);
  return g ? align256(g) + tr_vectors_bytes(n, d) : 0;
}

trstmi_status trstmi_tr_step(int64_t n, int64_t d, double* frame, const trstmi_tr_params* tp, trstmi_tr_report* rep,
                             void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (d > 64) return fail(TRSTMI_E_UNSUPPORTED, "the trust-region step supports d <= 64");
  if (!tp || !rep) return fail(TRSTMI_E_INVALID_ARG, "params and report must be host pointers");
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  if (!pos(tp->delta) || !pos(tp->radius) || !pos(tp->cg_tol) || !(tp->fd_step == 0.0 || pos(tp->fd_step)) ||
      !(tp->radius_max >= tp->radius) || !std::isfinite(tp->radius_max) || !(tp->eta >= 0.0 && tp->eta < 0.25) ||
      tp->cg_max_iter < 1)
    return fail(TRSTMI_E_INVALID_ARG, "invalid trust-region parameters");
  if (!frame) return fail(TRSTMI_E_INVALID_ARG, "frame must be a device pointer");
  if ((uintptr_t)frame & 15) return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  const size_t need = trstmi_tr_workspace_bytes(n, d);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  const size_t lws = align256(trstmi_lse_grad_workspace_bytes(n, d));
  st = tr_step_impl(n, d, frame, tp, rep, (char*)workspace, lws, stream);
  if (st == TRSTMI_E_HIP) return fail(TRSTMI_E_HIP, "trust-region step: a HIP call failed");
  if (st == TRSTMI_E_INVALID_ARG) return fail(TRSTMI_E_INVALID_ARG, "the frame has a zero or non-finite column");
  return st;
}

static size_t optimize_slot_bytes(int64_t n, int64_t d) {
  const size_t t = trstmi_tr_workspace_bytes(n, d);
  if (!t) return 0;
  const size_t frame = align256((size_t)2 * d * n * 8);
  return align256(t) + frame + align256(trstmi_coherence_workspace_bytes(n, d, 0)) + 256 + frame;
}

size_t trstmi_optimize_workspace_bytes(int64_t n, int64_t d, int32_t concurrency) {
  if (concurrency < 1 || concurrency > 64) return 0;
  return (size_t)concurrency * optimize_slot_bytes(n, d);
}

namespace {

// One worker's share of the starts: l = first, first + stride, ...; keeps
// the best (mu, l) of its share and that frame in its slot.
struct OptWorker {
  int64_t n, d;
  const trstmi_opt_params* op;
  char* slot;
  hipStream_t stream;
  int32_t first, stride;
  std::atomic<bool>* abort;  // set when any worker fails: the others stop at their next start
  double best_mu = __builtin_inf();
  int32_t best_l = -1;
  trstmi_status st = TRSTMI_OK;
  std::string err;

  double* best_frame() const {
    const size_t frame = align256((size_t)2 * d * n * 8);
    return (double*)(slot + optimize_slot_bytes(n, d) - frame);
  }

  trstmi_status run() {
    const size_t tws = align256(trstmi_tr_workspace_bytes(n, d));
    const size_t lws = align256(trstmi_lse_grad_workspace_bytes(n, d));
    double* W = (double*)(slot + tws);
    char* cws = slot + tws + align256((size_t)2 * d * n * 8);
    const size_t cws_bytes = trstmi_coherence_workspace_bytes(n, d, 0);
    double* mu_dev = (double*)(cws + align256(cws_bytes));
    trstmi_status rs;
    for (int32_t l = op->first_restart + first; l < op->first_restart + op->restarts; l += stride) {
      if (abort->load(std::memory_order_relaxed)) break;
      PerturbArgs pa{};
      pa.n = n;
      pa.d = (int32_t)d;
      pa.seed = (uint32_t)op->seed;
      pa.stream_id = (uint32_t)l;
      pa.have_z = 1;
      pa.base = nullptr;
      pa.tag = 1;
      pa.t_const = 0;
      pa.c0 = 0;
      pa.out = W;
      pa.out_kind = kOutF64;
      pa.out_ld = (int32_t)(2 * d);
      pa.out_slot_stride = 2 * d * n;
      TRY_HIP(launch_perturb(pa, 1, stream), "optimise: random start");
      for (int32_t k = 0; k < op->n_deltas; ++k) {
        trstmi_tr_params tp{};
        tp.delta = op->deltas[k];
        tp.radius = op->radius0;
        tp.radius_max = op->radius_max;
        tp.eta = op->eta;
        tp.cg_tol = op->cg_tol;
        tp.cg_max_iter = op->cg_max_iter ? op->cg_max_iter : (int32_t)(2 * d * n);
        tp.fd_step = op->fd_step;
        for (int32_t s = 0; s < op->steps_per_delta; ++s) {
          trstmi_tr_report rep{};
          rs = tr_step_impl(n, d, W, &tp, &rep, slot, lws, stream);
          if (rs == TRSTMI_E_HIP) return fail(TRSTMI_E_HIP, "optimise: a HIP call failed");
          if (rs != TRSTMI_OK) return fail(rs, "optimise: trust-region step failed");
          tp.radius = rep.new_radius;
          if (tp.radius < op->radius_min || rep.cg_exit == TRSTMI_CG_ZERO_GRADIENT) break;
        }
      }
      if ((rs = trstmi_coherence(n, d, TRSTMI_MODE_FP64, W, mu_dev, cws, cws_bytes, stream))) return rs;
      double mu = 0.0;
      TRY_HIP(hipMemcpyAsync(&mu, mu_dev, sizeof(double), hipMemcpyDeviceToHost, stream), "optimise: read mu");
      TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
      if (mu < best_mu) {
        best_mu = mu;
        best_l = l;
        TRY_HIP(hipMemcpyAsync(best_frame(), W, (size_t)2 * d * n * 8, hipMemcpyDeviceToDevice, stream),
                "optimise: copy");
      }
    }
    TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
    return TRSTMI_OK;
  }
};

}  // namespace

trstmi_status trstmi_optimize(int64_t n, int64_t d, const trstmi_opt_params* op, double* best_frame, double* best_mu,
                              int32_t* best_restart, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (d > 64) return fail(TRSTMI_E_UNSUPPORTED, "the optimiser supports d <= 64");
  if (!op || !best_mu || !best_restart) return fail(TRSTMI_E_INVALID_ARG, "params, best_mu and best_restart are host pointers");
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  bool ok = op->restarts >= 1 && op->n_deltas >= 1 && op->deltas && op->steps_per_delta >= 1 && pos(op->radius0) &&
            op->radius_min >= 0.0 && op->radius_max >= op->radius0 && std::isfinite(op->radius_max) &&
            op->eta >= 0.0 && op->eta < 0.25 && pos(op->cg_tol) && op->cg_max_iter >= 0 && (op->fd_step == 0.0 || pos(op->fd_step)) &&
            op->concurrency >= 1 && op->concurrency <= 64 && op->first_restart >= 0 &&
            (int64_t)op->first_restart + op->restarts <= INT32_MAX;
  for (int32_t k = 0; ok && k < op->n_deltas; ++k) ok = pos(op->deltas[k]);
  if (!ok) return fail(TRSTMI_E_INVALID_ARG, "invalid optimiser parameters");
  if (!best_frame || ((uintptr_t)best_frame & 15)) return fail(TRSTMI_E_INVALID_ARG, "best_frame: null or misaligned");
  const size_t need = trstmi_optimize_workspace_bytes(n, d, op->concurrency);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  const int32_t P = std::min(op->concurrency, op->restarts);
  const size_t slot_bytes = optimize_slot_bytes(n, d);

  std::atomic<bool> abort{false};
  std::vector<OptWorker> work(P);
  for (int32_t t = 0; t < P; ++t) {
    work[t].abort = &abort;
    work[t].n = n;
    work[t].d = d;
    work[t].op = op;
    work[t].slot = (char*)workspace + (size_t)t * slot_bytes;
    work[t].stream = stream;
    work[t].first = t;
    work[t].stride = P;
  }
  if (P == 1) {
    work[0].st = work[0].run();
  } else {
    int dev = 0;
    TRY_HIP(hipGetDevice(&dev), "optimise: device");
    TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
    for (int32_t t = 0; t < P; ++t) {
      hipError_t e = hipStreamCreateWithFlags(&work[t].stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        for (int32_t u = 0; u < t; ++u) (void)hipStreamDestroy(work[u].stream);
        return hip_fail(e, "optimise: stream");
      }
    }
    std::vector<std::thread> threads;
    for (int32_t t = 0; t < P; ++t)
      threads.emplace_back([&work, t, dev]() {
        OptWorker& w = work[t];
        hipError_t e = hipSetDevice(dev);
        w.st = e == hipSuccess ? w.run() : hip_fail(e, "optimise: device");
        if (w.st != TRSTMI_OK) {
          w.err = g_last_error;
          w.abort->store(true, std::memory_order_relaxed);
        }
      });
    for (auto& th : threads) th.join();
    for (int32_t t = 0; t < P; ++t) (void)hipStreamDestroy(work[t].stream);
    for (int32_t t = 0; t < P; ++t)
      if (work[t].st != TRSTMI_OK) return fail(work[t].st, work[t].err);
  }
  if (work[0].st != TRSTMI_OK) return work[0].st;
  int32_t w_best = -1;
  for (int32_t t = 0; t < P; ++t) {
    const OptWorker& w = work[t];
    if (w.best_l < 0) continue;
    if (w_best < 0 || w.best_mu < work[w_best].best_mu ||
        (w.best_mu == work[w_best].best_mu && w.best_l < work[w_best].best_l))
      w_best = t;
  }
  *best_mu = __builtin_inf();
  *best_restart = -1;
  if (w_best >= 0) {
    *best_mu = work[w_best].best_mu;
    *best_restart = work[w_best].best_l;
    TRY_HIP(hipMemcpyAsync(best_frame, work[w_best].best_frame(), (size_t)2 * d * n * 8, hipMemcpyDeviceToDevice,
                           stream), "optimise: copy");
  }
  TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
  return TRSTMI_OK;
}

size_t trstmi_optimize_batched_workspace_bytes(int64_t n, int64_t d, int32_t restarts) {
  if (n < 2 || n > kOptMaxN || d < 1 || d > kOptMaxD || restarts < 1) return 0;
  return align256((size_t)restarts * opt_batch_stride(n, d) * 8) + align256((size_t)restarts * 8) + 256 * 8;
}

trstmi_status trstmi_optimize_batched(int64_t n, int64_t d, const trstmi_opt_params* op, double* best_frame,
                                      double* best_mu, int32_t* best_restart, void* workspace,
                                      size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if (n > kOptMaxN || d > kOptMaxD)
    return fail(TRSTMI_E_UNSUPPORTED, "the batched optimiser holds a start in one block: n <= 128, d <= 16");
  if (!op || !best_mu || !best_restart) return fail(TRSTMI_E_INVALID_ARG, "params, best_mu and best_restart are host pointers");
  auto pos = [](double x) { return x > 0.0 && std::isfinite(x); };
  bool ok = op->restarts >= 1 && op->n_deltas >= 1 && op->n_deltas <= 256 && op->deltas && op->steps_per_delta >= 1 &&
            pos(op->radius0) && op->radius_min >= 0.0 && op->radius_max >= op->radius0 &&
            std::isfinite(op->radius_max) && op->eta >= 0.0 && op->eta < 0.25 && pos(op->cg_tol) &&
            op->cg_max_iter >= 0 && op->first_restart >= 0 && (int64_t)op->first_restart + op->restarts <= INT32_MAX;
  for (int32_t k = 0; ok && k < op->n_deltas; ++k) ok = pos(op->deltas[k]);
  if (!ok) return fail(TRSTMI_E_INVALID_ARG, "invalid optimiser parameters");
  if (op->fd_step != 0.0) return fail(TRSTMI_E_UNSUPPORTED, "the batched optimiser uses exact Hessian products (fd_step 0)");
  if (!best_frame || ((uintptr_t)best_frame & 15)) return fail(TRSTMI_E_INVALID_ARG, "best_frame: null or misaligned");
  const size_t need = trstmi_optimize_batched_workspace_bytes(n, d, op->restarts);
  if ((st = check_ws(workspace, workspace_bytes, need))) return st;
  char* ws = (char*)workspace;
  const size_t stride = opt_batch_stride(n, d);
  const size_t work_bytes = align256((size_t)op->restarts * stride * 8);
  double* mu = (double*)(ws + work_bytes);
  double* deltas = (double*)(ws + work_bytes + align256((size_t)op->restarts * 8));
  OptBatchArgs a{};
  a.n = (int32_t)n;
  a.d = (int32_t)d;
  a.starts = op->restarts;
  a.first = op->first_restart;
  a.seed = (uint32_t)op->seed;
  a.n_deltas = op->n_deltas;
  a.steps_per_delta = op->steps_per_delta;
  a.cg_max_iter = op->cg_max_iter ? op->cg_max_iter : (int32_t)(2 * d * n);
  a.deltas = deltas;
  a.radius0 = op->radius0;
  a.radius_min = op->radius_min;
  a.radius_max = op->radius_max;
  a.eta = op->eta;
  a.cg_tol = op->cg_tol;
  a.work = (double*)ws;
  a.stride = (int64_t)stride;
  a.mu = mu;
  TRY_HIP(hipMemcpyAsync(deltas, op->deltas, (size_t)op->n_deltas * 8, hipMemcpyHostToDevice, stream), "deltas");
  TRY_HIP(TIMED("opt_batch", stream, launch_opt_batch(a, stream)), "optimise (batched)");
  std::vector<double> host_mu(op->restarts);
  TRY_HIP(hipMemcpyAsync(host_mu.data(), mu, (size_t)op->restarts * 8, hipMemcpyDeviceToHost, stream), "read mu");
  TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
  int32_t best = -1;
  for (int32_t l = 0; l < op->restarts; ++l)
    if (host_mu[l] == host_mu[l] && (best < 0 || host_mu[l] < host_mu[best])) best = l;
  *best_mu = best >= 0 ? host_mu[best] : __builtin_inf();
  *best_restart = best >= 0 ? op->first_restart + best : -1;
  if (best >= 0) {
    TRY_HIP(hipMemcpyAsync(best_frame, a.work + (size_t)best * stride, (size_t)2 * d * n * 8, hipMemcpyDeviceToDevice,
                           stream), "optimise: copy");
    TRY_HIP(hipStreamSynchronize(stream), "optimise: sync");
  }
  return TRSTMI_OK;
}

trstmi_status trstmi_init_haar(const trstmi_params* p, const trstmi_state* state, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
  trstmi_status st = check_params(p);
  if (st) return st;
  if ((st = check_state(state))) return st;
  const Layout L = layout_of(p);
  if ((st = check_ws(workspace, workspace_bytes, L.total))) return st;
  char* ws = (char*)workspace;
  uint64_t* mx = (uint64_t*)(ws + L.cand_max);

  PerturbArgs pa = perturb_base(p);
  pa.base = nullptr;
  pa.tag = 1;
  pa.t_const = 0;
  pa.c0 = 0;
  pa.out = state->frame;
  pa.out_kind = kOutF64;
  pa.out_ld = (int32_t)(2 * p->d);
  pa.out_slot_stride = 2 * p->d * p->n;
  pa.zero_max = mx;
  TRY_HIP(launch_perturb(pa, 1, stream), "haar");
  const bool f32 = p->mode == TRSTMI_MODE_FP32;
  if (f32) {
    float* buf = (float*)(ws + L.cand);
    TRY_HIP(launch_convert_f32(state->frame, p->n, (int32_t)p->d, buf, L.ld, mx, stream), "convert");
    GramArgs g = gram_base(p->n, p->d, buf, p->n * L.ld, L.ld, kTileF32, mx, nullptr);
    TRY_HIP(launch_gram_f32(g, 1, stream), "gram_f32");
  } else {
    GramArgs g = gram_base(p->n, p->d, state->frame, 2 * p->d * p->n, (int32_t)(2 * p->d), kTileF64, mx, nullptr);
    TRY_HIP(launch_gram_f64(g, 1, stream), "gram_f64");
  }
  InitFinishArgs f{};
  f.max_bits = mx;
  f.is_f32 = f32 ? 1 : 0;
  f.mu = state->mu;
  f.radius = state->radius;
  f.step = state->step;
  f.flags = state->flags;
  f.radius0 = p->radius0;
  f.max_steps = p->max_steps;
  f.target_mu = p->target_mu;
  TRY_HIP(launch_init_finish(f, stream), "init_finish");
  return TRSTMI_OK;
}

trstmi_status trstmi_candidates(const trstmi_params* p, const double* frame, const double* radius, int64_t t,
                                int32_t c0, int32_t count, const double* explicit_z, double* out,
                                hipStream_t stream) {
  trstmi_status st = check_params(p);
  if (st) return st;
  if (!frame || !radius || !out) return fail(TRSTMI_E_INVALID_ARG, "frame, radius and out must be device pointers");
  if (((uintptr_t)frame & 15) || ((uintptr_t)out & 15)) return fail(TRSTMI_E_INVALID_ARG, "misaligned pointer");
  if (count < 1 || c0 < 0 || t < 0 || t >= ((int64_t)1 << 32) || (int64_t)c0 + count > ((int64_t)1 << 31))
    return fail(TRSTMI_E_INVALID_ARG, "bad candidate range or step");
  if (count > 65535) return fail(TRSTMI_E_INVALID_ARG, "count must be <= 65535");
  if (explicit_z && (int64_t)c0 + count > p->candidates)
    return fail(TRSTMI_E_INVALID_ARG, "explicit_z holds params.candidates draws: need c0 + count <= candidates");
  PerturbArgs pa = perturb_base(p);
  pa.base = frame;
  pa.radius = radius;
  pa.t_const = t;
  pa.c0 = c0;
  pa.z_explicit = explicit_z;
  pa.out = out;
  pa.out_kind = kOutF64;
  pa.out_ld = (int32_t)(2 * p->d);
  pa.out_slot_stride = 2 * p->d * p->n;
  TRY_HIP(launch_perturb(pa, count, stream), "candidates");
  return TRSTMI_OK;
}

trstmi_status trstmi_step(const trstmi_params* p, const trstmi_state* state, void* workspace, size_t workspace_bytes,
                          const double* explicit_z, const trstmi_report* report, hipStream_t stream) {
  trstmi_status st = check_params(p);
  if (st) return st;
  if ((st = check_state(state))) return st;
  const Layout L = layout_of(p);
  if ((st = check_ws(workspace, workspace_bytes, L.total))) return st;
  if (explicit_z && ((uintptr_t)explicit_z & 15)) return fail(TRSTMI_E_INVALID_ARG, "explicit_z misaligned");
  return enqueue_step(p, state, (char*)workspace, explicit_z, report, stream);
}

trstmi_status trstmi_solve(const trstmi_params* p, const trstmi_state* state, void* workspace,
                           size_t workspace_bytes, int32_t chunk, hipStream_t stream) {
  trstmi_status st = check_params(p);
  if (st) return st;
  if ((st = check_state(state))) return st;
  const Layout L = layout_of(p);
  if ((st = check_ws(workspace, workspace_bytes, L.total))) return st;
  if (chunk < 1) return fail(TRSTMI_E_INVALID_ARG, "chunk must be >= 1");
  char* ws = (char*)workspace;

  int64_t t0 = 0;
  int32_t flags = 0;
  TRY_HIP(hipMemcpyAsync(&t0, state->step, sizeof(t0), hipMemcpyDeviceToHost, stream), "read step");
  TRY_HIP(hipMemcpyAsync(&flags, state->flags, sizeof(flags), hipMemcpyDeviceToHost, stream), "read flags");
  TRY_HIP(hipStreamSynchronize(stream), "sync");
  if (flags & TRSTMI_FLAG_DONE) return TRSTMI_OK;
  const int64_t left = p->max_steps > t0 ? p->max_steps - t0 : 0;
  const int64_t max_chunks = left / chunk + 2;

  // Capture one chunk of steps into a graph (relaxed mode: calls made by other
  // threads cannot invalidate it).  If capture is not possible the chunk is
  // launched directly instead.
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (stream != nullptr && hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
    trstmi_status cst = TRSTMI_OK;
    for (int i = 0; i < chunk && cst == TRSTMI_OK; ++i) cst = enqueue_step(p, state, ws, nullptr, nullptr, stream);
    const hipError_t e2 = hipStreamEndCapture(stream, &graph);
    if (cst == TRSTMI_OK && e2 == hipSuccess && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
      exec = nullptr;
    if (!exec) {
      if (graph) (void)hipGraphDestroy(graph);
      graph = nullptr;
      (void)hipGetLastError();
      g_last_error.clear();
    }
  }
  trstmi_status result = TRSTMI_OK;
  for (int64_t it = 0; it < max_chunks; ++it) {
    if (exec) {
      hipError_t e = hipGraphLaunch(exec, stream);
      if (e != hipSuccess) {
        result = hip_fail(e, "graph launch");
        break;
      }
    } else {
      for (int i = 0; i < chunk && result == TRSTMI_OK; ++i)
        result = enqueue_step(p, state, ws, nullptr, nullptr, stream);
      if (result != TRSTMI_OK) break;
    }
    hipError_t e = hipMemcpyAsync(&flags, state->flags, sizeof(flags), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "poll");
      break;
    }
    if (flags & TRSTMI_FLAG_DONE) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  return result;
}

trstmi_status trstmi_timing_enable(int32_t on) {
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  T.on = on != 0;
  return TRSTMI_OK;
}

trstmi_status trstmi_timing_only(const char* kernel) {
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  T.only = kernel ? kernel : "";
  return TRSTMI_OK;
}

trstmi_status trstmi_timing_reset(void) {
  trstmi_status st = drain_timing();
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  T.totals.clear();
  return st;
}

trstmi_status trstmi_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return fail(TRSTMI_E_INVALID_ARG, "timing_read: NULL argument");
  trstmi_status st = drain_timing();
  if (st) return st;
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  auto it = T.totals.find(kernel);
  *total_ms = it == T.totals.end() ? 0.0 : it->second.first;
  *launches = it == T.totals.end() ? 0 : it->second.second;
  return TRSTMI_OK;
}

size_t trstmi_batch_workspace_bytes(const trstmi_batch_params* p, const trstmi_batch_instance* inst) {
  BatchLayout L;
  if (batch_layout(p, inst, L)) return 0;
  return L.total;
}

trstmi_status trstmi_batch_init(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                                size_t workspace_bytes, hipStream_t stream) {
  BatchLayout L;
  trstmi_status st = batch_prepare(p, inst, workspace, workspace_bytes, L);
  if (st) return st;
  char* ws = (char*)workspace;
  std::vector<char> host_inst((size_t)p->count * batch_inst_bytes());
  for (int32_t i = 0; i < p->count; ++i)
    batch_fill_inst(host_inst.data() + (size_t)i * batch_inst_bytes(), inst[i].n, inst[i].d, L.wpi[i], inst[i].seed,
                    inst[i].stream_id, L.frame_off[i], inst[i].target_mu, inst[i].max_steps);
  std::vector<char> zeros(256 + (size_t)p->count * batch_state_bytes(), 0);
  TRY_HIP(hipMemcpyAsync(ws + L.hdr, zeros.data(), 256, hipMemcpyHostToDevice, stream), "batch header");
  TRY_HIP(hipMemcpyAsync(ws + L.state, zeros.data(), (size_t)p->count * batch_state_bytes(), hipMemcpyHostToDevice,
                         stream), "batch state");
  TRY_HIP(hipMemcpyAsync(ws + L.inst, host_inst.data(), host_inst.size(), hipMemcpyHostToDevice, stream), "batch inst");
  TRY_HIP(hipMemcpyAsync(ws + L.units, L.unit_list.data(), L.unit_list.size() * sizeof(int2), hipMemcpyHostToDevice,
                         stream), "batch units");
  const BatchArgs b = batch_args(p, L, ws);
  TRY_HIP(TIMED("batch_init", stream, launch_batch_init(b, p->count, p->radius0, stream)), "batch init");
  TRY_HIP(hipStreamSynchronize(stream), "batch init sync");  // host buffers above must outlive the copies
  return TRSTMI_OK;
}

trstmi_status trstmi_batch_step(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                                size_t workspace_bytes, int32_t launches, double* rep_mu, int32_t* rep_best,
                                hipStream_t stream) {
  BatchLayout L;
  trstmi_status st = batch_prepare(p, inst, workspace, workspace_bytes, L);
  if (st) return st;
  if (launches < 0) return fail(TRSTMI_E_INVALID_ARG, "launches must be >= 0");
  BatchArgs b = batch_args(p, L, (char*)workspace);
  b.rep_mu = rep_mu;
  b.rep_best = rep_best;
  const int grid = batch_grid(L);
  for (int32_t l = 0; l < launches; ++l)
    TRY_HIP(TIMED("batch_step", stream, launch_batch_step(b, grid, stream)), "batch step");
  return TRSTMI_OK;
}

trstmi_status trstmi_batch_run(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                               size_t workspace_bytes, int32_t chunk, int64_t max_chunks, int32_t* all_done,
                               hipStream_t stream) {
  BatchLayout L;
  trstmi_status st = batch_prepare(p, inst, workspace, workspace_bytes, L);
  if (st) return st;
  if (chunk < 1 || max_chunks < 0) return fail(TRSTMI_E_INVALID_ARG, "chunk must be >= 1, max_chunks >= 0");
  char* ws = (char*)workspace;
  const BatchArgs b = batch_args(p, L, ws);
  int32_t done = 0;
  if (all_done) *all_done = 0;
  TRY_HIP(hipMemcpyAsync(&done, b.done_instances, 4, hipMemcpyDeviceToHost, stream), "batch poll");
  TRY_HIP(hipStreamSynchronize(stream), "batch poll");
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (stream != nullptr && done < p->count && max_chunks > 0) {
    TRY_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed), "batch capture");
    hipError_t le = hipSuccess;
    for (int32_t l = 0; l < chunk && le == hipSuccess; ++l) le = launch_batch_step(b, batch_grid(L), stream);
    hipError_t ce = hipStreamEndCapture(stream, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(le != hipSuccess ? le : ce, "batch capture");
    }
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(ie, "batch graph instantiate");
    }
  }
  trstmi_status result = TRSTMI_OK;
  for (int64_t k = 0; k < max_chunks && done < p->count; ++k) {
    hipError_t e = hipSuccess;
    if (exec) {
      e = hipGraphLaunch(exec, stream);
    } else {
      for (int32_t l = 0; l < chunk && e == hipSuccess; ++l) e = launch_batch_step(b, batch_grid(L), stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&done, b.done_instances, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "batch run");
      break;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (result == TRSTMI_OK && all_done) *all_done = done >= p->count ? 1 : 0;
  return result;
}

trstmi_status trstmi_batch_query(const trstmi_batch_params* p, const trstmi_batch_instance* inst,
                                 const void* workspace, size_t workspace_bytes, double* mu, double* radius,
                                 int64_t* step, int32_t* flags, int32_t* done_instances, hipStream_t stream) {
  BatchLayout L;
  trstmi_status st = batch_prepare(p, inst, workspace, workspace_bytes, L);
  if (st) return st;
  const char* ws = (const char*)workspace;
  std::vector<char> buf((size_t)p->count * batch_state_bytes());
  int32_t hdr[4] = {0, 0, 0, 0};
  TRY_HIP(hipMemcpyAsync(buf.data(), ws + L.state, buf.size(), hipMemcpyDeviceToHost, stream), "batch query");
  TRY_HIP(hipMemcpyAsync(hdr, ws + L.hdr, sizeof(hdr), hipMemcpyDeviceToHost, stream), "batch query");
  TRY_HIP(hipStreamSynchronize(stream), "batch query");
  const size_t sb = batch_state_bytes();
  for (int32_t i = 0; i < p->count; ++i) {
    const char* s = buf.data() + (size_t)i * sb;  // {double mu, double radius, int64 step, int32 flags, int32 count}
    if (mu) std::memcpy(&mu[i], s, 8);
    if (radius) std::memcpy(&radius[i], s + 8, 8);
    if (step) std::memcpy(&step[i], s + 16, 8);
    if (flags) std::memcpy(&flags[i], s + 24, 4);
  }
  if (done_instances) *done_instances = hdr[2];
  return TRSTMI_OK;
}

trstmi_status trstmi_batch_frame(const trstmi_batch_params* p, const trstmi_batch_instance* inst,
                                 const void* workspace, size_t workspace_bytes, int32_t i, double* out,
                                 hipStream_t stream) {
  BatchLayout L;
  trstmi_status st = batch_prepare(p, inst, workspace, workspace_bytes, L);
  if (st) return st;
  if (i < 0 || i >= p->count || !out) return fail(TRSTMI_E_INVALID_ARG, "bad instance index or output");
  const char* ws = (const char*)workspace;
  const size_t bytes = (size_t)2 * inst[i].d * inst[i].n * 8;
  TRY_HIP(hipMemcpyAsync(out, ws + L.frames + (size_t)L.frame_off[i] * 8, bytes, hipMemcpyDeviceToDevice, stream),
          "batch frame");
  return TRSTMI_OK;
}

const char* trstmi_last_error(void) { return g_last_error.c_str(); }

double trstmi_bf16_screen_bound(int64_t d) { return d >= 1 ? screen_eps(d) : NAN; }

double trstmi_batch_screen_bound(int32_t d) { return d >= 1 && d <= 16 ? batch_screen_eps(d) : NAN; }

trstmi_status trstmi_shutdown(void) {
  Timing& T = timing();
  std::lock_guard<std::mutex> g(T.mu);
  for (auto& r : T.pending) {
    (void)hipEventSynchronize(r.stop);
    T.pool.push_back(r.start);
    T.pool.push_back(r.stop);
  }
  T.pending.clear();
  for (hipEvent_t e : T.pool) (void)hipEventDestroy(e);
  T.pool.clear();
  T.totals.clear();
  T.on = false;
  T.only.clear();
  return TRSTMI_OK;
}

int32_t trstmi_abi_version(void) { return 14; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Coherence without allocation: the workspace is a fixed device array of the
// library (each GPU the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address is looked up once per device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocBytes = ((size_t)16 << 20) + 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

trstmi_status scratch_of_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "device");
  if (dev < 0 || dev >= kMaxDevices) return fail(TRSTMI_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TRSTMI_OK;
}

}  // namespace

extern "C" {

size_t trstmi_coherence_noalloc_max_bytes(void) { return kNoAllocBytes; }

trstmi_status trstmi_coherence_noalloc(int64_t n, int64_t d, int32_t mode, const double* frame, double* mu_out,
                                       hipStream_t stream) {
  trstmi_status st = check_size(n, d);
  if (st) return st;
  if ((st = check_mode(mode))) return st;
  const size_t need = trstmi_coherence_workspace_bytes(n, d, mode);
  if (need > kNoAllocBytes)
    return fail(TRSTMI_E_UNSUPPORTED, "frame too large for the fixed workspace: needs " + std::to_string(need) +
                                          " bytes, the library holds " + std::to_string(kNoAllocBytes));
  void* ws = nullptr;
  if ((st = scratch_of_device(&ws))) return st;
  return trstmi_coherence(n, d, mode, frame, mu_out, ws, kNoAllocBytes, stream);
}

}  // extern "C"
