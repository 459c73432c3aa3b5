// Select / accept / radius update, top-k screening selection, and the
// finishing kernels of the random start and of the coherence entry point.
//
// All run as a single 256-thread block on the stream after the Gram kernels,
// so a step never waits on the host.  Candidate maxima arrive as IEEE bit
// patterns of max |G|^2 (double, or float widened to 64 bits); a pattern at
// or above +inf is an invalid candidate.  mu_c = sqrt(max |G|^2) in FP64.
// The best candidate is the minimum of (mu_c, c), ties to the lower index;
// it is accepted iff mu_c* < mu (strict); the radius is multiplied by grow
// on accept and by shrink otherwise, clamped to [radius_min, radius_max].

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kThreads = 256;
constexpr int kTopkThreads = 1024;  // the tile list of the top-k is built in one or two passes
constexpr int kBitmapWords = 65536 / 32;  // one bit per candidate
constexpr int kRankMax = 1024;            // rank selection up to this many candidates

__device__ __forceinline__ double bits_to_mu(uint64_t b, int is_f32) {
  if (is_f32) {
    const uint32_t f = (uint32_t)b;
    if (f >= kInfBits32) return __builtin_inf();
    return sqrt((double)__uint_as_float(f));
  }
  if (b >= kInfBits64) return __builtin_inf();
  return sqrt(__longlong_as_double((int64_t)b));
}

// (value, index) lexicographic min, and the smallest value of any other entry.
struct Best2 {
  double v1;
  int c1;
  double v2;
};

__device__ __forceinline__ void best2_push(Best2& b, double v, int c) {
  if (v < b.v1 || (v == b.v1 && c < b.c1)) {
    b.v2 = b.v1;
    b.v1 = v;
    b.c1 = c;
  } else if (v < b.v2) {
    b.v2 = v;
  }
}

__device__ __forceinline__ void best2_merge(Best2& a, const Best2& o) {
  if (o.c1 >= 0) best2_push(a, o.v1, o.c1);
  if (o.v2 < a.v2) a.v2 = o.v2;
}

__device__ __forceinline__ void select_body(const SelectArgs& a) {
  __shared__ Best2 sh[kThreads];
  const int tid = threadIdx.x;
  if (*a.flags & kFlagDone) {
    if (tid == 0) a.dec->commit = 0;
    return;
  }
  Best2 b = {__builtin_inf(), -1, __builtin_inf()};
  for (int s = tid; s < a.count; s += kThreads) {
    const double mu = bits_to_mu(a.cand_max[s], a.is_f32);
    const int c = a.slot_cand ? a.slot_cand[s] : s;
    if (a.rep_cand_mu) a.rep_cand_mu[s] = mu;
    if (mu < __builtin_inf()) best2_push(b, mu, c);
  }
  sh[tid] = b;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      Best2 x = sh[tid];
      best2_merge(x, sh[tid + off]);
      sh[tid] = x;
    }
    __syncthreads();
  }
  if (tid != 0) return;
  const Best2 r = sh[0];
  const double mu_t = *a.mu;
  const double rad = *a.radius;
  const int64_t t = *a.step;
  const bool valid = r.c1 >= 0;
  const bool accept = valid && r.v1 < mu_t;
  bool near = valid && fabs(r.v1 - mu_t) <= a.tau;
  if (valid && r.v2 - r.v1 <= a.tau) near = true;
  if (a.use_screen_near && a.dec->screen_near) near = true;

  a.dec->best = r.c1;
  a.dec->t_old = t;
  a.dec->radius_old = rad;
  a.dec->commit = accept ? 1 : 0;
  double new_mu = mu_t;
  double new_rad;
  if (accept) {
    new_mu = r.v1;
    new_rad = fmin(rad * a.grow, a.radius_max);
  } else {
    new_rad = fmax(rad * a.shrink, a.radius_min);
  }
  const int64_t nt = t + 1;
  const bool done = (a.target_mu > 0.0 && new_mu <= a.target_mu) || nt >= a.max_steps;
  *a.mu = new_mu;
  *a.radius = new_rad;
  *a.step = nt;
  *a.flags = (accept ? kFlagAccepted : 0) | (near ? kFlagNearTie : 0) | (valid ? 0 : kFlagNoValid) |
             (done ? kFlagDone : 0);
  if (a.rep_best) *a.rep_best = r.c1;
}

__global__ __launch_bounds__(kThreads) void k_select(SelectArgs a) { select_body(a); }

// The same for a group of searches: search blockIdx.x of the table.
__global__ __launch_bounds__(kThreads) void k_select_tab(TabRef t) {
  const SelectArgs a = *(const SelectArgs*)(t.base + (size_t)t.list[blockIdx.x] * t.stride);
  select_body(a);
}

// k smallest screened values by (mu_screen, c); thresholds for certified pruning.
__device__ __forceinline__ void topk_body(const TopkArgs& a) {
  __shared__ double sv[kTopkThreads];
  __shared__ int sc[kTopkThreads];
  __shared__ uint32_t taken[kBitmapWords];
  __shared__ int sel_c[64];
  __shared__ double sel_thr[64];
  __shared__ int list_n;
  __shared__ uint64_t keys[kRankMax];
  __shared__ double kth[2];
  const int tid = threadIdx.x;
  if (*a.flags & kFlagDone) return;
  for (int c = tid; c < a.C && a.rep_cand_mu; c += kTopkThreads) a.rep_cand_mu[c] = bits_to_mu(a.cand_max[c], 1);
  if (a.C <= kRankMax) {
    // Rank selection: key = (screened bits clamped at +inf, c) orders like
    // (mu_screen, c); the candidate of rank r < k is the r-th rechecked one.
    for (int c = tid; c < a.C; c += kTopkThreads) {
      const uint32_t b = (uint32_t)a.cand_max[c];
      keys[c] = ((uint64_t)(b < kInfBits32 ? b : kInfBits32) << 32) | (uint32_t)c;
    }
    if (tid < 2) kth[tid] = 0.0;
    __syncthreads();
    for (int c = tid; c < a.C; c += kTopkThreads) {
      const uint64_t key = keys[c];
      int rank = 0;
      for (int o = 0; o < a.C; ++o) rank += keys[o] < key ? 1 : 0;
      if (rank <= a.k) {
        const double v = bits_to_mu(a.cand_max[c], 1);
        if (rank < a.k) {
          a.rechecked[rank] = c;
          // an invalid (non-finite) screened value disables pruning for that candidate
          a.thr[rank] = v < __builtin_inf() ? v - 2.0 * a.eps : -__builtin_inf();
          sel_c[rank] = c;
          sel_thr[rank] = a.thr[rank];
          if (a.rep_rechecked) a.rep_rechecked[rank] = c;
        }
        if (rank == a.k - 1) kth[0] = v;
        if (rank == a.k) kth[1] = v;
      }
    }
    __syncthreads();
    if (tid == 0) a.dec->screen_near = (a.k < a.C && kth[1] - kth[0] <= a.screen_tie) ? 1 : 0;
  } else {
    for (int q = tid; q < kBitmapWords; q += kTopkThreads) taken[q] = 0;
    __syncthreads();
    double prev = 0.0;
    for (int round = 0; round <= a.k && round < a.C; ++round) {
      double bv = __builtin_inf();
      int bc = 0x7fffffff;
      for (int c = tid; c < a.C; c += kTopkThreads) {
        if (taken[c >> 5] & (1u << (c & 31))) continue;
        const double mu = bits_to_mu(a.cand_max[c], 1);
        if (mu < bv || (mu == bv && c < bc)) {
          bv = mu;
          bc = c;
        }
      }
      sv[tid] = bv;
      sc[tid] = bc;
      __syncthreads();
      for (int off = kTopkThreads / 2; off > 0; off >>= 1) {
        if (tid < off) {
          const double ov = sv[tid + off];
          const int oc = sc[tid + off];
          if (ov < sv[tid] || (ov == sv[tid] && oc < sc[tid])) {
            sv[tid] = ov;
            sc[tid] = oc;
          }
        }
        __syncthreads();
      }
      const double v = sv[0];
      const int c = sc[0];
      __syncthreads();
      if (round < a.k) {
        if (tid == 0) {
          taken[c >> 5] |= 1u << (c & 31);
          a.rechecked[round] = c;
          // an invalid (non-finite) screened value disables pruning for that candidate
          a.thr[round] = v < __builtin_inf() ? v - 2.0 * a.eps : -__builtin_inf();
          sel_c[round] = c;
          sel_thr[round] = a.thr[round];
          if (a.rep_rechecked) a.rep_rechecked[round] = c;
        }
        prev = v;
      } else if (tid == 0) {
        a.dec->screen_near = (v - prev <= a.screen_tie) ? 1 : 0;
      }
      __syncthreads();
    }
    if (tid == 0 && a.k >= a.C) a.dec->screen_near = 0;
  }

  // Certified pruning.  For every pair |screened - exact| <= eps, so a screen
  // tile whose screened maximum is below (candidate's screened max - 2 eps)
  // cannot hold the candidate's exact maximum.  List the remaining screen
  // tiles of every rechecked candidate (an invalid candidate needs none: its
  // FP64 value is invalid as well).  Appends are aggregated per wavefront.
  if (tid == 0) list_n = 0;
  __syncthreads();
  const int sn = a.screen_nt * (a.screen_nt + 1) / 2;
  const int lane = tid & 63;
  constexpr int kU = 4;  // entries per thread per pass, loaded before any is used
  for (int e0 = 0; e0 < a.k * sn; e0 += kTopkThreads * kU) {
    uint4 tm[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * kTopkThreads + tid;
      tm[u] = make_uint4(0u, 0u, 0u, 0u);
      if (e < a.k * sn) {
        const int slot = e / sn;
        if (sel_thr[slot] > -__builtin_inf())
          tm[u] = *(const uint4*)(a.tile_max + ((size_t)sel_c[slot] * sn + (e - slot * sn)) * 4);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * kTopkThreads + tid;
      bool keep = false;
      int slot = 0, st = 0, qmask = 0;
      if (e < a.k * sn) {
        slot = e / sn;
        st = e - slot * sn;
        if (sel_thr[slot] > -__builtin_inf()) {
          // entry q bounds the screened values of the tile's rows 32 q ..
          // 32 q + 31 (the Gram kernels write one entry per 32-row quarter,
          // or per 64-row half into both of its quarters, or one value into
          // all four); bit q of the mask marks a quarter that can qualify
          // (squares compared against thr^2 lowered by 1e-12 relative: at
          // worst a quarter on the boundary is kept; a NaN entry is kept)
          const double t = sel_thr[slot];
          const double t2 = t > 0.0 ? t * t * (1.0 - 1e-12) : -__builtin_inf();
          const uint32_t e4[4] = {tm[u].x, tm[u].y, tm[u].z, tm[u].w};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (!((double)__uint_as_float(e4[q]) < t2)) qmask |= 1 << q;
          keep = qmask != 0;
        }
      }
      const uint64_t ballot = __ballot(keep);
      int base = 0;
      if (lane == 0 && ballot) base = atomicAdd(&list_n, __popcll(ballot));
      base = __shfl(base, 0, 64);
      if (keep) {
        const int pos = base + __popcll(ballot & ((1ull << lane) - 1));
        if (pos < a.list_cap) a.list[pos] = make_int2(slot | (qmask << 8), st);
      }
    }
  }
  __syncthreads();
  if (tid == 0) *a.list_count = list_n < a.list_cap ? list_n : a.list_cap;
}

__global__ __launch_bounds__(kTopkThreads) void k_topk(TopkArgs a) { topk_body(a); }

__global__ __launch_bounds__(kTopkThreads) void k_topk_tab(TabRef t) {
  const TopkArgs a = *(const TopkArgs*)(t.base + (size_t)t.list[blockIdx.x] * t.stride);
  topk_body(a);
}

// State of every listed search after a run of group steps: (flags, step, mu)
// through the state pointers of its select record.
__global__ __launch_bounds__(64) void k_poll_tab(TabRef t, PollRecord* out) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= t.count) return;
  const SelectArgs& a = *(const SelectArgs*)(t.base + (size_t)t.list[i] * t.stride);
  PollRecord r;
  r.flags = *a.flags;
  r.pad = 0;
  r.step = *a.step;
  r.mu = *a.mu;
  out[i] = r;
}

__global__ void k_init_finish(InitFinishArgs a) {
  if (threadIdx.x != 0) return;
  const double mu = bits_to_mu(*a.max_bits, a.is_f32);
  if (a.mu_out) {
    *a.mu_out = mu;
    return;
  }
  *a.mu = mu;
  *a.radius = a.radius0;
  *a.step = 0;
  const bool done = (a.target_mu > 0.0 && mu <= a.target_mu) || a.max_steps <= 0;
  *a.flags = done ? kFlagDone : 0;
}

}  // namespace

hipError_t launch_select(const SelectArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_topk(const TopkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(kTopkThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_select_tab(const TabRef& t, hipStream_t s) {
  hipLaunchKernelGGL(k_select_tab, dim3(t.count), dim3(kThreads), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_topk_tab(const TabRef& t, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_tab, dim3(t.count), dim3(kTopkThreads), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_poll_tab(const TabRef& t, PollRecord* out, hipStream_t s) {
  hipLaunchKernelGGL(k_poll_tab, dim3((t.count + 63) / 64), dim3(64), 0, s, t, out);
  return hipGetLastError();
}

hipError_t launch_init_finish(const InitFinishArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace trstmi
