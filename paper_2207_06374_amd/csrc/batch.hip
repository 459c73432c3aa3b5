// Batched form: many independent, uneven searches advanced together, one
// persistent kernel launch for every candidate of every instance plus one
// finalizing launch per step.
//
// Every instance i is an independent search (its own N_i, d_i, frame, radius,
// step and RNG stream) with the candidate rule of the single-frame path:
// candidate c at step t is Y = Phi + (radius / sqrt(d)) Z(i, c, t),
// renormalised; the best candidate by (mu_c, c) is accepted iff it lowers mu.
//
// Work: a unit is 1, 2 or 4 candidates of one instance, processed by one
// block of 4 wavefronts split into groups of `wpi` waves per candidate (the
// per-instance tile choice).  With one wave per candidate the phases below
// are separated by wave-level synchronisation only, so the block's waves
// run out of phase.  The step kernel is launched with at most as
// many blocks as the device holds at once; block b takes units b, b + grid,
// ... of the list (largest instances first), so no work counter is shared.
// Per candidate the group
//   1. draws and renormalises the candidate in FP64 (FP64 copy to global
//      scratch; to LDS, every real rounded to FP32 and held as two bfloat16
//      parts hi + lo);
//   2. screens every pair j < k with v_mfma_f32_16x16x32_bf16: Re and Im are
//      each the three products hi hi' + hi lo' + lo hi' of the split copies
//      (an FP32-class screen at three bfloat16 products instead of the FP32
//      matrix rate, which is no faster than the FP32 vector rate), keeping
//      the maximum of every 16 x 16 pair block;
//   3. re-evaluates exactly in FP64 the pairs whose screened |G| is within
//      2 eps of the screened maximum (eps bounds |screened - exact| for unit
//      columns, so the exact maximiser is among them): every candidate ends
//      with its exact FP64 coherence, stored with a plain write.
// The finalizing kernel (one block per instance) then selects, accepts,
// updates the radius and regenerates the accepted candidate in FP64 into the
// frame.  Handing the candidates' values over at the kernel boundary replaces
// a device-scope release per candidate (each of which writes back the L2 of
// its XCD) by the one at the end of the launch.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kThreads = 256;
// LDS words for the split copies of the candidates of one unit: N * ldk per
// group, summed over groups (ldk = split_row_words(d) <= 36 at d <= 16).
constexpr int kLdsWords = 9216;

struct alignas(16) BInst {
  int32_t n, d, wpi, ldk;  // ldk: words per column of the LDS split copy (split_row_words)
  uint32_t seed, stream_id;
  int64_t frame_off;       // doubles into the frame arena
  double target_mu;
  int64_t max_steps;
};

struct alignas(16) BState {
  double mu;
  double radius;
  int64_t step;
  int32_t flags;
  int32_t pad;
};

// Words per column of a candidate's LDS split copy: the hi parts of its 2d
// reals padded with zeros to kp = 2d rounded up to 8, then the lo parts
// likewise, then 16 bytes of padding (rows stay 16-byte aligned and the
// column-strided fragment reads spread over the banks).
__host__ __device__ constexpr int split_kp(int d) { return (2 * d + 7) / 8 * 8; }
__host__ __device__ constexpr int split_row_words(int d) { return split_kp(d) + 4; }

__host__ __device__ inline double eps_split(int d) {
  // |screened - exact| for unit columns, d <= 16.  Inputs: each real is
  // rounded to FP32 (f, relative 2^-24) and held as hi + lo (hi = bf16 of
  // f, lo = bf16 of the exact remainder r = f - hi).  With 2^e <= |f|,
  // |r| <= 2^(e-8); at equality r is a power of two and lo = r, otherwise r
  // lies at least nine binades below f and |lo - r| <= 2^-17 |f|.  So
  // hi + lo is within delta = 2^-17 (1 + 2^-24) + 2^-24 of the entry and the
  // inner product of two unit columns moves by at most 2 delta + delta^2.
  // Products: |lo| <= (1 + u) |r| <= u (1 + u) |f| (u = 2^-8), so the dropped
  // lo lo' add up to at most 2^-16 (1 + u)^2 (1 + 2^-24)^2 in each of Re and
  // Im.
  // Accumulation: 96 products (32 reals, zero padded, three products each)
  // summed in FP32 with faithful additions, gamma_96 (unit 2^-23) times at
  // most (1 + u)^2 (1 + 2u) (1 + 2^-24)^2.  Re and Im together give sqrt 2;
  // the tail covers the epilogue.
  (void)d;
  const double u = 0x1p-8, v = 0x1p-24, w = 0x1p-23;
  const double delta = 0x1p-17 * (1 + v) + v;
  const double unit = (1 + v) * (1 + v);
  const double dropped = 0x1p-16 * (1 + u) * (1 + u) * unit;
  const double g = 96 * w / (1.0 - 96 * w);
  const double acc = g * (1 + u) * (1 + u) * (1 + 2 * u) * unit;
  return (2 * delta + delta * delta) + 1.4142135623730951 * (dropped + acc) + 16 * v + 1e-12;
}

// x = hi + lo for two FP32 values: hi = bf16(x), lo = bf16(x - hi), both
// round to nearest even (x - hi is exact in FP32); packed with x[0] in the
// low half.
__device__ __forceinline__ void split_bf16x2(f32x2 x, uint32_t& hi, uint32_t& lo) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2));
  const float h0 = __uint_as_float(h << 16), h1 = __uint_as_float(h & 0xFFFF0000u);
  const f32x2 r = {x[0] - h0, x[1] - h1};
  hi = h;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
}

// Candidate c of instance I at step t, column col, Philox block q (entries 2q, 2q+1).
__device__ __forceinline__ void draw_block(const BInst& I, const double* frame, double s, int c, int64_t t,
                                           int64_t col, int q, const GaussTab& tab, double y[4], bool& two) {
  const int d = I.d;
  const int nb = (d + 1) >> 1;
  const int i0 = 2 * q;
  two = (i0 + 1) < d;
  const u32x4 ctr = {(uint32_t)(col * nb + q), (uint32_t)c, (uint32_t)t, 0u};
  const u32x4 w = philox4x32_10(ctr, I.seed, I.stream_id);
  double r0, c0, s0, r1, c1, s1;
  cn_polar(w.x, w.y, tab, r0, c0, s0);
  cn_polar(w.z, w.w, tab, r1, c1, s1);
  r0 *= s;
  r1 *= s;
  const double* bp = frame + 2 * ((size_t)col * d + i0);
  y[0] = fma(r0, c0, bp[0]);
  y[1] = fma(r0, s0, bp[1]);
  y[2] = two ? fma(r1, c1, bp[2]) : 0.0;
  y[3] = two ? fma(r1, s1, bp[3]) : 0.0;
}

// Lanes [0, nl) of the calling wave group regenerate candidate c (FP64, unit
// columns) into `out` (column stride 2d) and, when lds != null, into the LDS
// split copy.  Lanes of one column are LPC consecutive lanes; the norm is
// reduced with DPP row permutes inside the column's lanes.
template <int LPC>
__device__ void gen_candidate(const BInst& I, const double* frame, double radius, int c, int64_t t, double* out,
                              uint32_t* lds, const GaussTab& tab, int lane_g, int nl) {
  const int d = I.d;
  const int nb = (d + 1) >> 1;
  const double s = radius / sqrt((double)d);
  const int cols_per_pass = nl / LPC;
  const int lq = lane_g % LPC;
  for (int64_t col0 = 0; col0 < I.n; col0 += cols_per_pass) {
    const int64_t col = col0 + lane_g / LPC;
    const bool active = col < I.n && lq < nb;
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    bool two = false;
    if (active) draw_block(I, frame, s, c, t, col, lq, tab, y, two);
    double nrm2 = (y[0] * y[0] + y[1] * y[1]) + (y[2] * y[2] + y[3] * y[3]);
    nrm2 = group_sum<LPC>(nrm2);  // DPP inside the column's lanes (every lane of the wave takes part)
    if (!active) continue;
    // 1 / ||y||; NaN for a zero or non-finite norm, which makes the column
    // (and so the candidate) invalid
    const double inv = rsqrt_pos(nrm2);
    const int i0 = 2 * lq;
    double* o = out + 2 * ((size_t)col * d + i0);
    o[0] = y[0] * inv;
    o[1] = y[1] * inv;
    if (two) {
      o[2] = y[2] * inv;
      o[3] = y[3] * inv;
    }
    if (lds) {
      // reals 2 i0 .. 2 i0 + 3 of the column: words i0, i0 + 1 of each plane
      // (zero past 2d); the last lane of the column also zeroes the planes'
      // padding [4 nb, kp)
      const int kp2 = (I.ldk - 4) / 2;  // words per plane
      uint32_t h01, l01, h23 = 0, l23 = 0;
      split_bf16x2(f32x2{(float)(y[0] * inv), (float)(y[1] * inv)}, h01, l01);
      if (two) split_bf16x2(f32x2{(float)(y[2] * inv), (float)(y[3] * inv)}, h23, l23);
      uint32_t* row = lds + (size_t)col * I.ldk;
      *(uint2*)(row + i0) = make_uint2(h01, h23);
      *(uint2*)(row + kp2 + i0) = make_uint2(l01, l23);
      if (lq == nb - 1)
        for (int k = 2 * nb; k < kp2; k += 2) {
          *(uint2*)(row + k) = make_uint2(0u, 0u);
          *(uint2*)(row + kp2 + k) = make_uint2(0u, 0u);
        }
    }
  }
}

__device__ __forceinline__ void gen_dispatch(const BInst& I, const double* frame, double radius, int c, int64_t t,
                                             double* out, uint32_t* lds, const GaussTab& tab, int lane_g, int nl) {
  // d <= 16: at most 8 blocks per column
  const int nb = (I.d + 1) >> 1;
  if (nb <= 1) gen_candidate<1>(I, frame, radius, c, t, out, lds, tab, lane_g, nl);
  else if (nb <= 2) gen_candidate<2>(I, frame, radius, c, t, out, lds, tab, lane_g, nl);
  else if (nb <= 4) gen_candidate<4>(I, frame, radius, c, t, out, lds, tab, lane_g, nl);
  else gen_candidate<8>(I, frame, radius, c, t, out, lds, tab, lane_g, nl);
}

// Fragments of the split copy for v_mfma_f32_16x16x32_bf16: lane l holds
// row / column 16 blk + l % 16, reals 8 (l / 16) .. + 7 of the hi and of the
// lo plane (zero past the row's kp reals or past n).
__device__ __forceinline__ void frag_split(const uint32_t* L, int ldk, int n, int blk, u32x4& hi, u32x4& lo) {
  const int lane = threadIdx.x & 63;
  const int r = blk * 16 + (lane & 15);
  const int w0 = 4 * (lane >> 4);  // first word of the lane's 8 reals
  const int kp2 = (ldk - 4) / 2;
  hi = u32x4{0u, 0u, 0u, 0u};
  lo = u32x4{0u, 0u, 0u, 0u};
  if (r < n && w0 < kp2) {
    const uint32_t* p = L + (size_t)r * ldk + w0;
    hi = *(const u32x4*)p;
    lo = *(const u32x4*)(p + kp2);
  }
}

// v = (b, -a) per complex entry (a + ib) of a packed word pair (a low, b
// high), so that Im = u_i . v_j: swap the halves, negate the new high half.
__device__ __forceinline__ u32x4 rot_entries(u32x4 u) {
  u32x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = __builtin_amdgcn_alignbit(u[e], u[e], 16) ^ 0x80000000u;
  return v;
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }

// |G|^2 of the 16 x 16 pair block (bi, bj) from the split fragments of row
// block bi (a) and column block bj (b): Re and Im each accumulate
// hi lo', lo hi' and hi hi'.  m[v] = output (row 4 (lane/16) + v, column
// lane % 16), 0 where the pair is not (j > i, j < n).
__device__ __forceinline__ void screen_split(u32x4 ah, u32x4 al, u32x4 bh, u32x4 bl, int n, int bi, int bj,
                                             float m[4]) {
  const int lane = threadIdx.x & 63;
  const u32x4 vh = rot_entries(bh), vl = rot_entries(bl);
  const v4f32 z = {0.f, 0.f, 0.f, 0.f};
  v4f32 R = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bl), z, 0, 0, 0);
  v4f32 I = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(vl), z, 0, 0, 0);
  R = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), as_bf16x8(bh), R, 0, 0, 0);
  I = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), as_bf16x8(vh), I, 0, 0, 0);
  R = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bh), R, 0, 0, 0);
  I = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(vh), I, 0, 0, 0);
  if (bi < bj && (bj + 1) * 16 <= n) {  // every pair of the block is j > i, j < n
#pragma unroll
    for (int v = 0; v < 4; ++v) m[v] = fmaf(R[v], R[v], I[v] * I[v]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bi * 16 + 4 * (lane >> 4) + v;
      const int j = bj * 16 + (lane & 15);
      m[v] = (i < j && j < n) ? fmaf(R[v], R[v], I[v] * I[v]) : 0.f;
    }
  }
}

__device__ __forceinline__ uint64_t pair_f64_b(const double* c64, int d, int j, int k) {
  const double2* x = (const double2*)(c64 + 2 * (size_t)j * d);
  const double2* y = (const double2*)(c64 + 2 * (size_t)k * d);
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int i = 0; i < d; ++i) {
    const double2 p = x[i], q = y[i];
    re += p.x * q.x + p.y * q.y;
    im += p.x * q.y - p.y * q.x;
  }
  return (uint64_t)__double_as_longlong(re * re + im * im);
}

__device__ __forceinline__ double bits_mu(uint64_t b) {
  if (b >= kInfBits64) return __builtin_inf();
  return sqrt(__longlong_as_double((int64_t)b));
}

// Select / accept / radius update and the in-place FP64 commit, one block per
// instance (grid-stride): wave 0 reduces the candidates' exact values, the
// whole block regenerates the accepted candidate.
__global__ __launch_bounds__(kThreads) void k_batch_finalize(BatchArgs a) {
  __shared__ int acc_s;
  __shared__ int best_s;
  __shared__ GaussTab gtab;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  fill_gauss_tab(&gtab);
  __syncthreads();
  for (int i = blockIdx.x; i < a.count; i += gridDim.x) {
    const BInst I = ((const BInst*)a.inst)[i];
    BState* S = (BState*)a.state + i;
    const BState S0 = *S;
    if (S0.flags & kFlagDone) continue;  // uniform across the block
    if (tid < 64) {
      double v1 = __builtin_inf(), v2 = __builtin_inf();
      int c1 = 0x7fffffff;
      for (int c = lane; c < a.C; c += 64) {
        const double mu = bits_mu(a.cand_max[(size_t)i * a.C + c]);
        if (a.rep_mu) a.rep_mu[(size_t)i * a.C + c] = mu;
        if (!(mu < __builtin_inf())) continue;
        if (mu < v1 || (mu == v1 && c < c1)) {
          v2 = v1;
          v1 = mu;
          c1 = c;
        } else if (mu < v2) {
          v2 = mu;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov1 = __shfl_xor(v1, off, 64), ov2 = __shfl_xor(v2, off, 64);
        const int oc1 = __shfl_xor(c1, off, 64);
        if (ov1 < v1 || (ov1 == v1 && oc1 < c1)) {
          v2 = fmin(v1, ov2);
          v1 = ov1;
          c1 = oc1;
        } else {
          v2 = fmin(v2, ov1);
        }
      }
      const bool valid = c1 != 0x7fffffff;
      const bool accept = valid && v1 < S0.mu;
      if (lane == 0) {
        acc_s = accept ? 1 : 0;
        best_s = c1;
        bool near = valid && fabs(v1 - S0.mu) <= a.tau;
        if (valid && v2 - v1 <= a.tau) near = true;
        const double new_mu = accept ? v1 : S0.mu;
        const double new_rad = accept ? fmin(S0.radius * a.grow, a.radius_max) : fmax(S0.radius * a.shrink, a.radius_min);
        const int64_t nt = S0.step + 1;
        const bool done = (I.target_mu > 0.0 && new_mu <= I.target_mu) || nt >= I.max_steps;
        S->mu = new_mu;
        S->radius = new_rad;
        S->step = nt;
        S->flags = (accept ? kFlagAccepted : 0) | (near ? kFlagNearTie : 0) | (valid ? 0 : kFlagNoValid) |
                   (done ? kFlagDone : 0);
        if (a.rep_best) a.rep_best[i] = valid ? c1 : -1;
        if (done) atomicAdd(a.done_instances, 1);
      }
    }
    __syncthreads();
    if (acc_s) {
      // regenerate candidate best of step t into the frame, in place (each
      // column is read and rewritten by the same lanes)
      double* frame = a.frames + I.frame_off;
      gen_dispatch(I, frame, S0.radius, best_s, S0.step, frame, nullptr, gtab, tid, kThreads);
    }
    __syncthreads();
  }
}

// Synchronisation of a candidate's group of waves: with one wave per
// candidate (wpi = 1) the group is the wave itself and its LDS region,
// maxima and scratch are its own, so completing its LDS and memory
// operations suffices and the block's waves drift out of phase (one wave's
// FP64 generation overlaps another's matrix products); with more waves per
// candidate, the whole block.  wpi is the same for every wave of a unit.
__device__ __forceinline__ void group_sync(bool solo) {
  if (solo) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Position of the k-th (from 0) set bit of m (k < popcount(m)).
__device__ __forceinline__ int kth_set_bit(uint64_t m, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = m & ((1ull << w) - 1);
    const int c = __popcll(low);
    if (k >= c) {
      k -= c;
      m >>= w;
      pos += w;
    } else {
      m = low;
    }
  }
  return pos;
}

// (bi, bj) of the pair block `step` places after (bi, bj) in row-by-row
// upper-triangle order (row bi holds bj = bi .. nbk - 1); step <= 4 and every
// row holds at least one block, so the loop runs at most four times.
__device__ __forceinline__ void tile_advance(int step, int nbk, int& bi, int& bj) {
  bj += step;
  while (bj >= nbk && bi < nbk) {
    bj -= nbk - (bi + 1);
    ++bi;
  }
}

__device__ void screen_phase(const BInst& I, const uint32_t* L, const double* c64, int nbk, int nblk, int wg,
                             int wpi, bool work, uint32_t* blkmax, uint32_t* smax, unsigned long long* umax) {
  const int lane = threadIdx.x & 63;
  const int n = I.n;
  u32x4 ah, al, bh, bl;
  if (work) {
    uint32_t wmax = 0;
    int cur = -1;
    int bi = 0, bj = 0;
    tile_advance(wg, nbk, bi, bj);
    for (int b = wg; b < nblk; b += wpi, tile_advance(wpi, nbk, bi, bj)) {
      if (bi != cur) {  // the A fragments serve the whole row of blocks
        frag_split(L, I.ldk, n, bi, ah, al);
        cur = bi;
      }
      frag_split(L, I.ldk, n, bj, bh, bl);
      float m[4];
      screen_split(ah, al, bh, bl, n, bi, bj, m);
      uint32_t bm = __float_as_uint(m[0]);
#pragma unroll
      for (int v = 1; v < 4; ++v) bm = __float_as_uint(m[v]) > bm ? __float_as_uint(m[v]) : bm;
      bm = wave_max_u32_dpp(bm);
      if (lane == 0) blkmax[b] = bm;
      wmax = bm > wmax ? bm : wmax;
    }
    if (lane == 0) atomicMax(smax, wmax);
  }
  group_sync(wpi == 1);
  if (work) {
    const uint32_t sb = *smax;
    if (sb >= kInfBits32) {
      if (wg == 0 && lane == 0) *umax = ~0ull;  // non-finite column: invalid candidate
    } else {
      const double thr = sqrt((double)__uint_as_float(sb)) - 2.0 * eps_split(I.d);
      const float thr_sq = thr > 0.0 ? (float)(thr * thr * (1.0 - 1e-6)) : 0.0f;
      uint64_t best = 0;
      for (int b = wg; b < nblk; b += wpi) {
        if (__uint_as_float(blkmax[b]) < thr_sq) continue;
        int bi, bj;
        tile_decode(b, nbk, bi, bj);
        frag_split(L, I.ldk, n, bi, ah, al);
        frag_split(L, I.ldk, n, bj, bh, bl);
        float m[4];
        screen_split(ah, al, bh, bl, n, bi, bj, m);
        // the block's pairs that can attain the maximum, in (v, lane) order
        uint64_t mk[4];
        int cnt = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = bi * 16 + 4 * (lane >> 4) + v;
          const int jj = bj * 16 + (lane & 15);
          mk[v] = __ballot(ii < jj && jj < n && !(m[v] < thr_sq));
          cnt += __popcll(mk[v]);
        }
        // four pairs per pass, 16 lanes per pair (one complex entry each,
        // d <= 16), summed with DPP inside the lanes' row
        for (int e0 = 0; e0 < cnt; e0 += 4) {
          const int e = e0 + (lane >> 4);
          const int s = lane & 15;
          double re = 0.0, im = 0.0;
          if (e < cnt) {
            const int c0 = __popcll(mk[0]), c1 = __popcll(mk[1]), c2 = __popcll(mk[2]);
            int k = e, v = 0;
            uint64_t msk = mk[0];
            if (k >= c0) { k -= c0; v = 1; msk = mk[1];
              if (k >= c1) { k -= c1; v = 2; msk = mk[2];
                if (k >= c2) { k -= c2; v = 3; msk = mk[3]; } } }
            const int src = kth_set_bit(msk, k);  // the lane that holds the pair
            const int ii = bi * 16 + 4 * (src >> 4) + v;
            const int jj = bj * 16 + (src & 15);
            if (s < I.d) {
              const double2 x = ((const double2*)(c64 + 2 * (size_t)ii * I.d))[s];
              const double2 y = ((const double2*)(c64 + 2 * (size_t)jj * I.d))[s];
              re = x.x * y.x + x.y * y.y;
              im = x.x * y.y - x.y * y.x;
            }
          }
          re = group_sum<16>(re);
          im = group_sum<16>(im);
          if (e < cnt && s == 0) {
            const uint64_t pb = (uint64_t)__double_as_longlong(re * re + im * im);
            best = pb > best ? pb : best;
          }
        }
      }
      best = wave_max_u64(best);
      if (lane == 0) atomicMax(umax, (unsigned long long)best);
    }
  }
  group_sync(wpi == 1);
}

// Four blocks per CU (the LDS and register use of one block fit four times):
// the Gaussian tables are read from the workspace copy the init launch
// filled (8 KiB, held in the CU's cache) rather than kept in LDS.
__global__ __launch_bounds__(kThreads, 4) void k_batch_step(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kLdsWords];
  __shared__ uint32_t blkmax[4][136];       // per group: max |G|^2 bits of each 16 x 16 pair block (N <= 256)
  __shared__ uint32_t smax[4];
  __shared__ unsigned long long umax[4];
  const GaussTab& gtab = *(const GaussTab*)a.tab;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;

  for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
    const int2 unit = a.units[u];
    const int i = unit.x;
    const BInst I = ((const BInst*)a.inst)[i];
    const BState S0 = ((const BState*)a.state)[i];
    const bool skip_inst = S0.flags & kFlagDone;
    const int wpi = I.wpi;
    const int g = wave / wpi;                 // group of this wave
    const int wg = wave % wpi;                // wave index inside the group
    const int c = unit.y + g;
    const bool work = !skip_inst && c < a.C;
    const int groups = 4 / wpi;
    uint32_t* L = lds + (size_t)g * (kLdsWords / groups);
    double* c64 = a.scratch + ((size_t)blockIdx.x * 4 + g) * a.scratch_stride;
    const int n = I.n;
    const int nbk = (n + 15) / 16;
    const int nblk = nbk * (nbk + 1) / 2;

    // 1. candidate (FP64 scratch + LDS split copy, zero padded to kp reals)
    const bool solo = wpi == 1;
    if (solo) {
      if (lane == 0) {
        smax[g] = 0;
        umax[g] = 0;
      }
    } else {
      // a wave may still be in a previous one-wave unit, on its own part of
      // the LDS regions that these groups share differently
      __syncthreads();
      if (tid < 4) {
        smax[tid] = 0;
        umax[tid] = 0;
      }
    }
    group_sync(solo);
    if (work) gen_dispatch(I, a.frames + I.frame_off, S0.radius, c, S0.step, c64, L, gtab, wg * 64 + lane, wpi * 64);
    __threadfence_block();
    group_sync(solo);

    // 2. split screen: block maxima and the candidate maximum;
    // 3. certified FP64 recheck of the pairs that can attain the maximum
    screen_phase(I, L, c64, nbk, nblk, wg, wpi, work, blkmax[g], &smax[g], &umax[g]);

    // 4. publish (read by the finalizing launch)
    if (work && wg == 0 && lane == 0) a.cand_max[(size_t)i * a.C + c] = umax[g];
    group_sync(solo);
  }
}

// Random start of every instance (tag 1) and its exact FP64 coherence, one
// block per instance (grid-stride).
__global__ __launch_bounds__(kThreads) void k_batch_init(BatchArgs a, int count, double radius0) {
  __shared__ unsigned long long umax;
  __shared__ GaussTab gtab;
  const int tid = threadIdx.x;
  fill_gauss_tab(&gtab);
  if (blockIdx.x == 0) fill_gauss_tab((GaussTab*)a.tab);  // the step launches' copy
  __syncthreads();
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const BInst I = ((const BInst*)a.inst)[i];
    double* frame = a.frames + I.frame_off;
    const int d = I.d;
    const int nb = (d + 1) >> 1;
    if (tid == 0) umax = 0;
    __syncthreads();
    // draw: one thread per (column, block); norm by a serial pass per column
    for (int e = tid; e < I.n * nb; e += kThreads) {
      const int col = e / nb, q = e % nb;
      const u32x4 ctr = {(uint32_t)(col * nb + q), 0u, 0u, 1u};
      const u32x4 w = philox4x32_10(ctr, I.seed, I.stream_id);
      double r0, c0, s0, r1, c1, s1;
      cn_polar(w.x, w.y, gtab, r0, c0, s0);
      cn_polar(w.z, w.w, gtab, r1, c1, s1);
      double* o = frame + 2 * ((size_t)col * d + 2 * q);
      o[0] = r0 * c0;
      o[1] = r0 * s0;
      if (2 * q + 1 < d) {
        o[2] = r1 * c1;
        o[3] = r1 * s1;
      }
    }
    __syncthreads();
    for (int col = tid; col < I.n; col += kThreads) {
      double* o = frame + 2 * (size_t)col * d;
      double s = 0.0;
      for (int q = 0; q < nb; ++q) {
        const int i0 = 2 * q;
        double p = o[2 * i0] * o[2 * i0] + o[2 * i0 + 1] * o[2 * i0 + 1];
        if (i0 + 1 < d) p += o[2 * i0 + 2] * o[2 * i0 + 2] + o[2 * i0 + 3] * o[2 * i0 + 3];
        s += p;
      }
      const double inv = 1.0 / sqrt(s);
      for (int k = 0; k < 2 * d; ++k) o[k] *= inv;
    }
    __threadfence_block();
    __syncthreads();
    uint64_t best = 0;
    const int64_t pairs = (int64_t)I.n * (I.n - 1) / 2;
    for (int64_t p = tid; p < pairs; p += kThreads) {
      // p -> (j, k), j < k, row by row
      int j = 0;
      int64_t rem = p;
      while (rem >= I.n - 1 - j) {
        rem -= I.n - 1 - j;
        ++j;
      }
      const int k = j + 1 + (int)rem;
      const uint64_t b = pair_f64_b(frame, d, j, k);
      best = b > best ? b : best;
    }
    best = wave_max_u64(best);
    if ((tid & 63) == 0) atomicMax(&umax, (unsigned long long)best);
    __syncthreads();
    if (tid == 0) {
      BState* S = (BState*)a.state + i;
      const double mu = bits_mu(umax);
      S->mu = mu;
      S->radius = radius0;
      S->step = 0;
      const bool done = (I.target_mu > 0.0 && mu <= I.target_mu) || I.max_steps <= 0;
      S->flags = done ? kFlagDone : 0;
      if (done) atomicAdd(a.done_instances, 1);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_batch_step(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_step, dim3(grid), dim3(kThreads), 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int fgrid = a.count < 4096 ? a.count : 4096;
  hipLaunchKernelGGL(k_batch_finalize, dim3(fgrid > 0 ? fgrid : 1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_init(const BatchArgs& a, int count, double radius0, hipStream_t s) {
  const int grid = count < 4096 ? count : 4096;
  hipLaunchKernelGGL(k_batch_init, dim3(grid), dim3(kThreads), 0, s, a, count, radius0);
  return hipGetLastError();
}

int batch_step_max_blocks() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_step, kThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return per_cu * cus;
}

size_t batch_inst_bytes() { return sizeof(BInst); }
size_t batch_state_bytes() { return sizeof(BState); }

void batch_fill_inst(void* dst, int32_t n, int32_t d, int32_t wpi, uint32_t seed, uint32_t stream_id,
                     int64_t frame_off, double target_mu, int64_t max_steps) {
  BInst I{};
  I.n = n;
  I.d = d;
  I.wpi = wpi;
  I.ldk = split_row_words(d);
  I.seed = seed;
  I.stream_id = stream_id;
  I.frame_off = frame_off;
  I.target_mu = target_mu;
  I.max_steps = max_steps;
  *(BInst*)dst = I;
}

int batch_lds_words() { return kLdsWords; }

int32_t batch_row_words(int32_t d) { return split_row_words(d); }

double batch_screen_eps(int32_t d) { return eps_split(d); }

size_t batch_tab_bytes() { return sizeof(GaussTab); }

}  // namespace trstmi
