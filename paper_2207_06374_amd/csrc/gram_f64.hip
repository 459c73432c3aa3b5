// FP64 Gram + fused max of |G_jk|^2 over j < k, on v_mfma_f64_16x16x4_f64.
//
// A complex column phi = a + i b is stored as the real 2d-vector
// u = (a_0, b_0, a_1, b_1, ...).  With v = (b_0, -a_0, b_1, -a_1, ...):
//   Re <phi_j, phi_k> = u_j . u_k,   Im <phi_j, phi_k> = u_j . v_k,
// so one tile of the Hermitian Gram is two real products sharing the A
// operand, K = 2d.  v is formed while reading B from LDS: v[k] = +u[k+1]
// for even k and -u[k-1] for odd k.
//
// Only tiles (bi <= bj) of the upper triangle are launched (section IV: the
// upper triangle suffices by symmetry); on a diagonal tile the wave whose
// quadrant lies strictly below the diagonal skips its MFMAs, and the epilogue
// keeps j > i only.  |G|^2 = Re^2 + Im^2 is reduced in registers and across
// the block, and one 64-bit atomic max per block (on the IEEE bit pattern,
// order-preserving for non-negative values; NaN patterns sort above +inf and
// mark an invalid candidate) updates the candidate's maximum.  The Gram is
// never stored.
//
// The same tiles also evaluate the smooth maximum of section IV,
// F_{s,delta}(x) = s + delta log sum_i exp((x_i - s) / delta) over
// x = |G_jk|^2 (or |G_jk|), j < k, with s = max x, in one pass: each block
// finds its own maximum x_b (and raises the global maximum with the atomic
// above), sums exp((x - x_b) / delta) over its pairs into a slot of its own
// together with x_b, and one block rescales the slots to the global s,
// S = sum_b S_b exp((x_b - s) / delta), adding them in a fixed order, so the
// result does not depend on scheduling.  Every exponent is <= 0.
//
// Tile: 64 x 64 complex outputs per 256-thread block, each wave a 32 x 32
// quadrant (2 x 2 MFMA blocks, Re and Im accumulators).  K is staged through
// LDS in chunks of 32 doubles, one double of padding per column so the 16
// lanes that read 16 columns at the same k hit distinct banks.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = kTileF64;
constexpr int KC = 32;
constexpr int LDA = KC + 1;

// Parameters of the sum-exp epilogue (null: the maximum epilogue).
struct SumExp {
  double inv_delta;
  int32_t squared;         // x = |G|^2 (1) or |G| (0)
  double* partial;         // [tile][2]: block sum S_b, block maximum x_b
};

// Epilogues of the tile: the maximum, the smooth maximum, or the search for
// the first pair attaining a known maximum.
enum { kEpiMax = 0, kEpiLse = 1, kEpiPair = 2 };

template <int EPI>
__device__ __forceinline__ void gram_f64_tile(const GramArgs& a, int slot, int bi, int bj, double* As, double* Bs,
                                              uint64_t* red, const SumExp& se, uint64_t* pair = nullptr) {
  const double* base = (const double*)a.cand + (size_t)slot * a.slot_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool skip = (bi == bj) && wr == 1 && wc == 0;
  const int K = 2 * a.d;

  v4f64 accR[2][2], accI[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accR[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
      accI[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
    }

  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < (T * KC / 2) / 256; ++it) {
      const int idx = it * 256 + tid;
      const int col = idx / (KC / 2);
      const int m = idx % (KC / 2);
      const int k = k0 + 2 * m;
      double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
      const int ci = bi * T + col, cj = bj * T + col;
      if (k < K) {
        if (ci < a.n) va = *(const double2*)(base + (size_t)ci * a.ldk + k);
        if (cj < a.n) vb = *(const double2*)(base + (size_t)cj * a.ldk + k);
      }
      As[col * LDA + 2 * m] = va.x;
      As[col * LDA + 2 * m + 1] = va.y;
      Bs[col * LDA + 2 * m] = vb.x;
      Bs[col * LDA + 2 * m + 1] = vb.y;
    }
    __syncthreads();
    if (!skip) {
      const int ksteps = (K - k0 < KC ? K - k0 : KC) / 4 + (((K - k0 < KC ? K - k0 : KC) % 4) ? 1 : 0);
      const int kl = lane >> 4;
      const bool odd = kl & 1;
      for (int kk = 0; kk < ksteps; ++kk) {
        const int k = kk * 4 + kl;
        double av[2], bu[2], bv[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) av[r] = As[(wr * 32 + r * 16 + (lane & 15)) * LDA + k];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int cc = (wc * 32 + c * 16 + (lane & 15)) * LDA;
          bu[c] = Bs[cc + k];
          const double x = Bs[cc + (k ^ 1)];
          bv[c] = odd ? -x : x;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            accR[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r], bu[c], accR[r][c], 0, 0, 0);
            accI[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r], bv[c], accI[r][c], 0, 0, 0);
          }
      }
    }
  }

  if constexpr (EPI == kEpiPair) {
    // the first pair (in the order i * n + j) whose |G|^2 has the bits of the
    // maximum found by the maximum epilogue with the same arithmetic
    const uint64_t target = a.cand_max[slot];
    uint64_t first = ~0ull;
    if (!skip) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = bi * T + wr * 32 + r * 16 + 4 * v + (lane >> 4);
            const int j = bj * T + wc * 32 + c * 16 + (lane & 15);
            const double re = accR[r][c][v], im = accI[r][c][v];
            const uint64_t mb = (uint64_t)__double_as_longlong(re * re + im * im);
            const uint64_t q = (uint64_t)i * (uint64_t)a.n + (uint64_t)j;
            if (i < j && j < a.n && mb == target && q < first) first = q;
          }
    }
    first = ~wave_max_u64(~first);
    if (lane == 0 && first != ~0ull) atomicMin((unsigned long long*)pair, (unsigned long long)first);
    return;
  }
  if constexpr (EPI == kEpiLse) {
    // the block's maximum of |G|^2 (bit patterns: NaN above +inf), then its sum
    uint64_t bm = 0;
    if (!skip) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = bi * T + wr * 32 + r * 16 + 4 * v + (lane >> 4);
            const int j = bj * T + wc * 32 + c * 16 + (lane & 15);
            const double re = accR[r][c][v], im = accI[r][c][v];
            const uint64_t mb = (uint64_t)__double_as_longlong(re * re + im * im);
            if (i < j && j < a.n && mb > bm) bm = mb;
          }
    }
    bm = wave_max_u64(bm);
    if (lane == 0) red[w] = bm;
    __syncthreads();
    bm = red[0];
    for (int q = 1; q < 4; ++q) bm = red[q] > bm ? red[q] : bm;
    const bool finite = bm < kInfBits64;
    const double m_b = finite ? __longlong_as_double((int64_t)bm) : 0.0;
    const double x_b = se.squared ? m_b : sqrt(m_b);
    double sum = 0.0;
    if (!skip && finite) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = bi * T + wr * 32 + r * 16 + 4 * v + (lane >> 4);
            const int j = bj * T + wc * 32 + c * 16 + (lane & 15);
            const double re = accR[r][c][v], im = accI[r][c][v];
            const double m = re * re + im * im;
            const double x = se.squared ? m : sqrt(m);
            if (i < j && j < a.n) sum += exp((x - x_b) * se.inv_delta);
          }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    __syncthreads();  // every wave has read red[]
    double* reds = (double*)red;
    if (lane == 0) reds[w] = sum;
    __syncthreads();
    if (tid == 0) {
      se.partial[2 * blockIdx.x] = (reds[0] + reds[1]) + (reds[2] + reds[3]);
      se.partial[2 * blockIdx.x + 1] = x_b;
      atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)bm);
    }
    return;
  }
  uint64_t best = 0;
  if (!skip) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // f64 16x16x4 output: register v of lane l holds row 4 v + l / 16, column l % 16
          const int i = bi * T + wr * 32 + r * 16 + 4 * v + (lane >> 4);
          const int j = bj * T + wc * 32 + c * 16 + (lane & 15);
          const double re = accR[r][c][v], im = accI[r][c][v];
          const double m = re * re + im * im;
          const uint64_t mb = (uint64_t)__double_as_longlong(m);
          if (i < j && j < a.n && mb > best) best = mb;
        }
  }
  best = wave_max_u64(best);
  if (lane == 0) red[w] = best;
  __syncthreads();
  if (tid == 0) {
    uint64_t m = red[0];
    for (int q = 1; q < 4; ++q) m = red[q] > m ? red[q] : m;
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)m);
  }
}

__global__ __launch_bounds__(256) void k_gram_f64(GramArgs a) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  __shared__ double As[T * LDA];
  __shared__ double Bs[T * LDA];
  __shared__ uint64_t red[4];
  int bi, bj;
  tile_decode(blockIdx.x, a.nt, bi, bj);
  gram_f64_tile<kEpiMax>(a, blockIdx.y, bi, bj, As, Bs, red, SumExp{});
}

__global__ __launch_bounds__(256) void k_gram_f64_lse(GramArgs a, SumExp se) {
  __shared__ double As[T * LDA];
  __shared__ double Bs[T * LDA];
  __shared__ uint64_t red[4];
  int bi, bj;
  tile_decode(blockIdx.x, a.nt, bi, bj);
  gram_f64_tile<kEpiLse>(a, 0, bi, bj, As, Bs, red, se);
}

__global__ __launch_bounds__(256) void k_gram_f64_pair(GramArgs a, uint64_t* pair) {
  __shared__ double As[T * LDA];
  __shared__ double Bs[T * LDA];
  __shared__ uint64_t red[4];
  int bi, bj;
  tile_decode(blockIdx.x, a.nt, bi, bj);
  gram_f64_tile<kEpiPair>(a, 0, bi, bj, As, Bs, red, SumExp{}, pair);
}

__global__ void k_pair_init(uint64_t* pair) { *pair = ~0ull; }

// mu = sqrt(max |G|^2) and the pair (j, k) = (q / n, q mod n); (-1, -1) and
// +inf for a zero or non-finite column.
__global__ void k_pair_finish(const uint64_t* max_bits, const uint64_t* pair, int64_t n, double* mu, int64_t* jk) {
  const uint64_t b = *max_bits, q = *pair;
  if (b >= kInfBits64 || q == ~0ull) {
    *mu = __builtin_inf();
    jk[0] = -1;
    jk[1] = -1;
    return;
  }
  *mu = sqrt(__longlong_as_double((int64_t)b));
  jk[0] = (int64_t)(q / (uint64_t)n);
  jk[1] = (int64_t)(q % (uint64_t)n);
}

// F = s + delta log S with S = sum_b S_b exp((x_b - s) / delta), added in a
// fixed order: thread t takes slots t, t + 256, ... in turn, then a fixed
// pairwise tree.
__global__ __launch_bounds__(256) void k_lse_finish(const uint64_t* s_bits, const double* partial, int64_t count,
                                                    double delta, int32_t squared, double* out, double* log_sum) {
  __shared__ double acc[256];
  const uint64_t b = *s_bits;
  const bool finite = b < kInfBits64;
  const double m = finite ? __longlong_as_double((int64_t)b) : 0.0;
  const double s = squared ? m : sqrt(m);
  const double inv_delta = 1.0 / delta;
  double sum = 0.0;
  if (finite)
    for (int64_t i = threadIdx.x; i < count; i += 256) sum += partial[2 * i] * exp((partial[2 * i + 1] - s) * inv_delta);
  acc[threadIdx.x] = sum;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) acc[threadIdx.x] += acc[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (!finite) {  // a zero or non-finite column
      out[0] = __builtin_inf();
      out[1] = __builtin_inf();
      if (log_sum) *log_sum = __builtin_inf();
      return;
    }
    const double ls = log(acc[0]);
    out[0] = s;
    out[1] = s + delta * ls;
    if (log_sum) *log_sum = ls;
  }
}

}  // namespace

hipError_t launch_gram_f64(const GramArgs& a, int slots, hipStream_t s) {
  const int tiles = a.nt * (a.nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_f64, dim3(tiles, slots), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gram_f64_pair(const GramArgs& a, uint64_t* pair, double* mu, int64_t* jk, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_init, dim3(1), dim3(1), 0, s, pair);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tiles = a.nt * (a.nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_f64_pair, dim3(tiles), dim3(256), 0, s, a, pair);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pair_finish, dim3(1), dim3(1), 0, s, a.cand_max, pair, (int64_t)a.n, mu, jk);
  return hipGetLastError();
}

hipError_t launch_lse_pass(const GramArgs& a, double delta, int32_t squared, double* partial, hipStream_t s) {
  const int tiles = a.nt * (a.nt + 1) / 2;
  SumExp se{1.0 / delta, squared, partial};
  hipLaunchKernelGGL(k_gram_f64_lse, dim3(tiles), dim3(256), 0, s, a, se);
  return hipGetLastError();
}

hipError_t launch_lse_finish(const uint64_t* s_bits, const double* partial, int64_t count, double delta,
                             int32_t squared, double* out, double* log_sum, hipStream_t s) {
  hipLaunchKernelGGL(k_lse_finish, dim3(1), dim3(256), 0, s, s_bits, partial, count, delta, squared, out, log_sum);
  return hipGetLastError();
}

}  // namespace trstmi
