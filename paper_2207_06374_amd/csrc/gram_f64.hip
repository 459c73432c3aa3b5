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

__device__ __forceinline__ void gram_f64_tile(const GramArgs& a, int slot, int bi, int bj, double* As, double* Bs,
                                              uint64_t* red) {
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
  gram_f64_tile(a, blockIdx.y, bi, bj, As, Bs, red);
}

}  // namespace

hipError_t launch_gram_f64(const GramArgs& a, int slots, hipStream_t s) {
  const int tiles = a.nt * (a.nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_f64, dim3(tiles, slots), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace trstmi
