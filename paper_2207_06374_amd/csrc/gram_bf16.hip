// BF16-screen Gram + fused max of |G_jk|^2 over j < k, on
// v_mfma_f32_16x16x32_bf16 (gfx950), FP32 accumulation.
//
// Inputs are the FP64 unit candidates rounded to bfloat16 (nearest-even) by
// the perturb kernel, column stride ldk (multiple of 8, zero padded).  As in
// the FP64 kernel, Re <phi_j,phi_k> = u_j . u_k and Im = u_j . v_k with v the
// (im, -re) swap of u; here v is built in registers from each 32-bit (re, im)
// pair of the B fragment with one funnel shift and one sign flip.
//
// Tile: 128 x 128 complex outputs per 256-thread block, each wave a 64 x 64
// quadrant = 4 x 4 MFMA blocks of 16 x 16 (Re and Im accumulators in 128
// VGPRs).  K is staged through LDS in chunks of 128 bf16 per column, 8 bf16 of
// padding per column so 16 lanes reading 16 columns at one k offset hit
// distinct banks with 16-byte reads.  The block writes its tile maximum
// (for certified pruning of the FP64 recheck) and updates the candidate's
// running maximum with one atomic.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = kTileBF16;
constexpr int KCB = 128;
constexpr int LDB = KCB + 8;

__device__ __forceinline__ u32x4 swap_negate(u32x4 u) {
  u32x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = __builtin_amdgcn_alignbit(u[e], u[e], 16) ^ 0x80000000u;
  return v;
}

__global__ __launch_bounds__(256) void k_gram_bf16(GramArgs a) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  const int slot = blockIdx.y;
  int bi, bj;
  tile_decode(blockIdx.x, a.nt, bi, bj);

  __shared__ __attribute__((aligned(16))) uint16_t As[T * LDB];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[T * LDB];
  __shared__ uint32_t red[4];

  const uint16_t* base = (const uint16_t*)a.cand + (size_t)slot * a.slot_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool skip = (bi == bj) && wr == 1 && wc == 0;

  v4f32 accR[4][4], accI[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      accR[r][c] = v4f32{0.f, 0.f, 0.f, 0.f};
      accI[r][c] = v4f32{0.f, 0.f, 0.f, 0.f};
    }

  const int K = a.ldk;  // padded with zeros beyond 2d
  for (int k0 = 0; k0 < K; k0 += KCB) {
    __syncthreads();
    // T columns x KCB bf16 per side = 2048 chunks of 16 bytes per side
#pragma unroll
    for (int it = 0; it < (T * KCB / 8) / 256; ++it) {
      const int idx = it * 256 + tid;
      const int col = idx / (KCB / 8);
      const int m = idx % (KCB / 8);
      const int k = k0 + 8 * m;
      u32x4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      const int ci = bi * T + col, cj = bj * T + col;
      if (k < K) {
        if (ci < a.n) va = *(const u32x4*)(base + (size_t)ci * a.ldk + k);
        if (cj < a.n) vb = *(const u32x4*)(base + (size_t)cj * a.ldk + k);
      }
      *(u32x4*)&As[col * LDB + 8 * m] = va;
      *(u32x4*)&Bs[col * LDB + 8 * m] = vb;
    }
    __syncthreads();
    if (!skip) {
      const int rem = K - k0 < KCB ? K - k0 : KCB;
      const int ksteps = (rem + 31) / 32;
      const int koff = 8 * (lane >> 4);
      for (int kk = 0; kk < ksteps; ++kk) {
        bf16x8 av[4];
        u32x4 bu[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          av[r] = __builtin_bit_cast(bf16x8, *(const u32x4*)&As[(wr * 64 + r * 16 + (lane & 15)) * LDB + kk * 32 + koff]);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          bu[c] = *(const u32x4*)&Bs[(wc * 64 + c * 16 + (lane & 15)) * LDB + kk * 32 + koff];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bU = __builtin_bit_cast(bf16x8, bu[c]);
          const bf16x8 bV = __builtin_bit_cast(bf16x8, swap_negate(bu[c]));
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            accR[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bU, accR[r][c], 0, 0, 0);
            accI[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bV, accI[r][c], 0, 0, 0);
          }
        }
      }
    }
  }

  uint32_t best = 0;
  if (!skip) {
    const bool interior = (bi < bj) && ((bj + 1) * T <= a.n);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float re = accR[r][c][v], im = accI[r][c][v];
          const float m = re * re + im * im;
          const uint32_t mb = __float_as_uint(m);
          bool ok = true;
          if (!interior) {
            const int i = bi * T + wr * 64 + r * 16 + 4 * (lane >> 4) + v;
            const int j = bj * T + wc * 64 + c * 16 + (lane & 15);
            ok = i < j && j < a.n;
          }
          if (ok && mb > best) best = mb;
        }
  }
  best = wave_max_u32(best);
  if (lane == 0) red[w] = best;
  __syncthreads();
  if (tid == 0) {
    uint32_t m = red[0];
    for (int q = 1; q < 4; ++q) m = red[q] > m ? red[q] : m;
    if (a.tile_max) a.tile_max[(size_t)slot * gridDim.x + blockIdx.x] = m;
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)m);
  }
}

}  // namespace

hipError_t launch_gram_bf16(const GramArgs& a, int slots, hipStream_t s) {
  const int tiles = a.nt * (a.nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_bf16, dim3(tiles, slots), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace trstmi
