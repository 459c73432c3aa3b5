// FP32 Gram + fused max of |G_jk|^2 over j < k, on v_mfma_f32_16x16x4_f32.
//
// Same decomposition as the FP64 kernel (Re = u_j . u_k, Im = u_j . v_k with
// v the (im, -re) swap of u, K = 2d real), FP32 inputs rounded from the FP64
// unit candidates, FP32 accumulation.  64 x 64 complex outputs per block of
// 256 threads, wave quadrants of 2 x 2 MFMA blocks, K staged through LDS in
// chunks of 64 floats (one float of padding per column: conflict-free reads
// of 16 columns at one k).  The max is kept as float bit patterns in a
// 64-bit slot (non-negative floats order like unsigned integers; NaN above
// +inf).

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = kTileF32;
constexpr int KC = 64;
constexpr int LDA = KC + 1;

__global__ __launch_bounds__(256) void k_gram_f32(GramArgs a) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  const int slot = blockIdx.y;
  int bi, bj;
  tile_decode(blockIdx.x, a.nt, bi, bj);

  __shared__ float As[T * LDA];
  __shared__ float Bs[T * LDA];
  __shared__ uint32_t red[4];

  const float* base = (const float*)a.cand + (size_t)slot * a.slot_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool skip = (bi == bj) && wr == 1 && wc == 0;
  const int K = 2 * a.d;

  v4f32 accR[2][2], accI[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accR[r][c] = v4f32{0.f, 0.f, 0.f, 0.f};
      accI[r][c] = v4f32{0.f, 0.f, 0.f, 0.f};
    }

  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
    // T columns x KC floats per side = 1024 float4 per side
#pragma unroll
    for (int it = 0; it < (T * KC / 4) / 256; ++it) {
      const int idx = it * 256 + tid;
      const int col = idx / (KC / 4);
      const int m = idx % (KC / 4);
      const int k = k0 + 4 * m;
      float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
      const int ci = bi * T + col, cj = bj * T + col;
      if (k < a.ldk) {
        if (ci < a.n) va = *(const float4*)(base + (size_t)ci * a.ldk + k);
        if (cj < a.n) vb = *(const float4*)(base + (size_t)cj * a.ldk + k);
      }
      float* pa = &As[col * LDA + 4 * m];
      float* pb = &Bs[col * LDA + 4 * m];
      pa[0] = va.x; pa[1] = va.y; pa[2] = va.z; pa[3] = va.w;
      pb[0] = vb.x; pb[1] = vb.y; pb[2] = vb.z; pb[3] = vb.w;
    }
    __syncthreads();
    if (!skip) {
      const int rem = K - k0 < KC ? K - k0 : KC;
      const int ksteps = (rem + 3) / 4;
      const int kl = lane >> 4;
      const bool odd = kl & 1;
      for (int kk = 0; kk < ksteps; ++kk) {
        const int k = kk * 4 + kl;
        float av[2], bu[2], bv[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) av[r] = As[(wr * 32 + r * 16 + (lane & 15)) * LDA + k];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int cc = (wc * 32 + c * 16 + (lane & 15)) * LDA;
          bu[c] = Bs[cc + k];
          const float x = Bs[cc + (k ^ 1)];
          bv[c] = odd ? -x : x;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            accR[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bu[c], accR[r][c], 0, 0, 0);
            accI[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv[c], accI[r][c], 0, 0, 0);
          }
      }
    }
  }

  uint32_t best = 0;
  if (!skip) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = bi * T + wr * 32 + r * 16 + 4 * (lane >> 4) + v;
          const int j = bj * T + wc * 32 + c * 16 + (lane & 15);
          const float re = accR[r][c][v], im = accI[r][c][v];
          const float m = re * re + im * im;
          const uint32_t mb = __float_as_uint(m);
          if (i < j && j < a.n && mb > best) best = mb;
        }
  }
  best = wave_max_u32(best);
  if (lane == 0) red[w] = best;
  __syncthreads();
  if (tid == 0) {
    uint32_t m = red[0];
    for (int q = 1; q < 4; ++q) m = red[q] > m ? red[q] : m;
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)m);
  }
}

}  // namespace

hipError_t launch_gram_f32(const GramArgs& a, int slots, hipStream_t s) {
  const int tiles = a.nt * (a.nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_f32, dim3(tiles, slots), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace trstmi
