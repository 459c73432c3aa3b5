// Beamforming-codebook quantiser of section III on v_mfma_f64_16x16x4_f64.
//
// For channels h_m (columns of H, d x M) and unit codewords phi_i (the
// normalised codebook, d x N): index_m = argmax_i |<phi_i, h_m>|^2 (the first
// of equal maxima), gain_m = that maximum, dist_m = 1 - gain_m / |h_m|^2 (the
// squared chordal distance from the line of h_m to its codeword).
//
// With phi = a + i b stored as u = (a_0, b_0, a_1, b_1, ...) and, for a
// channel, v = (b_0, -a_0, ...): Re <phi, h> = u_phi . u_h and
// Im <phi, h> = u_phi . v_h, so one tile of Phi^* H is two real products
// with K = 2d sharing the codeword operand.  A block owns 64 channels and
// walks every 64-codeword tile in the same order as all other blocks (so a
// codeword tile is read from L2 by the whole grid at about the same time);
// each wave computes a 32 x 32 quadrant (codewords x channels) and keeps,
// per lane and channel column, the running maximum and its index.  Within a
// lane the codeword index only grows, so a strict comparison keeps the
// first of equal maxima; the final reduction across lanes and waves breaks
// ties by the lower index.  |h|^2 is summed from the channel chunks while
// the first codeword tile is computed.  Per-block sums of dist and gain go
// to fixed slots and one block adds them in a fixed order, so the means do
// not depend on scheduling.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = 64;        // codewords and channels per block tile
constexpr int KC = 32;       // K chunk staged through LDS
constexpr int LDA = KC + 1;  // padded LDS column

// Merge the per-lane (max, index, NaN) of NS slots per channel (slot =
// wave row x lane group), write the channel outputs and the block sums.
template <int NS>
__device__ __forceinline__ void finish_block(const MisoArgs& a, int64_t j0, int wr, int wc, const double* best,
                                             const int32_t* bidx, const bool* nan, double h2, double* redg,
                                             int32_t* redi, int32_t* redn, double* h2s) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int slot = wr * 4 + (lane >> 4);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = wc * 32 + c * 16 + (lane & 15);
    redg[slot * T + col] = best[c];
    redi[slot * T + col] = bidx[c];
    redn[slot * T + col] = nan[c] ? 1 : 0;
  }
  if (tid < T) h2s[tid] = h2;
  __syncthreads();
  double dist = 0.0, gain = 0.0;
  if (tid < T) {
    double g = redg[tid];
    int32_t gi = redi[tid];
    int32_t bad = redn[tid];
    for (int q = 1; q < NS; ++q) {
      const double x = redg[q * T + tid];
      const int32_t xi = redi[q * T + tid];
      if (x > g || (x == g && xi < gi)) {
        g = x;
        gi = xi;
      }
      bad |= redn[q * T + tid];
    }
    const int64_t j = j0 + tid;
    const double hh = h2s[tid];
    const bool finite_h = hh - hh == 0.0;
    if (bad || !finite_h) {
      gi = -1;
      g = __longlong_as_double(0x7FF8000000000000LL);
      dist = g;
    } else {
      dist = 1.0 - g / hh;
    }
    gain = g;
    if (j < a.m) {
      if (a.index) a.index[j] = gi;
      if (a.gain) a.gain[j] = g;
      if (a.dist) a.dist[j] = dist;
    } else {
      dist = 0.0;
      gain = 0.0;
    }
  }
  if (a.partial && tid < 64) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      dist += __shfl_xor(dist, off, 64);
      gain += __shfl_xor(gain, off, 64);
    }
    if (tid == 0) {
      a.partial[2 * blockIdx.x] = dist;
      a.partial[2 * blockIdx.x + 1] = gain;
    }
  }
}

// One K chunk of the codeword tile bi and of the block's channels, held in
// registers between its global load and its store to LDS.
struct Chunk {
  double2 a[(T * KC / 2) / 256];
  double2 b[(T * KC / 2) / 256];
};

__device__ __forceinline__ void load_chunk(const MisoArgs& a, int bi, int k0, int64_t j0, int K, Chunk& c) {
#pragma unroll
  for (int it = 0; it < (T * KC / 2) / 256; ++it) {
    const int idx = it * 256 + threadIdx.x;
    const int col = idx / (KC / 2);
    const int k = k0 + 2 * (idx % (KC / 2));
    const int ci = bi * T + col;
    const int64_t cj = j0 + col;
    c.a[it] = make_double2(0.0, 0.0);
    c.b[it] = make_double2(0.0, 0.0);
    if (k < K) {
      if (ci < a.n) c.a[it] = *(const double2*)(a.codebook + (size_t)ci * a.ldk + k);
      if (cj < a.m) c.b[it] = *(const double2*)(a.channels + (size_t)cj * K + k);
    }
  }
}

__device__ __forceinline__ void store_chunk(const Chunk& c, double* As, double* Bs) {
#pragma unroll
  for (int it = 0; it < (T * KC / 2) / 256; ++it) {
    const int idx = it * 256 + threadIdx.x;
    const int col = idx / (KC / 2);
    const int m = idx % (KC / 2);
    As[col * LDA + 2 * m] = c.a[it].x;
    As[col * LDA + 2 * m + 1] = c.a[it].y;
    Bs[col * LDA + 2 * m] = c.b[it].x;
    Bs[col * LDA + 2 * m + 1] = c.b[it].y;
  }
}

// The chunks (codeword tile bi, K offset k0) are taken in one flat sequence;
// the next chunk's global loads are issued before the current chunk's
// products, into registers, and stored to the other LDS buffer afterwards,
// so one barrier per chunk separates the two buffers' uses.
__global__ __launch_bounds__(256) void k_miso_quantize(MisoArgs a) {
  __shared__ double As[2][T * LDA];
  __shared__ double Bs[2][T * LDA];
  __shared__ double h2s[T];
  __shared__ double redg[8][T];
  __shared__ int32_t redi[8][T];
  __shared__ int32_t redn[8][T];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int K = 2 * a.d;
  const int64_t j0 = (int64_t)blockIdx.x * T;
  const int ntile = (a.n + T - 1) / T;
  const int nk = (K + KC - 1) / KC;
  const int nq = ntile * nk;

  double best[2] = {-1.0, -1.0};
  int32_t bidx[2] = {0, 0};
  bool nan[2] = {false, false};
  double h2 = 0.0;

  v4f64 accR[2][2], accI[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accR[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
      accI[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
    }

  Chunk nxt;
  load_chunk(a, 0, 0, j0, K, nxt);
  store_chunk(nxt, As[0], Bs[0]);
  __syncthreads();

  int bi = 0, kc = 0;
  for (int q = 0; q < nq; ++q) {
    const int buf = q & 1;
    const bool more = q + 1 < nq;
    if (more) {
      const int nbi = kc + 1 < nk ? bi : bi + 1;
      const int nkc = kc + 1 < nk ? kc + 1 : 0;
      load_chunk(a, nbi, nkc * KC, j0, K, nxt);
    }
    const double* Ab = As[buf];
    const double* Bb = Bs[buf];
    const int k0 = kc * KC;
    const int kn = K - k0 < KC ? K - k0 : KC;
    if (bi == 0 && tid < T) {
      for (int k = 0; k < kn; ++k) {
        const double x = Bb[tid * LDA + k];
        h2 = fma(x, x, h2);
      }
    }
    const int ksteps = (kn + 3) / 4;
    const int kl = lane >> 4;
    const bool odd = kl & 1;
    for (int kk = 0; kk < ksteps; ++kk) {
      const int k = kk * 4 + kl;
      double av[2], bu[2], bv[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) av[r] = Ab[(wr * 32 + r * 16 + (lane & 15)) * LDA + k];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int cc = (wc * 32 + c * 16 + (lane & 15)) * LDA;
        bu[c] = Bb[cc + k];
        const double x = Bb[cc + (k ^ 1)];
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
    if (kc + 1 == nk) {
      // output register v of lane l: codeword row 4 v + l / 16, channel column l % 16
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = bi * T + wr * 32 + r * 16 + 4 * v + (lane >> 4);
          if (i < a.n) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double re = accR[r][c][v], im = accI[r][c][v];
              const double g = re * re + im * im;
              if (g > best[c]) {
                best[c] = g;
                bidx[c] = i;
              }
              nan[c] |= (g != g);
            }
          }
        }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          accR[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
          accI[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
        }
      kc = 0;
      ++bi;
    } else {
      ++kc;
    }
    if (more) store_chunk(nxt, As[buf ^ 1], Bs[buf ^ 1]);
    __syncthreads();
  }

  finish_block<8>(a, j0, wr, wc, best, bidx, nan, h2, &redg[0][0], &redi[0][0], &redn[0][0], h2s);
}

// Resident form for 2d <= 128: the block's 64 channels are loaded into LDS
// once, with the whole K, and only the codeword chunks stream (prefetched
// one chunk ahead into registers, double-buffered in LDS).  Eight waves
// (4 codeword rows x 2 channel halves of 32 x 32) share a 128-codeword tile,
// so each channel chunk is read from LDS, not from L2, for every tile.
constexpr int TR = 128;           // codewords per tile in the resident form
constexpr int KRMAX = 128;        // largest K (rounded up to 4) held resident
constexpr int LDBMAX = KRMAX + 1; // odd column stride of the resident channels

struct ChunkR {
  double2 a[(TR * KC / 2) / 512];
};

__device__ __forceinline__ void load_chunk_r(const MisoArgs& a, int bi, int k0, int K, ChunkR& c) {
#pragma unroll
  for (int it = 0; it < (TR * KC / 2) / 512; ++it) {
    const int idx = it * 512 + threadIdx.x;
    const int col = idx / (KC / 2);
    const int k = k0 + 2 * (idx % (KC / 2));
    const int ci = bi * TR + col;
    c.a[it] = make_double2(0.0, 0.0);
    if (k < K && ci < a.n) c.a[it] = *(const double2*)(a.codebook + (size_t)ci * a.ldk + k);
  }
}

__device__ __forceinline__ void store_chunk_r(const ChunkR& c, double* As) {
#pragma unroll
  for (int it = 0; it < (TR * KC / 2) / 512; ++it) {
    const int idx = it * 512 + threadIdx.x;
    const int col = idx / (KC / 2);
    const int m = idx % (KC / 2);
    As[col * LDA + 2 * m] = c.a[it].x;
    As[col * LDA + 2 * m + 1] = c.a[it].y;
  }
}

__global__ __launch_bounds__(512) void k_miso_quantize_res(MisoArgs a) {
  __shared__ double Bs[T * LDBMAX];
  __shared__ double As[2][TR * LDA];
  __shared__ double h2s[T];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int K = 2 * a.d;
  const int KR = (K + 3) & ~3;     // K rounded up to whole MFMA k-steps (zero filled)
  const int ldb = KR + 1;
  const int64_t j0 = (int64_t)blockIdx.x * T;
  const int ntile = (a.n + TR - 1) / TR;
  const int nk = (K + KC - 1) / KC;
  const int nq = ntile * nk;

  for (int idx = tid; idx < T * (KR / 2); idx += 512) {
    const int col = idx / (KR / 2);
    const int k = 2 * (idx % (KR / 2));
    const int64_t cj = j0 + col;
    double2 v = make_double2(0.0, 0.0);
    if (k < K && cj < a.m) v = *(const double2*)(a.channels + (size_t)cj * K + k);
    Bs[col * ldb + k] = v.x;
    Bs[col * ldb + k + 1] = v.y;
  }
  ChunkR nxt;
  load_chunk_r(a, 0, 0, K, nxt);
  store_chunk_r(nxt, As[0]);
  __syncthreads();
  double h2 = 0.0;
  if (tid < T)
    for (int k = 0; k < K; ++k) {
      const double x = Bs[tid * ldb + k];
      h2 = fma(x, x, h2);
    }

  double best[2] = {-1.0, -1.0};
  int32_t bidx[2] = {0, 0};
  bool nan[2] = {false, false};
  v4f64 accR[2][2], accI[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accR[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
      accI[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
    }

  int bi = 0, kc = 0;
  for (int q = 0; q < nq; ++q) {
    const int buf = q & 1;
    const bool more = q + 1 < nq;
    if (more) {
      const int nbi = kc + 1 < nk ? bi : bi + 1;
      const int nkc = kc + 1 < nk ? kc + 1 : 0;
      load_chunk_r(a, nbi, nkc * KC, K, nxt);
    }
    const double* Ab = As[buf];
    const int k0 = kc * KC;
    const int kn = K - k0 < KC ? K - k0 : KC;
    const int ksteps = (kn + 3) / 4;
    const int kl = lane >> 4;
    const bool odd = kl & 1;
    for (int kk = 0; kk < ksteps; ++kk) {
      const int k = kk * 4 + kl;
      double av[2], bu[2], bv[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) av[r] = Ab[(wr * 32 + r * 16 + (lane & 15)) * LDA + k];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int cc = (wc * 32 + c * 16 + (lane & 15)) * ldb + k0;
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
    if (kc + 1 == nk) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = bi * TR + wr * 32 + r * 16 + 4 * v + (lane >> 4);
          if (i < a.n) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double re = accR[r][c][v], im = accI[r][c][v];
              const double g = re * re + im * im;
              if (g > best[c]) {
                best[c] = g;
                bidx[c] = i;
              }
              nan[c] |= (g != g);
            }
          }
        }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          accR[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
          accI[r][c] = v4f64{0.0, 0.0, 0.0, 0.0};
        }
      kc = 0;
      ++bi;
    } else {
      ++kc;
    }
    if (more) store_chunk_r(nxt, As[buf ^ 1]);
    __syncthreads();
  }
  // the codeword buffers are free after the last barrier: 16 slots of the merge there
  double* redg = &As[0][0];
  int32_t* redi = (int32_t*)(redg + 16 * T);
  int32_t* redn = redi + 16 * T;
  finish_block<16>(a, j0, wr, wc, best, bidx, nan, h2, redg, redi, redn, h2s);
}

// summary = (sum of dist, sum of gain) / m over the block slots, added in a
// fixed order: thread t takes slots t, t + 256, ... in turn, then a fixed
// pairwise tree.
__global__ __launch_bounds__(256) void k_miso_finish(const double* partial, int64_t count, int64_t m,
                                                     double* summary) {
  __shared__ double acc[2][256];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) {
    s0 += partial[2 * i];
    s1 += partial[2 * i + 1];
  }
  acc[0][threadIdx.x] = s0;
  acc[1][threadIdx.x] = s1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      acc[0][threadIdx.x] += acc[0][threadIdx.x + h];
      acc[1][threadIdx.x] += acc[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nan = __longlong_as_double(0x7FF8000000000000LL);
    summary[0] = m > 0 ? acc[0][0] / (double)m : nan;
    summary[1] = m > 0 ? acc[1][0] / (double)m : nan;
  }
}

}  // namespace

int64_t miso_blocks(int64_t m) { return (m + T - 1) / T; }

hipError_t launch_miso(const MisoArgs& a, double* summary, hipStream_t s) {
  const int64_t blocks = miso_blocks(a.m);
  if (blocks > 0) {
    if (2 * a.d <= KRMAX)
      hipLaunchKernelGGL(k_miso_quantize_res, dim3((unsigned)blocks), dim3(512), 0, s, a);
    else
      hipLaunchKernelGGL(k_miso_quantize, dim3((unsigned)blocks), dim3(256), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (summary) {
    hipLaunchKernelGGL(k_miso_finish, dim3(1), dim3(256), 0, s, a.partial, blocks, a.m, summary);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace trstmi
