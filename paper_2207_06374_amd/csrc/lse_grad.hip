// Gradient of the smooth maximum of section IV with respect to the
// unconstrained frame Y (the objective normalises Y's columns first):
//   w_jk = exp((x_jk - s) / delta) / S   (x = |G|^2, S = sum over j < k),
//   D = Phi (W o G)                        (W symmetric, zero diagonal),
//   g_k = 2 (D_k - phi_k Re(phi_k^H D_k)) / ||y_k||,
// so that dF = sum Re(conj(g) dY).
//
// k_lse_grad: a block owns 64 output columns k (tile kb) and a run of row
// tiles jb.  Both 64-column tiles of the normalised frame sit in LDS with
// the whole K = 2d (d <= 64).  Eight waves share them: wave w takes the 16
// columns k of group w mod 4 and the 32 rows j of half w / 4 of tile jb
// (two waves per SIMD, so one wave's exponentials and barriers overlap the
// other's matrix products).  A wave computes G for its rows and columns on
// v_mfma_f64_16x16x4f64, turns it into B = W o G in registers, and feeds B
// straight into the second product P = U_jb B over its rows (U: the real
// 2d-vectors of tile jb, rows m): the output layout
// of a 16 x 16 block (register v of lane l: row 4 v + l / 16, column
// l % 16) is the B-operand layout of the K step 4 v of the next product, so
// no data moves between the two.  Re and Im of D come from the two real
// products P1 = U Re(B), P2 = U Im(B) (D_re[i] = P1[2i] - P2[2i+1],
// D_im[i] = P2[2i] + P1[2i+1]).  Each wave writes its partial P1, P2 (its
// columns over its row half) to a slot of its own; k_lse_grad_finish adds
// the slots of a column in a fixed order and applies the projection through
// the normalisation, so repeated calls give the same bits.  The next row
// tile is loaded into registers while the current one is multiplied.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = 64;
constexpr int kMaxLdp = 129;  // 2d rounded up to 16, plus one (d <= 64)
constexpr int kThreadsG = 512;

__device__ __forceinline__ void stage_cols(const double* base, int ld, int n, int d, int c0, int ldp, double* Us) {
  // columns c0 .. c0 + 63 of the normalised frame, entries 0 .. ldp - 2,
  // zero past 2d and past column n
  for (int idx = threadIdx.x; idx < T * (ldp - 1); idx += blockDim.x) {
    const int col = idx / (ldp - 1), m = idx % (ldp - 1);
    const int c = c0 + col;
    Us[col * ldp + m] = (c < n && m < 2 * d) ? base[(size_t)c * ld + m] : 0.0;
  }
}

// The next row tile in registers while the current one is multiplied.  The
// LDS column holds L = ldp - 1 doubles, a power of two (16 .. 128), so a
// thread's 16-byte pieces sit at a fixed column stride: pair p = tid mod L/2
// of columns tid / (L/2) + q (1024 / L), q = 0 .. L/64 - 1 (at least one).
constexpr int kPre = T * (kMaxLdp - 1) / 2 / kThreadsG;  // double2 per thread, at most

__device__ __forceinline__ void fetch_cols(const double* base, int ld, int n, int d, int c0, int ldp,
                                           double2 pre[kPre]) {
  const int L2 = (ldp - 1) / 2;
  const int p = threadIdx.x % L2;
  const int col0 = threadIdx.x / L2, cstep = kThreadsG / L2;
  const int nq = T / cstep;
#pragma unroll
  for (int q = 0; q < kPre; ++q) {
    const int c = c0 + col0 + q * cstep;
    pre[q] = (q < nq && c < n && 2 * p < 2 * d) ? *(const double2*)(base + (size_t)c * ld + 2 * p)
                                               : make_double2(0.0, 0.0);
  }
}

__device__ __forceinline__ void put_cols(const double2 pre[kPre], int ldp, double* Us) {
  const int L2 = (ldp - 1) / 2;
  const int p = threadIdx.x % L2;
  const int col0 = threadIdx.x / L2, cstep = kThreadsG / L2;
  const int nq = T / cstep;
#pragma unroll
  for (int q = 0; q < kPre; ++q) {
    if (q < nq && col0 + q * cstep < T) {
      double* dst = Us + (col0 + q * cstep) * ldp + 2 * p;
      dst[0] = pre[q].x;
      dst[1] = pre[q].y;
    }
  }
}

// MB = 16-row blocks of the 2d output rows (1 .. 8).  The second product's
// k steps (8 per wave and tile) are spread over Q = 8 / MB accumulator sets
// per row block, so that for small d they form Q independent chains instead
// of one serial chain; the sets are added in a fixed order at the end.  The
// LDS column stride follows from MB: 2d rounded up to a power of two >= 16,
// plus one.
template <int MB>
__global__ __launch_bounds__(kThreadsG, 1) void k_lse_grad(GradArgs a) {
  constexpr int Q = 8 / MB;
  constexpr int NSL = MB * Q;
  constexpr int LDP = (MB <= 1 ? 16 : MB <= 2 ? 32 : MB <= 4 ? 64 : 128) + 1;
  __shared__ double Uk[T * kMaxLdp];
  __shared__ double Uj[T * kMaxLdp];
  const int kb = blockIdx.x, ch = blockIdx.y;
  const int nkb = gridDim.x, nch = gridDim.y;
  const int jb0 = (int)(((int64_t)ch * nkb) / nch), jb1 = (int)(((int64_t)(ch + 1) * nkb) / nch);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int cg = w & 3;   // column group: columns 16 cg .. 16 cg + 15 of tile kb
  const int rh = w >> 2;  // row half: rows 32 rh .. 32 rh + 31 of tile jb
  constexpr int ldp = LDP;
  const uint64_t sb = *a.s_bits;
  const bool valid = sb < kInfBits64;
  const double s = __longlong_as_double((int64_t)sb);
  const double logS = *a.log_sum;
  const double inv_delta = a.inv_delta;

  stage_cols(a.frame, a.ld, a.n, a.d, kb * T, ldp, Uk);

  v4f64 P1[NSL], P2[NSL];
#pragma unroll
  for (int q = 0; q < NSL; ++q) {
    P1[q] = v4f64{0.0, 0.0, 0.0, 0.0};
    P2[q] = v4f64{0.0, 0.0, 0.0, 0.0};
  }
  const int kl = lane >> 4;
  const bool odd = kl & 1;
  const int kcol = 16 * cg + (lane & 15);  // this lane's column within tile kb
  const int kglob = kb * T + kcol;

  double2 pre[kPre];
  fetch_cols(a.frame, a.ld, a.n, a.d, jb0 * T, ldp, pre);
  for (int jb = jb0; jb < jb1; ++jb) {
    __syncthreads();  // Uj free (and Uk staged on the first pass)
    put_cols(pre, ldp, Uj);
    __syncthreads();
    if (jb + 1 < jb1) fetch_cols(a.frame, a.ld, a.n, a.d, (jb + 1) * T, ldp, pre);
    v4f64 R[2], I[2];
#pragma unroll
    for (int jl = 0; jl < 2; ++jl) {
      R[jl] = v4f64{0.0, 0.0, 0.0, 0.0};
      I[jl] = v4f64{0.0, 0.0, 0.0, 0.0};
    }
    // the whole staged width (entries past 2d are zero), a compile-time count
#pragma unroll
    for (int kk = 0; kk < (LDP - 1) / 4; ++kk) {
      const int k = 4 * kk + kl;
      const double bu = Uk[kcol * ldp + k];
      const double x = Uk[kcol * ldp + (k ^ 1)];
      const double bv = odd ? -x : x;
#pragma unroll
      for (int jl = 0; jl < 2; ++jl) {
        const double av = Uj[(32 * rh + 16 * jl + (lane & 15)) * ldp + k];
        R[jl] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bu, R[jl], 0, 0, 0);
        I[jl] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, I[jl], 0, 0, 0);
      }
    }
    // B = W o G in the output layout: register v of lane l is row
    // j = 32 rh + 16 jl + 4 v + l / 16 of tile jb, column kcol
#pragma unroll
    for (int jl = 0; jl < 2; ++jl)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jglob = jb * T + 32 * rh + 16 * jl + 4 * v + kl;
        const double re = R[jl][v], im = I[jl][v];
        const double xv = re * re + im * im;
        const bool use = valid && jglob != kglob && jglob < a.n && kglob < a.n;
        const double wt = use ? exp((xv - s) * inv_delta - logS) : 0.0;
        R[jl][v] = wt * re;
        I[jl][v] = wt * im;
      }
    // P += U_jb B over this wave's rows: K runs over them in steps of 4
#pragma unroll
    for (int jl = 0; jl < 2; ++jl)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 32 * rh + 16 * jl + 4 * v + kl;
        const int sl = ((4 * jl + v) % Q) * MB;  // this k step's accumulator set
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const double am = Uj[j * ldp + 16 * mb + (lane & 15)];
          P1[sl + mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, R[jl][v], P1[sl + mb], 0, 0, 0);
          P2[sl + mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, I[jl][v], P2[sl + mb], 0, 0, 0);
        }
      }
  }
  // add the accumulator sets in order
#pragma unroll
  for (int q = 1; q < Q; ++q)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      P1[mb] += P1[q * MB + mb];
      P2[mb] += P2[q * MB + mb];
    }
  // partial slot (kb, ch, rh): [2][64 columns][2d rows]
  double* dst = a.partial + ((size_t)((kb * nch + ch) * 2 + rh) * 2) * T * (2 * a.d);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 16 * mb + 4 * v + kl;
      if (m < 2 * a.d) {
        dst[(size_t)kcol * (2 * a.d) + m] = P1[mb][v];
        dst[(size_t)T * (2 * a.d) + (size_t)kcol * (2 * a.d) + m] = P2[mb][v];
      }
    }
  }
}

// One wave per column k: add the slots (kb, ch, rh) in order, combine
// into D_k, project and scale.  Lane i takes entries i, i + 64, ...
__global__ __launch_bounds__(64) void k_lse_grad_finish(GradArgs a, int nch) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const int d = a.d;
  const int kb = k / T, kc = k % T;
  const bool valid = *a.s_bits < kInfBits64;
  double yy = 0.0, c = 0.0;
  // first pass: the column's raw norm and c = Re(phi^H D)
  for (int i = lane; i < d; i += 64) {
    const double ya = a.raw[(size_t)k * 2 * d + 2 * i], yb = a.raw[(size_t)k * 2 * d + 2 * i + 1];
    yy += ya * ya + yb * yb;
  }
  double dre[8], dim[8];  // d <= 64: at most one entry per lane, kept for both passes
#pragma unroll
  for (int q = 0; q < 8; ++q) dre[q] = dim[q] = 0.0;
  for (int i = lane, q = 0; i < d; i += 64, ++q) {
    double p1e = 0.0, p1o = 0.0, p2e = 0.0, p2o = 0.0;
    for (int sl = 0; sl < 2 * nch; ++sl) {  // slots (ch, rh) in order
      const double* src = a.partial + ((size_t)(kb * nch * 2 + sl) * 2) * T * (2 * d) + (size_t)kc * (2 * d);
      p1e += src[2 * i];
      p1o += src[2 * i + 1];
      p2e += src[(size_t)T * (2 * d) + 2 * i];
      p2o += src[(size_t)T * (2 * d) + 2 * i + 1];
    }
    dre[q] = p1e - p2o;
    dim[q] = p2e + p1o;
    const double pa = a.frame[(size_t)k * a.ld + 2 * i], pb = a.frame[(size_t)k * a.ld + 2 * i + 1];
    c += pa * dre[q] + pb * dim[q];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    yy += __shfl_xor(yy, off, 64);
    c += __shfl_xor(c, off, 64);
  }
  const double r = sqrt(yy);
  const double scale = valid ? 2.0 / r : __builtin_nan("");
  for (int i = lane, q = 0; i < d; i += 64, ++q) {
    const double pa = a.frame[(size_t)k * a.ld + 2 * i], pb = a.frame[(size_t)k * a.ld + 2 * i + 1];
    a.grad[(size_t)k * 2 * d + 2 * i] = scale * (dre[q] - c * pa);
    a.grad[(size_t)k * 2 * d + 2 * i + 1] = scale * (dim[q] - c * pb);
  }
}

}  // namespace

int lse_grad_chunks(int nkb) {
  // One 512-thread block fits a CU (LDS), so blocks run in rounds of 256
  // (the CU count).  Row tiles are split into nch runs: at least enough for
  // one round of blocks, at most runs of 4 tiles, and within that range the
  // smallest count whose grid fills its last round to 97 % (else the best
  // fill).  Each run writes its own partial sums (2 x 64 x 2d doubles per
  // wave pair), so fewer runs also mean less traffic: at N = 4096 four runs
  // (256 blocks, one full round) write half the partials of eight.  At
  // N = 18000 (282 tiles a side), 282 x 2 = 564 blocks took three rounds
  // with the last one 22 % full; 282 x 8 = 2256 fill nine rounds to 98 %.
  constexpr int kCUs = 256;
  int lo = (kCUs + nkb - 1) / nkb;
  lo = lo < 1 ? 1 : (lo > nkb ? nkb : lo);
  const int hi = nkb / 4 > lo ? nkb / 4 : lo;
  int best = lo;
  double best_fill = -1.0;
  for (int c = lo; c <= hi; ++c) {
    const int64_t blocks = (int64_t)nkb * c;
    const int64_t rounds = (blocks + kCUs - 1) / kCUs;
    const double f = (double)blocks / (double)(rounds * kCUs);
    if (f >= 0.97) return c;
    if (f > best_fill) {
      best_fill = f;
      best = c;
    }
  }
  return best;
}

hipError_t launch_lse_grad(const GradArgs& a, hipStream_t s) {
  const int nkb = (a.n + T - 1) / T;
  const int nch = lse_grad_chunks(nkb);
  const dim3 grid(nkb, nch), block(kThreadsG);
  switch ((2 * a.d + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_lse_grad<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_lse_grad<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_lse_grad<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_lse_grad<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_lse_grad<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_lse_grad<6>, grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_lse_grad<7>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_lse_grad<8>, grid, block, 0, s, a); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lse_grad_finish, dim3(a.n), dim3(64), 0, s, a, nch);
  return hipGetLastError();
}

}  // namespace trstmi
