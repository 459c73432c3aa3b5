// Exact Hessian-vector product of the smooth maximum of section IV (Alg. 1
// takes B_k to be the Hessian of the objective) with respect to the
// unconstrained frame Y, in a direction V (same layout as Y).
//
// Forward differentiation of the gradient's chain (see lse_grad.hip):
//   r_k = |y_k|, phi_k = y_k / r_k:   dr_k = Re(phi_k^H v_k),
//                                     dphi_k = (v_k - phi_k dr_k) / r_k;
//   G = Phi^H Phi:                    dG = dPhi^H Phi + Phi^H dPhi;
//   x = |G|^2:                        dx = 2 Re(conj(G) dG);
//   w = exp((x - s) / delta) / S:     dw = w (dx - sigma) / delta,
//                                     sigma = sum_{j<k} w_jk dx_jk;
//   D = Phi (W o G):                  dD = dPhi (W o G) + Phi (dW o G + W o dG)
//                                        = E - (sigma / delta) D,
//     E = dPhi (W o G) + Phi (W o (dx / delta) o G + W o dG);
//   c_k = Re(phi_k^H D_k):            dc_k = Re(dphi_k^H D_k + phi_k^H dD_k);
//   g_k = 2 (D_k - phi_k c_k) / r_k:  Hv_k = 2 (dD_k - dphi_k c_k - phi_k dc_k) / r_k
//                                             - g_k dr_k / r_k.
// sigma is a sum over all pairs, so the tile pass accumulates D and E
// (which do not need it) and its partial sums; the finishing kernel forms dD
// once sigma is known.  The tile pass weights the pairs with the unnormalised
// e = exp((x - s) / delta) of its own x and sums e as well, and the finishing
// kernels divide by that sum S: the weights then add up to one for the x
// this pass computed.  (Normalising with the sum of the smooth-maximum pass
// instead, whose x differ from these in the last bits, leaves the weights'
// total off by about 1e-13 at delta = 1e-3, which the (sigma / delta) D term
// turns into a relative error of about 1e-11 in Hv.)
//
// k_hv_prep: one wave per column (d <= 64: one entry per lane) forms r, dr,
// phi and dphi.  k_lse_hv: a block of eight waves owns 32 columns k (two
// 16-column blocks; phi and dphi of them in LDS) and a run of 16-row tiles j
// (phi and dphi of the tile staged in LDS, the next tile prefetched into
// registers).  Per tile, on v_mfma_f64_16x16x4f64:
//   forward: G and dG of the 16 x 32 pairs as four real products per
//     16 x 16 block, Re G = U_j . U_k, Im G = U_j . V_k (V: each (re, im)
//     pair swapped, the second negated), Re dG = dU_j . U_k + U_j . dU_k,
//     Im dG = dU_j . V_k + U_j . dV_k; wave w takes block w mod 2 and one of
//     the four (the two-product ones paired on a SIMD with a one-product
//     one), and leaves its result in LDS;
//   weights: one thread per pair forms e, its shares of S and of sigma,
//     B = e G and B1 = e (dx / delta) G + e dG in place;
//   backward: wave w takes the 16 real rows 16 w .. 16 w + 15 of the 2d-row
//     outputs P1 = U_j Re B, P2 = U_j Im B, Q1 = dU_j Re B + U_j Re B1,
//     Q2 = dU_j Im B + U_j Im B1 for both column blocks, accumulated over all
//     of the block's tiles in registers.
// Each block writes P1, P2, Q1, Q2 of its columns and its shares of S and
// sigma to slots of its own; the finishing kernels add them in a fixed order (so
// repeated calls give the same bits) and combine D_re[i] = P1[2i] - P2[2i+1],
// D_im[i] = P2[2i] + P1[2i+1] (E likewise from Q1, Q2).

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kTK = 32;         // columns k per block
constexpr int kTJ = 16;         // rows j per staged row tile
constexpr int kThreadsH = 512;  // eight waves
constexpr int kMaxLdpH = 129;   // LDS column stride: 2d rounded up to a power of two >= 16, plus one (d <= 64)
constexpr int kFS = kTK + 1;    // row stride of the per-pair arrays
constexpr int kPreH = 2 * kTJ * (kMaxLdpH - 1) / kThreadsH;  // prefetched doubles per thread, at most

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same bits (each step adds the
  // same two values on both lanes)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(64) void k_hv_prep(HvArgs a) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const int L = 2 * a.d;
  double ya = 0.0, yb = 0.0, va = 0.0, vb = 0.0;
  if (lane < a.d) {
    const double2 y = *(const double2*)(a.raw + (size_t)k * L + 2 * lane);
    const double2 v = *(const double2*)(a.v + (size_t)k * L + 2 * lane);
    ya = y.x;
    yb = y.y;
    va = v.x;
    vb = v.y;
  }
  const double r = sqrt(wave_sum(ya * ya + yb * yb));
  const double pa = ya / r, pb = yb / r;
  const double dr = wave_sum(pa * va + pb * vb);
  if (lane < a.d) {
    *(double2*)(a.phi + (size_t)k * L + 2 * lane) = make_double2(pa, pb);
    *(double2*)(a.dphi + (size_t)k * L + 2 * lane) = make_double2((va - pa * dr) / r, (vb - pb * dr) / r);
  }
  if (lane == 0) {
    a.r[k] = r;
    a.dr[k] = dr;
  }
}

// Columns c0 .. c0 + cnt - 1 of src (column stride L) into dst (column
// stride ldp): entries 0 .. ldp - 2, zero past L and past column n.
__device__ __forceinline__ void stage_h(const double* src, int n, int L, int c0, int cnt, int ldp, double* dst) {
  for (int idx = threadIdx.x; idx < cnt * (ldp - 1); idx += kThreadsH) {
    const int col = idx / (ldp - 1), m = idx - col * (ldp - 1);
    const int c = c0 + col;
    dst[col * ldp + m] = (c < n && m < L) ? src[(size_t)c * L + m] : 0.0;
  }
}

// The row tile j0 .. j0 + 15 of phi and dphi: element idx = tid + q * 512 of
// the (array, row, entry) space, entries 0 .. ldp - 2.
__device__ __forceinline__ void fetch_rows(const HvArgs& a, int j0, int ldp, double pre[kPreH]) {
  const int W = ldp - 1, per = kTJ * W, L = 2 * a.d;
#pragma unroll
  for (int q = 0; q < kPreH; ++q) {
    const int idx = (int)threadIdx.x + q * kThreadsH;
    double v = 0.0;
    if (idx < 2 * per) {
      const int arr = idx / per, rem = idx - arr * per;
      const int row = rem / W, m = rem - row * W;
      const int j = j0 + row;
      if (j < a.n && m < L) v = (arr ? a.dphi : a.phi)[(size_t)j * L + m];
    }
    pre[q] = v;
  }
}

__device__ __forceinline__ void put_rows(const double pre[kPreH], int ldp, double* Uj, double* dUj) {
  const int W = ldp - 1, per = kTJ * W;
#pragma unroll
  for (int q = 0; q < kPreH; ++q) {
    const int idx = (int)threadIdx.x + q * kThreadsH;
    if (idx < 2 * per) {
      const int arr = idx / per, rem = idx - arr * per;
      const int row = rem / W, m = rem - row * W;
      (arr ? dUj : Uj)[row * ldp + m] = pre[q];
    }
  }
}

// Forward product(s) of one 16 x 16 pair block: rows j of the tile (A
// operand: lane l holds row l % 16 at real index 4 ks + l / 16), columns
// kcol of the k tile (B operand).  Q: 0 Re G, 1 Im G, 2 Re dG, 3 Im dG.
template <int Q, int LDP>
__device__ __forceinline__ v4f64 fwd_block(const double* Uj, const double* dUj, const double* Uk, const double* dUk,
                                           int kcol) {
  constexpr int ldp = LDP;
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kl = lane >> 4;
  const bool odd = kl & 1;
  v4f64 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // the whole staged width (entries past 2d are zero), a compile-time count
#pragma unroll
  for (int ks = 0; ks < (LDP - 1) / 4; ++ks) {
    const int m = 4 * ks + kl;
    const double au = Uj[l16 * ldp + m];
    if constexpr (Q == 0) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, Uk[kcol * ldp + m], acc0, 0, 0, 0);
    } else if constexpr (Q == 1) {
      const double x = Uk[kcol * ldp + (m ^ 1)];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, odd ? -x : x, acc0, 0, 0, 0);
    } else if constexpr (Q == 2) {
      const double adu = dUj[l16 * ldp + m];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(adu, Uk[kcol * ldp + m], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, dUk[kcol * ldp + m], acc1, 0, 0, 0);
    } else {
      const double adu = dUj[l16 * ldp + m];
      const double x = Uk[kcol * ldp + (m ^ 1)], y = dUk[kcol * ldp + (m ^ 1)];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(adu, odd ? -x : x, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, odd ? -y : y, acc1, 0, 0, 0);
    }
  }
  if constexpr (Q >= 2) acc0 += acc1;
  return acc0;
}

// MB = 16-row blocks of the 2d real output rows (1 .. 8): waves w < MB take
// block w in the backward products.
template <int MB>
__global__ __launch_bounds__(kThreadsH, 1) void k_lse_hv(HvArgs a) {
  constexpr int LDP = (MB <= 1 ? 16 : MB <= 2 ? 32 : MB <= 4 ? 64 : 128) + 1;
  __shared__ double Uk[kTK * kMaxLdpH], dUk[kTK * kMaxLdpH];
  __shared__ double Uj[kTJ * kMaxLdpH], dUj[kTJ * kMaxLdpH];
  __shared__ double F[4][kTJ * kFS];  // R, I, dR, dI of the tile's pairs, then Re B, Im B, Re B1, Im B1
  __shared__ double red[2 * (kThreadsH / 64)];
  const int kb = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
  const int n = a.n, L = 2 * a.d;
  const int njt = (n + kTJ - 1) / kTJ;
  const int jt0 = (int)(((int64_t)ch * njt) / nch), jt1 = (int)(((int64_t)(ch + 1) * njt) / nch);
  const int tid = threadIdx.x;
  const int lane = tid & 63, l16 = lane & 15, kl = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cbf = w & 1, qf = w >> 1;  // forward: column block and quantity
  const uint64_t sb = *a.s_bits;
  const bool valid = sb < kInfBits64;
  const double s = __longlong_as_double((int64_t)sb);
  const double inv_delta = a.inv_delta;

  stage_h(a.phi, n, L, kb * kTK, kTK, LDP, Uk);
  stage_h(a.dphi, n, L, kb * kTK, kTK, LDP, dUk);

  v4f64 P1[2], P2[2], Q1[2], Q2[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) P1[cb] = P2[cb] = Q1[cb] = Q2[cb] = v4f64{0.0, 0.0, 0.0, 0.0};
  double sig = 0.0, esum = 0.0;

  double pre[kPreH];
  if (jt0 < jt1) fetch_rows(a, jt0 * kTJ, LDP, pre);
  for (int jt = jt0; jt < jt1; ++jt) {
    __syncthreads();  // Uj, dUj and F free (and Uk, dUk staged on the first pass)
    put_rows(pre, LDP, Uj, dUj);
    __syncthreads();
    if (jt + 1 < jt1) fetch_rows(a, (jt + 1) * kTJ, LDP, pre);

    // forward: this wave's quantity for column block cbf
    {
      const int kcol = 16 * cbf + l16;
      v4f64 r;
      if (qf == 0)
        r = fwd_block<0, LDP>(Uj, dUj, Uk, dUk, kcol);
      else if (qf == 1)
        r = fwd_block<1, LDP>(Uj, dUj, Uk, dUk, kcol);
      else if (qf == 2)
        r = fwd_block<2, LDP>(Uj, dUj, Uk, dUk, kcol);
      else
        r = fwd_block<3, LDP>(Uj, dUj, Uk, dUk, kcol);
#pragma unroll
      for (int v = 0; v < 4; ++v) F[qf][(4 * v + kl) * kFS + kcol] = r[v];
    }
    __syncthreads();

    // weights, one pair per thread, in place
    {
      const int jj = tid >> 5, kk = tid & (kTK - 1);
      const int o = jj * kFS + kk;
      const int j = jt * kTJ + jj, k = kb * kTK + kk;
      const double gr = F[0][o], gi = F[1][o], hr = F[2][o], hi = F[3][o];
      const double x = gr * gr + gi * gi;
      const double dx = 2.0 * (gr * hr + gi * hi);
      const bool use = valid && j != k && j < n && k < n;
      const double wt = use ? exp((x - s) * inv_delta) : 0.0;
      esum += wt;
      sig = fma(wt, dx, sig);
      const double f = wt * dx * inv_delta;
      F[0][o] = wt * gr;
      F[1][o] = wt * gi;
      F[2][o] = fma(f, gr, wt * hr);
      F[3][o] = fma(f, gi, wt * hi);
    }
    __syncthreads();

    // backward: real rows 16 w .. 16 w + 15 of the outputs, both column blocks
    if (w < MB) {
#pragma unroll
      for (int ks = 0; ks < kTJ / 4; ++ks) {
        const int jr = 4 * ks + kl;  // B operand row (k index) of this lane
        const double au = Uj[jr * LDP + 16 * w + l16];
        const double adu = dUj[jr * LDP + 16 * w + l16];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int o = jr * kFS + 16 * cb + l16;
          const double bre = F[0][o], bim = F[1][o], b1re = F[2][o], b1im = F[3][o];
          P1[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bre, P1[cb], 0, 0, 0);
          P2[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bim, P2[cb], 0, 0, 0);
          Q1[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(adu, bre, Q1[cb], 0, 0, 0);
          Q2[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(adu, bim, Q2[cb], 0, 0, 0);
          Q1[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, b1re, Q1[cb], 0, 0, 0);
          Q2[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, b1im, Q2[cb], 0, 0, 0);
        }
      }
    }
  }

  // partial slot (ch, k): [4][2d] = P1, P2, Q1, Q2 over real rows m
  if (w < MB) {
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int k = kb * kTK + 16 * cb + l16;
      if (k < n) {
        double* dst = a.partial + ((size_t)ch * n + k) * 4 * L;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * w + 4 * v + kl;
          if (m < L) {
            dst[m] = P1[cb][v];
            dst[L + m] = P2[cb][v];
            dst[2 * L + m] = Q1[cb][v];
            dst[3 * L + m] = Q2[cb][v];
          }
        }
      }
    }
  }
  sig = wave_sum(sig);
  esum = wave_sum(esum);
  if (lane == 0) {
    red[tid >> 6] = sig;
    red[kThreadsH / 64 + (tid >> 6)] = esum;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0, u = 0.0;
    for (int i = 0; i < kThreadsH / 64; ++i) {
      t += red[i];
      u += red[kThreadsH / 64 + i];
    }
    a.sigpart[kb * nch + ch] = t;
    a.esumpart[kb * nch + ch] = u;
  }
}

// S = (1/2) sum of the e partials and sigma = (1/2) sum of the e dx partials
// / S (each pair was counted as (j, k) and (k, j)), added by one block in a
// fixed order.
__global__ __launch_bounds__(256) void k_hv_sigma(HvArgs a, int count) {
  __shared__ double acc[2][256];
  double v = 0.0, u = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) {
    v += a.sigpart[i];
    u += a.esumpart[i];
  }
  acc[0][threadIdx.x] = v;
  acc[1][threadIdx.x] = u;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      acc[0][threadIdx.x] += acc[0][threadIdx.x + h];
      acc[1][threadIdx.x] += acc[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double S = 0.5 * acc[1][0];
    a.sigma[0] = 0.5 * acc[0][0] / S;
    a.sigma[1] = 1.0 / S;
  }
}

// One wave per column k: D, E from the row-run slots in order, then dD, c,
// dc and the product.
__global__ __launch_bounds__(64) void k_hv_finish(HvArgs a, int nch) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = a.n, d = a.d, L = 2 * d;
  const bool valid = *a.s_bits < kInfBits64;
  const double sigma = a.sigma[0], invS = a.sigma[1];
  double Dr = 0.0, Di = 0.0, Er = 0.0, Ei = 0.0, pa = 0.0, pb = 0.0, qa = 0.0, qb = 0.0;
  if (lane < d) {
    double p1e = 0.0, p1o = 0.0, p2e = 0.0, p2o = 0.0, q1e = 0.0, q1o = 0.0, q2e = 0.0, q2o = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      const double* src = a.partial + ((size_t)ch * n + k) * 4 * L;
      const double2 p1 = *(const double2*)(src + 2 * lane);
      const double2 p2 = *(const double2*)(src + L + 2 * lane);
      const double2 q1 = *(const double2*)(src + 2 * L + 2 * lane);
      const double2 q2 = *(const double2*)(src + 3 * L + 2 * lane);
      p1e += p1.x;
      p1o += p1.y;
      p2e += p2.x;
      p2o += p2.y;
      q1e += q1.x;
      q1o += q1.y;
      q2e += q2.x;
      q2o += q2.y;
    }
    Dr = (p1e - p2o) * invS;
    Di = (p2e + p1o) * invS;
    Er = (q1e - q2o) * invS;
    Ei = (q2e + q1o) * invS;
    const double2 p = *(const double2*)(a.phi + (size_t)k * L + 2 * lane);
    const double2 q = *(const double2*)(a.dphi + (size_t)k * L + 2 * lane);
    pa = p.x;
    pb = p.y;
    qa = q.x;
    qb = q.y;
  }
  const double sd = sigma * a.inv_delta;
  const double dDr = Er - sd * Dr, dDi = Ei - sd * Di;
  const double c = wave_sum(pa * Dr + pb * Di);
  const double dc = wave_sum(qa * Dr + qb * Di + pa * dDr + pb * dDi);
  const double r = a.r[k], dr = a.dr[k];
  if (lane < d) {
    const double gr = 2.0 * (Dr - pa * c) / r, gi = 2.0 * (Di - pb * c) / r;
    double hr = 2.0 * (dDr - qa * c - pa * dc) / r - gr * dr / r;
    double hi = 2.0 * (dDi - qb * c - pb * dc) / r - gi * dr / r;
    if (!valid) hr = hi = __builtin_nan("");
    *(double2*)(a.out + (size_t)k * L + 2 * lane) = make_double2(hr, hi);
  }
}

int hv_chunks(int n) {
  // one 512-thread block per CU (LDS): about one round of blocks over the
  // 256 CUs
  const int nkb = (n + kTK - 1) / kTK, njt = (n + kTJ - 1) / kTJ;
  int c = (256 + nkb - 1) / nkb;
  return c < 1 ? 1 : (c > njt ? njt : c);
}

}  // namespace

size_t hv_scratch_bytes(int64_t n, int64_t d) {
  const size_t vec = ((size_t)(2 * d * n) * 8 + 255) / 256 * 256;
  const size_t col = ((size_t)n * 8 + 255) / 256 * 256;
  const int nkb = (int)((n + kTK - 1) / kTK);
  const int nch = hv_chunks((int)n);
  const size_t part = ((size_t)nch * n * 4 * 2 * d * 8 + 255) / 256 * 256;
  const size_t sig = ((size_t)nkb * nch * 8 + 255) / 256 * 256;
  return 2 * vec + 2 * col + part + 2 * sig + 256;
}

void hv_layout(HvArgs& a, char* scratch, int64_t n, int64_t d) {
  const size_t vec = ((size_t)(2 * d * n) * 8 + 255) / 256 * 256;
  const size_t col = ((size_t)n * 8 + 255) / 256 * 256;
  const int nkb = (int)((n + kTK - 1) / kTK);
  const int nch = hv_chunks((int)n);
  const size_t part = ((size_t)nch * n * 4 * 2 * d * 8 + 255) / 256 * 256;
  const size_t sig = ((size_t)nkb * nch * 8 + 255) / 256 * 256;
  char* p = scratch;
  a.phi = (double*)p;
  p += vec;
  a.dphi = (double*)p;
  p += vec;
  a.r = (double*)p;
  p += col;
  a.dr = (double*)p;
  p += col;
  a.partial = (double*)p;
  p += part;
  a.sigpart = (double*)p;
  p += sig;
  a.esumpart = (double*)p;
  p += sig;
  a.sigma = (double*)p;
  a.n = (int32_t)n;
  a.d = (int32_t)d;
}

hipError_t launch_lse_hv(const HvArgs& a, hipStream_t s) {
  const int nkb = (a.n + kTK - 1) / kTK;
  const int nch = hv_chunks(a.n);
  hipLaunchKernelGGL(k_hv_prep, dim3(a.n), dim3(64), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid(nkb, nch);
  switch ((2 * a.d + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_lse_hv<1>, grid, dim3(kThreadsH), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_lse_hv<2>, grid, dim3(kThreadsH), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_lse_hv<3>, grid, dim3(kThreadsH), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_lse_hv<4>, grid, dim3(kThreadsH), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_lse_hv<5>, grid, dim3(kThreadsH), 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_lse_hv<6>, grid, dim3(kThreadsH), 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_lse_hv<7>, grid, dim3(kThreadsH), 0, s, a); break;
    default: hipLaunchKernelGGL(k_lse_hv<8>, grid, dim3(kThreadsH), 0, s, a); break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hv_sigma, dim3(1), dim3(256), 0, s, a, nkb * nch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hv_finish, dim3(a.n), dim3(64), 0, s, a, nch);
  return hipGetLastError();
}

}  // namespace trstmi
