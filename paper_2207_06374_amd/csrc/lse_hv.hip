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
// once sigma is known.
//
// k_hv_prep: one wave per column (d <= 64: one entry per lane) forms r, dr,
// phi and dphi.  k_lse_hv: a block owns 32 columns k and a run of 16-row
// tiles j; the k tile (phi, dphi) stays in LDS, each row tile is staged in
// turn.  Phase A: every thread takes two pairs (j, k) and forms G, dG, w,
// the weights B = w G and B1 = w (dx / delta) G + w dG into LDS, and its
// share of sigma.  Phase B: every thread accumulates D and E for 8 entries of
// one column k over the tile's 16 rows.  Each block writes its D and E
// partial sums and its sigma partial to slots of its own; the finishing
// kernels add them in a fixed order, so repeated calls give the same bits.
// FP64 throughout (vector FMA: the pair work mixes three products and a
// transcendental per entry, not one dense contraction).

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kTK = 32;       // columns k per block
constexpr int kTJ = 16;       // rows j per staged row tile
constexpr int kThreadsH = 256;
constexpr int kMaxDH = 64;
constexpr int kLdH = 2 * kMaxDH + 1;  // LDS column stride in doubles (odd: lanes reading 32 columns hit distinct banks)

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

__device__ __forceinline__ void stage(const double* src, int n, int L, int c0, int cols, double* dst) {
  for (int idx = threadIdx.x; idx < cols * L; idx += kThreadsH) {
    const int col = idx / L, m = idx - col * L;
    const int c = c0 + col;
    dst[col * kLdH + m] = c < n ? src[(size_t)c * L + m] : 0.0;
  }
}

template <int M>  // M = ceil(d / 8) entries per thread in phase B
__global__ __launch_bounds__(kThreadsH) void k_lse_hv(HvArgs a) {
  __shared__ double Pk[kTK * kLdH], dPk[kTK * kLdH], Pj[kTJ * kLdH], dPj[kTJ * kLdH];
  __shared__ double2 Bs[kTJ * kTK], B1s[kTJ * kTK];
  __shared__ double red[kThreadsH / 64];
  const int kb = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
  const int n = a.n, d = a.d, L = 2 * d;
  const int njt = (n + kTJ - 1) / kTJ;
  const int jt0 = (int)(((int64_t)ch * njt) / nch), jt1 = (int)(((int64_t)(ch + 1) * njt) / nch);
  const int tid = threadIdx.x;
  const uint64_t sb = *a.s_bits;
  const bool valid = sb < kInfBits64;
  const double s = __longlong_as_double((int64_t)sb);
  const double logS = *a.log_sum;
  const double inv_delta = a.inv_delta;

  stage(a.phi, n, L, kb * kTK, kTK, Pk);
  stage(a.dphi, n, L, kb * kTK, kTK, dPk);

  double Dre[M], Dim[M], Ere[M], Eim[M];
#pragma unroll
  for (int m = 0; m < M; ++m) Dre[m] = Dim[m] = Ere[m] = Eim[m] = 0.0;
  double sig = 0.0;
  const int kkB = tid >> 3, i0 = tid & 7;  // phase B: column kkB, entries i0 + 8 m

  for (int jt = jt0; jt < jt1; ++jt) {
    __syncthreads();  // the previous tile's phase B is done with Pj, Bs
    stage(a.phi, n, L, jt * kTJ, kTJ, Pj);
    stage(a.dphi, n, L, jt * kTJ, kTJ, dPj);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = tid + q * kThreadsH;
      const int kk = p & (kTK - 1), jj = p >> 5;
      const int j = jt * kTJ + jj, k = kb * kTK + kk;
      const double* pj = Pj + jj * kLdH;
      const double* dpj = dPj + jj * kLdH;
      const double* pk = Pk + kk * kLdH;
      const double* dpk = dPk + kk * kLdH;
      double gr = 0.0, gi = 0.0, hr = 0.0, hi = 0.0;  // G and dG
      for (int i = 0; i < d; ++i) {
        const double ar = pj[2 * i], ai = pj[2 * i + 1];
        const double br = pk[2 * i], bi = pk[2 * i + 1];
        const double er = dpj[2 * i], ei = dpj[2 * i + 1];
        const double fr = dpk[2 * i], fi = dpk[2 * i + 1];
        gr = fma(ar, br, fma(ai, bi, gr));
        gi = fma(ar, bi, fma(-ai, br, gi));
        // conj(dphi_j) phi_k + conj(phi_j) dphi_k
        hr = fma(er, br, fma(ei, bi, fma(ar, fr, fma(ai, fi, hr))));
        hi = fma(er, bi, fma(-ei, br, fma(ar, fi, fma(-ai, fr, hi))));
      }
      const double x = gr * gr + gi * gi;
      const double dx = 2.0 * (gr * hr + gi * hi);
      const bool use = valid && j != k && j < n && k < n;
      const double w = use ? exp((x - s) * inv_delta - logS) : 0.0;
      sig = fma(w, dx, sig);
      const double f = w * dx * inv_delta;
      Bs[jj * kTK + kk] = make_double2(w * gr, w * gi);
      B1s[jj * kTK + kk] = make_double2(fma(f, gr, w * hr), fma(f, gi, w * hi));
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < kTJ; ++jj) {
      const double2 b = Bs[jj * kTK + kkB], b1 = B1s[jj * kTK + kkB];
      const double* pj = Pj + jj * kLdH;
      const double* dpj = dPj + jj * kLdH;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int i = i0 + 8 * m;
        if (i < d) {
          const double pr = pj[2 * i], pi = pj[2 * i + 1];
          const double qr = dpj[2 * i], qi = dpj[2 * i + 1];
          // D += phi_j b;  E += dphi_j b + phi_j b1
          Dre[m] = fma(pr, b.x, fma(-pi, b.y, Dre[m]));
          Dim[m] = fma(pr, b.y, fma(pi, b.x, Dim[m]));
          Ere[m] = fma(qr, b.x, fma(-qi, b.y, fma(pr, b1.x, fma(-pi, b1.y, Ere[m]))));
          Eim[m] = fma(qr, b.y, fma(qi, b.x, fma(pr, b1.y, fma(pi, b1.x, Eim[m]))));
        }
      }
    }
  }
  const int k = kb * kTK + kkB;
  if (k < n) {
    double* dst = a.partial + ((size_t)ch * n + k) * 2 * L;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int i = i0 + 8 * m;
      if (i < d) {
        *(double2*)(dst + 2 * i) = make_double2(Dre[m], Dim[m]);
        *(double2*)(dst + L + 2 * i) = make_double2(Ere[m], Eim[m]);
      }
    }
  }
  sig = wave_sum(sig);
  if ((tid & 63) == 0) red[tid >> 6] = sig;
  __syncthreads();
  if (tid == 0) a.sigpart[kb * nch + ch] = (red[0] + red[1]) + (red[2] + red[3]);
}

// sigma = (1/2) sum of the partials (each pair was counted as (j, k) and
// (k, j)), added by one block in a fixed order.
__global__ __launch_bounds__(256) void k_hv_sigma(HvArgs a, int count) {
  __shared__ double acc[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) v += a.sigpart[i];
  acc[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) acc[threadIdx.x] += acc[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.sigma = 0.5 * acc[0];
}

// One wave per column k: D, E from the row-run slots in order, then dD, c,
// dc and the product.
__global__ __launch_bounds__(64) void k_hv_finish(HvArgs a, int nch) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = a.n, d = a.d, L = 2 * d;
  const bool valid = *a.s_bits < kInfBits64;
  const double sigma = *a.sigma;
  double Dr = 0.0, Di = 0.0, Er = 0.0, Ei = 0.0, pa = 0.0, pb = 0.0, qa = 0.0, qb = 0.0;
  if (lane < d) {
    for (int ch = 0; ch < nch; ++ch) {
      const double* src = a.partial + ((size_t)ch * n + k) * 2 * L;
      const double2 Dv = *(const double2*)(src + 2 * lane);
      const double2 Ev = *(const double2*)(src + L + 2 * lane);
      Dr += Dv.x;
      Di += Dv.y;
      Er += Ev.x;
      Ei += Ev.y;
    }
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
  const int nkb = (n + kTK - 1) / kTK, njt = (n + kTJ - 1) / kTJ;
  int c = (512 + nkb - 1) / nkb;  // about two rounds of blocks over 256 CUs
  return c < 1 ? 1 : (c > njt ? njt : c);
}

}  // namespace

size_t hv_scratch_bytes(int64_t n, int64_t d) {
  const size_t vec = ((size_t)(2 * d * n) * 8 + 255) / 256 * 256;
  const size_t col = ((size_t)n * 8 + 255) / 256 * 256;
  const int nkb = (int)((n + kTK - 1) / kTK);
  const int nch = hv_chunks((int)n);
  const size_t part = ((size_t)nch * n * 2 * 2 * d * 8 + 255) / 256 * 256;
  const size_t sig = ((size_t)nkb * nch * 8 + 255) / 256 * 256;
  return 2 * vec + 2 * col + part + sig + 256;
}

void hv_layout(HvArgs& a, char* scratch, int64_t n, int64_t d) {
  const size_t vec = ((size_t)(2 * d * n) * 8 + 255) / 256 * 256;
  const size_t col = ((size_t)n * 8 + 255) / 256 * 256;
  const int nkb = (int)((n + kTK - 1) / kTK);
  const int nch = hv_chunks((int)n);
  const size_t part = ((size_t)nch * n * 2 * 2 * d * 8 + 255) / 256 * 256;
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
  switch ((a.d + 7) / 8) {
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
