// The paper's outer procedure (Alg. 2) with every random start advanced by
// one block of a single launch: the Haar start of stream l, then for each
// smoothing delta of the schedule up to steps_per_delta trust-region steps
// (Alg. 1: Steihaug CG with exact Hessian-vector products, read with the
// textbook's completion of the printed listing, then the ratio test and
// radius rule), and finally the exact FP64 coherence of the frame.
//
// For frames small enough to sit in one block (n <= 128, d <= 16: the
// sizes of Table II) the host-driven step (trust_region.hip), which reads a
// few scalars per CG iteration and launches every vector operation, is
// bound by launches and synchronisations; here the block keeps the
// normalised frame (and its derivative along the CG direction) in LDS and
// the CG vectors in its part of the workspace, every thread owns at most
// one column k (the column sums over j of the gradient and the Hessian
// product stay in its registers), and every scalar decision is taken by all
// threads from the same block-reduced values (fixed-order reductions, so
// all threads agree bit for bit and repeated runs give the same bits).
//
// Per column k (phi_j normalised columns, G_jk = <phi_j, phi_k>, x = |G|^2,
// w_jk = exp((x_jk - s) / delta) / S):
//   gradient  D_k = sum_j phi_j w_jk G_jk,  g_k = 2 (D_k - phi_k c_k) / r_k,
//             c_k = Re(phi_k^H D_k);
//   Hessian along V: dr_k = Re(phi_k^H v_k), dphi_k = (v_k - phi_k dr_k) / r_k,
//             dG = dphi_j^H phi_k + phi_j^H dphi_k, dx = 2 Re(conj(G) dG),
//             E_k = sum_j [dphi_j w G + phi_j (w (dx / delta) G + w dG)],
//             sigma = (1/2) sum_{j != k} w dx, dD = E - (sigma / delta) D,
//             dc = Re(dphi_k^H D_k + phi_k^H dD_k),
//             Hv_k = 2 (dD_k - dphi_k c_k - phi_k dc_k) / r_k - g_k dr_k / r_k.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kThreadsO = 256;
constexpr int kWavesO = kThreadsO / 64;

struct OptSmem {
  double phi[kOptMaxN * 2 * kOptMaxD];
  double dphi[kOptMaxN * 2 * kOptMaxD];
  double rn[kOptMaxN];
  double drn[kOptMaxN];
  double red[kWavesO];
  GaussTab tab;
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// NaN-propagating maximum (a NaN value marks an invalid frame).
__device__ __forceinline__ double nmax(double a, double b) { return (a != a || b != b) ? __builtin_nan("") : (a > b ? a : b); }

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Fixed-order block reductions; every thread returns the same bits.
__device__ double block_sum(double v, OptSmem& S) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (S.red[0] + S.red[1]) + (S.red[2] + S.red[3]);
}

__device__ double block_max(double v, OptSmem& S) {
  v = wmax(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = v;
  __syncthreads();
  return nmax(nmax(S.red[0], S.red[1]), nmax(S.red[2], S.red[3]));
}

struct Dims {
  int n, d, L;  // L = 2 d n reals
};

__device__ double dot(const Dims& z, const double* u, const double* v, OptSmem& S) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < z.L; i += kThreadsO) acc = fma(u[i], v[i], acc);
  return block_sum(acc, S);
}

// out = a x + b y (out may alias x or y: each element is read and written by one thread)
__device__ void lincomb(const Dims& z, double a, const double* x, double b, const double* y, double* out) {
  for (int i = threadIdx.x; i < z.L; i += kThreadsO) out[i] = fma(b, y[i], a * x[i]);
  __syncthreads();
}

__device__ void zerov(const Dims& z, double* out) {
  for (int i = threadIdx.x; i < z.L; i += kThreadsO) out[i] = 0.0;
  __syncthreads();
}

__device__ void copyv(const Dims& z, const double* x, double* out) {
  for (int i = threadIdx.x; i < z.L; i += kThreadsO) out[i] = x[i];
  __syncthreads();
}

// phi = the columns of Y normalised, rn = their norms (LDS).
__device__ void normalize(const Dims& z, const double* Y, OptSmem& S) {
  const int k = threadIdx.x;
  if (k < z.n) {
    const double* y = Y + (size_t)k * 2 * z.d;
    double s = 0.0;
    for (int i = 0; i < 2 * z.d; ++i) s = fma(y[i], y[i], s);
    const double r = sqrt(s);
    S.rn[k] = r;
    for (int i = 0; i < 2 * z.d; ++i) S.phi[k * 2 * kOptMaxD + i] = y[i] / r;
  }
  __syncthreads();
}

__device__ __forceinline__ void gram_entry(const double* a, const double* b, int d, double& re, double& im) {
  re = 0.0;
  im = 0.0;
  for (int i = 0; i < d; ++i) {
    const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
    re = fma(ar, br, fma(ai, bi, re));
    im = fma(ar, bi, fma(-ai, br, im));
  }
}

// s = max over j < k of x, log S and F of the frame held in phi.
__device__ void smooth_max(const Dims& z, double delta, OptSmem& S, double& s, double& logS, double& F) {
  const int k = threadIdx.x;
  double m = 0.0;
  if (k < z.n)
    for (int j = 0; j < k; ++j) {
      double re, im;
      gram_entry(S.phi + j * 2 * kOptMaxD, S.phi + k * 2 * kOptMaxD, z.d, re, im);
      m = nmax(m, fma(re, re, im * im));
    }
  s = block_max(m, S);
  double acc = 0.0;
  if (k < z.n)
    for (int j = 0; j < k; ++j) {
      double re, im;
      gram_entry(S.phi + j * 2 * kOptMaxD, S.phi + k * 2 * kOptMaxD, z.d, re, im);
      acc += exp((fma(re, re, im * im) - s) / delta);
    }
  const double tot = block_sum(acc, S);
  logS = log(tot);
  F = s + delta * logS;
}

// Gradient of F at the frame held in phi (column k by thread k).
template <int DM>
__device__ void gradient(const Dims& z, double delta, double s, double logS, double* g, OptSmem& S) {
  const int k = threadIdx.x;
  if (k < z.n) {
    const double* pk = S.phi + k * 2 * kOptMaxD;
    double D[2 * DM];
#pragma unroll
    for (int i = 0; i < 2 * DM; ++i) D[i] = 0.0;
    for (int j = 0; j < z.n; ++j) {
      if (j == k) continue;
      const double* pj = S.phi + j * 2 * kOptMaxD;
      double re, im;
      gram_entry(pj, pk, z.d, re, im);
      const double w = exp((fma(re, re, im * im) - s) / delta - logS);
      const double br = w * re, bi = w * im;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < z.d) {
          D[2 * i] = fma(pj[2 * i], br, fma(-pj[2 * i + 1], bi, D[2 * i]));
          D[2 * i + 1] = fma(pj[2 * i], bi, fma(pj[2 * i + 1], br, D[2 * i + 1]));
        }
    }
    double c = 0.0;
#pragma unroll
    for (int i = 0; i < 2 * DM; ++i)
      if (i < 2 * z.d) c = fma(pk[i], D[i], c);
    const double r = S.rn[k];
#pragma unroll
    for (int i = 0; i < 2 * DM; ++i)
      if (i < 2 * z.d) g[(size_t)k * 2 * z.d + i] = 2.0 * (D[i] - pk[i] * c) / r;
  }
  __syncthreads();
}

// H v at the frame held in phi (same s, log S), v and out in the frame layout.
template <int DM>
__device__ void hess_vec(const Dims& z, double delta, double s, double logS, const double* v, double* out,
                         OptSmem& S) {
  const int k = threadIdx.x;
  if (k < z.n) {
    const double* pk = S.phi + k * 2 * kOptMaxD;
    const double* vk = v + (size_t)k * 2 * z.d;
    double dr = 0.0;
    for (int i = 0; i < 2 * z.d; ++i) dr = fma(pk[i], vk[i], dr);
    const double r = S.rn[k];
    S.drn[k] = dr;
    for (int i = 0; i < 2 * z.d; ++i) S.dphi[k * 2 * kOptMaxD + i] = (vk[i] - pk[i] * dr) / r;
  }
  __syncthreads();
  double D[2 * DM], E[2 * DM];
#pragma unroll
  for (int i = 0; i < 2 * DM; ++i) D[i] = E[i] = 0.0;
  double sig = 0.0;
  const double inv_delta = 1.0 / delta;
  if (k < z.n) {
    const double* pk = S.phi + k * 2 * kOptMaxD;
    const double* qk = S.dphi + k * 2 * kOptMaxD;
    for (int j = 0; j < z.n; ++j) {
      if (j == k) continue;
      const double* pj = S.phi + j * 2 * kOptMaxD;
      const double* qj = S.dphi + j * 2 * kOptMaxD;
      double gr, gi, ar, ai, br2, bi2;
      gram_entry(pj, pk, z.d, gr, gi);
      gram_entry(qj, pk, z.d, ar, ai);
      gram_entry(pj, qk, z.d, br2, bi2);
      const double hr = ar + br2, hi = ai + bi2;
      const double x = fma(gr, gr, gi * gi);
      const double dx = 2.0 * fma(gr, hr, gi * hi);
      const double w = exp((x - s) * inv_delta - logS);
      sig = fma(w, dx, sig);
      const double f = w * dx * inv_delta;
      const double Br = w * gr, Bi = w * gi;
      const double Cr = fma(f, gr, w * hr), Ci = fma(f, gi, w * hi);
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < z.d) {
          const double p0 = pj[2 * i], p1 = pj[2 * i + 1], q0 = qj[2 * i], q1 = qj[2 * i + 1];
          D[2 * i] = fma(p0, Br, fma(-p1, Bi, D[2 * i]));
          D[2 * i + 1] = fma(p0, Bi, fma(p1, Br, D[2 * i + 1]));
          E[2 * i] = fma(q0, Br, fma(-q1, Bi, fma(p0, Cr, fma(-p1, Ci, E[2 * i]))));
          E[2 * i + 1] = fma(q0, Bi, fma(q1, Br, fma(p0, Ci, fma(p1, Cr, E[2 * i + 1]))));
        }
    }
  }
  const double sigma = 0.5 * block_sum(sig, S);
  if (k < z.n) {
    const double* pk = S.phi + k * 2 * kOptMaxD;
    const double* qk = S.dphi + k * 2 * kOptMaxD;
    const double sd = sigma * inv_delta;
    double c = 0.0, dc = 0.0;
#pragma unroll
    for (int i = 0; i < 2 * DM; ++i)
      if (i < 2 * z.d) {
        const double dD = E[i] - sd * D[i];
        c = fma(pk[i], D[i], c);
        dc = fma(qk[i], D[i], fma(pk[i], dD, dc));
      }
    const double r = S.rn[k], dr = S.drn[k];
#pragma unroll
    for (int i = 0; i < 2 * DM; ++i)
      if (i < 2 * z.d) {
        const double dD = E[i] - sd * D[i];
        const double g = 2.0 * (D[i] - pk[i] * c) / r;
        out[(size_t)k * 2 * z.d + i] = 2.0 * (dD - qk[i] * c - pk[i] * dc) / r - g * dr / r;
      }
  }
  __syncthreads();
}

// The two t with |z + t d| = radius (t_minus <= 0 <= t_plus when |z| <= radius).
__device__ void to_boundary(const Dims& dm, const double* zv, const double* dv, double radius, OptSmem& S, double& tm,
                            double& tp) {
  const double a = dot(dm, dv, dv, S);
  const double b = 2.0 * dot(dm, zv, dv, S);
  const double c = dot(dm, zv, zv, S) - radius * radius;
  const double disc = sqrt(fmax(b * b - 4.0 * a * c, 0.0));
  tm = (-b - disc) / (2.0 * a);
  tp = (-b + disc) / (2.0 * a);
}

// Per-start vectors in the workspace.
struct Vecs {
  double *Y, *g, *z, *zn, *r, *rn, *dv, *Bd, *Bz, *Yp;
};

// One trust-region step on F_delta at Y (in place when taken); returns the
// new radius and the CG exit code.
template <int DM>
__device__ void tr_step(const Dims& dm, const OptBatchArgs& a, double delta, double radius, const Vecs& V,
                        OptSmem& S, double& new_radius, int& exit_code) {
  double s, logS, f0;
  normalize(dm, V.Y, S);
  smooth_max(dm, delta, S, s, logS, f0);
  gradient<DM>(dm, delta, s, logS, V.g, S);
  const int max_iter = a.cg_max_iter;
  // Steihaug CG for min g.p + p.B p / 2, |p| <= radius
  zerov(dm, V.z);
  zerov(dm, V.Bz);
  copyv(dm, V.g, V.r);
  lincomb(dm, -1.0, V.g, 0.0, V.g, V.dv);
  double rr = dot(dm, V.r, V.r, S);
  int code = TRSTMI_CG_MAX_ITER;
  if (sqrt(rr) < a.cg_tol) {
    code = TRSTMI_CG_ZERO_GRADIENT;
  } else {
    for (int j = 0; j < max_iter; ++j) {
      hess_vec<DM>(dm, delta, s, logS, V.dv, V.Bd, S);
      const double dBd = dot(dm, V.dv, V.Bd, S);
      if (dBd <= 0.0) {
        double tm, tp;
        to_boundary(dm, V.z, V.dv, radius, S, tm, tp);
        const double gz = dot(dm, V.g, V.z, S), gd = dot(dm, V.g, V.dv, S);
        const double zBz = dot(dm, V.z, V.Bz, S), dBz = dot(dm, V.dv, V.Bz, S);
        const double mm = gz + tm * gd + 0.5 * (zBz + 2.0 * tm * dBz + tm * tm * dBd);
        const double mp = gz + tp * gd + 0.5 * (zBz + 2.0 * tp * dBz + tp * tp * dBd);
        const double t = mm < mp ? tm : tp;
        lincomb(dm, 1.0, V.z, t, V.dv, V.z);
        lincomb(dm, 1.0, V.Bz, t, V.Bd, V.Bz);
        code = TRSTMI_CG_NEGATIVE_CURVATURE;
        break;
      }
      const double alpha = rr / dBd;
      lincomb(dm, 1.0, V.z, alpha, V.dv, V.zn);
      if (sqrt(dot(dm, V.zn, V.zn, S)) >= radius) {
        double tm, tp;
        to_boundary(dm, V.z, V.dv, radius, S, tm, tp);
        lincomb(dm, 1.0, V.z, tp, V.dv, V.z);
        lincomb(dm, 1.0, V.Bz, tp, V.Bd, V.Bz);
        code = TRSTMI_CG_BOUNDARY;
        break;
      }
      lincomb(dm, 1.0, V.r, alpha, V.Bd, V.rn);
      lincomb(dm, 1.0, V.Bz, alpha, V.Bd, V.Bz);
      const double rr_new = dot(dm, V.rn, V.rn, S);
      if (sqrt(rr_new) < a.cg_tol) {
        copyv(dm, V.zn, V.z);
        code = TRSTMI_CG_SMALL_RESIDUAL;
        break;
      }
      const double beta = rr_new / rr;
      lincomb(dm, -1.0, V.rn, beta, V.dv, V.dv);
      copyv(dm, V.zn, V.z);
      copyv(dm, V.rn, V.r);
      rr = rr_new;
    }
  }
  exit_code = code;
  // ratio test and radius rule
  const double snorm = sqrt(dot(dm, V.z, V.z, S));
  const double pred = -(dot(dm, V.g, V.z, S) + 0.5 * dot(dm, V.z, V.Bz, S));
  if (snorm == 0.0 || !(pred > 0.0)) {
    new_radius = radius / 4;
    return;
  }
  lincomb(dm, 1.0, V.Y, 1.0, V.z, V.Yp);
  double s1, logS1, f1;
  normalize(dm, V.Yp, S);
  smooth_max(dm, delta, S, s1, logS1, f1);
  const double rho = (f0 - f1) / pred;
  double nr = radius;
  if (rho < 0.25)
    nr = radius / 4;
  else if (rho > 0.75 && snorm >= radius * (1 - 1e-12))
    nr = fmin(2 * radius, a.radius_max);
  new_radius = nr;
  if (rho > a.eta) copyv(dm, V.Yp, V.Y);
}

template <int DM>
__global__ __launch_bounds__(kThreadsO) void k_opt_batch(OptBatchArgs a) {
  __shared__ OptSmem S;
  const int l = blockIdx.x;
  const Dims dm{a.n, a.d, 2 * a.d * a.n};
  double* base = a.work + (size_t)l * a.stride;
  const Vecs V{base,          base + dm.L,     base + 2 * dm.L, base + 3 * dm.L, base + 4 * dm.L,
               base + 5 * dm.L, base + 6 * dm.L, base + 7 * dm.L, base + 8 * dm.L, base + 9 * dm.L};
  fill_gauss_tab(&S.tab);
  __syncthreads();
  // random start (Alg. 2, first step): the draws of trstmi_init_haar for
  // stream first + l (tag 1, candidate 0, step 0), columns normalised
  const int nb = (a.d + 1) >> 1;
  for (int e = threadIdx.x; e < a.n * nb; e += kThreadsO) {
    const int col = e / nb, q = e - col * nb;
    const u32x4 ctr = {(uint32_t)(col * nb + q), 0u, 0u, 1u};
    const u32x4 w = philox4x32_10(ctr, a.seed, (uint32_t)(a.first + l));
    double r0, c0, s0, r1, c1, s1;
    cn_polar(w.x, w.y, S.tab, r0, c0, s0);
    cn_polar(w.z, w.w, S.tab, r1, c1, s1);
    double* o = V.Y + 2 * ((size_t)col * a.d + 2 * q);
    o[0] = r0 * c0;
    o[1] = r0 * s0;
    if (2 * q + 1 < a.d) {
      o[2] = r1 * c1;
      o[3] = r1 * s1;
    }
  }
  __syncthreads();
  normalize(dm, V.Y, S);
  for (int i = threadIdx.x; i < dm.L; i += kThreadsO) V.Y[i] = S.phi[(i / (2 * a.d)) * 2 * kOptMaxD + i % (2 * a.d)];
  __syncthreads();

  for (int kd = 0; kd < a.n_deltas; ++kd) {
    const double delta = a.deltas[kd];
    double radius = a.radius0;
    for (int st = 0; st < a.steps_per_delta; ++st) {
      double nr;
      int code;
      tr_step<DM>(dm, a, delta, radius, V, S, nr, code);
      radius = nr;
      if (radius < a.radius_min || code == TRSTMI_CG_ZERO_GRADIENT) break;
    }
  }
  // exact FP64 coherence of the result
  normalize(dm, V.Y, S);
  const int k = threadIdx.x;
  double m = 0.0;
  if (k < dm.n)
    for (int j = 0; j < k; ++j) {
      double re, im;
      gram_entry(S.phi + j * 2 * kOptMaxD, S.phi + k * 2 * kOptMaxD, dm.d, re, im);
      m = nmax(m, fma(re, re, im * im));
    }
  const double mx = block_max(m, S);
  if (threadIdx.x == 0) a.mu[l] = sqrt(mx);
}

}  // namespace

size_t opt_batch_stride(int64_t n, int64_t d) { return ((size_t)(10 * 2 * d * n) + 31) / 32 * 32; }

hipError_t launch_opt_batch(const OptBatchArgs& a, hipStream_t s) {
  const dim3 grid(a.starts), block(kThreadsO);
  if (a.d <= 4)
    hipLaunchKernelGGL(k_opt_batch<4>, grid, block, 0, s, a);
  else if (a.d <= 8)
    hipLaunchKernelGGL(k_opt_batch<8>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_opt_batch<16>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace trstmi
