// Trust-region step of the paper's optimiser on the smooth maximum (section
// IV): Steihaug's truncated CG for the trust-region subproblem (Alg. 1, with
// the textbook's completion of the garbled listing: boundary test on the new
// iterate, residual test on the new residual, and the beta / direction
// update), then the textbook ratio test and radius rule.
//
// Vectors are the real coordinates of the complex d x N frame (2dN doubles).
// All vector work runs in the kernels below: dot products over a fixed
// block partition with a fixed-order finish (repeatable bits), and linear
// combinations.  Hessian-vector products are exact (lse_hv.hip: B is the
// Hessian of the smooth maximum, as Alg. 1 states), or, as an option,
// central differences of the gradient (trstmi_lse_grad) along the unit
// direction.  The host part makes
// the scalar decisions of the algorithm, reading a few doubles per CG
// iteration.

#include <cmath>
#include <cstring>

#include "device_common.h"
#include "launch.h"
#include "trstmi.h"

namespace trstmi {

namespace {

constexpr int kDotBlocks = 256;
constexpr int kThreads = 256;

// partial[k][b] = sum over block b's range of u_k . v_k (k < nk).
__global__ __launch_bounds__(kThreads) void k_dot3(const double* u0, const double* v0, const double* u1,
                                                   const double* v1, const double* u2, const double* v2, int nk,
                                                   int64_t L, double* partial) {
  __shared__ double acc[3][kThreads];
  const int64_t chunk = (L + kDotBlocks - 1) / kDotBlocks;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < L ? lo + chunk : L;
  const double* U[3] = {u0, u1, u2};
  const double* V[3] = {v0, v1, v2};
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    if (k < nk)
      for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) s += U[k][i] * V[k][i];
    acc[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 3; ++k) acc[k][threadIdx.x] += acc[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[threadIdx.x * kDotBlocks + blockIdx.x] = acc[threadIdx.x][0];
}

__global__ __launch_bounds__(kDotBlocks) void k_dot3_finish(const double* partial, double* out) {
  __shared__ double acc[3][kDotBlocks];
  for (int k = 0; k < 3; ++k) acc[k][threadIdx.x] = partial[k * kDotBlocks + threadIdx.x];
  __syncthreads();
  for (int h = kDotBlocks / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 3; ++k) acc[k][threadIdx.x] += acc[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = acc[threadIdx.x][0];
}

// out = a x + b y (y may be null: out = a x; x may be null: out = b y).
__global__ __launch_bounds__(kThreads) void k_lincomb(double a, const double* x, double b, const double* y,
                                                      int64_t L, double* out) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < L; i += (int64_t)gridDim.x * kThreads) {
    double v = 0.0;
    if (x) v = a * x[i];
    if (y) v = x ? fma(b, y[i], v) : b * y[i];
    out[i] = v;
  }
}

struct Ctx {
  int64_t n, d, L;
  hipStream_t s;
  double* dots;      // device [3]
  double* partial;   // device [3][kDotBlocks]
  char* lws;         // trstmi_lse_grad workspace
  size_t lws_bytes;
  double* out2;      // device (s, F)
};

hipError_t lincomb(const Ctx& c, double a, const double* x, double b, const double* y, double* out) {
  int64_t blocks = (c.L + kThreads - 1) / kThreads;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_lincomb, dim3((int)blocks), dim3(kThreads), 0, c.s, a, x, b, y, c.L, out);
  return hipGetLastError();
}

// up to three dot products, read back to the host
hipError_t dots(const Ctx& c, int nk, const double* u0, const double* v0, const double* u1, const double* v1,
                const double* u2, const double* v2, double res[3]) {
  hipLaunchKernelGGL(k_dot3, dim3(kDotBlocks), dim3(kThreads), 0, c.s, u0, v0, u1, v1, u2, v2, nk, c.L, c.partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot3_finish, dim3(1), dim3(kDotBlocks), 0, c.s, c.partial, c.dots);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(res, c.dots, 3 * sizeof(double), hipMemcpyDeviceToHost, c.s)) != hipSuccess) return e;
  return hipStreamSynchronize(c.s);
}

}  // namespace

size_t tr_vectors_bytes(int64_t n, int64_t d) {
  const size_t vec = ((size_t)(2 * d * n) * 8 + 255) / 256 * 256;
  return 9 * vec + 256 + 3 * kDotBlocks * 8 + hv_scratch_bytes(n, d);
}

// The trust-region step itself (arguments validated by the caller).
trstmi_status tr_step_impl(int64_t n, int64_t d, double* frame, const trstmi_tr_params* tp, trstmi_tr_report* rep,
                           char* ws, size_t lws_bytes, hipStream_t stream) {
  Ctx c{};
  c.n = n;
  c.d = d;
  c.L = 2 * d * n;
  c.s = stream;
  c.lws = ws;
  c.lws_bytes = lws_bytes;
  const size_t vec = ((size_t)c.L * 8 + 255) / 256 * 256;
  char* p = ws + lws_bytes;
  double* V[9];
  for (int i = 0; i < 9; ++i) V[i] = (double*)(p + i * vec);
  double *g = V[0], *z = V[1], *r = V[2], *dd = V[3], *Bd = V[4], *Bz = V[5], *Yp = V[6], *gp = V[7], *gm = V[8];
  char* q = p + 9 * vec;
  c.out2 = (double*)q;
  c.dots = (double*)(q + 64);
  c.partial = (double*)(q + 256);
  const bool exact = !(tp->fd_step > 0.0);
  HvArgs hv{};
  if (exact) {
    hv_layout(hv, q + 256 + 3 * kDotBlocks * 8, n, d);
    const double* unused_log_sum = nullptr;  // the product normalises with its own sum
    lse_grad_scalars(n, d, ws, &hv.s_bits, &unused_log_sum);
    hv.raw = frame;
    hv.inv_delta = 1.0 / tp->delta;
  }

#define TR_HIP(expr)                                    \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return TRSTMI_E_HIP;          \
  } while (0)
#define TR_CALL(expr)                                   \
  do {                                                  \
    trstmi_status st_ = (expr);                         \
    if (st_ != TRSTMI_OK) return st_;                   \
  } while (0)

  auto grad_at = [&](const double* Y, double* gout) -> trstmi_status {
    return trstmi_lse_grad(n, d, Y, tp->delta, c.out2, gout, c.lws, c.lws_bytes, stream);
  };
  double h2[2];
  double res[3];
  // f and g at the frame
  TR_CALL(grad_at(frame, g));
  TR_HIP(hipMemcpyAsync(h2, c.out2, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  TR_HIP(hipStreamSynchronize(stream));
  const double f0 = h2[1];
  std::memset(rep, 0, sizeof(*rep));
  rep->f_old = f0;
  rep->f_new = f0;
  rep->new_radius = tp->radius / 4;
  if (!std::isfinite(f0)) return TRSTMI_E_INVALID_ARG;  // a zero or non-finite column

  // Steihaug CG on m(p) = g.p + p.B p / 2, |p| <= radius
  const double radius = tp->radius;
  TR_HIP(lincomb(c, 0.0, nullptr, 0.0, nullptr, z));
  TR_HIP(lincomb(c, 0.0, nullptr, 0.0, nullptr, Bz));
  TR_HIP(lincomb(c, 1.0, g, 0.0, nullptr, r));
  TR_HIP(lincomb(c, -1.0, g, 0.0, nullptr, dd));
  TR_HIP(dots(c, 1, r, r, nullptr, nullptr, nullptr, nullptr, res));
  double rr = res[0];
  int iters = 0, code = TRSTMI_CG_MAX_ITER;
  if (std::sqrt(rr) < tp->cg_tol) {
    code = TRSTMI_CG_ZERO_GRADIENT;
  } else {
    for (int j = 0; j < tp->cg_max_iter; ++j) {
      iters = j + 1;
      TR_HIP(dots(c, 1, dd, dd, nullptr, nullptr, nullptr, nullptr, res));
      const double nd = std::sqrt(res[0]);
      if (exact) {
        // B d with B the Hessian at the frame (s and log S of the frame stay
        // in the gradient's workspace: no gradient is evaluated elsewhere)
        hv.v = dd;
        hv.out = Bd;
        TR_HIP(launch_lse_hv(hv, stream));
      } else {
        // B d by central differences along d / |d|
        const double hs = tp->fd_step / nd;
        TR_HIP(lincomb(c, 1.0, frame, hs, dd, Yp));
        TR_CALL(grad_at(Yp, gp));
        TR_HIP(lincomb(c, 1.0, frame, -hs, dd, Yp));
        TR_CALL(grad_at(Yp, gm));
        TR_HIP(lincomb(c, nd / (2.0 * tp->fd_step), gp, -nd / (2.0 * tp->fd_step), gm, Bd));
      }
      TR_HIP(dots(c, 3, dd, Bd, z, dd, z, z, res));
      const double dBd = res[0], zd = res[1], zz = res[2];
      const double d2 = nd * nd;
      // roots of |z + t d|^2 = radius^2
      const double bq = 2.0 * zd, cq = zz - radius * radius;
      const double disc = std::sqrt(std::fmax(bq * bq - 4.0 * d2 * cq, 0.0));
      const double tm = (-bq - disc) / (2.0 * d2), tpl = (-bq + disc) / (2.0 * d2);
      if (dBd <= 0.0) {
        TR_HIP(dots(c, 3, g, z, g, dd, z, Bz, res));
        const double gz = res[0], gd = res[1], zBz = res[2];
        TR_HIP(dots(c, 1, dd, Bz, nullptr, nullptr, nullptr, nullptr, res));
        const double dBz = res[0];
        auto model = [&](double t) { return gz + t * gd + 0.5 * (zBz + 2 * t * dBz + t * t * dBd); };
        const double t = model(tm) < model(tpl) ? tm : tpl;
        TR_HIP(lincomb(c, 1.0, z, t, dd, z));
        TR_HIP(lincomb(c, 1.0, Bz, t, Bd, Bz));
        code = TRSTMI_CG_NEGATIVE_CURVATURE;
        break;
      }
      const double alpha = rr / dBd;
      // |z + alpha d| >= radius: stop on the boundary along d
      const double zn2 = zz + 2.0 * alpha * zd + alpha * alpha * d2;
      if (std::sqrt(zn2) >= radius) {
        TR_HIP(lincomb(c, 1.0, z, tpl, dd, z));
        TR_HIP(lincomb(c, 1.0, Bz, tpl, Bd, Bz));
        code = TRSTMI_CG_BOUNDARY;
        break;
      }
      TR_HIP(lincomb(c, 1.0, z, alpha, dd, z));
      TR_HIP(lincomb(c, 1.0, r, alpha, Bd, r));
      TR_HIP(lincomb(c, 1.0, Bz, alpha, Bd, Bz));
      TR_HIP(dots(c, 1, r, r, nullptr, nullptr, nullptr, nullptr, res));
      const double rr_new = res[0];
      if (std::sqrt(rr_new) < tp->cg_tol) {
        code = TRSTMI_CG_SMALL_RESIDUAL;
        break;
      }
      const double beta = rr_new / rr;
      TR_HIP(lincomb(c, -1.0, r, beta, dd, dd));
      rr = rr_new;
    }
  }
  rep->cg_iters = iters;
  rep->cg_exit = code;

  // ratio test and radius rule
  TR_HIP(dots(c, 3, z, z, g, z, z, Bz, res));
  const double snorm = std::sqrt(res[0]);
  const double pred = -(res[1] + 0.5 * res[2]);
  rep->step_norm = snorm;
  if (snorm == 0.0 || !(pred > 0.0)) return TRSTMI_OK;  // no step; radius / 4
  TR_HIP(lincomb(c, 1.0, frame, 1.0, z, Yp));
  TR_CALL(trstmi_lse(n, d, Yp, tp->delta, 1, c.out2, c.lws, c.lws_bytes, stream));
  TR_HIP(hipMemcpyAsync(h2, c.out2, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  TR_HIP(hipStreamSynchronize(stream));
  const double f1 = h2[1];
  const double rho = (f0 - f1) / pred;
  rep->f_new = f1;
  rep->rho = rho;
  double nr = radius;
  if (rho < 0.25) nr = radius / 4;
  else if (rho > 0.75 && snorm >= radius * (1 - 1e-12)) nr = std::fmin(2 * radius, tp->radius_max);
  rep->new_radius = nr;
  rep->accepted = rho > tp->eta ? 1 : 0;
  if (rep->accepted) TR_HIP(lincomb(c, 1.0, Yp, 0.0, nullptr, frame));
  return TRSTMI_OK;
#undef TR_HIP
#undef TR_CALL
}

}  // namespace trstmi
