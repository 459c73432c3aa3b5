// Candidate generation: trust-region perturbation and column renormalisation.
//
// For candidate c at step t:  Y = Phi + (radius / sqrt(d)) Z,  Z i.i.d. CN(0,1)
// from Philox4x32-10, then every column is divided by its Euclidean norm (the
// unconstrained formulation of section IV divides each column by its norm).
// The same kernel draws the random start (Alg. 2 step 1: y = z, tag 1),
// normalises a caller frame (y = Phi), and commits an accepted candidate in
// place (regenerating it from the same counters).
//
// Work split: a column of d complex entries is ceil(d/2) Philox blocks (one
// block = 4 words = 2 complex entries).  LPC lanes (a power of two <= 64)
// share a column, each holding kMaxQ = 4 blocks in registers; the norm is
// reduced across the LPC lanes with DPP row permutes (xor-shuffles across
// rows), so a column never leaves the wavefront.  Every output kind uses the
// same split for a given d, so a candidate's FP64 bits are the same in every
// launch that writes it and its screen copies are their roundings.  Loads
// and stores are 16-byte and consecutive lanes touch consecutive entries of
// a column.

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxQ = 4;  // blocks per lane: d <= 2 * 64 * kMaxQ = 512 (Q below is the compiled bound)

template <int OUT>
__device__ __forceinline__ void store_pair(const PerturbArgs& a, size_t slot, int64_t col, int i,
                                           double re0, double im0, double re1, double im1, bool two) {
  const size_t off = slot * (size_t)a.out_slot_stride + (size_t)col * a.out_ld + 2 * (size_t)i;
  if constexpr (OUT == kOutF64) {
    double* o = (double*)a.out + off;
    *(double2*)o = make_double2(re0, im0);
    if (two) *(double2*)(o + 2) = make_double2(re1, im1);
  } else if constexpr (OUT == kOutF32) {
    float* o = (float*)a.out + off;
    if (two) {
      *(float4*)o = make_float4((float)re0, (float)im0, (float)re1, (float)im1);
    } else {
      *(float2*)o = make_float2((float)re0, (float)im0);
    }
  } else {
    uint16_t* o = (uint16_t*)a.out + off;
    const uint32_t w0 = bf16x2_rne(re0, im0);
    const uint32_t w1 = bf16x2_rne(re1, im1);
    if (two) {
      *(uint2*)o = make_uint2(w0, w1);
    } else {
      *(uint32_t*)o = w0;
    }
  }
}

template <int OUT>
__device__ __forceinline__ void store_zero_pad(const PerturbArgs& a, size_t slot, int64_t col) {
  // elements [2d, out_ld) of the column
  const size_t off = slot * (size_t)a.out_slot_stride + (size_t)col * a.out_ld;
  for (int k = 2 * a.d; k < a.out_ld; ++k) {
    if constexpr (OUT == kOutF64) {
      ((double*)a.out)[off + k] = 0.0;
    } else if constexpr (OUT == kOutF32) {
      ((float*)a.out)[off + k] = 0.0f;
    } else {
      ((uint16_t*)a.out)[off + k] = 0;
    }
  }
}

// DRAW: compiled for the candidate form only (base frame present, Philox
// draws, no explicit perturbation); otherwise the three fields decide.
// FULL (with DRAW): d is even and the LPC lanes of a column hold exactly its
// ceil(d/2) blocks (LPC * Q == d / 2), so no block is partial or missing;
// lanes of columns past n compute on the last column and store nothing.
template <int LPC, int Q, int OUT, bool DRAW, bool FULL>
__device__ __forceinline__ void perturb_body(const PerturbArgs& a, int bx, int gx, int slot) {
  static_assert(DRAW || !FULL, "the full split is compiled for the candidate form only");
  if (a.gate && ((*a.gate & a.gate_mask) != a.gate_want)) return;
  const double* const base = a.base;
  const bool has_base = DRAW || a.base != nullptr;
  const bool have_z = DRAW || a.have_z != 0;
  const double* const z_explicit = DRAW ? nullptr : a.z_explicit;
  __shared__ GaussTab gtab_s;
  GaussTab* const gtab = &gtab_s;
  fill_gauss_tab(gtab);
  __syncthreads();
  if (a.zero_max && bx == 0 && threadIdx.x == 0) a.zero_max[slot] = 0;

  const int c = a.cand_idx ? a.cand_idx[slot] : a.c0 + slot;
  const int64_t t = a.tstep ? *a.tstep : a.t_const;
  const int d = a.d;
  const int nb = FULL ? LPC * Q : (d + 1) >> 1;
  double s = 0.0;
  if (has_base && have_z) s = *a.radius / sqrt((double)d);

  constexpr int kColsPerWave = 64 / LPC;
  constexpr int kColsPerIter = (kThreads / 64) * kColsPerWave;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lq = lane & (LPC - 1);

  for (int64_t col0 = (int64_t)bx * kColsPerIter; col0 < a.n; col0 += (int64_t)gx * kColsPerIter) {
    const int64_t col = col0 + wave * kColsPerWave + lane / LPC;
    const bool active = col < a.n;  // whole LPC groups share `active`
    const int64_t colr = FULL ? (active ? col : a.n - 1) : col;  // column read
    double y[Q][4];
    double nrm2 = 0.0;
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
      const int q = lq + qi * LPC;
      if constexpr (!FULL) {
        y[qi][0] = y[qi][1] = y[qi][2] = y[qi][3] = 0.0;
        if (!active || q >= nb) continue;
      }
      const int i0 = 2 * q;
      const bool two = FULL || (i0 + 1) < d;
      double p[4] = {0.0, 0.0, 0.0, 0.0};
      if (has_base) {
        const double* bp = base + 2 * ((size_t)colr * d + i0);
        const double2 p0 = *(const double2*)bp;
        p[0] = p0.x;
        p[1] = p0.y;
        if (two) {
          const double2 p1 = *(const double2*)(bp + 2);
          p[2] = p1.x;
          p[3] = p1.y;
        }
      }
      if (has_base && !have_z) {
#pragma unroll
        for (int e = 0; e < 4; ++e) y[qi][e] = p[e];
      } else if (z_explicit) {
        const double* zp = z_explicit + 2 * (((size_t)c * a.n + col) * d + i0);
        double z[4] = {zp[0], zp[1], 0.0, 0.0};
        if (two) {
          z[2] = zp[2];
          z[3] = zp[3];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) y[qi][e] = has_base ? p[e] + s * z[e] : z[e];
      } else {
        // two complex draws; y = Phi + s z with the step scale folded into
        // the modulus of each draw
        const u32x4 ctr = {(uint32_t)(col * nb + q), (uint32_t)c, (uint32_t)t, a.tag};
        const u32x4 w = philox4x32_10_uniform_key(ctr, a.seed, a.stream_id);
        double r0, c0, s0, r1, c1, s1;
        cn_polar(w.x, w.y, *gtab, r0, c0, s0);
        cn_polar(w.z, w.w, *gtab, r1, c1, s1);
        if (has_base) {
          r0 *= s;
          r1 *= s;
          y[qi][0] = fma(r0, c0, p[0]);
          y[qi][1] = fma(r0, s0, p[1]);
          y[qi][2] = fma(r1, c1, p[2]);
          y[qi][3] = fma(r1, s1, p[3]);
        } else {
          y[qi][0] = r0 * c0;
          y[qi][1] = r0 * s0;
          y[qi][2] = r1 * c1;
          y[qi][3] = r1 * s1;
        }
      }
      if (!two) {
        y[qi][2] = 0.0;
        y[qi][3] = 0.0;
      }
      nrm2 = fma(y[qi][3], y[qi][3], fma(y[qi][2], y[qi][2], fma(y[qi][1], y[qi][1], fma(y[qi][0], y[qi][0], nrm2))));
    }
    nrm2 = group_sum<LPC>(nrm2);
    if (!active) continue;
    // 1 / ||y||; NaN for a zero or non-finite norm, which makes the column
    // (and so the candidate) invalid
    const double inv = rsqrt_pos(nrm2);
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
      const int q = lq + qi * LPC;
      if (!FULL && q >= nb) continue;
      const int i0 = 2 * q;
      const bool two = FULL || (i0 + 1) < d;
      double o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = y[qi][e] * inv;
      store_pair<OUT>(a, slot, col, i0, o[0], o[1], o[2], o[3], two);
      if (q == nb - 1 && a.out_ld > 2 * d) store_zero_pad<OUT>(a, slot, col);
    }
  }
}

template <int LPC, int Q, int OUT, bool DRAW, bool FULL>
__global__ __launch_bounds__(kThreads) void k_perturb(PerturbArgs a) {
  perturb_body<LPC, Q, OUT, DRAW, FULL>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

// The same for a group of searches: search blockIdx.z of the table.
template <int LPC, int Q, int OUT, bool DRAW, bool FULL>
__global__ __launch_bounds__(kThreads) void k_perturb_tab(TabRef t) {
  const PerturbArgs a = *(const PerturbArgs*)(t.base + (size_t)t.list[blockIdx.z] * t.stride);
  perturb_body<LPC, Q, OUT, DRAW, FULL>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

// Commit by copy.  Every output kind of a candidate comes from the same
// column split for a given d, so the FP64 columns written earlier in the step
// have the bits the regeneration would write; copying them replaces drawing
// the accepted candidate again.
__global__ __launch_bounds__(kThreads) void k_commit_copy(CommitCopyArgs a) {
  if (a.dec->commit != 1) return;
  const int best = a.dec->best;
  int slot = best;
  if (a.slot_cand) {
    slot = -1;
    for (int s = 0; s < a.k; ++s)
      if (a.slot_cand[s] == best) slot = s;
    if (slot < 0) return;  // the selection only picks listed candidates
  }
  const double* src = a.src + (size_t)slot * a.src_slot_stride;
  const int h = a.d;  // double2 per column
  const int64_t total = a.n * h;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    const int64_t col = e / h;
    const int m = (int)(e - col * h);
    ((double2*)(a.frame + (size_t)col * 2 * a.d))[m] = ((const double2*)(src + (size_t)col * a.src_ld))[m];
  }
}

// FP64 frame -> FP32 copy with zero padding (no renormalisation).
__global__ __launch_bounds__(kThreads) void k_convert_f32(const double* frame, int64_t n, int d, float* out,
                                                          int out_ld, uint64_t* zero_max) {
  if (zero_max && blockIdx.x == 0 && threadIdx.x == 0) zero_max[0] = 0;
  const int64_t total = n * out_ld;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    const int64_t col = e / out_ld;
    const int k = (int)(e - col * out_ld);
    out[e] = k < 2 * d ? (float)frame[2 * col * d + k] : 0.0f;
  }
}

// x[i] -> bfloat16 bits, the rounding of the BF16 screen copies (pairs of
// entries; an odd count pads the last pair with 0).
__global__ __launch_bounds__(kThreads) void k_round_bf16(const double* x, int64_t count, uint16_t* out) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; 2 * p < count;
       p += (int64_t)gridDim.x * kThreads) {
    const bool two = 2 * p + 1 < count;
    const uint32_t w = bf16x2_rne(x[2 * p], two ? x[2 * p + 1] : 0.0);
    out[2 * p] = (uint16_t)w;
    if (two) out[2 * p + 1] = (uint16_t)(w >> 16);
  }
}

// A group launch (tab != null) covers tab->count searches with the largest
// n among them (a.n) and the same d.
template <int LPC, int Q, int OUT, bool DRAW = false, bool FULL = false>
hipError_t launch_lpc(const PerturbArgs& a, int slots, hipStream_t s, const TabRef* tab) {
  constexpr int kColsPerIter = (kThreads / 64) * (64 / LPC);
  int64_t groups = (a.n + kColsPerIter - 1) / kColsPerIter;
  // about 2048 blocks across all slots (8 per CU, two resident rounds at 4
  // waves per SIMD), each looping over column groups, so that the per-block
  // table fill is spread over more entries
  const int64_t total = (int64_t)slots * (tab ? tab->count : 1);
  int64_t want = (2048 + total - 1) / total;
  if (want < 1) want = 1;
  const int gx = (int)(groups < want ? groups : want);
  if (tab)
    hipLaunchKernelGGL((k_perturb_tab<LPC, Q, OUT, DRAW, FULL>), dim3(gx, slots, tab->count), dim3(kThreads), 0, s,
                       *tab);
  else
    hipLaunchKernelGGL((k_perturb<LPC, Q, OUT, DRAW, FULL>), dim3(gx, slots), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// 4 blocks per lane, so the column's inverse norm is shared by more entries.
// Every output kind of a candidate uses this same split, so a candidate's
// FP64 bits are the same in every launch that writes it and its BF16 / FP32
// screen copies are the roundings of those FP64 values.
template <int OUT, bool DRAW>
hipError_t launch_q4(const PerturbArgs& a, int nb, int slots, hipStream_t s, const TabRef* tab) {
  if (DRAW && a.d % 2 == 0) {
    // full splits: d = 8, 16, 32, 64, 128, 256, 512
    switch (nb) {
      case 4: return launch_lpc<1, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 8: return launch_lpc<2, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 16: return launch_lpc<4, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 32: return launch_lpc<8, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 64: return launch_lpc<16, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 128: return launch_lpc<32, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      case 256: return launch_lpc<64, 4, OUT, DRAW, DRAW>(a, slots, s, tab);
      default: break;
    }
  }
  if (nb <= 4) return launch_lpc<1, 4, OUT, DRAW>(a, slots, s, tab);
  if (nb <= 8) return launch_lpc<2, 4, OUT, DRAW>(a, slots, s, tab);
  if (nb <= 16) return launch_lpc<4, 4, OUT, DRAW>(a, slots, s, tab);
  if (nb <= 32) return launch_lpc<8, 4, OUT, DRAW>(a, slots, s, tab);
  if (nb <= 64) return launch_lpc<16, 4, OUT, DRAW>(a, slots, s, tab);
  if (nb <= 128) return launch_lpc<32, 4, OUT, DRAW>(a, slots, s, tab);
  return launch_lpc<64, kMaxQ, OUT, DRAW>(a, slots, s, tab);
}

}  // namespace

namespace {
hipError_t launch_perturb_any(const PerturbArgs& a, int slots, hipStream_t s, const TabRef* tab) {
  const int nb = (a.d + 1) / 2;
  const bool draw = a.base && a.have_z && !a.z_explicit;
  switch (a.out_kind) {
    case kOutF64:
      return draw ? launch_q4<kOutF64, true>(a, nb, slots, s, tab) : launch_q4<kOutF64, false>(a, nb, slots, s, tab);
    case kOutF32:
      return draw ? launch_q4<kOutF32, true>(a, nb, slots, s, tab) : launch_q4<kOutF32, false>(a, nb, slots, s, tab);
    default:
      return draw ? launch_q4<kOutBF16, true>(a, nb, slots, s, tab)
                  : launch_q4<kOutBF16, false>(a, nb, slots, s, tab);
  }
}
}  // namespace

hipError_t launch_commit_copy(const CommitCopyArgs& a, hipStream_t s) {
  const int64_t total = a.n * a.d;
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_commit_copy, dim3((int)(g > 0 ? g : 1)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_perturb(const PerturbArgs& a, int slots, hipStream_t s) {
  return launch_perturb_any(a, slots, s, nullptr);
}

hipError_t launch_perturb_tab(const TabRef& t, const PerturbArgs& shape, int slots, hipStream_t s) {
  return launch_perturb_any(shape, slots, s, &t);
}

hipError_t launch_convert_f32(const double* frame, int64_t n, int32_t d, float* out, int32_t out_ld,
                              uint64_t* zero_max, hipStream_t s) {
  const int64_t total = n * out_ld;
  int64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_convert_f32, dim3((int)blocks), dim3(kThreads), 0, s, frame, n, d, out, out_ld, zero_max);
  return hipGetLastError();
}

hipError_t launch_round_bf16(const double* x, int64_t count, uint16_t* out, hipStream_t s) {
  int64_t blocks = (count / 2 + kThreads) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_round_bf16, dim3((int)blocks), dim3(kThreads), 0, s, x, count, out);
  return hipGetLastError();
}

}  // namespace trstmi
