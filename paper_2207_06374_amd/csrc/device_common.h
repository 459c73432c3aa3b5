// Device-side building blocks shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trstmi {

typedef double v4f64 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kFlagAccepted = 1;
constexpr int kFlagDone = 2;
constexpr int kFlagNearTie = 4;
constexpr int kFlagNoValid = 8;

// Bit pattern of +inf; a stored maximum at or above it (as an unsigned
// integer) is +inf or NaN, i.e. an invalid candidate.
constexpr uint64_t kInfBits64 = 0x7FF0000000000000ull;
constexpr uint32_t kInfBits32 = 0x7F800000u;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds on a 4-word
// counter, 2-word key bumped by the Weyl constants between rounds.
// One 32x32->64 multiply per product (v_mad_u64_u32) gives both halves, and
// each three-way xor is one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// The same generator for key words that are uniform across the wavefront.
// The round keys are bumped in scalar registers inside every round: left to
// itself the compiler precomputes all twenty of them once per kernel, and in
// a kernel with many live scalars they spill to vector lanes and are read
// back with one vector instruction each.  The empty asm hides the bumped key
// from that hoisting; it emits no instruction.
__device__ __forceinline__ u32x4 philox4x32_10_uniform_key(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    asm volatile("" : "+s"(k0), "+s"(k1));
  }
  return c;
}

// Word -> uniform in (0, 1): (w + 1/2) 2^-32, exact in FP64.
__device__ __forceinline__ double word_to_unit(uint32_t w) {
  return ((double)w + 0.5) * 0x1p-32;
}

// ---------------------------------------------------------------------------
// FP64 elementary functions for the uniforms of word_to_unit, u in
// [2^-33, 1 - 2^-33].  Written for this argument range only (no special
// cases), each within a few ulp; the series are Taylor series truncated where
// the first omitted term is below 2^-56 of the result.
// ---------------------------------------------------------------------------

// Reciprocal of d > 0: hardware estimate, two Newton steps, then the quotient
// n / d with one residual correction.
__device__ __forceinline__ double div_pos(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
}

// ln x for a positive normal x (used to fill the log table below).
// x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) with
// s = (m - 1) / (m + 1), |s| <= 0.1716, so s^2 <= 0.0295 and the odd series
// 2 (s + s^3/3 + ... + s^19/19) leaves < 2^-57; e ln 2 uses a two-part ln 2
// whose leading part times e is exact.
__device__ __forceinline__ double log_pos(double u) {
  double m = __builtin_amdgcn_frexp_mant(u);  // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(u);
  if (m < 0.7071067811865476) {
    m += m;
    e -= 1;
  }
  const double s = div_pos(m - 1.0, m + 1.0);
  const double z = s * s;
  double p = 2.0 / 19;
  p = fma(p, z, 2.0 / 17);
  p = fma(p, z, 2.0 / 15);
  p = fma(p, z, 2.0 / 13);
  p = fma(p, z, 2.0 / 11);
  p = fma(p, z, 2.0 / 9);
  p = fma(p, z, 2.0 / 7);
  p = fma(p, z, 2.0 / 5);
  p = fma(p, z, 2.0 / 3);
  const double lnm = fma(s, z * p, s + s);
  const double ln2_hi = 0x1.62e42feep-1;           // ln 2 to 32 bits
  const double ln2_lo = 0x1.a39ef35793c76p-33;     // ln 2 - ln2_hi
  const double fe = (double)e;
  return fma(fe, ln2_hi, fma(fe, ln2_lo, lnm));
}

// sqrt(a) for a > 0 in the normal range: hardware 1/sqrt estimate, one
// coupled Newton (Goldschmidt) step, one residual correction.
__device__ __forceinline__ double sqrt_pos(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, a), h, g);
}

// 1/sqrt(x) for a positive normal x: hardware estimate, one coupled Newton
// (Goldschmidt) step on g ~ sqrt(x) and h ~ 1/(2 sqrt(x)), then one more on
// h.  Zero, infinite and NaN x give NaN (0 inf or inf 0 in g).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  h = fma(h, r, h);
  return h + h;
}

// One FP64 value from the lane selected by a DPP row permute (dpp_ctrl).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum over each aligned group of G consecutive lanes (G a power of two <= 64),
// left in every lane of the group with the same bits: quad swaps, half-row
// and row mirrors inside a 16-lane row, then xor-shuffles across rows.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// (sin 2 pi u, cos 2 pi u).  j = rint(4u) quarter turns and t = u - j/4 in
// [-1/8, 1/8] are exact; x = 2 pi t, |x| <= pi/4, sin x through x^17 and
// cos x through x^16; the quarter turns rotate the pair.
__device__ __forceinline__ void sincos_2pi(double u, double& sn, double& cs) {
  const double j = rint(4.0 * u);
  const double t = fma(j, -0.25, u);
  const double x = t * 6.283185307179586;  // 2 pi
  const double z = x * x;
  double ps = 1.0 / 355687428096000.0;                  // 1/17!
  ps = fma(ps, z, -1.0 / 1307674368000.0);              // 1/15!
  ps = fma(ps, z, 1.0 / 6227020800.0);                  // 1/13!
  ps = fma(ps, z, -1.0 / 39916800.0);                   // 1/11!
  ps = fma(ps, z, 1.0 / 362880.0);                      // 1/9!
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  const double sx = fma(x * z, ps, x);
  double pc = 1.0 / 20922789888000.0;                   // 1/16!
  pc = fma(pc, z, -1.0 / 87178291200.0);                // 1/14!
  pc = fma(pc, z, 1.0 / 479001600.0);                   // 1/12!
  pc = fma(pc, z, -1.0 / 3628800.0);                    // 1/10!
  pc = fma(pc, z, 1.0 / 40320.0);
  pc = fma(pc, z, -1.0 / 720.0);
  pc = fma(pc, z, 1.0 / 24.0);
  pc = fma(pc, z, -0.5);
  const double cx = fma(z, pc, 1.0);
  const int q = (int)j & 3;
  const double a = (q & 1) ? cx : sx;
  const double b = (q & 1) ? sx : cx;
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

// Tables of the Gaussian draws, filled into LDS by every kernel that draws
// (the same function fills them everywhere).
//  sc[i] = (cos, sin)(2 pi i / 256), i = 0..255.
//  lg[i] = (r_i, ln r_i) for the mantissa bin m in [(256 + i)/512,
//          (257 + i)/512): r_i is 1/c_i (c_i the bin centre) rounded to a
//          multiple of 2^-12, except r_255 = 1 so that the bin just below 1
//          reduces exactly; |m r_i - 1| <= 2^-9 + 2^-13 in every bin.
constexpr int kSinCosTab = 256;
constexpr int kLogTab = 256;

struct GaussTab {
  double2 sc[kSinCosTab];
  double2 lg[kLogTab];
};

__device__ __forceinline__ void fill_gauss_tab(GaussTab* tab) {
  for (int i = threadIdx.x; i < kSinCosTab; i += blockDim.x) {
    double sn, cs;
    sincos_2pi(i * (1.0 / kSinCosTab), sn, cs);
    tab->sc[i] = make_double2(cs, sn);
  }
  for (int i = threadIdx.x; i < kLogTab; i += blockDim.x) {
    double r = 1.0;
    if (i < kLogTab - 1) r = rint(0x1p12 * 512.0 / (256.5 + i)) * 0x1p-12;
    tab->lg[i] = make_double2(r, log_pos(r));
  }
}

// (sin, cos)(2 pi u) for u = (w + 1/2) 2^-32: the top 8 bits of w select the
// table angle a = 2 pi i / 256, the rest give b = 2 pi ((w mod 2^24) + 1/2)
// 2^-32 in (0, 2 pi / 256), exactly reduced; sin b through b^7 and 1 - cos b
// through b^8 (first omitted terms below 2^-60 of the result), then the
// angle-sum rotation.
__device__ __forceinline__ void sincos_2pi_word(uint32_t w, const double2* tab, double& sn, double& cs) {
  const double2 t = tab[w >> 24];
  const double b = ((double)(w & 0xFFFFFFu) + 0.5) * (6.283185307179586 * 0x1p-32);  // exact power-of-two scaling
  const double z = b * b;
  const double sb = fma(b * z, fma(z, fma(z, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), b);
  const double cm = z * fma(z, fma(z, fma(z, -1.0 / 40320.0, 1.0 / 720.0), -1.0 / 24.0), 0.5);
  cs = fma(-t.y, sb, fma(-t.x, cm, t.x));
  sn = fma(t.x, sb, fma(-t.y, cm, t.y));
}

// -ln u for u = (w + 1/2) 2^-32 (Tang's table-driven reduction): u = m 2^e
// with m in [1/2, 1) (so e <= 0 and ln m <= 0: no term cancels another);
// eight mantissa bits pick the bin, t = m r_i - 1 (one rounding, exact in
// the last bin where r = 1) and ln m = ln(1 + t) - ln r_i, with ln(1 + t)
// through t^6 (first omitted term below 2^-56 of it for |t| <= 2^-8.9).
__device__ __forceinline__ double neg_log_word(uint32_t w, const double2* lg) {
  const double v = (double)w + 0.5;  // u 2^32: same mantissa as u, exponent larger by 32
  const double m = __builtin_amdgcn_frexp_mant(v);
  const int e = __builtin_amdgcn_frexp_exp(v) - 32;
  const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(m) >> 32);
  const double2 T = lg[(hi >> 12) & 0xFFu];
  const double t = fma(m, T.x, -1.0);
  double q = fma(t, -1.0 / 6.0, 1.0 / 5.0);
  q = fma(q, t, -0.25);
  q = fma(q, t, 1.0 / 3.0);
  q = fma(q, t, -0.5);
  const double lp = fma(t * t, q, t);               // ln(1 + t)
  const double ln2_hi = 0x1.62e42feep-1;            // ln 2 to 32 bits
  const double ln2_lo = 0x1.a39ef35793c76p-33;      // ln 2 - ln2_hi
  const double fe = (double)e;
  return fma(-fe, ln2_hi, fma(-fe, ln2_lo, T.y - lp));
}

// One complex CN(0, 1) draw in polar form (Box-Muller 1958, each part of
// variance 1/2): modulus rho = sqrt(-ln u0) = sqrt(-2 ln u0) sqrt(1/2) and
// angle 2 pi u1; the draw is rho (cos, sin).  Callers scale rho first when
// they add a multiple of the draw.
__device__ __forceinline__ void cn_polar(uint32_t w0, uint32_t w1, const GaussTab& tab, double& rho, double& cs,
                                         double& sn) {
  rho = sqrt_pos(neg_log_word(w0, tab.lg));
  sincos_2pi_word(w1, tab.sc, sn, cs);
}

// ---------------------------------------------------------------------------
// FP64 -> bfloat16, round to nearest, ties to even, computed directly from
// the double (no intermediate float rounding).  A bfloat16 keeps 8
// significant bits: with |x| = m 2^e, 1/2 <= m < 1, the result is an integer
// multiple of 2^(e-8) (spacing fixed at 2^-133 below the normal range).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x) {
  if (x != x) return 0x7FC0;
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  int e = (int)((bits >> 52) & 0x7FF) - 1022;  // frexp exponent for normal x (0 or subnormal -> tiny)
  if (e < -125) e = -125;
  const double up = __longlong_as_double((int64_t)(1023 + 8 - e) << 52);    // 2^(8-e)
  const double down = __longlong_as_double((int64_t)(1023 - 8 + e) << 52);  // 2^(e-8)
  const double r = rint(x * up) * down;  // exact: representable in bfloat16
  const float f = (float)r;               // exact
  return (uint16_t)(__float_as_uint(f) >> 16);
}

// Two doubles -> two bfloat16 (round to nearest even, as if rounded directly
// from the double), packed with x0 in the low half.  Rounding to FP32 first
// and then to bfloat16 gives the same result unless the FP32 value lands
// exactly on a bfloat16 midpoint (x may lie on either side of it) or is an
// FP32 subnormal; those rare lanes use f64_to_bf16_rne.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// A float f is unsafe for the second rounding when it is a bfloat16 midpoint
// (low 16 bits exactly 0x8000) or an FP32 subnormal (class mask 0x90: the
// negative and positive subnormal classes of v_cmp_class_f32).
__device__ __forceinline__ bool bf16_via_f32_unsafe(float f) {
  return (unsigned)((__float_as_uint(f) & 0xFFFFu) == 0x8000u) | (unsigned)__builtin_amdgcn_classf(f, 0x90);
}

__device__ __forceinline__ uint32_t bf16x2_rne(double x0, double x1) {
  const f32x2 f = {(float)x0, (float)x1};
  const bool slow = (unsigned)bf16_via_f32_unsafe(f[0]) | (unsigned)bf16_via_f32_unsafe(f[1]);
  if (__ballot(slow) && slow)
    return (uint32_t)f64_to_bf16_rne(x0) | ((uint32_t)f64_to_bf16_rne(x1) << 16);
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

// ---------------------------------------------------------------------------
// Upper-triangle tile enumeration: tile t in [0, nt(nt+1)/2) <-> (bi, bj),
// bi <= bj, row by row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_decode(int t, int nt, int& bi, int& bj) {
  int row = 0;
  int rem = t;
  while (rem >= nt - row) {
    rem -= nt - row;
    ++row;
  }
  bi = row;
  bj = row + rem;
}

__device__ __forceinline__ int tile_linear(int bi, int bj, int nt) {
  // number of tiles in rows 0..bi-1 plus offset in row bi
  return bi * nt - (bi * (bi - 1)) / 2 + (bj - bi);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Max over the 64 lanes with DPP row permutes (no LDS traffic): quad swaps,
// half-row and row mirrors leave every lane of a 16-lane row with the row
// maximum; the four row maxima are combined through scalar registers.
__device__ __forceinline__ uint32_t wave_max_u32_dpp(uint32_t v) {
  uint32_t o;
  o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  v = o > v ? o : v;
  o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  v = o > v ? o : v;
  o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v = o > v ? o : v;
  o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v = o > v ? o : v;
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
  const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
  const uint32_t a = r0 > r1 ? r0 : r1;
  const uint32_t b = r2 > r3 ? r2 : r3;
  return a > b ? a : b;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace trstmi
