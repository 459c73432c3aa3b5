// BF16-screen Gram + fused max of |G_jk|^2 over j < k, on
// v_mfma_f32_16x16x32_bf16 (gfx950), FP32 accumulation.
//
// Inputs are the FP64 unit candidates rounded to bfloat16 (nearest-even) by
// the perturb kernel, column stride ldk = 2d rounded up to a multiple of 32,
// zero padded.  A complex column is the real 2d-vector u = (a_0, b_0, ...);
// with v = (b_0, -a_0, b_1, -a_1, ...):
//   Re <phi_j, phi_k> = u_j . u_k,   Im <phi_j, phi_k> = -(v_j . u_k),
// so both parts share the B operand u_k, and v_j is formed in registers from
// the A rows (one funnel shift and one sign flip per 32-bit (re, im) pair).
//
// Wide kernel (2d <= 128): a 256-thread block owns a row segment: two tile
// rows (256 frame columns) against up to kSegK consecutive 128-column tiles
// of the strict upper triangle.  Each wave keeps 64 rows (u and v for the
// whole K) in VGPRs for the whole segment, so the A side is read and
// converted once per segment, and every B column staged in LDS feeds 256
// rows.  The 128 B columns of one tile sit in LDS (16 bytes of padding per
// column: 16 lanes reading 16 columns at one k offset hit distinct banks);
// the next tile's columns are prefetched into registers while the current
// tile is computed and stored into a second LDS buffer, so each tile costs
// one barrier.  Per tile, the wave sweeps 8 column blocks of 16 columns:
// 4 x 2 x K/32 MFMAs per block, row block by row block (the 2 K/32 products
// of one 16-row block back to back).  The accumulators of a row block are
// folded (|G|^2 = Re^2 + Im^2, running max on the float bit patterns; the
// integer max keeps NaN, which marks an invalid candidate, above every
// finite value) under the products of the row block two places later, and
// scheduling groups spread that epilogue and the LDS reads of the next
// column block over the MFMAs.  Diagonal tiles skip the column blocks wholly
// below the wave's rows and keep j > i; rows/columns past N are zero and
// contribute 0.
//
// Narrow kernel (any 2d <= 256; the form for 128 < 2d): one tile row (128
// frame columns) per segment, 32 rows per wave, the same pipelining with two
// accumulator sets.  For 2d > 160 a lean variant without the register
// prefetch of the next tile and with fragments read per column block keeps
// two blocks per CU (about 244 registers per lane instead of 300).
//
// Blocks are mapped XCD-aware: the dispatcher deals consecutive block ids to
// the 8 XCDs in turn, so block b runs on XCD b mod 8; all segments of
// candidate c go to blocks with b mod 8 = c mod 8, which keeps a candidate's
// columns in one XCD's L2.
//
// Each wave keeps its maximum for every tile in a lane and writes them once
// per segment (they prune the FP64 recheck); the block updates the
// candidate's running maximum with one atomic.  The FP64 recheck of the best
// screened candidates (k_recheck_pairs) screens again the tiles that can hold
// the exact maximum, one wave per 32 x 32 sub-block, and evaluates only the
// pairs that can attain it in FP64.
//
// Fallback kernel (2d > 256, coherence entry point only): 128 x 128 tiles, K
// looped in LDS chunks of 128.

#include <mutex>
#include <vector>

#include "device_common.h"
#include "launch.h"

namespace trstmi {

namespace {

constexpr int T = kTileBF16;

__device__ __forceinline__ u32x4 swap_negate(u32x4 u) {
  u32x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = __builtin_amdgcn_alignbit(u[e], u[e], 16) ^ 0x80000000u;
  return v;
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t bc = b > c ? b : c;  // folded into v_max3_u32
  return a > bc ? a : bc;
}

__device__ __forceinline__ bool xcd_slot(const GramArgs& a, int tiles, int& slot, int& tile) {
  const int b = blockIdx.x;
  const int local = b >> 3;
  slot = (local / tiles) * 8 + (b & 7);
  tile = local % tiles;
  return slot < a.slots;
}

// The 32 rows of wave w (u for Re, v for -Im, whole K) in registers.
template <int KS>
struct ARows {
  u32x4 u[2][KS];
  u32x4 v[2][KS];
};

template <int KS>
__device__ __forceinline__ void load_rows(const uint16_t* base, int ldk, int n, int bi, ARows<KS>& A) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const int row = bi * T + w * 32 + rb * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      u32x4 u = {0u, 0u, 0u, 0u};
      if (row < n) u = *(const u32x4*)(base + (size_t)row * ldk + ks * 32 + 8 * (lane >> 4));
      A.u[rb][ks] = u;
      A.v[rb][ks] = swap_negate(u);
    }
  }
}

// The B columns of tile column block bj: 128 columns x 4 KS chunks of 16 bytes,
// 2 KS chunks per thread, fetched into registers and stored into LDS.  Chunk
// idx = it * 256 + thread is column idx / (4 KS), part idx % (4 KS); since the
// column stride is 32 KS elements, the tile's columns are contiguous in
// memory and chunk idx sits at element 8 idx of the tile.
template <int KS>
__device__ __forceinline__ void fetch_cols(const uint16_t* base, int n, int bj, u32x4 pf[2 * KS]) {
  constexpr int LDK = 32 * KS;
  const uint16_t* p = base + (size_t)bj * T * LDK + 8 * threadIdx.x;
  if ((bj + 1) * T <= n) {
#pragma unroll
    for (int it = 0; it < 2 * KS; ++it) pf[it] = *(const u32x4*)(p + it * 256 * 8);
  } else {
#pragma unroll
    for (int it = 0; it < 2 * KS; ++it) {
      const int col = (it * 256 + (int)threadIdx.x) / (KS * 4);
      u32x4 v = {0u, 0u, 0u, 0u};
      if (bj * T + col < n) v = *(const u32x4*)(p + it * 256 * 8);
      pf[it] = v;
    }
  }
}

template <int KS>
__device__ __forceinline__ void store_cols(const u32x4 pf[2 * KS], uint16_t* Bs) {
  constexpr int LDL = 32 * KS + 8;
#pragma unroll
  for (int it = 0; it < 2 * KS; ++it) {
    const int idx = it * 256 + threadIdx.x;
    const int col = idx / (KS * 4);
    const int ch = idx % (KS * 4);
    *(u32x4*)&Bs[col * LDL + ch * 8] = pf[it];
  }
}

// B fragments of column block cb from LDS.
template <int KS>
__device__ __forceinline__ void read_frags(const uint16_t* Bs, int cb, u32x4 bq[KS]) {
  constexpr int LDL = 32 * KS + 8;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) bq[ks] = *(const u32x4*)&Bs[(cb * 16 + (lane & 15)) * LDL + ks * 32 + 8 * (lane >> 4)];
}

// MFMAs of one column block: Re and -Im of the 2 x (16 x 16) outputs.
template <int KS>
__device__ __forceinline__ void mma_frags(const ARows<KS>& A, const u32x4 bq[KS], v4f32 accR[2], v4f32 accI[2]) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    accR[rb] = v4f32{0.f, 0.f, 0.f, 0.f};
    accI[rb] = v4f32{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const bf16x8 b = as_bf16x8(bq[ks]);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      accR[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.u[rb][ks]), b, accR[rb], 0, 0, 0);
      accI[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.v[rb][ks]), b, accI[rb], 0, 0, 0);
    }
  }
}

template <int KS>
__device__ __forceinline__ void mma_block(const ARows<KS>& A, const uint16_t* Bs, int cb, v4f32 accR[2],
                                          v4f32 accI[2]) {
  u32x4 bq[KS];
  read_frags<KS>(Bs, cb, bq);
  mma_frags<KS>(A, bq, accR, accI);
}

// |G|^2 float bits of the outputs: m[rb * 4 + v] is tile row
// 32 w + 16 rb + 4 (lane / 16) + v, tile column 16 cb + lane % 16.
__device__ __forceinline__ void sq_mag(const v4f32 accR[2], const v4f32 accI[2], uint32_t m[8]) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float re = accR[rb][v], im = accI[rb][v];
      m[rb * 4 + v] = __float_as_uint(fmaf(re, re, im * im));
    }
}

__device__ __forceinline__ uint32_t max_of(uint32_t best, const uint32_t m[8]) {
  const uint32_t a = max3u(m[0], m[1], m[2]);
  const uint32_t b = max3u(m[3], m[4], m[5]);
  const uint32_t c = max3u(m[6], m[7], best);
  return max3u(a, b, c);
}

// Max |G|^2 bits over this wave's rows of one tile held in LDS.
template <int KS>
__device__ __forceinline__ uint32_t tile_max_wave(const ARows<KS>& A, const uint16_t* Bs, bool diag) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  uint32_t best = 0;
  uint32_t m[8];
  if (!diag) {
    // fragments of block cb + 1 are read while block cb multiplies; the
    // epilogue of block cb - 1 runs in the second half of block cb's MFMAs,
    // when those results are complete.  The scheduling groups pin this order
    // (the compiler would otherwise sink the LDS reads next to their use).
    v4f32 xR[2], xI[2], yR[2], yI[2];
    u32x4 bp[KS], bq[KS];
    read_frags<KS>(Bs, 0, bp);
    read_frags<KS>(Bs, 1, bq);
    mma_frags<KS>(A, bp, xR, xI);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cb = 1; cb < T / 16; ++cb) {
      if (cb & 1) {
        if (cb + 1 < T / 16) read_frags<KS>(Bs, cb + 1, bp);
        mma_frags<KS>(A, bq, yR, yI);
        sq_mag(xR, xI, m);
      } else {
        if (cb + 1 < T / 16) read_frags<KS>(Bs, cb + 1, bq);
        mma_frags<KS>(A, bp, xR, xI);
        sq_mag(yR, yI, m);
      }
      best = max_of(best, m);
#pragma unroll
      for (int i = 0; i < KS; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
      }
#pragma unroll
      for (int i = KS; i < 2 * KS; ++i) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
      for (int i = 2 * KS; i < 4 * KS; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // epilogue VALU
      }
      __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    sq_mag(yR, yI, m);
    return max_of(best, m);
  }
  for (int cb = 2 * w; cb < T / 16; ++cb) {
    v4f32 xR[2], xI[2];
    mma_block<KS>(A, Bs, cb, xR, xI);
    sq_mag(xR, xI, m);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = w * 32 + (q >> 2) * 16 + 4 * (lane >> 4) + (q & 3);
      const int j = cb * 16 + (lane & 15);
      if (i >= j) m[q] = 0u;
    }
    best = max_of(best, m);
  }
  return best;
}

// The same for the lean form (K >= 192): fragments read per column block
// just before its products, no register double buffering; latency is
// covered by the second wavefront on the SIMD that the saved registers allow.
template <int KS>
__device__ __forceinline__ uint32_t tile_max_wave_lean(const ARows<KS>& A, const uint16_t* Bs, bool diag) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  uint32_t best = 0;
  uint32_t m[8];
  for (int cb = diag ? 2 * w : 0; cb < T / 16; ++cb) {
    v4f32 xR[2], xI[2];
    mma_block<KS>(A, Bs, cb, xR, xI);
    sq_mag(xR, xI, m);
    if (diag) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = w * 32 + (q >> 2) * 16 + 4 * (lane >> 4) + (q & 3);
        const int j = cb * 16 + (lane & 15);
        if (i >= j) m[q] = 0u;
      }
    }
    best = max_of(best, m);
  }
  return best;
}

// Column tile bj from global memory into LDS in one pass (zero past n).
template <int KS>
__device__ __forceinline__ void copy_cols(const uint16_t* base, int n, int bj, uint16_t* Bs) {
  u32x4 pf[2 * KS];
  fetch_cols<KS>(base, n, bj, pf);
  store_cols<KS>(pf, Bs);
}

// Segment s of the row-segment enumeration: row block bi in order, each row
// block split into ceil((nt - bi) / seg) runs of at most seg column tiles.
__device__ __forceinline__ void seg_decode(int s, int nt, int seg, int& bi, int& bj0, int& bj1) {
  int r = 0;
  int rem = s;
  for (;;) {
    const int ns = (nt - r + seg - 1) / seg;
    if (rem < ns) break;
    rem -= ns;
    ++r;
  }
  bi = r;
  bj0 = r + rem * seg;
  bj1 = bj0 + seg < nt ? bj0 + seg : nt;
}

// Narrow kernel, two blocks per CU: double-buffered tiles and the register
// prefetch while the whole-K rows leave room (2d <= 160), the lean variant
// (one tile buffer, one copy pass per tile) beyond that.
template <int KS>
__device__ __forceinline__ void gram_bf16_narrow(const GramArgs& a, int b) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  const int local = b >> 3;
  const int slot = (local / a.nseg) * 8 + (b & 7);
  const int seg = local % a.nseg;
  if (slot >= a.slots) return;
  int bi, bj0, bj1;
  seg_decode(seg, a.nt, a.segk, bi, bj0, bj1);
  const int tiles = a.nt * (a.nt + 1) / 2;

  // Two B tiles while two blocks still fit in LDS: tile bj + 1 is stored
  // into the buffer tile bj - 1 used, so one barrier per tile suffices.  One
  // tile (and a barrier before the store) beyond that.
  constexpr int kBuf = T * (32 * KS + 8);
  constexpr int kNB = KS <= 4 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kNB * kBuf];
  __shared__ uint32_t red[4];
  const uint16_t* base = (const uint16_t*)a.cand + (size_t)slot * a.slot_stride;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;

  uint32_t cmax = 0;
  uint32_t tile_lane = 0;
  ARows<KS> A;
  if constexpr (KS >= 6) {
    // lean form: two blocks per CU (the registers of one block's waves fit
    // twice), each tile copied in one pass between two barriers
    copy_cols<KS>(base, a.n, bj0, Bs);
    load_rows<KS>(base, a.ldk, a.n, bi, A);
    __syncthreads();
    for (int bj = bj0; bj < bj1; ++bj) {
      const uint32_t tmax = tile_max_wave_lean<KS>(A, Bs, bj == bi);
      cmax = tmax > cmax ? tmax : cmax;
      if (a.tile_max) {
        const uint32_t wm = wave_max_u32_dpp(tmax);
        if (lane == bj - bj0) tile_lane = wm;
      }
      if (bj + 1 < bj1) {
        __syncthreads();  // every wave is done with this tile's columns
        copy_cols<KS>(base, a.n, bj + 1, Bs);
        __syncthreads();
      }
    }
  } else {
    u32x4 pf[2 * KS];
    fetch_cols<KS>(base, a.n, bj0, pf);
    load_rows<KS>(base, a.ldk, a.n, bi, A);
    store_cols<KS>(pf, Bs);
    __syncthreads();
    if (bj0 + 1 < bj1) fetch_cols<KS>(base, a.n, bj0 + 1, pf);
    for (int bj = bj0; bj < bj1; ++bj) {
      const int buf = kNB == 2 ? (bj - bj0) & 1 : 0;
      const uint32_t tmax = tile_max_wave<KS>(A, Bs + buf * kBuf, bj == bi);
      cmax = tmax > cmax ? tmax : cmax;
      if (a.tile_max) {
        // lane k keeps the wave maximum of tile bj0 + k; stored after the
        // segment, so no tile waits on a global store
        const uint32_t wm = wave_max_u32_dpp(tmax);
        if (lane == bj - bj0) tile_lane = wm;
      }
      if (bj + 1 < bj1) {
        if (kNB == 1) __syncthreads();  // every wave is done with this tile's columns
        store_cols<KS>(pf, Bs + (kNB == 2 ? buf ^ 1 : 0) * kBuf);
        __syncthreads();  // tile bj + 1 is in LDS; every wave is past tile bj
        if (bj + 2 < bj1) fetch_cols<KS>(base, a.n, bj + 2, pf);
      }
    }
  }

  if (a.tile_max && lane < bj1 - bj0)
    a.tile_max[((size_t)slot * tiles + tile_linear(bi, bj0 + lane, a.nt)) * 4 + w] = tile_lane;
  cmax = wave_max_u32_dpp(cmax);
  if (lane == 0) red[w] = cmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t mx = max3u(red[0], red[1], red[2] > red[3] ? red[2] : red[3]);
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)mx);
  }
}

// ---------------------------------------------------------------------------
// Wide kernel helpers: 64 rows per wave.
// ---------------------------------------------------------------------------
template <int KS>
struct QRows {
  u32x4 u[4][KS];
  u32x4 v[4][KS];
};

template <int KS>
__device__ __forceinline__ void load_rows_q(const uint16_t* base, int ldk, int n, int row0, QRows<KS>& A) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int row = row0 + rb * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      u32x4 u = {0u, 0u, 0u, 0u};
      if (row < n) u = *(const u32x4*)(base + (size_t)row * ldk + ks * 32 + 8 * (lane >> 4));
      A.u[rb][ks] = u;
      A.v[rb][ks] = swap_negate(u);
    }
  }
}

// |G|^2 bits of row block rb's 16 x 16 outputs folded into best.
__device__ __forceinline__ uint32_t fold_rb(uint32_t best, v4f32 R, v4f32 I) {
  uint32_t m[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) m[v] = __float_as_uint(fmaf(R[v], R[v], I[v] * I[v]));
  return max3u(max3u(m[0], m[1], m[2]), m[3], best);
}

// One column block: the epilogue of the previous block (R, I on entry) is
// folded row block by row block just before the first MFMAs that overwrite
// those accumulators, then the remaining K steps follow.
template <int KS, bool EPI>
__device__ __forceinline__ void qblock(const QRows<KS>& A, const u32x4 b[KS], v4f32 R[4], v4f32 I[4],
                                       uint32_t& best) {
  const v4f32 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    if (EPI) best = fold_rb(best, R[rb], I[rb]);
    R[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.u[rb][0]), as_bf16x8(b[0]), z, 0, 0, 0);
    I[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.v[rb][0]), as_bf16x8(b[0]), z, 0, 0, 0);
  }
#pragma unroll
  for (int ks = 1; ks < KS; ++ks)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      R[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.u[rb][ks]), as_bf16x8(b[ks]), R[rb], 0, 0, 0);
      I[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.v[rb][ks]), as_bf16x8(b[ks]), I[rb], 0, 0, 0);
    }
}

// Row-block-major form of one column block: the 2 KS products of row block
// rb run back to back, and the |G|^2 / max fold of row block rb - 2 (of the
// previous column block for rb < 2) runs under them, so the fold of a row
// block is spread over another row block's products instead of being packed
// before the next column block.  Row block rb's accumulators are rewritten
// only at row block rb of the next column block, after their fold.
template <int KS, bool EPI>
__device__ __forceinline__ void qblock_rm(const QRows<KS>& A, const u32x4 b[KS], v4f32 R[4], v4f32 I[4],
                                          uint32_t& best) {
  const v4f32 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int fr = (rb + 2) & 3;
    if (EPI || rb >= 2) best = fold_rb(best, R[fr], I[fr]);
    R[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.u[rb][0]), as_bf16x8(b[0]), z, 0, 0, 0);
    I[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.v[rb][0]), as_bf16x8(b[0]), z, 0, 0, 0);
#pragma unroll
    for (int ks = 1; ks < KS; ++ks) {
      R[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.u[rb][ks]), as_bf16x8(b[ks]), R[rb], 0, 0, 0);
      I[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A.v[rb][ks]), as_bf16x8(b[ks]), I[rb], 0, 0, 0);
    }
  }
}

template <int KS>
__device__ __forceinline__ void sched_qblock_rm(bool epi, bool reads) {
  // per row block: its 2 KS products, the fold (10 VALU) in pairs after the
  // first five, one LDS read of the next column block's fragments after the
  // first product (KS reads over the first KS row blocks)
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const bool fold = epi || rb >= 2;
#pragma unroll
    for (int j = 0; j < 2 * KS; ++j) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      if (j == 0 && reads && rb < KS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      if (fold && j < 5) __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    }
  }
}

// Max |G|^2 bits over this wave's 64 rows (tile offset roff) against the 128
// LDS columns of one tile; on a diagonal tile only pairs with j > i count.
template <int KS>
__device__ __forceinline__ uint32_t tile_max_k(const QRows<KS>& A, const uint16_t* Bs, bool diag, int roff) {
  const int lane = threadIdx.x & 63;
  uint32_t best = 0;
  v4f32 R[4], I[4];
  u32x4 b0[KS], b1[KS];
  if (!diag) {
    read_frags<KS>(Bs, 0, b0);
    read_frags<KS>(Bs, 1, b1);
    qblock_rm<KS, false>(A, b0, R, I, best);
    sched_qblock_rm<KS>(false, false);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cb = 1; cb < T / 16; ++cb) {
      if (cb & 1) {
        if (cb + 1 < T / 16) read_frags<KS>(Bs, cb + 1, b0);
        qblock_rm<KS, true>(A, b1, R, I, best);
      } else {
        if (cb + 1 < T / 16) read_frags<KS>(Bs, cb + 1, b1);
        qblock_rm<KS, true>(A, b0, R, I, best);
      }
      sched_qblock_rm<KS>(true, cb + 1 < T / 16);
      __builtin_amdgcn_sched_barrier(0);
    }
    best = fold_rb(best, R[2], I[2]);
    best = fold_rb(best, R[3], I[3]);
    return best;
  }
  // diagonal tile: column blocks wholly below this wave's rows are skipped
  for (int c = roff / 16; c < T / 16; ++c) {
    read_frags<KS>(Bs, c, b0);
    qblock<KS, false>(A, b0, R, I, best);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      uint32_t m[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        m[v] = __float_as_uint(fmaf(R[rb][v], R[rb][v], I[rb][v] * I[rb][v]));
        const int i = roff + rb * 16 + 4 * (lane >> 4) + v;
        const int j = c * 16 + (lane & 15);
        if (i >= j) m[v] = 0u;
      }
      best = max3u(max3u(m[0], m[1], m[2]), m[3], best);
    }
  }
  return best;
}

// Row segments of 256-row blocks: row block r (tile rows 2r, 2r + 1) against
// runs of column tiles bj >= 2r; the nt - 2r tiles of row block r are split
// into ceil((nt - 2r) / seg) runs of equal length (within one tile), so
// every block does about the same work and the A rows are loaded once per
// run of up to seg tiles (6 measured best at N = 4096, d = 64 among 3..16).
__device__ __forceinline__ void seg_decode_k(int s, int nt, int seg, int& r, int& bj0, int& bj1) {
  r = 0;
  int rem = s;
  for (;;) {
    const int ns = (nt - 2 * r + seg - 1) / seg;
    if (rem < ns) break;
    rem -= ns;
    ++r;
  }
  const int L = nt - 2 * r;
  const int ns = (L + seg - 1) / seg;
  bj0 = 2 * r + (rem * L) / ns;
  bj1 = 2 * r + ((rem + 1) * L) / ns;
}

template <int KS>
__device__ __forceinline__ void gram_bf16_wide(const GramArgs& a, int b) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  const int local = b >> 3;
  const int slot = (local / a.nseg) * 8 + (b & 7);
  const int seg = local % a.nseg;
  if (slot >= a.slots) return;
  int r, bj0, bj1;
  seg_decode_k(seg, a.nt, a.segk, r, bj0, bj1);
  const int tiles = a.nt * (a.nt + 1) / 2;

  constexpr int kBuf = T * (32 * KS + 8);
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2 * kBuf];
  __shared__ uint32_t red[4];
  const uint16_t* base = (const uint16_t*)a.cand + (size_t)slot * a.slot_stride;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int tr = 2 * r + (w >> 1);   // this wave's tile row
  const int roff = 64 * (w & 1);     // its rows' offset in that tile row

  u32x4 pf[2 * KS];
  fetch_cols<KS>(base, a.n, bj0, pf);
  QRows<KS> A;
  load_rows_q<KS>(base, a.ldk, a.n, tr * T + roff, A);
  store_cols<KS>(pf, Bs);
  __syncthreads();
  if (bj0 + 1 < bj1) fetch_cols<KS>(base, a.n, bj0 + 1, pf);

  uint32_t cmax = 0;
  uint32_t tile_lane = 0;
  for (int bj = bj0; bj < bj1; ++bj) {
    const int buf = (bj - bj0) & 1;
    uint32_t tmax = 0;
    if (bj >= tr && tr < a.nt) tmax = tile_max_k<KS>(A, Bs + buf * kBuf, bj == tr, roff);
    cmax = tmax > cmax ? tmax : cmax;
    if (a.tile_max) {
      const uint32_t wm = wave_max_u32_dpp(tmax);
      if (lane == bj - bj0) tile_lane = wm;
    }
    if (bj + 1 < bj1) {
      store_cols<KS>(pf, Bs + (buf ^ 1) * kBuf);
      __syncthreads();
      if (bj + 2 < bj1) fetch_cols<KS>(base, a.n, bj + 2, pf);
    }
  }
  // tile (tr, bj) is covered by the two waves of tile row tr: each fills two
  // of its four entries
  if (a.tile_max && lane < bj1 - bj0 && bj0 + lane >= tr && tr < a.nt) {
    uint32_t* dst = a.tile_max + ((size_t)slot * tiles + tile_linear(tr, bj0 + lane, a.nt)) * 4 + 2 * (w & 1);
    *(uint2*)dst = make_uint2(tile_lane, tile_lane);
  }
  cmax = wave_max_u32_dpp(cmax);
  if (lane == 0) red[w] = cmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t mx = max3u(red[0], red[1], red[2] > red[3] ? red[2] : red[3]);
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)mx);
  }
}

template <int KS>
__global__ __launch_bounds__(256, 2) void k_gram_bf16(GramArgs a) {
  gram_bf16_narrow<KS>(a, blockIdx.x);
}

template <int KS>
__global__ __launch_bounds__(256, 2) void k_gram_bf16_k(GramArgs a) {
  gram_bf16_wide<KS>(a, blockIdx.x);
}

// Group launches: search blockIdx.y of the table (each record with its own
// slots and nseg; blocks past a search's own grid return at once).
template <int KS>
__global__ __launch_bounds__(256, 2) void k_gram_bf16_tab(TabRef t) {
  const GramArgs a = *(const GramArgs*)(t.base + (size_t)t.list[blockIdx.y] * t.stride);
  gram_bf16_narrow<KS>(a, blockIdx.x);
}

template <int KS>
__global__ __launch_bounds__(256, 2) void k_gram_bf16_k_tab(TabRef t) {
  const GramArgs a = *(const GramArgs*)(t.base + (size_t)t.list[blockIdx.y] * t.stride);
  gram_bf16_wide<KS>(a, blockIdx.x);
}

int k_segments(int nt, int seg) {
  int total = 0;
  for (int r = 0; 2 * r < nt; ++r) total += (nt - 2 * r + seg - 1) / seg;
  return total;
}

// Exact FP64 <phi_j, phi_k> partial sums for 16 lanes per pair: lane sub of
// the group takes entries sub, sub + 16, ... (loads of a 64-entry chunk
// issued together); the caller combines the sixteen with group_sum<16>
// (commutative steps, so every lane of the group ends with the same bits,
// whichever pair or item it is).
__device__ __forceinline__ void pair_f64_part(const double* c64, int ld, int d, int j, int k, int sub, double& re,
                                              double& im) {
  const double2* x = (const double2*)(c64 + (size_t)j * ld);
  const double2* y = (const double2*)(c64 + (size_t)k * ld);
  re = 0.0;
  im = 0.0;
  for (int i0 = 0; i0 < d; i0 += 64) {
    double2 p[4], q[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = i0 + sub + 16 * t;
      p[t] = i < d ? x[i] : make_double2(0.0, 0.0);
      q[t] = i < d ? y[i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      re += p[t].x * q[t].x + p[t].y * q[t].y;
      im += p[t].x * q[t].y - p[t].y * q[t].x;
    }
  }
}

// Pair-level FP64 recheck.  For a rechecked candidate with screened maximum s
// and certified screen error eps, the exact maximiser has screened value
// >= s - 2 eps = thr (its exact value is >= the exact value at the screened
// maximiser >= s - eps).  Each listed screen tile is screened again (any
// screen within eps of the exact values serves) and every pair whose screened
// value reaches thr is evaluated exactly in FP64 from the FP64 candidate.
// One wave per work item: 32 rows x 32 columns (sub-block sb of 16) of a
// listed screen tile, A and B fragments read straight from global memory (no
// LDS, no barrier), so every item of every listed tile runs at once.
template <int KS>
__device__ __forceinline__ void recheck_body(const RecheckArgs& a, int bx, int gx) {
  if (*a.flags & kFlagDone) return;
  __shared__ int2 hits[32 * 32];
  __shared__ int nhits;
  const int lane = threadIdx.x;
  if (bx == 0 && lane < a.k && !(a.thr[lane] > -__builtin_inf()))
    atomicMax((unsigned long long*)&a.recheck_max[lane], ~0ull);  // invalid candidate
  const int items = *a.count * 16;
  for (int it = bx; it < items; it += gx) {
    const int2 item = a.list[it >> 4];
    const int rq = (it >> 2) & 3, cq = it & 3;
    int bi, bj;
    tile_decode(item.y, a.nt, bi, bj);
    if (bi == bj && rq > cq) continue;  // wholly below the diagonal (uniform: no barrier skipped unevenly)
    if (!((item.x >> (8 + rq)) & 1)) continue;  // row quarter below the threshold (uniform as well)
    const int slot = item.x & 0xFF;
    const double thr = a.thr[slot];
    const float thr_sq = thr > 0.0 ? (float)(thr * thr * (1.0 - 1e-6)) : 0.0f;
    const uint16_t* base = a.screen + (size_t)a.rechecked[slot] * a.screen_stride;
    const double* c64 = a.cand64 + (size_t)slot * a.stride64;
    const int r0 = bi * T + 32 * rq, c0 = bj * T + 32 * cq;
    u32x4 au[2][KS], av[2][KS], bu[2][KS];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = r0 + 16 * h + (lane & 15);
      const int col = c0 + 16 * h + (lane & 15);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = ks * 32 + 8 * (lane >> 4);
        au[h][ks] = row < a.n ? *(const u32x4*)(base + (size_t)row * a.ldk16 + k) : u32x4{0u, 0u, 0u, 0u};
        bu[h][ks] = col < a.n ? *(const u32x4*)(base + (size_t)col * a.ldk16 + k) : u32x4{0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[h][ks] = swap_negate(au[h][ks]);
    // qualifying pairs go to a list first, so the FP64 code below exists once
    // (it runs rarely and would otherwise be fetched cold in many copies)
    if (lane == 0) nhits = 0;
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      v4f32 xR[2], xI[2];
      uint32_t m[8];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        xR[rb] = v4f32{0.f, 0.f, 0.f, 0.f};
        xI[rb] = v4f32{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          xR[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(au[rb][ks]), as_bf16x8(bu[cb][ks]), xR[rb], 0, 0, 0);
          xI[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(av[rb][ks]), as_bf16x8(bu[cb][ks]), xI[rb], 0, 0, 0);
        }
      sq_mag(xR, xI, m);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = r0 + (q >> 2) * 16 + 4 * (lane >> 4) + (q & 3);
        const int j = c0 + cb * 16 + (lane & 15);
        if (i < j && j < a.n && !(__uint_as_float(m[q]) < thr_sq)) hits[atomicAdd(&nhits, 1)] = make_int2(i, j);
      }
    }
    __syncthreads();
    const int nh = nhits;
    uint64_t best = 0;
    // 4 pairs at a time, 16 lanes per pair, so the loads of all of them are
    // in flight together
    for (int e0 = 0; e0 < nh; e0 += 4) {
      const int e = e0 + (lane >> 4);
      double re = 0.0, im = 0.0;
      if (e < nh) {
        const int2 h = hits[e];
        pair_f64_part(c64, a.ld64, a.d, h.x, h.y, lane & 15, re, im);
      }
      re = group_sum<16>(re);
      im = group_sum<16>(im);
      if (e < nh) {
        const uint64_t mb = (uint64_t)__double_as_longlong(re * re + im * im);
        best = mb > best ? mb : best;
      }
    }
    __syncthreads();  // the list is rebuilt by the next item
    best = wave_max_u64(best);
    if (lane == 0 && best) atomicMax((unsigned long long*)&a.recheck_max[slot], (unsigned long long)best);
  }
}

template <int KS>
__global__ __launch_bounds__(64) void k_recheck_pairs(RecheckArgs a) {
  recheck_body<KS>(a, blockIdx.x, gridDim.x);
}

template <int KS>
__global__ __launch_bounds__(64) void k_recheck_pairs_tab(TabRef t) {
  const RecheckArgs a = *(const RecheckArgs*)(t.base + (size_t)t.list[blockIdx.y] * t.stride);
  recheck_body<KS>(a, blockIdx.x, gridDim.x);
}

// General K: chunks of 128 bf16 through LDS, each wave a 64 x 64 quadrant.
constexpr int KCB = 128;
constexpr int LDB = KCB + 8;

__global__ __launch_bounds__(256) void k_gram_bf16_chunked(GramArgs a) {
  if (a.flags && (*a.flags & kFlagDone)) return;
  const int tiles = a.nt * (a.nt + 1) / 2;
  int slot, tile;
  if (!xcd_slot(a, tiles, slot, tile)) return;
  int bi, bj;
  tile_decode(tile, a.nt, bi, bj);

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

  const int K = a.ldk;
  for (int k0 = 0; k0 < K; k0 += KCB) {
    __syncthreads();
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
        u32x4 au[4];
        bf16x8 bb[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) au[r] = *(const u32x4*)&As[(wr * 64 + r * 16 + (lane & 15)) * LDB + kk * 32 + koff];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          bb[c] = as_bf16x8(*(const u32x4*)&Bs[(wc * 64 + c * 16 + (lane & 15)) * LDB + kk * 32 + koff]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bf16x8 aU = as_bf16x8(au[r]);
          const bf16x8 aV = as_bf16x8(swap_negate(au[r]));
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            accR[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aU, bb[c], accR[r][c], 0, 0, 0);
            accI[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aV, bb[c], accI[r][c], 0, 0, 0);
          }
        }
      }
    }
  }

  uint32_t best = 0;
  if (!skip) {
    const bool diag = bi == bj;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float re = accR[r][c][v], im = accI[r][c][v];
          uint32_t mb = __float_as_uint(fmaf(re, re, im * im));
          if (diag) {
            const int i = wr * 64 + r * 16 + 4 * (lane >> 4) + v;
            const int j = wc * 64 + c * 16 + (lane & 15);
            if (i >= j) mb = 0u;
          }
          best = mb > best ? mb : best;
        }
  }
  best = wave_max_u32(best);
  if (lane == 0) red[w] = best;
  __syncthreads();
  if (tid == 0) {
    const uint32_t mx = max3u(red[0], red[1], red[2] > red[3] ? red[2] : red[3]);
    if (a.tile_max)
      for (int q = 0; q < 4; ++q) a.tile_max[((size_t)slot * tiles + tile) * 4 + q] = mx;
    atomicMax((unsigned long long*)&a.cand_max[slot], (unsigned long long)mx);
  }
}

template <int KS>
hipError_t launch_rp(const RecheckArgs& a, int grid, hipStream_t s, const TabRef* tab) {
  if (tab)
    hipLaunchKernelGGL(k_recheck_pairs_tab<KS>, dim3(grid, tab->count), dim3(64), 0, s, *tab);
  else
    hipLaunchKernelGGL(k_recheck_pairs<KS>, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

// grid: blocks of the prepared record (or, for a group, the largest over
// the group)
template <int KS>
hipError_t launch_ks(const GramArgs& a, int grid, hipStream_t s, const TabRef* tab) {
  bool wide = false;
  if constexpr (KS <= 4) wide = a.form == 0;
  if (wide) {
    if constexpr (KS <= 4) {
      if (tab)
        hipLaunchKernelGGL(k_gram_bf16_k_tab<KS>, dim3(grid, tab->count), dim3(256), 0, s, *tab);
      else
        hipLaunchKernelGGL(k_gram_bf16_k<KS>, dim3(grid), dim3(256), 0, s, a);
    }
  } else {
    if (tab)
      hipLaunchKernelGGL(k_gram_bf16_tab<KS>, dim3(grid, tab->count), dim3(256), 0, s, *tab);
    else
      hipLaunchKernelGGL(k_gram_bf16<KS>, dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_gram_any(const GramArgs& a, int grid, hipStream_t s, const TabRef* tab) {
  const int ks = a.ldk / 32;
  switch (a.ldk % 32 == 0 ? ks : 0) {
    case 1: return launch_ks<1>(a, grid, s, tab);
    case 2: return launch_ks<2>(a, grid, s, tab);
    case 3: return launch_ks<3>(a, grid, s, tab);
    case 4: return launch_ks<4>(a, grid, s, tab);
    case 5: return launch_ks<5>(a, grid, s, tab);
    case 6: return launch_ks<6>(a, grid, s, tab);
    case 7: return launch_ks<7>(a, grid, s, tab);
    case 8: return launch_ks<8>(a, grid, s, tab);
    default: {
      if (tab) return hipErrorInvalidValue;  // the group form needs 2d <= 256
      const long tiles = (long)a.nt * (a.nt + 1) / 2;
      hipLaunchKernelGGL(k_gram_bf16_chunked, dim3((int)(tiles * ((a.slots + 7) / 8 * 8))), dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
}

hipError_t launch_rp_any(const RecheckArgs& a, int grid, hipStream_t s, const TabRef* tab) {
  switch (a.ldk16 / 32) {
    case 1: return launch_rp<1>(a, grid, s, tab);
    case 2: return launch_rp<2>(a, grid, s, tab);
    case 3: return launch_rp<3>(a, grid, s, tab);
    case 4: return launch_rp<4>(a, grid, s, tab);
    case 5: return launch_rp<5>(a, grid, s, tab);
    case 6: return launch_rp<6>(a, grid, s, tab);
    case 7: return launch_rp<7>(a, grid, s, tab);
    case 8: return launch_rp<8>(a, grid, s, tab);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int bf16_segments(int nt, int seg) {
  int total = 0;
  for (int r = 0; r < nt; ++r) total += (nt - r + seg - 1) / seg;
  return total;
}

namespace {
std::mutex g_tiles_mu;
std::vector<ScreenTile> g_tiles;
}  // namespace

void screen_tiles_set(const ScreenTile* e, int32_t count) {
  std::lock_guard<std::mutex> g(g_tiles_mu);
  g_tiles.assign(e, e + count);
}

void screen_tile_choose(int64_t n, int32_t ks, int32_t* form, int32_t* seg) {
  *form = ks <= 4 ? 0 : 1;
  *seg = ks <= 4 ? 6 : 8;
  std::lock_guard<std::mutex> g(g_tiles_mu);
  const ScreenTile* best = nullptr;
  for (const ScreenTile& t : g_tiles)
    if (t.ks == ks && t.n_max >= n && (!best || t.n_max < best->n_max)) best = &t;
  if (best) {
    *form = best->form;
    *seg = best->seg;
  }
}

int gram_bf16_prepare(GramArgs& a, int slots) {
  a.slots = slots;
  const long slots8 = (slots + 7) / 8 * 8;
  const int ks = a.ldk % 32 == 0 ? a.ldk / 32 : 0;
  if (ks >= 1 && ks <= 8) {
    screen_tile_choose(a.n, ks, &a.form, &a.segk);
    if (ks > 4) a.form = 1;  // 256-row blocks hold the whole K only up to 2d = 128
    a.nseg = a.form == 0 ? k_segments(a.nt, a.segk) : bf16_segments(a.nt, a.segk);
    return (int)((long)a.nseg * slots8);
  }
  a.nseg = 0;
  return (int)((long)a.nt * (a.nt + 1) / 2 * slots8);
}

hipError_t launch_gram_bf16(const GramArgs& a_in, int slots, hipStream_t s) {
  GramArgs a = a_in;
  const int grid = gram_bf16_prepare(a, slots);
  return launch_gram_any(a, grid, s, nullptr);
}

hipError_t launch_gram_bf16_tab(const TabRef& t, int ldk, int form, int grid, hipStream_t s) {
  GramArgs shape{};
  shape.ldk = ldk;
  shape.form = form;
  return launch_gram_any(shape, grid, s, &t);
}

int recheck_grid(int list_cap) {
  const long items = 16L * list_cap;
  return (int)(items < 4096 ? items : 4096);
}

hipError_t launch_recheck_pairs(const RecheckArgs& a, hipStream_t s) {
  return launch_rp_any(a, recheck_grid(a.list_cap), s, nullptr);
}

hipError_t launch_recheck_tab(const TabRef& t, int ldk16, int grid, hipStream_t s) {
  RecheckArgs shape{};
  shape.ldk16 = ldk16;
  return launch_rp_any(shape, grid, s, &t);
}

}  // namespace trstmi
