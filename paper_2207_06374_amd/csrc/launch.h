// Host-side launchers of the library's kernels and their argument records.
// Shared by the kernel translation units and the C-ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "trstmi.h"

namespace trstmi {

enum OutKind { kOutF64 = 0, kOutF32 = 1, kOutBF16 = 2 };

// Decision record written by the select kernel and read by the commit.
struct Decision {
  int32_t commit;        // 1: regenerate candidate `best` into the frame
  int32_t best;          // selected candidate, -1 if none valid
  int64_t t_old;         // step index the candidates were drawn at
  double radius_old;     // radius the candidates were drawn with
  int32_t screen_near;   // BF16 screen: k-th and (k+1)-th screened values nearly tie
  int32_t pad;
};

// Perturb + renormalise (also: random start, normalise-only, commit).
struct PerturbArgs {
  const double* base;       // frame (2*d*n doubles, column stride 2d) or null (y = z)
  const double* radius;     // device scalar radius (used when base and draws are both present)
  const int64_t* tstep;     // device scalar step index, or null -> t_const
  int64_t t_const;
  const int32_t* cand_idx;  // device list slot -> candidate, or null -> c0 + slot
  int32_t c0;
  int32_t have_z;           // 0: y = base (normalise only)
  const int32_t* gate;      // run only if (*gate & gate_mask) == gate_want (null: always)
  int32_t gate_mask;
  int32_t gate_want;
  const double* z_explicit; // [c][n][d] complex, or null -> Philox draws
  int64_t n;
  int32_t d;
  uint32_t seed;
  uint32_t stream_id;
  uint32_t tag;
  void* out;                // candidate buffer
  int32_t out_kind;         // OutKind
  int32_t out_ld;           // elements per column in `out` (>= 2d; padding written as zero)
  int64_t out_slot_stride;  // elements per slot in `out`
  uint64_t* zero_max;       // if not null: zero_max[slot] <- 0 (block 0)
};

// Gram + fused max of |G|^2 over the strict upper triangle.
struct GramArgs {
  const void* cand;          // slot-major candidates
  int64_t slot_stride;       // elements per slot
  int32_t ldk;               // elements per column (>= 2d, multiple of 8, zero padded)
  int32_t n;
  int32_t d;
  int32_t nt;                // tiles per side
  int32_t slots;             // candidates in this launch (set by the launcher)
  int32_t nseg;              // BF16: row segments per candidate (set by the launcher)
  uint64_t* cand_max;        // [slot] running max (bits of the float type)
  const int32_t* flags;      // DONE gate (null: always run)
  uint32_t* tile_max;        // screen: [slot][ntiles][4] max bits per tile and wave (null: not kept)
  int32_t form;              // BF16 screen: 0 = 256-row blocks (2d <= 128), 1 = 128-row blocks (set by the launcher)
  int32_t segk;              // BF16 screen: column tiles per block run (set by the launcher from the tile table)
};

struct SelectArgs {
  const uint64_t* cand_max;  // [count] max bits (double, or float if is_f32)
  int32_t count;
  int32_t is_f32;
  const int32_t* slot_cand;  // slot -> candidate (null: identity)
  double tau;                // near-tie threshold
  int32_t use_screen_near;   // also report dec->screen_near as a near tie
  double* mu;
  double* radius;
  int64_t* step;
  int32_t* flags;
  double grow, shrink, radius_min, radius_max;
  int64_t max_steps;
  double target_mu;
  Decision* dec;
  double* rep_cand_mu;       // [count] (null: not written)
  int32_t* rep_best;         // [1]
};

struct TopkArgs {
  const uint64_t* cand_max;  // [C] float bits of the screened max |G|^2
  int32_t C;
  int32_t k;
  double eps;                // certified screen error bound (|G| units)
  double screen_tie;         // gap below which membership of the top-k is a near tie
  const int32_t* flags;
  int32_t* rechecked;        // [k] out
  double* thr;               // [k] out: per rechecked candidate, mu_screen - 2 eps
  Decision* dec;
  double* rep_cand_mu;       // [C] screened mu (null: not written)
  int32_t* rep_rechecked;    // [k]
  // certified pruning of the FP64 recheck: screen tile maxima in, list of
  // screen tiles that may hold a rechecked candidate's exact maximum out
  const uint32_t* tile_max;  // [C][screen tiles][4] float bits of max |G|^2 (per wave)
  int32_t screen_nt;         // screen tiles per side
  int2* list;                // out: (slot | row-quarter mask << 8, screen tile) items
  int32_t* list_count;       // out
  int32_t list_cap;
};

// Pair-level FP64 recheck over the listed screen tiles.
struct RecheckArgs {
  const uint16_t* screen;    // BF16 candidates, indexed by candidate
  int64_t screen_stride;     // elements per candidate
  int32_t ldk16;             // BF16 column stride (multiple of 32, <= 256)
  const double* cand64;      // FP64 candidates of the rechecked slots
  int64_t stride64;          // doubles per slot
  int32_t ld64;              // FP64 column stride (doubles)
  int32_t n, d, nt, k;       // nt: screen tiles per side; k: rechecked slots
  const int2* list;          // (slot | row-quarter mask << 8, screen tile)
  const int32_t* count;
  int32_t list_cap;
  const int32_t* rechecked;  // slot -> candidate
  const double* thr;         // slot -> screened max - 2 eps (-inf: invalid candidate)
  uint64_t* recheck_max;     // [k] FP64 max |G|^2 bits (zeroed before)
  const int32_t* flags;
};

// Every argument record of one step of one search in the BF16-screen form,
// as the single-search launches use them.  The serving engine keeps one per
// admitted search in a device table and launches each kernel once for a
// group of searches of the same d: the search is a grid dimension and each
// block reads its record from the table, so every search runs exactly the
// arithmetic of its own single-search step.
struct StepArgs {
  PerturbArgs pa;   // candidates (BF16 screen copies)
  GramArgs g;       // screen (slots and nseg filled in)
  TopkArgs ta;
  PerturbArgs pr;   // FP64 regeneration of the rechecked candidates
  RecheckArgs ra;
  SelectArgs sa;
  PerturbArgs pc;   // commit of the accepted candidate
};

// A group of records in a device table: record i of the group is at
// base + list[i] * stride (base points at the member the kernel reads).
struct TabRef {
  const char* base;
  size_t stride;
  const int32_t* list;  // device [count]
  int32_t count;
};

struct PollRecord {
  int32_t flags;
  int32_t pad;
  int64_t step;
  double mu;
};

struct InitFinishArgs {
  const uint64_t* max_bits;  // one value
  int32_t is_f32;
  double* mu;
  double* radius;
  int64_t* step;
  int32_t* flags;
  double radius0;
  int64_t max_steps;
  double target_mu;
  double* mu_out;            // coherence entry: write mu here instead (state pointers null)
};

// Batched form (batch.hip).  launch_batch_step enqueues the step kernel
// (`grid` blocks, at most the resident capacity) and the finalizing kernel.
struct BatchArgs {
  const void* inst;          // [count] instance descriptors
  void* state;               // [count] per-instance state
  const int2* units;         // (instance, first candidate) work units, largest instances first
  int32_t nunits;
  int32_t C;                 // candidates per instance per step
  double* frames;            // frame arena
  uint64_t* cand_max;        // [count][C] exact FP64 max |G|^2 bits of the step's candidates
  double* scratch;           // per block and group: one FP64 candidate
  int64_t scratch_stride;    // doubles per scratch slot
  int32_t count;             // instances
  int32_t* done_instances;   // instances that reached DONE
  double tau, grow, shrink, radius_min, radius_max;
  double* rep_mu;            // [count][C] or null
  int32_t* rep_best;         // [count] or null
  void* tab;                 // the Gaussian draw tables (a GaussTab, filled by the init launch)
};

hipError_t launch_batch_step(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_init(const BatchArgs& a, int count, double radius0, hipStream_t s);
int batch_step_max_blocks();
size_t batch_inst_bytes();
size_t batch_state_bytes();
void batch_fill_inst(void* dst, int32_t n, int32_t d, int32_t wpi, uint32_t seed, uint32_t stream_id,
                     int64_t frame_off, double target_mu, int64_t max_steps);
int batch_lds_words();
int32_t batch_row_words(int32_t d);  // LDS words per column of a candidate's split copy
double batch_screen_eps(int32_t d);    // the split screen's certified bound (d <= 16)
size_t batch_tab_bytes();

hipError_t launch_perturb(const PerturbArgs& a, int slots, hipStream_t s);

// Commit by copy: when dec->commit is set, the accepted candidate's FP64
// columns, already written earlier in the step (the FP64 candidates, or the
// FP64 copies of the rechecked ones), are copied into the frame.
struct CommitCopyArgs {
  const Decision* dec;
  const int32_t* slot_cand;  // slot -> candidate (k entries), or null: slot = candidate
  int32_t k;
  const double* src;         // slot s at src + s * src_slot_stride, column stride src_ld
  int64_t src_slot_stride;
  int32_t src_ld;
  double* frame;             // column stride 2d
  int64_t n;
  int32_t d;
};
hipError_t launch_commit_copy(const CommitCopyArgs& a, hipStream_t s);
hipError_t launch_gram_f64(const GramArgs& a, int slots, hipStream_t s);
// After launch_gram_f64 on one frame (slot 0): the first pair j < k in the
// order j * n + k whose |G|^2 has the maximum's bits, into *pair (scratch),
// then mu = sqrt(max) and jk = (j, k) (or +inf and (-1, -1)).
hipError_t launch_gram_f64_pair(const GramArgs& a, uint64_t* pair, double* mu, int64_t* jk, hipStream_t s);
// Smooth maximum (one frame, slot 0), one pass over the tiles: per block
// (S_b, x_b) into partial[tile][2] and the maximum |G|^2 bits into
// a.cand_max[0] (zeroed beforehand); then F = s + delta log S into
// out = (s, F).
hipError_t launch_lse_pass(const GramArgs& a, double delta, int32_t squared, double* partial, hipStream_t s);
hipError_t launch_lse_finish(const uint64_t* s_bits, const double* partial, int64_t count, double delta,
                             int32_t squared, double* out, double* log_sum, hipStream_t s);

// Gradient of the smooth maximum (x = |G|^2, d <= 64) with respect to the
// unconstrained frame.
struct GradArgs {
  const double* frame;      // normalised frame (column stride ld)
  const double* raw;        // the caller's frame (column stride 2d), for the column norms
  int32_t ld;
  int32_t ldp;              // LDS column stride: 2d rounded up to a power of two >= 16, plus one
  int32_t n, d;
  const uint64_t* s_bits;   // max |G|^2 bits
  const double* log_sum;    // log of sum exp((x - s) / delta) over j < k
  double inv_delta;
  double* partial;          // [nkb][nch][2 row halves][2][64][2d]
  double* grad;             // out: column stride 2d, (re, im) interleaved
};
int lse_grad_chunks(int nkb);
hipError_t launch_lse_grad(const GradArgs& a, hipStream_t s);

// Exact Hessian-vector product of the smooth maximum (lse_hv.hip, d <= 64).
struct HvArgs {
  const double* raw;        // the frame Y (column stride 2d)
  const double* v;          // the direction V (same layout)
  const uint64_t* s_bits;   // max |G|^2 bits of Y
  double inv_delta;
  double* out;              // Hv (same layout)
  // scratch, laid out by hv_layout
  double* phi;              // normalised columns (stride 2d)
  double* dphi;             // their derivative along V
  double* r;                // [n] column norms
  double* dr;               // [n] their derivative
  double* partial;          // [chunks][n][4][2d] partial sums of U Re B, U Im B, dU Re B + U Re B1, dU Im B + U Im B1
  double* sigpart;          // [blocks] partial sums of sum e dx (e = exp((x - s) / delta), unnormalised)
  double* esumpart;         // [blocks] partial sums of e
  double* sigma;            // [2]: sigma and 1 / S (S = sum of e over j < k)
  int32_t n, d;
};
size_t hv_scratch_bytes(int64_t n, int64_t d);
void hv_layout(HvArgs& a, char* scratch, int64_t n, int64_t d);
hipError_t launch_lse_hv(const HvArgs& a, hipStream_t s);
// Alg. 2 with one block per random start (opt_batch.hip): n <= kOptMaxN,
// d <= kOptMaxD, exact Hessian products.
constexpr int kOptMaxN = 128;
constexpr int kOptMaxD = 16;
struct OptBatchArgs {
  int32_t n, d, starts, first;  // starts l = 0 .. starts - 1 use stream first + l
  uint32_t seed;
  int32_t n_deltas, steps_per_delta, cg_max_iter;
  const double* deltas;         // device [n_deltas]
  double radius0, radius_min, radius_max, eta, cg_tol;
  double* work;                 // [starts][stride]: the frame, then nine CG vectors of 2dn doubles
  int64_t stride;               // doubles per start (opt_batch_stride)
  double* mu;                   // [starts] exact FP64 coherence of each final frame
};
size_t opt_batch_stride(int64_t n, int64_t d);
hipError_t launch_opt_batch(const OptBatchArgs& a, hipStream_t s);

// Where trstmi_lse_grad leaves s (max |G|^2 bits) and log S in its workspace.
void lse_grad_scalars(int64_t n, int64_t d, char* ws, const uint64_t** s_bits, const double** log_sum);

// Beamforming-codebook quantiser (miso.hip).
struct MisoArgs {
  const double* codebook;   // normalised codewords (column stride ldk, zero padded)
  int32_t ldk;
  int32_t n, d;
  const double* channels;   // the caller's channels (column stride 2d)
  int64_t m;
  int32_t* index;           // [m] argmax codeword, -1 if undefined (null: not written)
  double* gain;             // [m] max |<phi_i, h>|^2 (null: not written)
  double* dist;             // [m] 1 - gain / |h|^2 (null: not written)
  double* partial;          // [blocks][2] block sums of dist and gain (null: not kept)
};
int64_t miso_blocks(int64_t m);
// The quantiser, then (if summary is not null) summary = (mean dist, mean gain).
hipError_t launch_miso(const MisoArgs& a, double* summary, hipStream_t s);

// Every record of one BF16-screen step of a search (validated parameters,
// mode TRSTMI_MODE_BF16_SCREEN) over its state and workspace, as
// trstmi_step launches them; z and rep as trstmi_step's (nullable).
StepArgs bf16_step_args(const trstmi_params* p, const trstmi_state* st, char* ws, const double* z,
                        const trstmi_report* rep);

// The calling thread's error message (what trstmi_last_error returns).
trstmi_status set_last_error(trstmi_status code, const std::string& msg);

// Trust-region step (trust_region.hip): the vectors' workspace bytes, and the
// step itself given a trstmi_lse_grad workspace of lws_bytes at ws.
size_t tr_vectors_bytes(int64_t n, int64_t d);
trstmi_status tr_step_impl(int64_t n, int64_t d, double* frame, const trstmi_tr_params* tp, trstmi_tr_report* rep,
                           char* ws, size_t lws_bytes, hipStream_t stream);
hipError_t launch_gram_f32(const GramArgs& a, int slots, hipStream_t s);
hipError_t launch_gram_bf16(const GramArgs& a, int slots, hipStream_t s);
// Fills a.slots, a.form, a.segk and a.nseg as launch_gram_bf16 does (form
// and run length from the screen tile table); returns that launch's grid.
int gram_bf16_prepare(GramArgs& a, int slots);
// The screen tile table (process-wide): form and run length by K steps
// (ks = 2d / 32 rounded up) and the smallest n_max >= n; without an entry,
// 256-row blocks with runs of 6 tiles for ks <= 4, 128-row blocks with runs of
// 8 tiles above.  The choice changes speed only, never a result.
struct ScreenTile {
  int32_t ks, n_max, form, seg;
};
void screen_tiles_set(const ScreenTile* e, int32_t count);
void screen_tile_choose(int64_t n, int32_t ks, int32_t* form, int32_t* seg);
int recheck_grid(int list_cap);
// Group launches over a table (see StepArgs).  shape: a record with the
// group's d, output kind and largest n; grid: the largest grid of the group.
hipError_t launch_perturb_tab(const TabRef& t, const PerturbArgs& shape, int slots, hipStream_t s);
hipError_t launch_gram_bf16_tab(const TabRef& t, int ldk, int form, int grid, hipStream_t s);
hipError_t launch_topk_tab(const TabRef& t, hipStream_t s);
hipError_t launch_recheck_tab(const TabRef& t, int ldk16, int grid, hipStream_t s);
hipError_t launch_select_tab(const TabRef& t, hipStream_t s);
hipError_t launch_poll_tab(const TabRef& t, PollRecord* out, hipStream_t s);
hipError_t launch_select(const SelectArgs& a, hipStream_t s);
hipError_t launch_topk(const TopkArgs& a, hipStream_t s);
hipError_t launch_recheck_pairs(const RecheckArgs& a, hipStream_t s);
hipError_t launch_init_finish(const InitFinishArgs& a, hipStream_t s);
hipError_t launch_round_bf16(const double* x, int64_t count, uint16_t* out, hipStream_t s);
hipError_t launch_convert_f32(const double* frame, int64_t n, int32_t d, float* out, int32_t out_ld,
                              uint64_t* zero_max, hipStream_t s);

// Tile edges of the Gram kernels (columns per tile side).
constexpr int kTileF64 = 64;
constexpr int kTileF32 = 64;
constexpr int kTileBF16 = 128;

}  // namespace trstmi
