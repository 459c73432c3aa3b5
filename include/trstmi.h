/*
 * trstmi.h -- C ABI of the MI355X (gfx950) candidate-coherence library.
 *
 * The library implements the data-parallel hot path of a stochastic
 * trust-region search for low-coherence complex frames (Park, Saltijeral,
 * Zhong, "Grassmannian packings: Trust-region stochastic tuning for matrix
 * incoherence", arXiv:2207.06374):
 *
 *   - random start: N unit vectors in C^d (Alg. 2 step 1);
 *   - per step: C random perturbations of the frame inside the trust radius,
 *     column renormalisation (section IV remark: every column is divided by
 *     its norm), the Hermitian Gram of each candidate, and the fused
 *     reduction to the coherence mu = max_{j<k} |<phi_j, phi_k>| (section I;
 *     only the upper triangle is needed, section IV);
 *   - select the best candidate, accept it if it lowers mu, grow or shrink
 *     the radius.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Frame layout: a d x N complex frame is 2*d*N doubles, column-major with
 *   interleaved (re, im): entry (i, j) is at [2*(j*d + i)] (re) and
 *   [2*(j*d + i) + 1] (im).  Column j is the vector phi_j.
 * Memory: every pointer marked "device" is HIP device memory owned by the
 *   caller.  The library never allocates or frees device memory; scratch
 *   space comes from the caller's workspace buffer (see
 *   trstmi_workspace_bytes), 256-byte aligned.
 * Streams: every call is ordered on the given stream (0 = null stream) and
 *   returns without waiting for the GPU, except trstmi_solve, which polls a
 *   device flag once per chunk of steps.
 * Errors: every function returns a trstmi_status.  Argument errors are found
 *   on the host before anything is launched and leave device memory
 *   untouched.  A HIP launch failure returns TRSTMI_E_HIP.  The text of the
 *   last error of the calling thread is returned by trstmi_last_error().
 * Randomness: draws come from Philox4x32-10 (Salmon et al., SC'11) keyed by
 *   (seed, stream_id) with counter (block, candidate, step, tag); results are
 *   a pure function of the inputs and parameters.
 */
#ifndef TRSTMI_H
#define TRSTMI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t trstmi_status;
enum {
  TRSTMI_OK = 0,
  TRSTMI_E_INVALID_ARG = 1,   /* a size, pointer, mode or parameter is out of range */
  TRSTMI_E_WORKSPACE = 2,     /* workspace null, misaligned or smaller than required */
  TRSTMI_E_HIP = 3,           /* a HIP call failed (message in trstmi_last_error) */
  TRSTMI_E_UNSUPPORTED = 4    /* valid request this build does not handle */
};

/* Arithmetic of the candidate evaluation. */
enum {
  TRSTMI_MODE_FP64 = 0,        /* candidates and Gram in FP64 */
  TRSTMI_MODE_FP32 = 1,        /* candidates rounded to FP32, Gram in FP32 (MFMA) */
  TRSTMI_MODE_BF16_SCREEN = 2  /* all candidates screened from BF16 inputs (MFMA, FP32
                                  accumulate); the recheck_topk best screened ones are
                                  re-evaluated exactly in FP64 and only FP64 values decide.
                                  Steps in this mode need d <= 128 (else E_UNSUPPORTED). */
};

/* Bits of *state.flags. */
#define TRSTMI_FLAG_ACCEPTED 1  /* the last step accepted a candidate */
#define TRSTMI_FLAG_DONE 2      /* mu <= target_mu or step == max_steps; steps are no-ops */
#define TRSTMI_FLAG_NEAR_TIE 4  /* the last decision compared values closer than near_tie */
#define TRSTMI_FLAG_NO_VALID 8  /* the last step had no valid candidate */

/* Limits of this build. */
#define TRSTMI_MAX_D 512
#define TRSTMI_MAX_CANDIDATES 32768
#define TRSTMI_MAX_TOPK 64

/*
 * Parameters of a search.  Sizes: n = N >= 2 vectors, 1 <= d <= TRSTMI_MAX_D,
 * n * ceil(d/2) < 2^32.  candidates = C in [1, TRSTMI_MAX_CANDIDATES].
 * recheck_topk = k in [1, min(C, TRSTMI_MAX_TOPK)] (BF16 screen only).
 * seed and stream_id must be < 2^32.  Radius rule: on accept
 * radius <- min(grow * radius, radius_max), else radius <- max(shrink * radius,
 * radius_min); 0 < radius_min <= radius0 <= radius_max, grow >= 1,
 * 0 < shrink <= 1.  A step perturbs every column by radius in RMS norm:
 * Y_c = Phi + (radius / sqrt(d)) Z_c with Z_c i.i.d. CN(0, 1).
 * target_mu <= 0 disables the target; 0 <= max_steps <= 2^32 - 1 (the step
 * index is one 32-bit word of the random-number counter, so more steps would
 * repeat draws; larger values are rejected).  near_tie <= 0 selects
 * the mode's default (2e-12 for FP64 decisions, 4e-6 for FP32).
 */
typedef struct trstmi_params {
  int64_t n;
  int64_t d;
  int32_t candidates;
  int32_t mode;
  int32_t recheck_topk;
  int32_t reserved0;
  uint64_t seed;
  uint64_t stream_id;
  double radius0;
  double grow;
  double shrink;
  double radius_min;
  double radius_max;
  int64_t max_steps;
  double target_mu;
  double near_tie;
} trstmi_params;

/* Search state: all device pointers, caller-owned.  frame holds 2*d*n doubles
 * (layout above) with unit columns; mu, radius, step and flags are scalars. */
typedef struct trstmi_state {
  double* frame;
  double* mu;
  double* radius;
  int64_t* step;
  int32_t* flags;
} trstmi_state;

/* Optional per-step outputs (device pointers; each may be NULL).
 * cand_mu[C]   : each candidate's coherence as the mode computes it (FP64,
 *                FP32, or the BF16-screened value); +inf for an invalid
 *                candidate (a column of zero or non-finite norm).
 * rechecked[k] : BF16 screen: the candidates re-evaluated in FP64, in order
 *                of screened value (ties to the lower index).
 * recheck_mu[k]: their FP64 coherence.
 * best[1]      : the selected candidate c* (-1 if none was valid).
 * Nothing is written when the state is already DONE. */
typedef struct trstmi_report {
  double* cand_mu;
  int32_t* rechecked;
  double* recheck_mu;
  int32_t* best;
} trstmi_report;

/* Fills *p with defaults for a frame of n vectors in C^d: 64 candidates,
 * FP64, k = 8, seed 0, radius0 0.1, grow 2, shrink 0.5, radius range
 * [1e-12, 1], 1000 steps, no target. */
void trstmi_default_params(trstmi_params* p, int64_t n, int64_t d);

/* Bytes of workspace trstmi_init_haar / trstmi_step / trstmi_solve need for
 * these parameters (0 if the parameters are invalid). */
size_t trstmi_workspace_bytes(const trstmi_params* p);

/* Bytes of workspace trstmi_coherence needs for an n x d frame in this mode. */
size_t trstmi_coherence_workspace_bytes(int64_t n, int64_t d, int32_t mode);

/*
 * Coherence of a frame (section I): the columns of `frame` (device, layout
 * above, any nonzero scale) are normalised, then
 * *mu_out (device double) = max_{j<k} |<phi_j, phi_k>|.
 * mode FP64: exact up to rounding; FP32: Gram in FP32 from FP32-rounded unit
 * columns; BF16_SCREEN: the screened value from BF16-rounded unit columns.
 * A column whose norm is zero or not finite gives *mu_out = +inf.
 * Requires n >= 2, 1 <= d <= TRSTMI_MAX_D.
 */
trstmi_status trstmi_coherence(int64_t n, int64_t d, int32_t mode, const double* frame,
                               double* mu_out, void* workspace, size_t workspace_bytes,
                               hipStream_t stream);

/*
 * trstmi_coherence for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and result as trstmi_coherence, with the
 * workspace taken from a fixed device array inside the library instead of
 * the caller's buffer.  The array holds trstmi_coherence_noalloc_max_bytes()
 * bytes (16 MiB + 256: an FP64 frame with n * (2d rounded up to 8) <= 2^21,
 * e.g. N = 8192 at d = 128); larger frames return TRSTMI_E_UNSUPPORTED
 * before anything is launched.  Each GPU holds its own array for the life of
 * the process; the first call on a device looks up its address.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one device (different streams or threads without
 * ordering) race and must be serialised by the caller.  Arguments, errors
 * and stream ordering as trstmi_coherence.
 */
size_t trstmi_coherence_noalloc_max_bytes(void);
trstmi_status trstmi_coherence_noalloc(int64_t n, int64_t d, int32_t mode, const double* frame,
                                       double* mu_out, hipStream_t stream);

/*
 * A pair attaining the coherence (section I definition, FP64): *mu_out
 * (device) <- mu as trstmi_coherence computes it in TRSTMI_MODE_FP64, and
 * pair_out[0..1] (device int64) <- (j, k), j < k, the first pair in the
 * order j * n + k whose |<phi_j, phi_k>|^2 has exactly the bits of the
 * maximum (the pair is not unique in general; the value is).  A zero or
 * non-finite column gives +inf and (-1, -1).  Costs a second pass over the
 * Gram tiles.  Workspace: trstmi_coherence_workspace_bytes(n, d,
 * TRSTMI_MODE_FP64).  Stream-ordered.
 */
trstmi_status trstmi_coherence_pair(int64_t n, int64_t d, const double* frame, double* mu_out, int64_t* pair_out,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Bytes of workspace trstmi_lse needs for an n x d frame. */
size_t trstmi_lse_workspace_bytes(int64_t n, int64_t d);

/*
 * Smooth maximum of section IV (the shifted log-sum-exp the paper's
 * optimiser minimises; its Proposition bounds it by s <= F <= s + delta log n):
 * the columns of `frame` (device, layout above, any nonzero scale) are
 * normalised in FP64, x runs over the n = N(N-1)/2 values |G_jk|^2
 * (squared = 1) or |G_jk| (squared = 0), j < k, s = max x, and
 *   out[0] = s,  out[1] = F = s + delta log sum exp((x - s) / delta)
 * (out: device, 2 doubles), all in FP64.  The sum is added in a fixed order,
 * so repeated calls give the same bits.  A column whose norm is zero or not
 * finite gives out = (+inf, +inf).  delta must be finite and > 0.
 * Requires n >= 2, 1 <= d <= TRSTMI_MAX_D; workspace of
 * trstmi_lse_workspace_bytes(n, d) bytes, else TRSTMI_E_WORKSPACE.
 * Stream-ordered.
 */
trstmi_status trstmi_lse(int64_t n, int64_t d, const double* frame, double delta, int32_t squared,
                         double* out, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Tile choice of the BF16 screen (speed only: every result is the same
 * under any choice).  An entry applies to frames with ks = ceil(2d / 32) K
 * steps of 32 and n <= n_max (the entry with the smallest such n_max):
 * form 0 = blocks of 256 frame rows (64 per wavefront, ks <= 4), form 1 =
 * blocks of 128 rows (32 per wavefront); seg = column tiles of 128 one block
 * sweeps after loading its rows (1 .. 64).  Without an entry: form 0 with
 * runs of 6 for ks <= 4, form 1 with runs of 8 above.  The table is
 * process-wide and copied; it applies to steps, solves and server
 * admissions prepared after the call (count 0 clears it).  Written by
 * paper_2207_06374_amd.autotune from timings on the device.
 */
typedef struct {
  int32_t ks, n_max, form, seg;
} trstmi_screen_tile;
trstmi_status trstmi_screen_tiles_set(const trstmi_screen_tile* entries, int32_t count);

/* Bytes of workspace trstmi_lse_grad needs (0 if invalid or d > 64). */
size_t trstmi_lse_grad_workspace_bytes(int64_t n, int64_t d);

/*
 * The smooth maximum of trstmi_lse over x = |G_jk|^2 and its gradient with
 * respect to the unconstrained frame (section IV: the objective divides each
 * column by its norm, so the frame itself is the free variable of the
 * paper's trust-region minimisation): out (device, 2 doubles) = (s, F);
 * grad (device, same layout and size as frame) = g with
 *   dF = sum over entries of Re(conj(g) dframe),
 * g_k = 2 (D_k - phi_k Re(phi_k^H D_k)) / |frame_k|, D = Phi (W o G),
 * W_jk = exp((x_jk - s) / delta) / sum_{j<k} exp((x - s) / delta) (zero
 * diagonal).  FP64, fixed summation order (repeatable bits).  A zero or
 * non-finite column gives out = (+inf, +inf) and a NaN gradient.
 * Requires n >= 2, 1 <= d <= 64 (TRSTMI_E_UNSUPPORTED above), delta finite
 * and > 0; workspace of trstmi_lse_grad_workspace_bytes(n, d) bytes.
 */
trstmi_status trstmi_lse_grad(int64_t n, int64_t d, const double* frame, double delta, double* out,
                              double* grad, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Bytes of workspace trstmi_lse_hvp needs (0 if invalid or d > 64). */
size_t trstmi_lse_hvp_workspace_bytes(int64_t n, int64_t d);

/*
 * Exact Hessian-vector product of the smooth maximum over x = |G_jk|^2 with
 * respect to the unconstrained frame (section IV; Alg. 1 takes B_k to be the
 * Hessian of the objective): out (device, 2 doubles) = (s, F) as
 * trstmi_lse_grad gives them; hv (device, frame layout) = H v, the
 * derivative of trstmi_lse_grad's gradient at `frame` along the direction v
 * (device, frame layout), so that sum Re(conj(u) hv) is the second
 * derivative of F along u and v.  Forward differentiation of the gradient's
 * chain (column norms, Gram, |G|^2, the weights exp((x - s)/delta) / S, the
 * product Phi (W o G) and the projection through the normalisation), in FP64
 * with a fixed summation order (repeatable bits); S is summed in the same
 * pass from the same x as the weights, so they add up to one.  The
 * workspace size depends on n and d only.  A zero or non-finite
 * column gives out = (+inf, +inf) and a NaN product.  Requires n >= 2,
 * 1 <= d <= 64 (TRSTMI_E_UNSUPPORTED above), delta finite and > 0; workspace
 * of trstmi_lse_hvp_workspace_bytes(n, d) bytes.  Stream-ordered.
 */
trstmi_status trstmi_lse_hvp(int64_t n, int64_t d, const double* frame, const double* v, double delta,
                             double* out, double* hv, void* workspace, size_t workspace_bytes,
                             hipStream_t stream);

/* Exit of Steihaug CG (trstmi_tr_report.cg_exit). */
enum {
  TRSTMI_CG_SMALL_RESIDUAL = 0,      /* |r| < cg_tol: interior step */
  TRSTMI_CG_NEGATIVE_CURVATURE = 1,  /* d.Bd <= 0: to the boundary point with the lower model value */
  TRSTMI_CG_BOUNDARY = 2,            /* the next iterate would leave the region: stop on the boundary */
  TRSTMI_CG_MAX_ITER = 3,            /* cg_max_iter iterations */
  TRSTMI_CG_ZERO_GRADIENT = 4        /* |g| < cg_tol: no step */
};

typedef struct {
  double delta;       /* smoothing of the maximum, > 0 */
  double radius;      /* trust radius of this step, > 0 */
  double radius_max;  /* cap of the radius rule, >= radius */
  double eta;         /* the step is taken when rho > eta, 0 <= eta < 1/4 */
  double cg_tol;      /* residual norm that ends CG, > 0 */
  int32_t cg_max_iter;/* >= 1 */
  double fd_step;     /* 0: exact Hessian-vector products (trstmi_lse_hvp); > 0: central
                         differences of the gradient with this step instead */
} trstmi_tr_params;

typedef struct {
  double f_old, f_new;  /* F at the frame and at frame + step (f_new = f_old if no step was tried) */
  double rho;           /* actual / predicted decrease */
  double step_norm;
  double new_radius;    /* radius for the next step */
  int32_t cg_iters, cg_exit, accepted;
} trstmi_tr_report;

/* Bytes of workspace trstmi_tr_step needs (0 if invalid or d > 64). */
size_t trstmi_tr_workspace_bytes(int64_t n, int64_t d);

/*
 * One trust-region step of the paper's optimiser (section IV) on the smooth
 * maximum over |G|^2 of the unconstrained frame (device, in/out): Alg. 1,
 * Steihaug's truncated CG for min g.p + p.B p / 2 over |p| <= radius, read
 * with the textbook's completion of the printed listing (boundary test on
 * the new iterate, residual test on the new residual, the beta / direction
 * update; negative curvature goes to the boundary point with the lower
 * model value); B p exactly (B = the Hessian at the frame, trstmi_lse_hvp),
 * or by central differences of trstmi_lse_grad along p/|p| if fd_step > 0.
 * Then rho = (F(frame) - F(frame + p)) / (m(0) - m(p)); rho < 1/4 divides
 * the radius by 4, rho > 3/4 with |p| = radius doubles it (up to
 * radius_max), and frame <- frame + p when rho > eta.  *rep (host) gets
 * the outcome.  All vector work runs on the GPU (fixed-order dot products:
 * repeatable bits); the call synchronises the stream a few times per CG
 * iteration to read scalars.  Requires n >= 2, 1 <= d <= 64; a frame with
 * a zero or non-finite column returns TRSTMI_E_INVALID_ARG (frame unchanged).
 */
trstmi_status trstmi_tr_step(int64_t n, int64_t d, double* frame, const trstmi_tr_params* params,
                             trstmi_tr_report* rep, void* workspace, size_t workspace_bytes,
                             hipStream_t stream);

typedef struct {
  uint64_t seed;           /* random starts: stream l of this seed, l = 0 .. restarts - 1 */
  int32_t restarts;        /* L >= 1 (the paper uses L = 2 d^2) */
  int32_t n_deltas;        /* >= 1 */
  const double* deltas;    /* host array of n_deltas decreasing smoothing values, each > 0 */
  int32_t steps_per_delta; /* trust-region steps per delta, >= 1 */
  double radius0;          /* radius at the start of every delta, > 0 */
  double radius_min;       /* a delta ends when the radius falls below this, >= 0 */
  double radius_max;       /* >= radius0 */
  double eta;              /* 0 <= eta < 1/4 */
  double cg_tol;           /* > 0 */
  int32_t cg_max_iter;     /* >= 1, or 0 for 2 d N */
  double fd_step;          /* 0: exact Hessian-vector products; > 0: central differences */
  int32_t concurrency;     /* starts run at once (one host thread and stream each), 1 .. 64 */
  int32_t first_restart;   /* the starts are l = first_restart .. first_restart + restarts - 1, >= 0
                              (one run of L starts may be split into several calls) */
} trstmi_opt_params;

/* Bytes of workspace trstmi_optimize needs with `concurrency` starts in
 * flight (0 if invalid or d > 64). */
size_t trstmi_optimize_workspace_bytes(int64_t n, int64_t d, int32_t concurrency);

/*
 * The paper's outer procedure (Alg. 2): for each of L random starts (the
 * Haar start of trstmi_init_haar with stream_id l), minimise the smooth
 * maximum F_{s,delta_k} over |G|^2 with trust-region steps (trstmi_tr_step)
 * for the decreasing deltas in turn, each continuing from the previous
 * minimiser (a delta ends after steps_per_delta steps, when the radius
 * falls below radius_min, or when the gradient vanishes); then the exact
 * FP64 coherence of the result.  best_frame (device, caller's layout)
 * receives the frame with the smallest coherence, *best_mu and
 * *best_restart (host) its coherence and start index (the lowest index
 * among equal coherences).  With concurrency P > 1 the starts are dealt to
 * P host threads, each with a stream of its own (created and destroyed by
 * the call, after the caller's stream has drained; start l goes to thread
 * l mod P); every start computes exactly what it computes alone, so the
 * result does not depend on P.  Synchronises the stream.  Requires n >= 2,
 * 1 <= d <= 64, and a workspace of trstmi_optimize_workspace_bytes(n, d, P).
 */
trstmi_status trstmi_optimize(int64_t n, int64_t d, const trstmi_opt_params* params, double* best_frame,
                              double* best_mu, int32_t* best_restart, void* workspace,
                              size_t workspace_bytes, hipStream_t stream);

/* Bytes of workspace trstmi_optimize_batched needs for `restarts` starts (0
 * if n > 128, d > 16 or an argument is invalid). */
size_t trstmi_optimize_batched_workspace_bytes(int64_t n, int64_t d, int32_t restarts);

/*
 * The same procedure as trstmi_optimize (Alg. 2 around Alg. 1 steps with
 * exact Hessian products; the same parameters, starts and result) with every
 * start advanced by one block of a single launch: each block draws its
 * start, runs every delta's trust-region steps (Steihaug CG, ratio test,
 * radius rule) with all vector work and every scalar decision on the device,
 * and ends with the exact FP64 coherence of its frame; the host then picks
 * the least coherence (lowest start index among equal values) and copies
 * that frame to best_frame.  No host synchronisation inside the procedure,
 * one launch for all starts.  For n <= 128, d <= 16 (the frame and its
 * normalisation sit in one block's LDS); larger sizes and fd_step != 0 give
 * TRSTMI_E_UNSUPPORTED.  params->concurrency is ignored.  Every start
 * follows the oracle's step (rounding aside), so results match
 * trstmi_optimize's to rounding, not bit for bit.  Synchronises the stream.
 */
trstmi_status trstmi_optimize_batched(int64_t n, int64_t d, const trstmi_opt_params* params, double* best_frame,
                                      double* best_mu, int32_t* best_restart, void* workspace,
                                      size_t workspace_bytes, hipStream_t stream);

/* Bytes of workspace trstmi_miso_quantize needs (0 if a size is invalid). */
size_t trstmi_miso_workspace_bytes(int64_t n, int64_t d, int64_t m);

/*
 * Beamforming-codebook quantiser of section III (the MISO application): the
 * codebook is n codewords phi_i (columns, normalised here as section III
 * takes unit codewords), the channels are m vectors h_j in C^d; both in the
 * frame layout (device, column j at offset 2*d*j as interleaved re, im).
 * For every channel, written where the pointer is not NULL (device):
 *   index[j] = argmax_i |<phi_i, h_j>|^2 (the first of equal maxima),
 *   gain[j]  = that maximum (the received SNR in units of E_s / sigma),
 *   dist[j]  = 1 - gain[j] / |h_j|^2 (squared chordal distance from the line
 *              of h_j to its codeword, section II),
 * and summary[0..1] = the means of dist and gain over the m channels (a
 * Monte-Carlo estimate of the codebook's distortion and mean SNR gain when
 * the channels are CN(0, I_d) draws), added in a fixed order (NaN if m = 0).
 * <phi, h> = sum conj(phi_k) h_k, computed in FP64.  A codeword of zero or
 * non-finite norm gives index -1 and NaN gain and dist for every channel; a
 * channel whose squared norm is not finite gives -1 and NaN for that
 * channel; a zero channel has gain 0 at index 0 and a NaN dist.
 * Stream-ordered.  1 <= n <= 262144, 1 <= d <= 512, 0 <= m < 2^31;
 * codebook and channels 16-byte aligned; the workspace (device, 256-byte
 * aligned) holds the normalised codebook and the block sums.
 */
trstmi_status trstmi_miso_quantize(const double* codebook, int64_t n, int64_t d, const double* channels, int64_t m,
                                   int32_t* index, double* gain, double* dist, double* summary, void* workspace,
                                   size_t workspace_bytes, hipStream_t stream);

/*
 * Random start (Alg. 2 step 1): state->frame <- N normalised CN(0, I_d)
 * columns drawn with tag 1 (candidate 0, step 0); *mu <- its coherence
 * (FP32 Gram in FP32 mode, exact FP64 otherwise); *radius <- radius0;
 * *step <- 0; *flags <- DONE if the target is already met or max_steps == 0.
 */
trstmi_status trstmi_init_haar(const trstmi_params* p, const trstmi_state* state,
                               void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * The rounding the BF16 screen applies to its inputs (precision form of the
 * step): x[i] (device, count doubles) -> out[i] (device, count bfloat16 bit
 * patterns), round to nearest with ties to even, taken directly from the
 * double (as if with unbounded precision); subnormal bfloat16 results are
 * kept, a NaN gives a NaN.  Stream-ordered.  count >= 0; NULL or misaligned
 * pointers (count > 0) return TRSTMI_E_INVALID_ARG.
 */
trstmi_status trstmi_round_bf16(const double* x, int64_t count, uint16_t* out, hipStream_t stream);

/*
 * The normalised FP64 candidates of one step, for inspection: for
 * i = 0..count-1, out + i*2*d*n <- normalise(frame + (radius / sqrt(d)) Z)
 * with Z the draws of candidate (c0 + i) at step t (or explicit_z, see
 * trstmi_step, if not NULL).  frame and radius are device pointers.  A column
 * of zero or non-finite norm comes out as NaN.
 */
trstmi_status trstmi_candidates(const trstmi_params* p, const double* frame, const double* radius,
                                int64_t t, int32_t c0, int32_t count, const double* explicit_z,
                                double* out, hipStream_t stream);

/*
 * One step of the search on *state (no-op if DONE).  The trust region is the
 * one of Alg. 1 (section IV): a radius that grows after a successful step and
 * shrinks after a failed one; the objective is the coherence of section I
 * (largest modulus of an off-diagonal Gram entry of the column-normalised
 * frame, section IV).  The paper fixes neither the random perturbation nor the
 * radius constants; this step reads them as stated under trstmi_params.
 * Draws the C perturbations of step *step (or reads explicit_z: device,
 * C x 2*d*n doubles, candidate c at offset c*2*d*n, same layout as a frame),
 * renormalises, evaluates every candidate's coherence in the mode's
 * arithmetic, selects c* = argmin over (mu_c, c), accepts iff mu_{c*} < *mu,
 * updates frame, mu, radius, step and flags.  report may be NULL.
 * Invalid candidates (a column of zero or non-finite norm) are not an error:
 * their coherence is +inf and they never win; a step whose candidates are all
 * invalid rejects and sets TRSTMI_FLAG_NO_VALID.
 * Errors: TRSTMI_E_INVALID_ARG (parameters, NULL or misaligned state
 * pointers), TRSTMI_E_UNSUPPORTED (BF16 screen with d > 128),
 * TRSTMI_E_WORKSPACE, TRSTMI_E_HIP; nothing is launched on an error found on
 * the host.
 */
trstmi_status trstmi_step(const trstmi_params* p, const trstmi_state* state, void* workspace,
                          size_t workspace_bytes, const double* explicit_z,
                          const trstmi_report* report, hipStream_t stream);

/*
 * One run of the search from *state until DONE (the target coherence is met
 * or step == max_steps): the inner loop of one random start of Alg. 2
 * (section IV), with trstmi_step as the iteration.  Checks the device flag
 * after every `chunk` steps (chunk >= 1).  Launches of each chunk are
 * captured once into a HIP graph and replayed.  Blocks the calling thread;
 * returns after the stream has finished the last chunk.  The result equals
 * that of calling trstmi_step until DONE, bit for bit.
 * Errors: as trstmi_step; chunk < 1 gives TRSTMI_E_INVALID_ARG.
 */
trstmi_status trstmi_solve(const trstmi_params* p, const trstmi_state* state, void* workspace,
                           size_t workspace_bytes, int32_t chunk, hipStream_t stream);

/*
 * Batched form: `count` independent searches of different sizes advanced
 * together: per step, one persistent kernel launch evaluates every candidate
 * of every instance and one finalizing launch selects, accepts and commits
 * for every instance.  Instance i has its own
 * N_i, d_i, seed and stream (its draws are those of a single search with the
 * same seed and stream_id), its own frame, radius, step and flags, and its own
 * target / step limit; the candidate count, radius rule and near-tie threshold
 * are shared.  Every candidate is screened to FP32-class accuracy on the
 * BF16 matrix cores (each real rounded to FP32 and held as two bfloat16
 * parts hi + lo; Re and Im from hi hi' + hi lo' + lo hi'; certified error
 * below 5.5e-5 for unit columns) and the pairs that can attain its maximum are
 * re-evaluated in FP64, so each candidate's coherence, the selection and the
 * accept test are exact FP64 (each instance follows the FP64 single search;
 * its result does not depend on the other instances in the batch or on its
 * waves_per_item).
 * Limits: 2 <= n <= 256, 1 <= d <= 16, n * (ceil(2d/8)*8 + 4) <= 9216 * wpi / 4
 * (LDS words of a candidate's split copy), 1 <= candidates <= 256.  All state
 * lives in the caller's workspace.
 */
typedef struct trstmi_batch_instance {
  int32_t n;
  int32_t d;
  uint32_t seed;
  uint32_t stream_id;
  double target_mu;        /* <= 0: no target */
  int64_t max_steps;
  int32_t waves_per_item;  /* wavefronts per candidate: 1, 2 or 4; 0 = smallest that fits */
  int32_t reserved;
} trstmi_batch_instance;

typedef struct trstmi_batch_params {
  int32_t count;
  int32_t candidates;
  double radius0;
  double grow;
  double shrink;
  double radius_min;
  double radius_max;
  double near_tie;         /* <= 0: 2e-12 */
} trstmi_batch_params;

/* Workspace bytes for this batch (0 if invalid).  `inst` is a host array. */
size_t trstmi_batch_workspace_bytes(const trstmi_batch_params* p, const trstmi_batch_instance* inst);

/* Lays out the batch in the workspace and draws every instance's random start
 * (tag 1) with its exact FP64 coherence.  Copies `inst` (host) to the device
 * and returns after the copy; the rest is ordered on `stream`. */
trstmi_status trstmi_batch_init(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* `launches` steps of every not-yet-DONE instance (one kernel launch each).
 * rep_mu (device [count][candidates], nullable) receives the candidates'
 * FP64 coherences and rep_best (device [count], nullable) c* (-1: none), both
 * for the last launch. */
trstmi_status trstmi_batch_step(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                                size_t workspace_bytes, int32_t launches, double* rep_mu, int32_t* rep_best,
                                hipStream_t stream);

/* Steps until every instance is DONE or max_chunks chunks have run: `chunk`
 * step launches are captured once into a HIP graph (on a non-null stream) and
 * replayed; the DONE count is polled after each chunk.  *all_done (host,
 * nullable) is set to 1 if every instance finished. */
trstmi_status trstmi_batch_run(const trstmi_batch_params* p, const trstmi_batch_instance* inst, void* workspace,
                               size_t workspace_bytes, int32_t chunk, int64_t max_chunks, int32_t* all_done,
                               hipStream_t stream);

/* Copies the per-instance scalars to host arrays (each nullable) and waits
 * for the stream. */
trstmi_status trstmi_batch_query(const trstmi_batch_params* p, const trstmi_batch_instance* inst,
                                 const void* workspace, size_t workspace_bytes, double* mu, double* radius,
                                 int64_t* step, int32_t* flags, int32_t* done_instances, hipStream_t stream);

/* Copies instance i's frame (2 d_i n_i doubles, frame layout) to `out` (device). */
trstmi_status trstmi_batch_frame(const trstmi_batch_params* p, const trstmi_batch_instance* inst,
                                 const void* workspace, size_t workspace_bytes, int32_t i, double* out,
                                 hipStream_t stream);

/*
 * Kernel timing.  trstmi_timing_enable(1) makes every later kernel launch of
 * the library record a HIP event before and after it on the launch's stream
 * (launches under graph capture are not timed).  trstmi_timing_read waits for
 * the recorded events and returns, for one kernel name, the summed elapsed
 * milliseconds and the number of timed launches since the last reset.  Names:
 * "perturb", "gram_f64", "gram_f32", "gram_bf16", "topk", "perturb_recheck",
 * "recheck", "select", "commit", "batch_step".  trstmi_timing_only(name)
 * limits timing to launches of that kernel (NULL or "": every kernel), so
 * that the events of the others do not add to a measured step.  Process-wide
 * settings; returns TRSTMI_OK.
 */
trstmi_status trstmi_timing_enable(int32_t on);
trstmi_status trstmi_timing_only(const char* kernel);
trstmi_status trstmi_timing_reset(void);
trstmi_status trstmi_timing_read(const char* kernel, double* total_ms, int64_t* launches);

/* Message of the last failed call on this thread ("" if none). */
const char* trstmi_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving form: a solve server with continuous batching on one GPU.
 * Requests are queued on submission.  One engine thread (with a HIP stream
 * of its own, default priority) keeps a table of admitted requests in
 * device memory and advances all of them together: per step, each kernel of
 * the BF16-screen step (trstmi_step's) is launched once per group of
 * admitted requests with the same d, every request running exactly its own
 * single-search arithmetic.  After every `chunk` steps the engine reads back
 * every request's state in one copy, retires the finished ones and admits
 * the requests at the head of the queue into the freed rows as long as
 * their footprint fits in the caller's pool (first in line is served first;
 * a request larger than the pool is rejected at once).  While the admitted
 * set is unchanged a chunk is captured once into a HIP graph and replayed.
 * Each result is what trstmi_init_haar + trstmi_solve give for the same
 * request alone (its own seed and stream id), bit for bit, in any mix.
 * ------------------------------------------------------------------------- */
enum {
  TRSTMI_REQ_QUEUED = 0,
  TRSTMI_REQ_RUNNING = 1,
  TRSTMI_REQ_DONE = 2,     /* finished states from here on */
  TRSTMI_REQ_ERROR = 3,
  TRSTMI_REQ_REJECTED = 4,
  TRSTMI_REQ_CANCELLED = 5
};

typedef struct trstmi_server trstmi_server;  /* opaque */

typedef struct {
  void* pool;              /* device memory owned by the caller, 256-byte aligned, kept until destroy;
                              its first trstmi_server_table_bytes(slots) bytes hold the engine table,
                              the rest the admitted requests */
  uint64_t pool_bytes;     /* > trstmi_server_table_bytes(slots) + 256 */
  int32_t slots;           /* requests admitted at once (rows of the table), 1 .. 1024 */
  int32_t chunk;           /* steps between admissions and state read-backs, >= 1 */
  int32_t candidates;      /* per step, >= 1 */
  int32_t mode;            /* TRSTMI_MODE_BF16_SCREEN (others: TRSTMI_E_UNSUPPORTED) */
  int32_t recheck_topk;    /* BF16 screen: candidates re-evaluated in FP64, >= 1 */
  int32_t reserved0;
  double radius0;          /* > 0 */
  double target_factor;    /* default target = target_factor x Welch bound, >= 0 */
} trstmi_server_params;

typedef struct {
  int64_t n, d;
  uint64_t seed, stream_id;  /* the random start and perturbations (each < 2^32) */
  double target_mu;          /* NaN: target_factor x Welch(n, d); <= 0: no target */
  int64_t max_steps;
} trstmi_request;

typedef struct {
  int32_t status;          /* TRSTMI_REQ_* */
  int32_t reached;         /* done with mu <= target_mu */
  double mu;               /* exact FP64 coherence of the final frame (NaN until done) */
  int64_t steps;
  double target_mu;
  double queue_s;          /* submission to admission (NaN if never admitted) */
  double run_s;            /* admission to completion (NaN until finished) */
  uint64_t footprint;      /* bytes of the pool the request holds while it runs */
} trstmi_request_result;

typedef struct {
  uint64_t pool_capacity, pool_used, pool_peak;
  int32_t active, queued;
  int64_t submitted;
} trstmi_server_stats;

/* Bytes of pool one request with these parameters holds while it runs
 * (workspace, frame and state scalars, each rounded up to 256 bytes); 0 if
 * the parameters are invalid. */
size_t trstmi_request_footprint(const trstmi_params* p);

/* Bytes at the start of the pool that hold the engine table for `slots`
 * rows (0 if slots is out of range). */
size_t trstmi_server_table_bytes(int32_t slots);

/* Certified bounds on |screened - exact| coherence for unit columns in C^d
 * (section I's mu), used to prune the FP64 rechecks of the two
 * reduced-precision screens; host functions, no device is touched, NaN for
 * d out of range:
 *  - trstmi_bf16_screen_bound: the BF16-screen form (TRSTMI_MODE_BF16_SCREEN
 *    of trstmi_step and trstmi_solve, and the serving engine), d >= 1;
 *  - trstmi_batch_screen_bound: the batched form's split screen (FP32 values
 *    as hi + lo bfloat16 parts, three products), 1 <= d <= 16. */
double trstmi_bf16_screen_bound(int64_t d);
double trstmi_batch_screen_bound(int32_t d);

/* The Welch bound sqrt((n - d) / (d (n - 1))) (0 for n <= d; section II),
 * the default target of a request is target_factor times it.  NaN for
 * n < 2 or d < 1. */
double trstmi_welch_bound(int64_t n, int64_t d);

/* Starts a server (its engine thread and stream) on the current device;
 * *out receives it. */
trstmi_status trstmi_server_create(const trstmi_server_params* params, trstmi_server** out);

/* Queues a request; *id (host) receives its id.  A request that cannot run
 * (invalid sizes, or a footprint above the pool) is recorded as
 * TRSTMI_REQ_REJECTED with a message (read it through poll). */
trstmi_status trstmi_server_submit(trstmi_server* server, const trstmi_request* request, int64_t* id);

/* Current state of a request, without waiting.  For a request that ended in
 * an error or was rejected, trstmi_last_error() then holds its message. */
trstmi_status trstmi_server_poll(trstmi_server* server, int64_t id, trstmi_request_result* out);

/* Waits until the request has finished (any finished state) or timeout_s
 * seconds have passed (timeout_s < 0: no limit), then reports as poll. */
trstmi_status trstmi_server_wait(trstmi_server* server, int64_t id, double timeout_s,
                                 trstmi_request_result* out);

/* Removes a still-queued request (TRSTMI_E_INVALID_ARG once it runs). */
trstmi_status trstmi_server_cancel(trstmi_server* server, int64_t id);

/* Drops the record of a finished request (any finished state), so that a
 * long-running server does not keep every result; its id is then unknown. */
trstmi_status trstmi_server_forget(trstmi_server* server, int64_t id);

/* Pool use (now and peak), running and queued requests, submissions. */
trstmi_status trstmi_server_get_stats(trstmi_server* server, trstmi_server_stats* out);

/* Lets the running requests finish, cancels the queued ones, joins the
 * engine thread and frees the server (the pool stays the caller's). */
trstmi_status trstmi_server_destroy(trstmi_server* server);

/* Releases the library's internal state (the pooled HIP events of kernel
 * timing, after waiting for any still pending; totals are cleared and timing
 * is switched off).  Call it before the process releases its devices; the
 * library stays usable and recreates what it needs on demand. */
trstmi_status trstmi_shutdown(void);

/* ABI version of this library (increases when a declaration changes). */
int32_t trstmi_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TRSTMI_H */
