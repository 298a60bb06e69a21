/*
 * msld.h -- C ABI of the MI355X (gfx950) multi-scale low-rank decomposition library.
 *
 * The library solves the convex multi-scale low-rank decomposition (Ong & Lustig,
 * "Beyond Low Rank + Sparse: Multi-scale Low Rank Matrix Decomposition", Sec. 3,
 * eq:cvx):
 *     minimise  sum_i lambda_i ||X_i||_(i)   subject to  sum_i X_i = Y,
 * where ||.||_(i) is the sum of nuclear norms of the m_i x n_i blocks of scale i,
 * with the ADMM iteration of Sec. 7 (eq:admm): a consensus X-update, a block-wise
 * singular value soft-threshold (eq:svt, eq:bsvt) per scale, and a scaled dual
 * update, optionally with the random cycle spinning of Sec. 9.
 *
 * Conventions for every entry point:
 *   - Matrices are float32, row-major. "d_" pointers are HIP device pointers on the
 *     device that is current when the call is made; other pointers are host memory.
 *   - Work is enqueued on the HIP stream given at msld_create (NULL = legacy default
 *     stream) and is stream-ordered; a call returns before the GPU work ends unless
 *     it says otherwise.
 *   - The caller owns every buffer it passes; the library never frees them. The
 *     library owns its handle and workspace (allocated in msld_create, released in
 *     msld_free).
 *   - Errors: invalid arguments return MSLD_EINVAL before anything is enqueued. A
 *     failing HIP call returns MSLD_EDEVICE and marks the handle failed: later
 *     calls on it return MSLD_EDEVICE. No C++ exception crosses this interface.
 *   - A handle must not be used from two host threads at once; distinct handles
 *     may run concurrently on distinct streams.
 */
#ifndef MSLD_H
#define MSLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSLD_MAX_SCALES 16

typedef enum {
  MSLD_OK = 0,
  MSLD_EINVAL = -1,    /* invalid argument or parameter set */
  MSLD_ENOMEM = -2,    /* device or host allocation failed */
  MSLD_EDEVICE = -3,   /* a HIP runtime call failed; the handle is now unusable */
  MSLD_ENUMERIC = -4,  /* the iterate became non-finite (NaN/Inf in Y or overflow) */
  MSLD_EBUSY = -5,     /* reserved for queue-full conditions */
  MSLD_ETOOLARGE = -6  /* the problem exceeds a fixed capacity (msld_bsvt_noalloc) */
} msld_status;

/* Problem and solver parameters (Sec. 2 partition, Sec. 4 lambda, Sec. 7 ADMM,
 * Sec. 9 cycle spinning).
 *   M, N        : Y is M x N, 1 <= M, N <= 2^20 and M*N < 2^31.
 *   L           : number of scales, 1 <= L <= MSLD_MAX_SCALES.
 *   block_m/n[i]: block size of scale i. Must divide M and N (contiguous tiling of
 *                 the partition of Sec. 2); (M, N) is the single full-size block.
 *                 Any shape that tiles M x N is accepted; 1 x 1 scales are
 *                 soft-thresholded inside the consensus pass.
 *   lambda[i]   : weight of scale i, > 0; a value <= 0 selects the default of the
 *                 boxed rule eq:lambda, sqrt(m)+sqrt(n)+sqrt(ln(MN/max(m,n))).
 *   rho         : ADMM parameter, > 0; scale i thresholds at lambda_i / rho.
 *   max_iters   : iteration count K (tol == 0) or cap (tol > 0), >= 1.
 *   tol         : 0 runs exactly max_iters iterations; > 0 also stops after
 *                 iteration k when (k+1) % check_every == 0 and the primal residual
 *                 r_k = sqrt(sum_i ||X_i - Z_i||_F^2) / ||Y||_F is <= tol.
 *   check_every : >= 1, residual cadence when tol > 0.
 *   cycle_spin  : 0 = fixed partition; 1 = random cycle spinning: scale i at
 *                 iteration k uses shift msld_cycle_shift(shift_seed, k, i, ...).
 *   shift_seed  : seed of the counter-based shift hash.
 *   lowrank_min : blocks whose shorter side is >= this use the certified low-rank
 *                 SVT (subspace iteration on the Gram matrix, one-sided Jacobi on the
 *                 reduced block, and an a-posteriori certificate that bounds the
 *                 error by the non-expansiveness of the prox; blocks that fail it
 *                 get an exact SVT: the LDS Jacobi tier, or the polar route for
 *                 blocks too large for LDS). Blocks up to 128 x 128 use a fused
 *                 one-kernel version. 0 selects the default (32); a negative value
 *                 disables the path. Blocks of 16 to 31 columns too tall for the LDS
 *                 and panel tiers (more than about 4800 rows) take it as well.
 *                 Results agree to rounding.
 *   kind[i]     : MSLD_KIND_BLOCK (0): block-wise nuclear norm over the partition;
 *                 MSLD_KIND_NOISE (1): the noise scale of Sec. 2, whose reshape takes
 *                 the whole matrix to an MN x 1 vector, so its norm is the Frobenius
 *                 norm and its Z-step z = v max(1 - tau / ||v||_F, 0); requires
 *                 block (M, N); no shift applies; the default lambda is eq:lambda on
 *                 the MN x 1 block, sqrt(MN) + 1. Zero-initialised params mean all 0.
 *   spin_count  : cycle spinning of Sec. 9 as an average (needs cycle_spin = 1).
 *                 0 or 1: one random shift per scale and iteration (above). c > 1:
 *                 the Z-step of every block scale other than 1 x 1 is the mean of
 *                 Shift_{-s}(BlockSVT(Shift_s(V))) over a shift set S. An axis the
 *                 block spans whole (m = M or n = N) has one distinct shift (a cyclic
 *                 shift only permutes inside each block there), so there are
 *                 mr x nc distinct shifts, mr = (m == M ? 1 : m), nc likewise. When
 *                 c >= mr nc, S is all of them in row-major order (full cycle
 *                 spinning, translation invariant); else the c shifts
 *                 msld_cycle_shift(shift_seed + j, k, i, ...), j = 0..c-1. Scales
 *                 with mr nc = 1 keep the single random shift. Costs |S| BlockSVTs
 *                 per averaged scale and iteration and two more M x N planes.
 *                 Must be >= 0.
 *   image_w     : for space-time scales: the rows of Y are the pixels of an
 *                 H x image_w image in row-major order (row y * image_w + x; M must
 *                 be H * image_w) and the columns are frames. 0 when unused.
 *   patch_w[i]  : MSLD_KIND_SPATIAL (2) scales (the general block reshape R_b of
 *                 Sec. 2, as in the video and DCE experiments of Sec. 10): a block is
 *                 a ph x pw pixel patch (pw = patch_w[i], ph = block_m[i] / pw) over
 *                 block_n[i] consecutive frames, reshaped to block_m[i] x block_n[i]
 *                 (block row dy * pw + dx is pixel (y0 + dy, x0 + dx)); pw must
 *                 divide block_m[i] and image_w, ph must divide H. Cycle spinning
 *                 shifts the video cyclically in (y, x, t); the hashed row residue
 *                 s_r in [0, ph pw) gives (sy, sx) = (s_r / pw, s_r % pw). Other
 *                 kinds ignore patch_w.
 *   fork_mode   : where the scales' BlockSVT work forks from the main stream (results
 *                 are identical, only the schedule changes): 0 = automatic (each
 *                 scale right after its own stream pass on planes of at most 2^24
 *                 elements, one fork after every pass on larger planes); 1 = always
 *                 right after each scale's own pass; 2 = always one fork after every
 *                 pass; 3 = no fork: every scale's BlockSVT runs on the handle's
 *                 stream, one scale after another (no two kernels of an iteration
 *                 overlap, so phase timings are each kernel's own). Other values:
 *                 MSLD_EINVAL. */
#define MSLD_KIND_BLOCK 0
#define MSLD_KIND_NOISE 1
#define MSLD_KIND_SPATIAL 2
typedef struct msld_params {
  int32_t M, N, L;
  int32_t block_m[MSLD_MAX_SCALES];
  int32_t block_n[MSLD_MAX_SCALES];
  float lambda[MSLD_MAX_SCALES];
  float rho;
  int32_t max_iters;
  float tol;
  int32_t check_every;
  int32_t cycle_spin;
  int32_t lowrank_min;
  uint64_t shift_seed;
  int32_t kind[MSLD_MAX_SCALES];
  int32_t spin_count;
  int32_t image_w;
  int32_t patch_w[MSLD_MAX_SCALES];
  int32_t fork_mode;
} msld_params;

/* Outcome of one msld_solve. primal_resid is r_k of the last iteration run
 * (computed when info is requested); dual_resid is rho ||Z^k - Z^(k-1)||_F / ||Y||_F
 * over all scales for that iteration (the change of the block-low-rank components,
 * the dual residual of ADMM; reported only, it stops nothing), -1 when not computed.
 * status is MSLD_ENUMERIC when Y holds a NaN or Inf (checked before the first
 * iteration) or the residual became non-finite. live[i] counts the blocks of scale i that
 * passed the singular-value bound test and were decomposed, summed over all
 * iterations; sweeps[i] sums the Jacobi sweeps run on them; rank[i] sums the
 * output ranks; certified[i] counts the blocks finished by the certified low-rank
 * path (the rest of live[i] ran full Jacobi); fail_coupling[i] / fail_bound[i]
 * count the blocks that path handed to Jacobi, by the test they failed. */
typedef struct msld_result {
  int32_t iters;
  int32_t status;
  double primal_resid;
  double dual_resid;
  uint64_t live[MSLD_MAX_SCALES];
  uint64_t sweeps[MSLD_MAX_SCALES];
  uint64_t rank[MSLD_MAX_SCALES];
  uint64_t certified[MSLD_MAX_SCALES];
  uint64_t fail_coupling[MSLD_MAX_SCALES];
  uint64_t fail_bound[MSLD_MAX_SCALES];
  uint64_t polar[MSLD_MAX_SCALES];        /* failed certificates finished by the polar route */
  uint64_t polar_steps[MSLD_MAX_SCALES];  /* its Newton-Schulz steps (polar + sign, per chunk) */
  uint64_t undecided[MSLD_MAX_SCALES];    /* low-rank blocks whose certificate needed the
                                             remainder Gram E^T E (the trace bound left them
                                             undecided) */
  uint64_t cw_certified[MSLD_MAX_SCALES]; /* of those, certified by the Collatz-Wielandt
                                             bound where the Frobenius bound alone failed */
  uint64_t gram_certified[MSLD_MAX_SCALES]; /* low-rank blocks certified to have no singular
                                               value above tau by the Collatz-Wielandt
                                               bound of their Gram matrix, before any
                                               subspace iteration (output zero) */
} msld_result;

typedef struct msld_solver msld_solver; /* opaque */

/* Validate p, plan the kernels of every scale and allocate the workspace on the
 * current device. hip_stream is a hipStream_t (NULL = default stream). On success
 * *out holds a new handle; on failure *out is NULL.
 * Each decomposed scale runs its BlockSVT on a stream the handle creates (forked from
 * and joined back into hip_stream every iteration). Streams run side by side only on
 * hardware queues of their own: HIP takes the count per process from the environment
 * variable GPU_MAX_HW_QUEUES (default 4) when it initialises. When the scale streams
 * outnumber the queues left beside the caller's, the low-rank scales' streams are
 * created first so that their long chains get queues of their own. */
msld_status msld_create(const msld_params *p, void *hip_stream, msld_solver **out);

/* Run the ADMM of eq:admm on Y (M x N, leading dimension ldY >= N, device) and
 * write the components Z_1..Z_L to d_Z (L x M x N contiguous, device, caller-owned;
 * it also serves as the iterate, so it must not alias d_Y). Starts from
 * Z_i = U_i = 0. If info is non-NULL the call synchronises the stream and fills
 * *info; with tol > 0 the call always synchronises (it reads the residual back).
 * Returns MSLD_ENUMERIC when the residual it reads back is not finite. */
msld_status msld_solve(msld_solver *s, const float *d_Y, int64_t ldY, float *d_Z,
                       msld_result *info);

/* Set the iterate to the ADMM starting point Z_i = U_i = 0 (d_Z is zeroed, the
 * internal D planes too), the iteration counter k to 0 and the statistics to 0. */
msld_status msld_reset(msld_solver *s, float *d_Z);

/* Run `count` >= 1 further ADMM iterations k, k+1, ... (k continues from the last
 * msld_reset / msld_step / msld_solve on this handle; cycle-spin shifts follow k)
 * on the iterate held in d_Z (L x M x N, device) and the handle's D planes. If
 * resid is non-NULL, the primal residual r of the last iteration is written to
 * *resid (host) and the call synchronises; MSLD_ENUMERIC if r is not finite. Pass
 * the same d_Y / d_Z as the msld_reset that started the run. */
msld_status msld_step(msld_solver *s, const float *d_Y, int64_t ldY, float *d_Z,
                      int32_t count, double *resid);

/* Iteration count and per-scale live / sweep / rank counters accumulated since the
 * last msld_reset (primal_resid is -1: use msld_step to obtain it). Synchronises. */
msld_status msld_stats(msld_solver *s, msld_result *info);

/* Autotuner of the BlockSVT launch choice per block size (not a step of the paper).
 * Times, on the current device and the given stream, the tiers and launch shapes that
 * apply to m x n blocks (register tier; fused certified low-rank kernel with first
 * subspace width p or 2p; LDS Jacobi tier with at most 1, 2, 4 or as many workgroups
 * per compute unit as fit; certified low-rank path on batched GEMMs), one block-wise
 * SVT call each on a synthetic matrix of up to 4096 such blocks (rank-1 blocks at about
 * twice the threshold on half of them, small noise), and records the fastest in a
 * process-wide cache keyed by (m, n, device architecture). Solvers, batches and server
 * classes created afterwards use the cached choice for every scale of that block size
 * (alone or in a batch alike; a plan's lowrank_min < 0 still excludes the low-rank
 * tiers), so results do not depend on batch composition; all candidates compute the
 * same block-wise SVT up to rounding. m, n in [1, 4096], not both 1. Allocates device
 * memory while it runs; call it when no solver is being created on another thread.
 * Errors: MSLD_EINVAL, MSLD_ENOMEM, MSLD_EDEVICE (no candidate could be timed). */
typedef struct msld_tune_result {
  int32_t tier;        /* chosen tier, msld_scale_tier numbering */
  int32_t lds_cap;     /* LDS tier: workgroups per compute unit (0: as many as fit) */
  int32_t lrs_wide;    /* fused low-rank kernel: 1 = first pass with 2p (no retry pass) */
  int32_t candidates;  /* configurations timed */
  float us_per_block;  /* time of the chosen one, microseconds per block */
  float us_default;    /* time of the built-in choice, microseconds per block */
} msld_tune_result;
msld_status msld_autotune(int32_t m, int32_t n, void* hip_stream, msld_tune_result* out);

/* Forget every autotuned choice; plans created afterwards use the built-in choice. */
void msld_autotune_clear(void);

/* Iterations as HIP graphs (not a step of the paper: launch overhead). When no scale
 * of the plan takes the low-rank path with blocks beyond the LDS Jacobi tier (its polar
 * fallback reads the failure count and per-block scalars on the host to size its step
 * counts), msld_step, msld_solve and msld_batch_solve capture one ADMM
 * iteration per D-buffer parity into a HIP graph on first use and replay it for every
 * iteration whose residual is not read; the shift seed and iteration counter then live
 * on the device. Graphs are keyed by the Y and Z buffers and the mask; new buffers are
 * captured again. Results equal those of plain launches.
 * enable != 0 allows graphs (the default), 0 forces plain launches. Returns 1 if
 * iterations will be replayed from graphs, 0 if not (disabled, or the plan needs host
 * waits), or a negative msld_status. Synchronises the solver's stream. */
int32_t msld_set_graph(msld_solver* s, int32_t enable);

/* Masked data consistency (the collaborative-filtering variant of Sec. 10): with a
 * mask set, the X-update of eq:admm applies its consensus correction only on observed
 * entries and keeps X_i = Z_i - U_i on the others, so the constraint sum_i X_i = Y
 * holds on the observed entries only; unobserved entries of Y are never read into
 * the iteration and the residual is relative to ||P_observed(Y)||_F. d_mask is an
 * M x N row-major byte array on the device (nonzero = observed), leading dimension
 * ldmask >= N; it is caller-owned and must stay valid for every msld_solve /
 * msld_reset / msld_step that follows. NULL clears the mask. Single solvers only
 * (MSLD_EINVAL for batch / server classes). */
msld_status msld_set_mask(msld_solver *s, const uint8_t *d_mask, int64_t ldmask);

/* Kernel timing with HIP events on the streams that run each part (the consensus on
 * the handle's stream, each scale on its own stream). msld_profile_begin(s, n)
 * creates events for the next n iterations (each iteration records them as it is
 * enqueued; later iterations are not recorded). msld_profile_end synchronises and
 * returns elapsed milliseconds summed over the recorded iterations in
 * ms[(L + 1) * 4 + L]: ms[4L] the consensus pass, ms[4L + 1] the stream pass of all
 * decomposed scales (one launch: shifted gather, bound test, speculative write);
 * for scale i, ms[4i + 1] the rest of the set-up (bound reduction, panel load),
 * ms[4i + 2] the SVD kernels (register / LDS / fused low-rank kernel, the batched
 * low-rank path, or all panel-round launches), ms[4i + 3] the rest (fallbacks,
 * gains, rebuild); ms[4i + 0] stays 0 (the stream pass is shared); ms[4(L + 1) + i]
 * the Gram kernel B^T B alone of a low-rank scale (inside ms[4i + 2]). Scales run
 * concurrently, so their times overlap. round_launches[L] receives the number of panel-round
 * kernel launches per scale, *iters_recorded the number of iterations covered. */
msld_status msld_profile_begin(msld_solver *s, int32_t max_iters);
msld_status msld_profile_end(msld_solver *s, double *ms, int64_t *round_launches,
                             int32_t *iters_recorded);

/* One block-wise SVT call with scale `scale`'s block shape and an explicit shift
 * (Sec. 7 eq:bsvt with Sec. 9 Shift): d_Z = Shift_{-s}(BSVT_tau(Shift_s(d_V))),
 * where Shift_s(A)[r][c] = A[(r+sr) mod M][(c+sc) mod N]. d_V and d_Z are M x N
 * contiguous device buffers; they may alias. 0 <= sr < block_m, 0 <= sc < block_n.
 * Uses the handle's workspace, so it must not overlap a msld_solve on the handle. */
msld_status msld_bsvt(msld_solver *s, int32_t scale, const float *d_V, float *d_Z,
                      float tau, int32_t sr, int32_t sc);

/* Release the handle and its workspace (waits for the handle's stream). NULL-safe. */
void msld_free(msld_solver *s);

/* Bytes of device workspace msld_create allocates for p (0 if p is invalid). */
size_t msld_workspace_bytes(const msld_params *p);

/* Human-readable name of a status code (static string). */
const char *msld_status_string(int32_t status);

/* Default weight of eq:lambda for an m x n block of an M x N matrix (host). */
msld_status msld_default_lambda(int32_t M, int32_t N, int32_t m, int32_t n, float *out);

/* Cycle-spin shift of scale i at iteration k (host computation; Sec. 9). The paper
 * leaves the draw unspecified; the library uses the SplitMix64 output mix
 * (Steele, Lea & Flood 2014) of seed + 0x9E3779B97F4A7C15 * (16k + i + 1) modulo
 * 2^64, and takes sr = (z >> 32) mod m, sc = (z mod 2^32) mod n. k >= 0,
 * 0 <= i < 16. */
msld_status msld_cycle_shift(uint64_t seed, int32_t k, int32_t i, int32_t m, int32_t n,
                             int32_t *sr, int32_t *sc);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the block-wise SVT of msld_bsvt
 * without a handle, d_Z = Shift_{-s}(BSVT_tau(Shift_s(d_V))) with m x n blocks, on the
 * caller's stream (NULL = legacy default stream), enqueued and not waited for. It calls
 * no allocating routine: its workspace (an M x N dual plane, the live-block list, bound
 * partials, counters) is a fixed 32 MiB device array inside the library, held by every
 * device the function runs on until the process ends, and every call on a device
 * shares it, so calls that overlap on one device (concurrent streams or threads) race:
 * serialise them. d_V and d_Z are M x N row-major device buffers of the current device
 * and may alias; 0 <= sr < m, 0 <= sc < n, tau >= 0. Block shapes of the register and
 * LDS tiers only (the blocks msld_bsvt decomposes with full one-sided Jacobi when its
 * handle has lowrank_min < 0); 1 x 1 blocks and blocks too large for LDS return
 * MSLD_EINVAL, a workspace beyond the 32 MiB (about M N <= 7 million elements, less for
 * tall blocks) returns MSLD_ETOOLARGE, both before anything is enqueued. Results equal
 * msld_bsvt's on a handle with lowrank_min < 0 bit for bit. */
msld_status msld_bsvt_noalloc(int32_t M, int32_t N, int32_t m, int32_t n, const float *d_V,
                              float *d_Z, float tau, int32_t sr, int32_t sc, void *hip_stream);

/* The same shifts computed by device code (the code the kernels run), for
 * count consecutive iterations k0..k0+count-1 of every scale of the handle's
 * ladder: out[(k - k0) * L * 2 + i * 2 + {0,1}] = (sr, sc). out is host memory of
 * 2 * L * count ints; the call synchronises. count >= 1. */
msld_status msld_device_shifts(msld_solver *s, int32_t k0, int32_t count, int32_t *out);

/* ------------------------------------------------------------------ batches
 * Many independent decompositions (of uneven sizes and ladders) solved together.
 * Instances whose parameters agree except for shift_seed form a class; the
 * instances of a class are stacked along the rows of one set of planes, so each
 * kernel of an ADMM iteration is launched once per class for all its instances and
 * the low-rank path's GEMMs are batched across them. Every instance keeps its own
 * shift seed (its cycle-spin shifts are those of a single solve with that seed), its
 * own iteration count and residual test, so its result equals its solve alone. */
typedef struct msld_batch msld_batch;

/* Plan n >= 1 instances (params[0..n-1], host array) and allocate their workspace
 * on the current device; work runs on hip_stream. */
msld_status msld_batch_create(int32_t n, const msld_params *params, void *hip_stream,
                              msld_batch **out);

/* Number of classes (stacked launch groups) of the batch, -1 for NULL. */
int32_t msld_batch_classes(const msld_batch *b);

/* Solve every instance i from Z = U = 0: d_Y[i] (M_i x N_i, leading dimension
 * ldY[i], device) in, d_Z[i] (L_i x M_i x N_i, device) out. d_Y, ldY, d_Z and info
 * are host arrays of n entries (info may be NULL). An instance with tol > 0 stops at
 * its own tolerance. Synchronises the stream. */
msld_status msld_batch_solve(msld_batch *b, const float *const *d_Y, const int64_t *ldY,
                             float *const *d_Z, msld_result *info);

void msld_batch_free(msld_batch *b);   /* NULL-safe */

/* ------------------------------------------------------------------ serving
 * Continuous batching of independent decompositions (a request loop). Requests wait
 * in a FIFO queue and are admitted, in order, while fewer than max_active are
 * running: a request takes a free slot of a class (a stacked solver for its problem
 * shape, min(max_active, 8) slots, as in the batches above); a new class is created
 * when its HBM footprint (workspace plus stacked Y and Z planes) fits in
 * hbm_budget_bytes, after releasing idle classes if needed. Each msld_server_step
 * runs one ADMM iteration (Sec. 7 eq:admm, from Z = U = 0) for all active slots of
 * each class with one set of launches (classes on the server's num_streams streams),
 * reads the per-slot residuals back, and retires every request whose residual is
 * <= its tol (checked every check_every iterations) or that reached max_iters,
 * copying its Z planes to the request's buffer. A request's result is the same
 * alone and in any mix: slots are independent instances of deterministic kernels. */
typedef struct msld_server msld_server;

/* max_active >= 1, hbm_budget_bytes > 0, 1 <= num_streams <= 64; streams are created
 * at the default priority on the current device. */
msld_status msld_server_create(int32_t max_active, size_t hbm_budget_bytes,
                               int32_t num_streams, msld_server **out);

/* Queue one request. d_Y (M x N, leading dimension ldY) and d_Z (L x M x N) are
 * caller-owned device buffers that must stay valid until the request is reported
 * done; d_Z receives Z_1..Z_L. MSLD_EINVAL if p is invalid or the footprint exceeds
 * the whole budget. Does not touch the device. */
msld_status msld_server_submit(msld_server *sv, const msld_params *p, const float *d_Y,
                               int64_t ldY, float *d_Z, int64_t request_id);

/* Admit, advance every active request by one iteration, retire, and report up to
 * max_out finished requests (id, iterations run, last residual, status) in the
 * caller's host arrays; *n_done receives the count, *n_active the running requests
 * and *n_queued the requests still waiting (plus finished ones not yet reported).
 * Synchronises the streams of requests due for a residual check. */
msld_status msld_server_step(msld_server *sv, int64_t *done_ids, int32_t *done_iters,
                             double *done_resid, int32_t *done_status, int32_t max_out,
                             int32_t *n_done, int32_t *n_active, int32_t *n_queued);

/* HBM bytes a server with this max_active charges against its budget for the class
 * of problem p (workspace plus stacked Y and Z planes of min(max_active, 8) slots),
 * as used by admission. Host only. MSLD_EINVAL if p is invalid. */
msld_status msld_server_class_bytes(const msld_params *p, int32_t max_active, size_t *out);

/* Free the server, its streams and the workspace of requests still active. NULL-safe. */
void msld_server_free(msld_server *sv);

/* Kernel tier the plan chose for scale i: 0 = 1x1 (fused in the consensus pass),
 * 1 = register tier (blocks up to 8 x 8), 2 = LDS tier, 3 = HBM panel tier,
 * 4 = certified low-rank path on batched GEMMs (failures: LDS tier or polar route),
 * 5 = fused certified low-rank kernel for blocks up to 64 x 128 (failures: LDS
 * tier), 6 = noise scale (Frobenius prox). Returns -1 for an invalid index. */
int32_t msld_scale_tier(const msld_solver *s, int32_t scale);

#ifdef __cplusplus
}
#endif
#endif /* MSLD_H */
