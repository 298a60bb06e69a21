// Internal declarations shared by the HIP kernels and the C-ABI runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/msld.h"

namespace msld {

// ---------------------------------------------------------------- shift hash
// Cycle-spin shift of scale i at iteration k (Sec. 9, random cycle spinning).
// Counter-based: SplitMix64 output mix (Steele, Lea & Flood 2014) of
// seed + 0x9E3779B97F4A7C15 * (16 k + i + 1) mod 2^64; rows use the high 32 bits,
// columns the low 32 bits, each reduced modulo the block size. One definition is
// compiled for host and device so the kernels and msld_cycle_shift agree bit for bit.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline void cycle_shift(uint64_t seed, int k, int i, int m, int n,
                                            int* sr, int* sc) {
  const uint64_t ctr = 16ull * (uint64_t)k + (uint64_t)i + 1ull;
  const uint64_t z = mix64(seed + 0x9E3779B97F4A7C15ull * ctr);
  *sr = (int)((z >> 32) % (uint64_t)m);
  *sc = (int)((z & 0xFFFFFFFFull) % (uint64_t)n);
}

// Shift of one scale for one launch: none, hashed from (seed, k, scale) on device,
// or explicit (sr, sc). Several independent instances of one shape can be stacked
// along the rows of one set of planes; then each instance z has its own seed and
// iteration counter (iseed[z], ik[z], device arrays) and an active flag.
struct ShiftSpec {
  uint64_t seed;
  int k;          // iteration
  int scale;      // scale index i
  int mode;       // 0: none, 1: hashed from (seed, k, scale), 2: explicit (sr, sc)
  int sr, sc;
  const unsigned long long* iseed;  // per-instance seeds (null: seed)
  const int* ik;                    // per-instance iteration (null: k)
  const int* iactive;               // per-instance active flag (null: all active)
  uint64_t seed_add = 0;            // added to the seed in mode 1 (j-th shift of a spin set)
};

__device__ inline void block_shift(const ShiftSpec& s, int z, int m, int n, int* sr, int* sc) {
  if (s.mode == 1) {
    const uint64_t seed = (s.iseed ? (uint64_t)s.iseed[z] : s.seed) + s.seed_add;
    const int k = s.ik ? s.ik[z] : s.k;
    cycle_shift(seed, k, s.scale, m, n, sr, sc);
  } else if (s.mode == 2) {
    *sr = s.sr;
    *sc = s.sc;
  } else {
    *sr = 0;
    *sc = 0;
  }
}

// One-sided Jacobi rotation test for a column pair with squared norms al, be and inner
// product ga: rotate while |ga| > tol sqrt(al) sqrt(be). A threshold needs no correctly
// rounded square root, so the hardware one (one instruction) serves.
__device__ inline bool jacobi_rotates(float ga, float al, float be, float tol) {
  return fabsf(ga) > tol * __builtin_amdgcn_sqrtf(al) * __builtin_amdgcn_sqrtf(be);
}

// Sum over the 64 lanes of a wave, returned to every lane, with DPP lane moves (register
// to register) rather than LDS permutes: pairs, quads, 8-lane halves and 16-lane rows by
// quad_perm / row_half_mirror / row_mirror (every lane of a row then holds the row's
// sum), rows 1 and 3 add the preceding row's sum (row_bcast:15), rows 2 and 3 the sum of
// rows 0-1 (row_bcast:31); lane 63 ends with the total, which readlane broadcasts.
// Every lane of the wave must be active.
__device__ inline float wave_sum_dpp(float v) {
  int x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));  // row_mirror
  x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = __float_as_int(v);
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// One-sided Jacobi rotation of columns with squared norms al, be and inner product ga
// (p' = c p - s q, q' = s p + c q): tan t of the smaller angle from zeta = (be - al) /
// (2 ga), formed with the hardware reciprocal, square root and reciprocal square root
// (about 1 ulp each). The angle need not be exact (the next sweep removes what is
// left); c = 1 / sqrt(1 + t^2) and s = t c keep the rotation orthogonal to float32
// rounding.
__device__ inline void jacobi_cs(float ga, float al, float be, float* c, float* s) {
  const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.f * ga);
  const float az = fabsf(zeta);
  const float t = az > 1e18f ? 0.5f * __builtin_amdgcn_rcpf(zeta)
                             : copysignf(__builtin_amdgcn_rcpf(
                                             az + __builtin_amdgcn_sqrtf(1.f + zeta * zeta)),
                                         zeta);
  const float cc = __builtin_amdgcn_rsqf(1.f + t * t);
  *c = cc;
  *s = cc * t;
}

__device__ inline bool inst_active(const ShiftSpec& s, int z) {
  return s.iactive == nullptr || s.iactive[z] != 0;
}

// ------------------------------------------------------------------ plans
enum Tier { TIER_1X1 = 0, TIER_REG = 1, TIER_LDS = 2, TIER_PANEL = 3, TIER_LRS = 5,
            TIER_FRO = 6 };
constexpr int kFroParts = 512;   // partial sums per instance of the noise scale's norm

// Geometry of one scale's partition. M counts the rows of all stacked instances
// (NI instances of IM rows each, IM = M for a single instance); P = NI * PI block rows.
struct ScaleGeom {
  int M, N;       // stacked matrix
  int m, n;       // block
  int P, Q;       // blocks per column / row of blocks (all instances)
  int trans;      // 1 if the logical block B is the transpose of the stored block
  int mb, nb;     // logical block rows / columns, mb >= nb (B = block or block^T)
  int IM, PI, NI; // rows and block rows per instance, number of instances
  int pw, ph;     // space-time blocks: pixel patch (0: contiguous row blocks)
  int iw, ih;     // image whose pixels are the rows of an instance (space-time only)
};

// Instance-local row of row i of the block-row pl under a row shift sr. Contiguous
// partitions: row pl m + i + sr with cyclic wrap. Space-time partitions: pixel
// (dy, dx) = (i / pw, i % pw) of patch pl (patches in row-major order over the
// image), under the patch shift (sy, sx) = (sr / pw, sr % pw), with wrap in y and x.
__device__ inline int local_row(const ScaleGeom& g, int pl, int i, int sr) {
  if (g.pw) {
    const int qx = g.iw / g.pw;
    const int py = pl / qx, px = pl - py * qx;
    const int sy = sr / g.pw, sx = sr - sy * g.pw;
    const int dy = i / g.pw, dx = i - dy * g.pw;
    int y = py * g.ph + dy + sy;
    if (y >= g.ih) y -= g.ih;
    int x = px * g.pw + dx + sx;
    if (x >= g.iw) x -= g.iw;
    return y * g.iw + x;
  }
  int local = pl * g.m + i + sr;
  if (local >= g.IM) local -= g.IM;
  return local;
}

// Stacked row of row i of block row p under a row shift sr: the shift wraps inside
// the block's own instance (Shift_s of Sec. 9 applied per instance).
__device__ inline int grow(const ScaleGeom& g, int p, int i, int sr) {
  const int z = p / g.PI;
  return z * g.IM + local_row(g, p - z * g.PI, i, sr);
}

__device__ inline int gcol(const ScaleGeom& g, int q, int j, int sc) {
  int c = q * g.n + j + sc;
  if (c >= g.N) c -= g.N;
  return c;
}

// 64-bit device counters per scale: [0] live blocks, [1] sweeps, [2] output rank,
// [3] certified, [4] coupling failures, [5] bound failures, [6] undecided by the trace
// bound, [7] certified by the Collatz-Wielandt bound only, [8] certified zero by the
// Gram matrix's Collatz-Wielandt bound before the subspace iteration.
constexpr int kStatsWords = 16;

// Per-scale device buffers and counters.
struct ScaleWork {
  float* spinAcc;       // averaged cycle spinning: [plane] sum over the shift set
  float* spinTmp;       // [plane] one shift's Z-step
  int lds_cap;          // LDS tier: workgroups per CU cap (0: as many as fit)
  int lrs_wide;         // fused low-rank kernel: first pass with 2p, no retry pass
  double* froPart;      // noise scale: [ninst][kFroParts] partial sums of squares
  float* froGain;       // noise scale: [ninst] gains max(1 - tau / ||v||_F, 0)
  int* live_count;      // [1] blocks that passed the bound test this pass
  int* live_list;       // [P*Q] block ids
  float* rowpart;       // [P*Q*spb*m] partial row sums (strips narrower than a block)
  float* fropart;       // [P*Q*spb] partial squared Frobenius norms
  unsigned long long* stats;  // [8]: live blocks, sweeps, output rank, certified,
                              //      coupling failures, bound failures, spare x2
  // panel tier
  float* pA;            // [slots][nbp][mb] column-major logical block
  float* pW;            // [slots][nbp][nb] column-major right rotations
  int* pflag;           // [slots][2]: rotated-in-sweep, converged
  float* pg;            // [slots][nbp] thresholding gains
  int slots;
  int nbp;              // nb padded to a multiple of 2 * panel width
  int pw;               // panel width
  // certified low-rank path (lowrank.hip); per slot unless noted
  int use_lr;
  float* lrG;           // [slots][nb*nb] Gram B^T B
  float* lrP;           // [slots][nb*nb] scratch for E^T E and its squarings
  float* lrQ;           // [slots][nb*nb]
  float* lrY;           // [slots][nb*p]
  float* lrX;           // [slots][nb*p] orthonormal subspace basis
  float* lrC;           // [slots][mb*p] B X, then the rotated columns a_l
  float* lrT;           // [slots][p*nb] A_f^T B
  float* lrW;           // [slots][nb*p] G V_r
  float* lrV;           // [slots][nb*p] right vectors V_r
  float* lrSig;         // [3][slots][p]: sigma, deflation mask, remainder-bound mask
  float* lrScal;        // [slots][8]
  float* lrRow;         // [slots][nb / 64 + 1][nb] row partials of |E^T E| and row sums
  float* lrOm;          // [nb*p] probe matrix
  float* lrSplit;       // [slots][chunks][nb*nb] split partials of tall blocks (null: none)
  int lrChunks;         // split_chunks(mb, nb)
  float* lrSkPart;      // [slots][sk_chunks(nb)][max(mb, nb)*p] split partials of the skinny
                        // products G X and B V_r of blocks 768 or more wide (null: none)
  int lrSkChunks;
  int* lrCount;         // [5] device counters: fallback, appends, undecided after the trace
                        // bound, undecided after the stage-0 bounds, A_f list
  int* lrFall;          // [5 slots] block ids, then slot indices, of failed certificates;
                        // then the slots left undecided by the stage-0 bound; then those
                        // left undecided by the trace bound (stage -1); then the slots
                        // that need A_f (rebuild or fallback)
  int lds_fallback;     // 1: fallback blocks fit the LDS Jacobi tier
  int* hostInts;        // pinned host ints [2]
  // polar fallback (polar.hip) for failed certificates of blocks beyond the LDS tier;
  // buffers hold plCap compacted blocks
  int plCap;
  float* plPart;        // [plCap][polar_part_floats(mb, nb)] split partial products of the
                        // polar route's GEMMs
  float* plX0;          // [plCap][mb*nb] E' / alpha, later the thresholded block
  float* plXa;          // [plCap][mb*nb] Newton-Schulz iterates
  float* plXb;
  float* plT;           // [plCap][nb*nb]
  float* plS;
  float* plY;
  float* plW;
  float* plScal;        // [plCap][4] alpha, alpha_S, deflated, ||B||_F
  int* plSteps;         // [plCap][2] each block's polar and sign step counts
  float* hostPl;        // pinned host copy of plScal
  int* hostSteps;       // pinned host staging of plSteps
  long long stats_host[3];   // polar blocks, polar steps, sign steps (host counters)
};

struct StreamPlan {
  int ws;        // strip width in columns
  int whole;     // 1: strips hold whole blocks (ws multiple of n), 0: blocks split
  int spb;       // strips per block (whole == 0)
  int kb;        // blocks per strip (whole == 1)
  int spr;       // strips per block row
  int rowbound;  // 1: row-weighted bound of Sec. 8 and Frobenius; 0: Frobenius only (blocks
                 // so tall that strips are under 8 columns: the row partials would be as
                 // large as the block)
  int cst;       // column strips per block (whole == 0); spb = cst * row chunks
  int rch;       // rows per strip (m unless rowbound == 0)
  int align;     // 1: strip edges on global 32-column (128-byte) boundaries: the first
                 // strip of a block takes the columns up to the first boundary, so
                 // cst = ceil(n / ws) + 1 and a strip may be empty
  int nt;        // threads per workgroup, 256 or 512
};

// Stream pass of every decomposed scale in one launch (kernel argument; plane i of a
// stacked plane array starts at plane * scale).
struct StreamScale {
  ScaleGeom g;
  StreamPlan sp;
  int scale;
  float tau2lim;
  int* live_count;
  int* live_list;
  float* rowpart;
  float* fropart;
};
struct StreamAll {
  int n;                       // decomposed scales
  int first[MSLD_MAX_SCALES + 1];  // first workgroup of each scale; first[n] = grid
  size_t plane;                // elements per plane
  StreamScale s[MSLD_MAX_SCALES];
};

// ----------------------------------------------------------- launchers (kernels.hip)
hipError_t launch_stream_all(const StreamAll& a, const float* Z, const float* R, float* D,
                             const ShiftSpec& sh, hipStream_t st,
                             hipEvent_t* after_scale = nullptr);
float stream_tau2lim(const ScaleGeom& g, float tau);
hipError_t launch_fill(float* p, float v, size_t count, hipStream_t st);
bool reg_tier_shape(int m, int n);   // block shapes of the register tier
hipError_t launch_spin_acc(float* acc, const float* zs, size_t n, size_t inst_elems,
                           const int* iactive, hipStream_t st);
hipError_t launch_spin_finish(float* Z, float* D, const float* R, const float* acc, float inv,
                              size_t n, size_t inst_elems, const int* iactive, hipStream_t st);
hipError_t launch_consensus(const float* Y, int64_t ldY, const float* Dcur, float* Dnext,
                            float* Z, float* R, int M, int N, int L, const int* scales1,
                            const float* taus1, int n1, int IM, const int* iactive,
                            const uint8_t* mask, int64_t ldmask, hipStream_t st);
// ev (optional, 5 events): recorded before the scale pass, after the stream pass,
// before the panel rounds, after the panel rounds and after the whole pass.
// deferred (optional): a low-rank scale whose fallback is the polar route only queues
// the copy of its fallback count, sets *deferred = 1 and returns; the caller then calls
// finish_fallback for it (on the same stream) once its other work is issued.
hipError_t launch_scale(const ScaleGeom& g, int tier, const StreamPlan& sp, ScaleWork& w,
                        const float* Zin, const float* R, float* Zout, float* Dout,
                        float tau, const ShiftSpec& sh, float jtol, int max_sweeps,
                        int panel_sweeps, int num_cus, hipStream_t st, hipEvent_t* ev,
                        int* round_launches,
                        bool stream_done, int* deferred = nullptr);
hipError_t finish_fallback(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                           const ShiftSpec& sh, hipStream_t st);
int lr_small_shape(int mb, int nb, int* NB, int* MB, int* P);
size_t lr_small_lds_bytes(int NB, int MB, int P);
hipError_t launch_lr_small(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout,
                           float tau, const ShiftSpec& sh, int num_cus, int pass,
                           const int* count, const int* list, int* fcount, int* flist,
                           hipStream_t st);
// Matrix-core kernels (mfma.hip). Slots walk up to a device count (dcount, or hcount
// when dcount is null); `slots` is the most a launch can see, which sizes its grid.
enum SkMode { SK_DENSE = 0, SK_B = 1, SK_BT = 2 };
// Row chunks of the split contractions of tall blocks (1: no split); depends on the
// block shape only. A split needs slots * chunks * nb * nb floats of partial sums.
int split_chunks(int mb, int nb);
// G = B^T B of the live blocks, B gathered from V = -Dout (tall and wide blocks split
// their rows over part when it is given). With rowpart, unsplit 64-wide tiles also write
// the per-tile |G| row sums (the layout of the Collatz-Wielandt steps); *rows_done says
// whether they did.
hipError_t launch_mf_gram(const ScaleGeom& g, const ShiftSpec& sh, const float* Dout,
                          const int* live_count, const int* live_list, int slots, float* G,
                          float* part, float* rowpart, bool* rows_done, hipStream_t st);
// C (M x 16) = A (M x K) X (K x 16): A dense column-major (SK_DENSE), the gathered
// block B (SK_B) or B^T (SK_BT); C column-major or row-major (rowmaj).
hipError_t launch_sk(int mode, bool rowmaj, const float* A, int64_t sA, int lda,
                     const float* Dout, const ScaleGeom& g, const ShiftSpec& sh,
                     const int* live_list, const float* X, int64_t sX, int M, int K, float* C,
                     int64_t sC, const int* dcount, int hcount, int slots, const int* slot_list,
                     float* part, int split, hipStream_t st);
// Y = A X (M x 16) for symmetric A, barrier-free; needs M % 16 == 0 and lda % 4 == 0.
// With part (slots x ceil(M / 256) x M x 16 floats), M >= 1024 splits the contraction
// (partials indexed by slot, also under a slot list).
hipError_t launch_sym_x(const float* A, int64_t sA, int lda, const float* X, int64_t sX, int M,
                        float* Y, int64_t sY, const int* dcount, int slots, const int* slot_list,
                        float* part, hipStream_t st);
// C = A^T A (M x M from the K x M column-major A), exactly symmetric (upper tiles formed
// and mirrored), batch entries c < count.
hipError_t launch_syrk(int M, int K, const float* A, int lda, int64_t sa, float* C, int ldc,
                       int64_t sc, const int* dcount, int hcount, int max_count, hipStream_t st);
// Contraction chunks of an M x N x K product (a function of the shape alone: fewer than
// 512 output tiles of 64 x 64 and a contraction of 256 or more split into up to 8 chunks
// of at least 128, about 1024 workgroups in all; kc their 32-aligned length); a split
// launch_gemm needs chunks x M x N floats of part per batch entry.
int gemm_split(int M, int N, int K, int* kc);
// C = op(A) B, column-major, batch entries c < count. With part (part_floats floats), a
// product with few output tiles splits its contraction as gemm_split says (partials
// summed in order), or not at all when part is too small for every entry.
hipError_t launch_gemm(bool ta, int M, int N, int K, const float* A, int lda, int64_t sa,
                       const float* B, int ldb, int64_t sb, float* C, int ldc, int64_t sc,
                       const int* dcount, int hcount, int max_count, hipStream_t st,
                       float* part = nullptr, int64_t part_floats = 0);
// C = A^T B for products known to be symmetric (M x M, contraction K, count batch
// entries): the upper 64 x 64 tiles, each mirrored below the diagonal, so C is exactly
// symmetric; part as for launch_gemm, at the split of the full product. With unsummed,
// a split product is left as its chunks in part (column-major M x M each, chunk z of
// entry c at (c chunks + z) M M) and *unsummed = chunks, for the caller to sum in order;
// otherwise (and with no split) *unsummed = 0 and C holds the product.
hipError_t launch_gemm_sym(int M, int K, const float* A, int lda, int64_t sa, const float* B,
                           int ldb, int64_t sb, float* C, int ldc, int64_t sc, int count,
                           hipStream_t st, float* part, int64_t part_floats,
                           int* unsummed = nullptr);
// Z = A_f diag(gains) V_r^T of the certified slots among slot_list[0 .. *count) (all
// slots < *count when the list is null), scattered with D' = 2 Z' - V.
hipError_t launch_mf_rebuild(const ScaleGeom& g, const ShiftSpec& sh, float* Zout, float* Dout,
                             const int* count, const int* slot_list, const int* live_list,
                             int slots, const int* pflag, const float* Af, const float* Vr,
                             const float* sig, const float* mask, float tau, hipStream_t st);
// E^T E = G - Q V^T - V Q^T (P = 16 columns) of the listed slots to Pm, with per-tile
// partial trace and squared norm (part) and per-row partial |.| sums (rowpart).
hipError_t launch_lr_ge(const float* G, const float* Q, const float* V, float* Pm, int nb,
                        float* part, float* rowpart, const int* list, const int* lcount,
                        int slots, hipStream_t st);
// Contraction chunks of the skinny products (G X, B V_r) of blocks 768 or more wide: 128
// columns each, a function of nb alone (B V_r of blocks 1024 or more wide uses the Gram's
// split buffer and 256-column chunks instead).
inline int sk_chunks(int nb) { return (nb + 127) / 128; }
// Split partial floats per block of the polar route's products (mb x nb blocks).
int64_t polar_part_floats(int mb, int nb);
hipError_t run_polar(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                     const ShiftSpec& sh, int nfall, hipStream_t st);
// Certified low-rank BlockSVT of the live blocks (count on the device); failed
// certificates are listed for the exact fallback (w.lrCount[0], w.lrFall).
hipError_t run_lowrank(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                       const ShiftSpec& sh, hipStream_t st, hipEvent_t* gram_ev = nullptr);
__global__ void k_zero_ints(int* p, int n);
__global__ void k_copy_count(const int* src, int* dst);
// Per-instance sums (instance z = rows [z IM, (z+1) IM)): out[z].
// Also the dual residual sums sum_i ||Z_i' - Z_i||^2 into out_dual[z].
hipError_t launch_resid(const float* Dold, const float* Dnew, const float* R, const float* Z,
                        int M, int N, int L, int IM, int NI, double* partial, int nparts,
                        double* out, double* out_dual, hipStream_t st);
hipError_t launch_sumsq(const float* Y, int64_t ldY, int IM, int N, int NI, const uint8_t* mask,
                        int64_t ldmask, double* partial, int nparts, double* out,
                        hipStream_t st);
hipError_t launch_device_shifts(uint64_t seed, int k0, int count, int L, const int* bm,
                                const int* bn, int* out, hipStream_t st);

}  // namespace msld
