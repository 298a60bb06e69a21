// Certified low-rank BlockSVT for large blocks.
//
// For a live block B (logical mb x nb, mb >= nb) the soft-threshold of eq:svt only
// needs the singular triplets with sigma > tau. A subspace iteration on the Gram
// G = B^T B finds an orthonormal X (nb x p); the SVD of the reduced block B X (from
// its float64 Gram) gives B V_r = A_f (orthogonal columns a_l = sigma_l u_l) with
// V_r = X W. Let L be the
// columns with sigma_l > tau (live), plus those with tau/2 < sigma_l <= tau whose own
// coupling c_l = ||u_l^T B - sigma_l v_l^T|| is tiny, and E_L = B (I - V_L V_L^T). The
// result Z = sum_{l in L} max(1 - tau/sigma_l, 0) a_l v_l^T is accepted only if
//   (i)  sigma_max(E_L) <= tau, checked with the upper bound
//        lambda_max(E_L^T E_L) <= max(max_{l in K} sigma_l^2, lambda_max(E^T E))
//                                 + (sum_{l in K} sigma_l^2 c_l^2)^(1/2)
//        (K: further well-converged directions outside L, E = B (I - V V^T) the
//        remainder after L and K; a 2 x 2 block split of E_L^T E_L), with
//        lambda_max(E^T E) <= min(||E^T E||_F, Collatz-Wielandt bound of |E^T E| with the
//        vector of its row sums), then tr * ||(E^T E / tr)^k||_F^(1/k), k = 2, 8, and
//   (ii) ||U_L^T E_L||_F is below a small fraction of ||B||_F.
// The bound of (i) is tried first with tr(E^T E) = ||B||_F^2 - sum ||B v_l||^2, which
// needs no E^T E; only the slots it leaves undecided get E^T E and the finer bounds.
// Then B0 = U_L S_L V_L^T + (I - U_L U_L^T) E_L decouples, SVT(B0) = Z (columns of L
// below tau threshold to zero), and since the proximal map is non-expansive
// ||SVT(B) - Z||_F <= ||B - B0||_F = ||U_L^T E_L||_F.
// Blocks that fail either test get an exact SVT: the LDS Jacobi tier when they fit
// in LDS, else the polar route (polar.hip). The matrix products (the Gram matrix, the
// subspace, coupling and remainder products, the squarings) and the rebuild are the
// matrix-core kernels of mfma.hip, which read each block straight from the iterate at
// its shifted coordinates; the orthonormalisation, the reduced SVD and the certificate
// are the kernels below. Every launch has a fixed grid and walks the live (or
// undecided) slots up to a count kept on the device: nothing here waits for the host.
#include "msld_internal.h"

namespace msld {

static constexpr float kCertMargin = 2e-3f;    // relative margin on tau^2 for test (i)
static constexpr float kCouplingTol = 1e-5f;   // test (ii): ||U_L^T E||_F <= tol ||B||_F

__device__ __forceinline__ int wrap_add2(int base, int off, int mod) {
  int v = base + off;
  return v >= mod ? v - mod : v;
}

__device__ __forceinline__ float block_sum(float v, float* red) {
  // 256-thread workgroup sum; red holds >= 4 floats
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float s = 0.f;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// Fixed +-1/sqrt(nb) probe matrix (column-major nb x p) from an integer hash.
__global__ void k_lr_omega(float* Om, int nb, int p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * p) return;
  uint64_t z = mix64(0x243F6A8885A308D3ull + (uint64_t)e);
  Om[e] = ((z >> 63) ? 1.f : -1.f) * rsqrtf((float)nb);
}

// tr(G) per slot.
__global__ void __launch_bounds__(256) k_lr_trace(const float* G, int nb, int64_t strideG,
                                                  float* scal, int which, const int* count) {
  __shared__ float red[8];
  const int cnt = *count;
  for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x) {
    const float* g = G + (int64_t)slot * strideG;
    float s = 0.f;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += g[(int64_t)i * nb + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) scal[slot * 8 + which] = s;
  }
}

// Rows of the P-column matrices staged in LDS per step of the fp64 Gram reductions.
constexpr int kRC = 128;

// Gram K = Y^T Z (P x P) of two nb x P column-major matrices, accumulated in float64 over
// row chunks staged in LDS; thread t (256 = P * P) owns entry (t / P, t % P).
template <int P>
__device__ __forceinline__ double gram64_pp(const float* y, const float* z, int nb,
                                            float (*ys)[P + 1], float (*zs)[P + 1]) {
  const int tid = threadIdx.x;
  const int a = tid / P, b = tid - (tid / P) * P;
  double acc = 0.0;
  for (int r0 = 0; r0 < nb; r0 += kRC) {
    const int rows = min(kRC, nb - r0);
    for (int e = tid; e < kRC * P; e += 256) {
      const int l = e / kRC, r = e - l * kRC;
      ys[r][l] = r < rows ? y[(int64_t)l * nb + r0 + r] : 0.f;
      zs[r][l] = r < rows ? z[(int64_t)l * nb + r0 + r] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < kRC; ++r) acc += (double)ys[r][a] * (double)zs[r][b];
    __syncthreads();
  }
  return acc;
}

// Float64 Gram K[a][b] = sum_r y[a nb + r] z[b nb + r] of two nb x P column-major panels
// by NT threads (NT / P^2 interleaved row groups per entry): rows are staged through
// LDS in chunks of kBC while the next chunk's loads are in flight (one load latency per
// panel rather than per chunk); rows past nb are zero. Thread e < P^2 returns entry
// (e / P, e % P), summed over the row groups in a fixed order; the others return 0.
// With y == z only ys is used (zs may alias it) and K[a][b], K[b][a] come out equal.
constexpr int kBC = 512;
template <int P, int NT>
__device__ double gram64_stream(const float* y, const float* z, int nb, float (*ys)[P + 1],
                                float (*zs)[P + 1], double* red) {
  constexpr int E = P * P, RG = NT / E, PER = kBC * P / NT;
  static_assert(NT % E == 0 && (kBC * P) % NT == 0, "thread layout");
  const int tid = threadIdx.x;
  const int e = tid % E, rg = tid / E;
  const int a = e / P, b = e - (e / P) * P;
  const bool same = y == z;
  float py[PER], pz[PER];
  auto load = [&](int r0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + NT * u;
      const int l = idx / kBC, r = idx - (idx / kBC) * kBC;
      const bool in = r0 + r < nb;
      py[u] = in ? y[(int64_t)l * nb + r0 + r] : 0.f;
      pz[u] = (in && !same) ? z[(int64_t)l * nb + r0 + r] : 0.f;
    }
  };
  double acc = 0.0;
  __syncthreads();   // earlier writes of the panels by this workgroup are visible
  load(0);
  for (int r0 = 0; r0 < nb; r0 += kBC) {
    __syncthreads();   // the previous chunk (and any earlier use of ys, zs) is read
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + NT * u;
      const int l = idx / kBC, r = idx - (idx / kBC) * kBC;
      ys[r][l] = py[u];
      if (!same) zs[r][l] = pz[u];
    }
    __syncthreads();
    if (r0 + kBC < nb) load(r0 + kBC);
    const float (*zz)[P + 1] = same ? ys : zs;
#pragma unroll 8
    for (int r = rg; r < kBC; r += RG) acc += (double)ys[r][a] * (double)zz[r][b];
  }
  red[tid] = acc;
  __syncthreads();
  double k = 0.0;
  if (tid < E)
    for (int g2 = 0; g2 < RG; ++g2) k += red[g2 * E + tid];
  __syncthreads();
  return k;
}

// Lane l's double, broadcast to the whole wave (l uniform).
__device__ __forceinline__ double bcast64(double v, int l) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_readlane(hi, l), __builtin_amdgcn_readlane(lo, l));
}

// Orthonormalisation of large panels (nb > 512, one workgroup of 1024 threads per slot)
// by Cholesky QR applied twice: the float64 Gram S = Z^T Z of the panel, its Cholesky
// factor R, then Z <- Z R^-1 in float64 per row. A column whose remaining squared norm
// is at most 1e-12 of its own (numerically dependent on the earlier ones) gets a zero
// output column and no part in the later ones. The second pass removes what rounding
// left of the first pass's departure from orthonormality.
template <int P>
__global__ void __launch_bounds__(1024) k_lr_orth_cq(const float* Y, float* X, int nb,
                                                     int64_t stride, const int* count,
                                                     const int* sl) {
  constexpr int NT = 1024;
  static_assert(P * P == 256, "the Gram entries fill a quarter of the workgroup");
  __shared__ float zs[kBC][P + 1];
  __shared__ double red[NT];
  __shared__ double S[P][P + 1];
  __shared__ double T[P][P + 1];
  const int cnt = *count;
  const int tid = threadIdx.x;
  for (int ci = blockIdx.x; ci < cnt; ci += gridDim.x) {
    const int slot = sl ? sl[ci] : ci;
    const float* y = Y + (int64_t)slot * stride;
    float* x = X + (int64_t)slot * stride;
    for (int pass = 0; pass < 2; ++pass) {
      const float* z = pass == 0 ? y : x;
      // (its first barrier orders the previous pass's writes of x before the reads)
      const double kv = gram64_stream<P, NT>(z, z, nb, zs, zs, red);
      if (tid < P * P) S[tid / P][tid % P] = kv;
      __syncthreads();
      if (tid < 64) {
        // Cholesky by wave 0 in registers: lane k (< P) holds column k of S, which
        // becomes column k of R (right-looking: row j of R, then the trailing upper
        // triangle, entry (i, k) by lane k); every other entry a lane needs is broadcast
        // from its owner with readlane. Then lane k solves R t = e_k for column k of
        // T = R^-1, bottom up, and writes it to LDS.
        const int lane = tid;
        double c[P];
#pragma unroll
        for (int i = 0; i < P; ++i) c[i] = lane < P ? S[i][lane] : 0.0;
        const double d0 = lane < P ? S[lane][lane] : 0.0;
        unsigned dep = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const double d = bcast64(c[j], j);
          const double s0 = bcast64(d0, j);
          const bool dj = !(s0 > 0.0) || !(d > 1e-12 * s0);
          if (dj) dep |= 1u << j;
          const double rjj = dj ? 1.0 : sqrt(d);
          if (lane == j) c[j] = rjj;
          else if (lane > j) c[j] = dj ? 0.0 : c[j] / rjj;
          const double rjk = c[j];
#pragma unroll
          for (int i = j + 1; i < P; ++i) {
            const double rji = bcast64(c[j], i);
            if (lane >= i) c[i] -= rji * rjk;
          }
        }
        const bool dk = lane < P && ((dep >> lane) & 1u);
        double t[P];
#pragma unroll
        for (int i = P - 1; i >= 0; --i) {
          const double rii = bcast64(c[i], i);
          if (i > lane) {
            t[i] = 0.0;
          } else if (i == lane) {
            t[i] = dk ? 0.0 : 1.0 / rii;
          } else {
            double v = 0.0;
#pragma unroll
            for (int m = i + 1; m < P; ++m) {
              const double rim = bcast64(c[i], m);
              if (m <= lane) v += rim * t[m];
            }
            t[i] = dk ? 0.0 : -v / rii;
          }
        }
        if (lane < P) {
#pragma unroll
          for (int i = 0; i < P; ++i) T[i][lane] = t[i];
        }
      }
      __syncthreads();
      for (int r = tid; r < nb; r += NT) {
        float zv[P];
#pragma unroll
        for (int j = 0; j < P; ++j) zv[j] = z[(int64_t)j * nb + r];
#pragma unroll 1
        for (int l = 0; l < P; ++l) {
          double o = 0.0;
#pragma unroll
          for (int j = 0; j < P; ++j) o += (double)zv[j] * T[j][l];
          x[(int64_t)l * nb + r] = (float)o;
        }
      }
    }
  }
}

__device__ __forceinline__ float wave_sum(float v) { return wave_sum_dpp(v); }

// Orthonormalisation with one wave per slot and the columns held in registers
// (lane l owns rows l + 64 r, r < RPL): no LDS and no workgroup barriers. Classical
// Gram-Schmidt with exactly two projection passes ("twice is enough"); a column whose
// norm drops below half in both passes is numerically dependent and set to zero. The
// fixed pass count keeps every register index static.
template <int P, int RPL>
__global__ void __launch_bounds__(256) k_lr_orth_w(const float* Y, float* X, int nb,
                                                   int64_t stride, const int* count,
                                                   const int* sl) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cnt = *count;
  for (int ci = blockIdx.x * 4 + wv; ci < cnt; ci += gridDim.x * 4) {
  const int slot = sl ? sl[ci] : ci;
  const float* y = Y + (int64_t)slot * stride;
  float* x = X + (int64_t)slot * stride;
  float v[P][RPL];
#pragma unroll
  for (int j = 0; j < P; ++j)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      v[j][r] = row < nb ? y[j * nb + row] : 0.f;
    }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    float n0 = 0.f;
#pragma unroll
    for (int r = 0; r < RPL; ++r) n0 += v[j][r] * v[j][r];
    n0 = wave_sum(n0);
    float nn = n0;
    bool kept = true;
    if (j > 0) {
      kept = false;
      float nprev = n0;
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        float c[P];
#pragma unroll
        for (int i = 0; i < j; ++i) {
          float sdot = 0.f;
#pragma unroll
          for (int r = 0; r < RPL; ++r) sdot += v[i][r] * v[j][r];
          c[i] = wave_sum(sdot);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          float t = v[j][r];
#pragma unroll
          for (int i = 0; i < j; ++i) t -= c[i] * v[i][r];
          v[j][r] = t;
        }
        float s = 0.f;
#pragma unroll
        for (int r = 0; r < RPL; ++r) s += v[j][r] * v[j][r];
        nn = wave_sum(s);
        kept = kept || nn >= 0.25f * nprev;
        nprev = nn;
      }
    }
    const float nrm = sqrtf(nn);
    const bool keep = kept && nrm > 1e-30f && nn > 1e-12f * n0;
    const float inv = keep ? 1.f / nrm : 0.f;
#pragma unroll
    for (int r = 0; r < RPL; ++r) v[j][r] *= inv;
  }
#pragma unroll
  for (int j = 0; j < P; ++j)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      if (row < nb) x[j * nb + row] = v[j][r];
    }
  }
}

// Round-robin pair order of a cyclic Jacobi sweep over ncols (even) indices: ncols - 1
// rounds of ncols / 2 disjoint pairs (the same order as the tiers in kernels.hip, which
// is not visible from this translation unit).
__device__ __forceinline__ void lr_pair(int round, int k, int ncols, int* a, int* b) {
  const int n1 = ncols - 1;
  *a = (k == 0) ? 0 : 1 + (k - 1 + round) % n1;
  *b = 1 + (ncols - 2 - k + round) % n1;
}

// Jacobi rotation annihilating the (p, q) entry of a symmetric matrix with diagonal
// entries app, aqq: columns p' = c p - s q, q' = s p + c q. The angle only has to be
// close to the annihilating one (the next sweep removes what is left), so tan is formed
// with the hardware's approximate reciprocal and reciprocal square root; c = 1 /
// sqrt(1 + t^2) then gets two Newton steps, so that c^2 + s^2 = 1 to float64 accuracy and
// every rotation stays orthogonal. False (c = 1, s = 0) when |apq| <= 1e-14 sqrt(app aqq).
__device__ __forceinline__ bool jacobi_rot64(double app, double aqq, double apq, double* c,
                                             double* s) {
  *c = 1.0;
  *s = 0.0;
  if (!(apq * apq > 1e-28 * fabs(app * aqq)) || apq == 0.0) return false;
  const double th = (aqq - app) * __builtin_amdgcn_rcp(2.0 * apq);
  double t;
  if (fabs(th) > 1e150) {
    t = 0.5 * __builtin_amdgcn_rcp(th);
  } else {
    const double h = th * th + 1.0;
    const double den = fabs(th) + h * __builtin_amdgcn_rsq(h);
    t = copysign(__builtin_amdgcn_rcp(den), th);
  }
  const double x = t * t + 1.0;
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  *c = y;
  *s = t * y;
  return true;
}

// SVD of the reduced block B X from the Gram matrix alone. With W0 = G X (nb x P),
// K = X^T W0 = (B X)^T (B X) is the Gram of the reduced block (float64, symmetrised);
// its eigen-decomposition K = W diag(lambda) W^T by cyclic two-sided Jacobi in float64
// (parallel pair order) gives sigma_l = sqrt(lambda_l), the right vectors
// V_r = X W (nb x P) and, since G is symmetric, T^T = G V_r = W0 W, the coupling
// product A_f^T B with A_f = B V_r (T stored row-major, T[c P + l]). A_f itself is
// formed later, only for the blocks whose rebuild or fallback needs it.
// A Jacobi round: thread (u, w) of the first wave owns the 2 x 2 sub-block of K at
// the rows of pair u and the columns of pair w; it forms both pairs' rotations from
// the current K (every thread that needs a rotation computes it from the same
// entries, so all copies agree bit for bit), writes its sub-block of J_u^T K J_w to the
// other buffer and applies J_w to its sub-block of W; one barrier per round.
template <int P>
__global__ void __launch_bounds__(256) k_lr_reduced(const float* X, const float* W0, int nb,
                                                    float* Vr, float* Tt, float* sig,
                                                    const int* count, const int* sl) {
  static_assert(P * P == 256, "one Gram entry per thread");
  static_assert((P / 2) * (P / 2) <= 64, "one wave of sub-blocks");
  __shared__ float ys[kRC][P + 1], zs[kRC][P + 1];
  __shared__ double Kb[2][P][P + 1];
  __shared__ double V[P][P + 1];
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  const int cnt = *count;
  for (int ci = blockIdx.x; ci < cnt; ci += gridDim.x) {
    const int slot = sl ? sl[ci] : ci;
    const float* x = X + (int64_t)slot * nb * P;
    const float* w0 = W0 + (int64_t)slot * nb * P;
    const double kv = gram64_pp<P>(x, w0, nb, ys, zs);
    Kb[1][tid / P][tid % P] = kv;
    __syncthreads();
    {
      const int a = tid / P, b = tid % P;
      Kb[0][a][b] = 0.5 * (Kb[1][a][b] + Kb[1][b][a]);
      V[a][b] = a == b ? 1.0 : 0.0;
    }
    int cur = 0;
    for (int sw = 0; sw < 40; ++sw) {
      if (tid == 0) s_rot = 0;
      __syncthreads();
      for (int rd = 0; rd < P - 1; ++rd) {
        if (tid < (P / 2) * (P / 2)) {
          const int u = tid / (P / 2), w = tid - (tid / (P / 2)) * (P / 2);
          int pu, qu, pw, qw;
          lr_pair(rd, u, P, &pu, &qu);
          lr_pair(rd, w, P, &pw, &qw);
          double (*K)[P + 1] = Kb[cur];
          double cu, su, cw, sw2;
          const bool ru = jacobi_rot64(K[pu][pu], K[qu][qu], K[pu][qu], &cu, &su);
          jacobi_rot64(K[pw][pw], K[qw][qw], K[pw][qw], &cw, &sw2);
          if (u == w && ru) s_rot = 1;
          const double k00 = K[pu][pw], k01 = K[pu][qw], k10 = K[qu][pw], k11 = K[qu][qw];
          // K J_w on rows pu, qu, then J_u^T on the left
          const double t00 = cw * k00 - sw2 * k01, t01 = sw2 * k00 + cw * k01;
          const double t10 = cw * k10 - sw2 * k11, t11 = sw2 * k10 + cw * k11;
          double (*Kn)[P + 1] = Kb[cur ^ 1];
          Kn[pu][pw] = cu * t00 - su * t10;
          Kn[pu][qw] = cu * t01 - su * t11;
          Kn[qu][pw] = su * t00 + cu * t10;
          Kn[qu][qw] = su * t01 + cu * t11;
          // W J_w on rows pu, qu (the rows of pair u cover every row once)
          const double v00 = V[pu][pw], v01 = V[pu][qw], v10 = V[qu][pw], v11 = V[qu][qw];
          V[pu][pw] = cw * v00 - sw2 * v01;
          V[pu][qw] = sw2 * v00 + cw * v01;
          V[qu][pw] = cw * v10 - sw2 * v11;
          V[qu][qw] = sw2 * v10 + cw * v11;
        }
        cur ^= 1;
        __syncthreads();
      }
      const int rot = s_rot;
      __syncthreads();
      if (!rot) break;
    }
    double (*K)[P + 1] = Kb[cur];
    if (tid < P) sig[slot * P + tid] = (float)sqrt(fmax(K[tid][tid], 0.0));
    float* vr = Vr + (int64_t)slot * nb * P;
    float* tt = Tt + (int64_t)slot * nb * P;
    // V_r = X W, T^T = W0 W: one row per thread, its 2 P inputs read once (coalesced
    // across the workgroup) and kept in registers
    for (int r = tid; r < nb; r += 256) {
      float xv[P], wv[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        xv[j] = x[(int64_t)j * nb + r];
        wv[j] = w0[(int64_t)j * nb + r];
      }
#pragma unroll 1
      for (int l = 0; l < P; ++l) {
        double o = 0.0, t = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const double vjl = V[j][l];
          o += (double)xv[j] * vjl;
          t += (double)wv[j] * vjl;
        }
        vr[(int64_t)l * nb + r] = (float)o;
        tt[(int64_t)r * P + l] = (float)t;
      }
    }
    __syncthreads();
  }
}

// Per direction l: c_l^2 = || T_l / sigma_l - sigma_l v_l^T ||^2 with T = A_f^T B
// (= ||u_l^T B - sigma_l v_l^T||^2). Deflation set L (mask): live (sigma > tau) always;
// near-live (tau/2 < sigma <= tau) when c_l <= 0.3 tol ||B||_F. scal[1] = sum of c_l^2
// over L. For the remainder bound, other well-converged directions l' (not in L, with
// sigma_l^2 c_l^2 <= (1e-3 tau^2)^2) are split off too: dmask marks L and them,
// scal[7] = max sigma_l'^2 (with a relative allowance for the residual
// non-orthogonality of the rotated columns) and scal[6] = sum sigma_l'^2 c_l'^2.
template <int P>
__global__ void __launch_bounds__(256) k_lr_coupling(const float* T, const float* sig,
                                                     const float* Vr, int nb, float tau,
                                                     float tol, float* scal, float* mask,
                                                     float* dmask, const int* count,
                                                     const int* sl) {
  __shared__ float red[8];
  __shared__ float cl[P];
  const int cnt = *count;
  for (int ci = blockIdx.x; ci < cnt; ci += gridDim.x) {
  const int slot = sl ? sl[ci] : ci;
  __syncthreads();
  const float* t = T + (int64_t)slot * P * nb;
  const float* vr = Vr + (int64_t)slot * nb * P;
  const float* sg = sig + slot * P;
  for (int l = 0; l < P; ++l) {
    const float s = sg[l];
    if (!(s > 0.f)) {                 // uniform branch: sg is shared by all threads
      if (threadIdx.x == 0) cl[l] = 0.f;
      continue;
    }
    const float inv = 1.f / s;
    float acc = 0.f;
    for (int cidx = threadIdx.x; cidx < nb; cidx += blockDim.x) {
      const float d = t[(int64_t)cidx * P + l] * inv - s * vr[l * nb + cidx];
      acc += d * d;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) cl[l] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float trG = scal[slot * 8 + 0];
    const float near_lim = 0.09f * tol * tol * trG;   // (0.3 tol ||B||_F)^2
    float c2 = 0.f, omax = 0.f, cross = 0.f;
    for (int l = 0; l < P; ++l) {
      const float s = sg[l];
      const bool live = s > tau;
      const bool near = !live && s > 0.5f * tau && cl[l] <= near_lim;
      const bool in = live || near;
      const float x = s * s * cl[l];
      const bool split = !in && s > 0.f && s * sqrtf(cl[l]) <= 1e-3f * tau * tau;
      mask[slot * P + l] = in ? 1.f : 0.f;
      dmask[slot * P + l] = (in || split) ? 1.f : 0.f;
      if (in) c2 += cl[l];
      if (split) {
        omax = fmaxf(omax, s * s);
        cross += x;
      }
    }
    scal[slot * 8 + 1] = c2;
    scal[slot * 8 + 6] = cross;
    scal[slot * 8 + 7] = omax * (1.f + 1e-4f);
  }
  }
}

// Q = W - V H / 2 over the columns the mask selects (others zero), with W = G V_r
// (row-major: the coupling product T^T) and H = V^T W (P x P, masked), so that
// E^T E = G - Q V^T - V Q^T for the remainder E = B (I - V V^T) of the masked columns
// V; for the slots of the undecided list.
template <int P>
__global__ void __launch_bounds__(256) k_lr_q(const float* Wg, const float* Vr, const float* mask,
                                              float* Qo, int nb, const int* list,
                                              const int* lcount) {
  static_assert(P * P == 256, "one H entry per thread");
  __shared__ float vs[kRC][P + 1], ws[kRC][P + 1];
  __shared__ float h[P * P];
  __shared__ float mk[P];
  const int tid = threadIdx.x;
  const int cnt = *lcount;
  for (int c = blockIdx.x; c < cnt; c += gridDim.x) {
    const int slot = list[c];
    const float* w = Wg + (int64_t)slot * nb * P;   // row-major: w[i P + k]
    const float* v = Vr + (int64_t)slot * nb * P;   // column-major: v[l nb + i]
    float* q = Qo + (int64_t)slot * nb * P;
    __syncthreads();
    if (tid < P) mk[tid] = mask[slot * P + tid];
    // H[k][l] = v_l . w_k over the masked pairs (thread (k, l), rows staged in LDS)
    const int k = tid / P, l = tid - (tid / P) * P;
    float hacc = 0.f;
    for (int r0 = 0; r0 < nb; r0 += kRC) {
      const int rows = min(kRC, nb - r0);
      __syncthreads();
      for (int e = tid; e < kRC * P; e += 256) {
        const int j = e / kRC, r = e - j * kRC;   // column j, row r (column-major reads)
        vs[r][j] = r < rows ? v[(int64_t)j * nb + r0 + r] : 0.f;
        const int rr = e / P, jj = e - rr * P;     // row rr, column jj (row-major reads)
        ws[rr][jj] = rr < rows ? w[(int64_t)(r0 + rr) * P + jj] : 0.f;
      }
      __syncthreads();
#pragma unroll 8
      for (int r = 0; r < kRC; ++r) hacc += vs[r][l] * ws[r][k];
    }
    h[k * P + l] = (mk[k] > 0.f && mk[l] > 0.f) ? hacc : 0.f;
    __syncthreads();
    // Q[:, k] = W[:, k] - V H[k][:]^T / 2 on masked k (one row per thread)
    for (int r = tid; r < nb; r += 256) {
      float vv[P];
#pragma unroll
      for (int j = 0; j < P; ++j) vv[j] = v[(int64_t)j * nb + r];
#pragma unroll 1
      for (int kk = 0; kk < P; ++kk) {
        float sv = 0.f;
        if (mk[kk] > 0.f) {
          float vh = 0.f;
#pragma unroll
          for (int j = 0; j < P; ++j) vh += vv[j] * h[kk * P + j];
          sv = w[(int64_t)r * P + kk] - 0.5f * vh;
        }
        q[(int64_t)kk * nb + r] = sv;
      }
    }
  }
}

// Per 64 x 64 tile of the Gram matrix G of each live slot, the partial sums of |G_ij|
// over the tile's columns for each of its rows (rowpart slice tj, the layout the
// Collatz-Wielandt steps below read); fixed summation order.
__global__ void __launch_bounds__(256) k_lr_gabs_rowpart(const float* G, int nb, float* rowpart,
                                                         const int* count) {
  __shared__ float ps[4][64];
  const int cnt = *count;
  const int tn = (nb + 63) / 64;
  const int ti = blockIdx.x % tn, tj = blockIdx.x / tn;
  const int i0 = ti * 64, j0 = tj * 64;
  const int il = threadIdx.x & 63, jg = threadIdx.x >> 6;
  const int i = i0 + il;
  for (int slot = blockIdx.y; slot < cnt; slot += gridDim.y) {
    const float* g = G + (int64_t)slot * nb * nb;
    float a = 0.f;
    if (i < nb)
      for (int jl = jg; jl < 64 && j0 + jl < nb; jl += 4) a += fabsf(g[(int64_t)(j0 + jl) * nb + i]);
    __syncthreads();
    ps[jg][il] = a;
    __syncthreads();
    if (threadIdx.x < 64 && i < nb)
      rowpart[(int64_t)slot * nb * (tn + 1) + (int64_t)tj * nb + i] =
          (ps[0][il] + ps[1][il]) + (ps[2][il] + ps[3][il]);
  }
}

// Zero-output certificate before the subspace iteration: sigma_max(B)^2 = lambda_max(G)
// is at most the Collatz-Wielandt bound of |G| (scal[5]); below tau^2 (with the
// certificate's margin) every singular value is thresholded to zero, which is the
// output the stream pass already wrote (Z' = 0, D' = -V). Such slots are settled here
// (no singular values, no rebuild); the others are listed for the subspace iteration
// (fall[5 slots ..], counts[5]).
__global__ void k_lr_gram_decide(const int* live, int slots, const float* scal, float* sig,
                                 float tau, int* pflag, int* counts, int* fall,
                                 unsigned long long* stats) {
  const int count = *live;
  const float lim = tau * tau * (1.f - kCertMargin);
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < count;
       slot += gridDim.x * blockDim.x) {
    const float b = scal[slot * 8 + 5];
    if (b <= lim && isfinite(b)) {
      for (int l = 0; l < 16; ++l) sig[slot * 16 + l] = 0.f;
      pflag[4 * slot + 1] = 1;
      pflag[4 * slot + 2] = 1;
      pflag[4 * slot + 3] = 0;
      atomicAdd(&stats[0], 1ull);
      atomicAdd(&stats[3], 1ull);
      atomicAdd(&stats[8], 1ull);
    } else {
      fall[5 * slots + atomicAdd(&counts[5], 1)] = slot;
    }
  }
}

// Collatz-Wielandt bound for the symmetric M = E^T E (in Pm): with r = |M| 1 and
// y = |M| r, lambda_max(M) <= rho(|M|) <= max_i y_i / r_i (a row with r_i = 0 is zero).
// Three small steps on the tile partials, all in a fixed summation order:
// k_lr_rsum: r_i = sum over tile columns of the row partials of E^T E (slice tn);
// k_lr_cwy: per 64 x 64 tile, partial y_i over its columns (slices 0..tn-1);
// k_lr_cwmax: y_i, the ratio, its maximum; scal[4] = min(||M||_F, bound) / tr(M).
__global__ void __launch_bounds__(256) k_lr_rsum(float* rowpart, int nb, const int* list,
                                                 const int* lcount) {
  const int cnt = *lcount;
  const int tn = (nb + 63) / 64;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  for (int cidx = blockIdx.y; cidx < cnt; cidx += gridDim.y) {
    const int slot = list ? list[cidx] : cidx;
    float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
    float v = 0.f;
    for (int t = 0; t < tn; ++t) v += rp[(int64_t)t * nb + i];
    rp[(int64_t)tn * nb + i] = v;
  }
}

__global__ void __launch_bounds__(256) k_lr_cwy(const float* Pm, float* rowpart, int nb,
                                                const int* list, const int* lcount) {
  __shared__ float rj[64];
  __shared__ float ys[4][64];
  const int cnt = *lcount;
  for (int cidx = blockIdx.y; cidx < cnt; cidx += gridDim.y) {
  const int slot = list ? list[cidx] : cidx;
  const int tn = (nb + 63) / 64;
  const int ti = blockIdx.x % tn, tj = blockIdx.x / tn;
  const int i0 = ti * 64, j0 = tj * 64;
  float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
  const float* pm = Pm + (int64_t)slot * nb * nb;
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) rj[tid] = j0 + tid < nb ? rp[(int64_t)tn * nb + j0 + tid] : 0.f;
  __syncthreads();
  const int il = tid & 63, i = i0 + il;
  float y = 0.f;
  if (i < nb)
    for (int jl = tid >> 6; jl < 64; jl += 4) {
      const int j = j0 + jl;
      if (j >= nb) break;
      y += fabsf(pm[(int64_t)j * nb + i]) * rj[jl];
    }
  ys[tid >> 6][il] = y;
  __syncthreads();
  if (tid < 64 && i < nb) rp[(int64_t)tj * nb + i] = ys[0][il] + ys[1][il] + ys[2][il] + ys[3][il];
  }
}

// mode 0: scal[4] = min(scal[4], bound / tr(E^T E)); mode 1: scal[5] = the bound itself
// (+inf when it cannot be formed).
__global__ void __launch_bounds__(256) k_lr_cwmax(const float* rowpart, int nb, float* scal,
                                                  const int* list, const int* lcount, int mode) {
  __shared__ float red[8];
  const int cnt = *lcount;
  for (int cidx = blockIdx.x; cidx < cnt; cidx += gridDim.x) {
  const int slot = list ? list[cidx] : cidx;
  const int tn = (nb + 63) / 64;
  const float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
  float best = 0.f;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    float y = 0.f;
    for (int t = 0; t < tn; ++t) y += rp[(int64_t)t * nb + i];
    const float ri = rp[(int64_t)tn * nb + i];
    if (ri > 0.f) best = fmaxf(best, y / ri);
    else if (y > 0.f) best = __int_as_float(0x7f800000);   // not for a symmetric M
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = fmaxf(best, __shfl_xor(best, o));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = fmaxf(b, red[w]);
    if (mode == 1) {
      scal[slot * 8 + 5] = isfinite(b) ? b : __int_as_float(0x7f800000);
    } else {
      const float tr = scal[slot * 8 + 2];
      if (tr > 0.f && isfinite(b)) scal[slot * 8 + 4] = fminf(scal[slot * 8 + 4], b / tr);
    }
  }
  }
}

// Reduce the per-tile partials of E^T E in a fixed order: scal[2] = tr(E^T E),
// scal[4] = ||E^T E||_F / tr(E^T E) (stage-0 bound factor).
// One workgroup per listed slot: thread t sums tiles t, t + 256, ... in order, then a
// fixed tree over the threads.
__device__ __forceinline__ float tree_sum256(float v, float* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(256) k_lr_ge_reduce(const float* part, int tiles, float* scal,
                                                      const int* list, const int* lcount) {
  __shared__ float red[256];
  const int cnt = *lcount;
  for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
    const int slot = list[idx];
    float tr = 0.f, f2 = 0.f;
    for (int t = threadIdx.x; t < tiles; t += 256) {
      tr += part[((int64_t)slot * tiles + t) * 2];
      f2 += part[((int64_t)slot * tiles + t) * 2 + 1];
    }
    tr = tree_sum256(tr, red);
    f2 = tree_sum256(f2, red);
    if (threadIdx.x == 0) {
      scal[slot * 8 + 2] = tr;
      scal[slot * 8 + 4] = tr > 0.f ? sqrtf(f2) / tr : 0.f;
      scal[slot * 8 + 3] = scal[slot * 8 + 4];   // the Frobenius factor alone (statistics)
    }
  }
}

// Gather the undecided slots' E^T E (slot-indexed Pm) into compact positions of Dst,
// scaled by 1 / tr(E^T E) (0 stays 0), so that the squarings only touch those slots.
__global__ void k_lr_gather_scale(const float* Pm, float* Dst, int nb, const int* list,
                                  const int* lcount, const float* scal) {
  const int cnt = *lcount;
  for (int c = blockIdx.y; c < cnt; c += gridDim.y) {
    const int slot = list[c];
    const float tr = scal[slot * 8 + 2];
    const float inv = tr > 0.f ? 1.f / tr : 0.f;
    const int64_t total = (int64_t)nb * nb;
    const float* src = Pm + (int64_t)slot * total;
    float* dst = Dst + (int64_t)c * total;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
      dst[e] = src[e] * inv;
  }
}

// ||Pm||_F per slot from per-tile partials (fixed reduction order).
__global__ void __launch_bounds__(256) k_lr_frob_part(const float* Pm, int nb, float* part,
                                                      const int* lcount) {
  __shared__ float red[8];
  const int cnt = *lcount;
  for (int slot = blockIdx.y; slot < cnt; slot += gridDim.y) {
    const float* pm = Pm + (int64_t)slot * nb * nb;
    const int64_t total = (int64_t)nb * nb;
    float acc = 0.f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
      acc += pm[e] * pm[e];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[(int64_t)slot * gridDim.x + blockIdx.x] = acc;
  }
}

// Compact entry c belongs to slot list[c]; one workgroup per entry (fixed order).
__global__ void __launch_bounds__(256) k_lr_frob_reduce(const float* part, int tiles,
                                                        const int* lcount, const int* list,
                                                        float* scal, int which) {
  __shared__ float red[256];
  const int cnt = *lcount;
  for (int c = blockIdx.x; c < cnt; c += gridDim.x) {
    float f2 = 0.f;
    for (int t = threadIdx.x; t < tiles; t += 256) f2 += part[(int64_t)c * tiles + t];
    f2 = tree_sum256(f2, red);
    if (threadIdx.x == 0) scal[list[c] * 8 + which] = sqrtf(f2);
  }
}

// Certificate decision; flags per slot: [1] converged (panel rounds skip it),
// [2] handled here (panel gain / rebuild skip it), [3] undecided after stage 0.
// Stage 0 uses the Frobenius bound lambda_max(E^T E) <= ||E^T E||_F; slots it cannot
// certify (but whose coupling passes) wait for stage 1, which uses the bound from the
// eighth power. Fallback slots are listed (block ids) for the LDS Jacobi tier.
__device__ __forceinline__ void lr_certify(int slot, const float* sig, float tau, int* pflag,
                                           unsigned long long* stats) {
  pflag[4 * slot + 1] = 1;
  pflag[4 * slot + 2] = 1;
  int k = 0;
  for (int l = 0; l < 16; ++l) k += sig[slot * 16 + l] > tau;
  atomicAdd(&stats[0], 1ull);
  atomicAdd(&stats[2], (unsigned long long)k);
  atomicAdd(&stats[3], 1ull);
}

// A slot whose certificate failed: its block id goes to fall[] (LDS Jacobi fallback) and
// its slot index to fall[slots + f] (polar fallback); scal[5] keeps the remainder bound
// on lambda_max(E^T E), or, when the coupling test failed (no deflation possible), minus
// the Collatz-Wielandt bound on sigma_max(B)^2 that the Gram bound left there (-inf when
// it is not a positive finite number).
__device__ __forceinline__ float undeflated(float cw) {
  return (cw > 0.f && isfinite(cw)) ? -cw : -__int_as_float(0x7f800000);
}

__device__ __forceinline__ void lr_fallback(int slot, int slots, int* pflag, int* counts,
                                            int* fall, const int* live_list, float* scal,
                                            float bound) {
  pflag[4 * slot + 2] = 0;
  scal[slot * 8 + 5] = bound;
  const int f = atomicAdd(&counts[0], 1);
  fall[f] = live_list[slot];
  fall[slots + f] = slot;
}

// Counters (counts[]): [0] fallback blocks, [1] appends of the stage being decided,
// [2] slots left undecided by the trace bound (listed at fall[3 slots ..]), [3] slots
// left undecided by the stage-0 bounds (listed at fall[2 slots ..]), [4] the A_f list,
// [5] slots the Gram bound left to the subspace iteration (fall[5 slots ..]). Stage -1
// walks that list, stage 0 the trace bound's list, stages 1 and 2 stage 0's.
__global__ void k_lr_decide(const int* live, int slots, float* scal, const float* sig,
                            const float* dmask, float tau, int* pflag, int* counts, int* fall,
                            const int* live_list, unsigned long long* stats, int stage,
                            int power) {
  (void)live;
  const int count = stage < 0 ? counts[5] : stage == 0 ? counts[2] : counts[3];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += gridDim.x * blockDim.x) {
    const int slot = stage < 0 ? fall[5 * slots + idx]
                     : stage == 0 ? fall[3 * slots + idx] : fall[2 * slots + idx];
    const float* sc = scal + slot * 8;
    const float trG = sc[0], c2 = sc[1], trE = sc[2];
    const float lim = tau * tau * (1.f - kCertMargin);
    if (stage < 0) {
      pflag[4 * slot + 3] = 0;
      const bool c_ok = c2 <= kCouplingTol * kCouplingTol * trG && isfinite(c2) && isfinite(trG);
      if (!c_ok) {
        lr_fallback(slot, slots, pflag, counts, fall, live_list, scal, undeflated(scal[slot * 8 + 5]));
        atomicAdd(&stats[4], 1ull);
        continue;
      }
      // lambda_max(E^T E) <= tr(E^T E) = ||B||_F^2 - sum_l ||B v_l||^2 over the deflated
      // and split-off directions (V_r orthonormal), with a rounding allowance of 1e-4
      // ||B||_F^2 for the cancellation; the same 2 x 2 split bound as stage 0
      float s2 = 0.f;
      for (int l = 0; l < 16; ++l) {
        const float sg = sig[slot * 16 + l];
        if (dmask[slot * 16 + l] > 0.f) s2 += sg * sg;
      }
      const float trEF = fmaxf(trG - s2, 0.f) + 1e-4f * trG;
      const float bF = fmaxf(sc[7], trEF) + sqrtf(sc[6]);
      if (bF <= lim && isfinite(bF)) {
        lr_certify(slot, sig, tau, pflag, stats);
      } else {
        const int u = atomicAdd(&counts[1], 1);
        fall[3 * slots + u] = slot;
        atomicAdd(&stats[6], 1ull);   // needs E^T E
      }
      continue;
    }
    if (stage == 0) {
      pflag[4 * slot + 3] = 0;
      const bool c_ok = c2 <= kCouplingTol * kCouplingTol * trG && isfinite(c2) && isfinite(trE);
      if (!c_ok) {
        lr_fallback(slot, slots, pflag, counts, fall, live_list, scal, undeflated(scal[slot * 8 + 5]));
        atomicAdd(&stats[4], 1ull);
        continue;
      }
      // lambda_max(E_L^T E_L) <= max(max_l' sigma_l'^2, lambda_max(E^T E)) + ||A'^T E||_2,
      // l' over the split-off directions, E the remainder after them and L, and
      // ||A'^T E||_F^2 <= sum sigma_l'^2 c_l'^2
      const float b0 = fmaxf(sc[7], trE > 0.f ? trE * sc[4] : 0.f) + sqrtf(sc[6]);
      if (b0 <= lim && isfinite(b0)) {
        lr_certify(slot, sig, tau, pflag, stats);
        // certified thanks to the Collatz-Wielandt bound (the Frobenius one alone fails)
        const float bfro = fmaxf(sc[7], trE > 0.f ? trE * sc[3] : 0.f) + sqrtf(sc[6]);
        if (!(bfro <= lim)) atomicAdd(&stats[7], 1ull);
      } else {
        pflag[4 * slot + 3] = 1;
        const int u = atomicAdd(&counts[1], 1);
        fall[2 * slots + u] = slot;
      }
      continue;
    }
    // sc[3] = ||(E^T E / tr)^power||_F, so lambda_max <= tr * sc[3]^(1/power)
    if (!pflag[4 * slot + 3]) continue;
    const float bp = fmaxf(sc[7], trE > 0.f ? trE * powf(sc[3], 1.f / (float)power) : 0.f) +
                     sqrtf(sc[6]);
    if (bp <= lim && isfinite(bp)) {
      pflag[4 * slot + 3] = 0;
      lr_certify(slot, sig, tau, pflag, stats);
    } else if (stage == 2) {
      pflag[4 * slot + 3] = 0;
      lr_fallback(slot, slots, pflag, counts, fall, live_list, scal, isfinite(bp) ? bp : -1.f);
      atomicAdd(&stats[5], 1ull);
    } else {
      atomicAdd(&counts[1], 1);   // still undecided after this stage
    }
  }
}

// Slots whose rebuild needs A_f = B V_r (a certificate passed with a direction above
// tau) or whose exact fallback deflates with it (a certificate failed), listed at
// list[0 .. *count).
template <int P>
__global__ void k_lr_aflist(const int* live, const int* pflag, const float* sig, float tau,
                            int* list, int* count) {
  const int cnt = *live;
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < cnt;
       slot += gridDim.x * blockDim.x) {
    bool need = !pflag[4 * slot + 2];
    if (!need)
      for (int l = 0; l < P; ++l) need = need || sig[slot * P + l] > tau;
    if (need) list[atomicAdd(count, 1)] = slot;
  }
}

// ------------------------------------------------------------------ driver
// Grid for per-slot kernels: a few workgroups per compute unit, at most one per slot.
static int slot_grid(int slots, int per_cu_target = 4096) {
  int g = per_cu_target;
  if (g > slots) g = slots;
  if (g < 1) g = 1;
  return g;
}

hipError_t run_lowrank(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                       const ShiftSpec& sh, hipStream_t st, hipEvent_t* gram_ev) {
  constexpr int P = 16;
  hipError_t e;
  const int mb = g.mb, nb = g.nb, S = w.slots;
  const int* live = w.live_count;
  const int* list = w.live_list;
  const int64_t sG = (int64_t)nb * nb;
  const int64_t sY = (int64_t)nb * P;
  const int64_t sC = (int64_t)mb * P;
  int* cnt = w.lrCount;
  hipLaunchKernelGGL(k_lr_omega, dim3((nb * P + 255) / 256), dim3(256), 0, st, w.lrOm, nb, P);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, cnt, 6);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // G = B^T B, gathered straight from the iterate (matrix cores)
  if (gram_ev && (e = hipEventRecord(gram_ev[0], st)) != hipSuccess) return e;
  bool rows_done = false;
  if ((e = launch_mf_gram(g, sh, Dout, live, list, S, w.lrG, w.lrSplit, w.lrRow, &rows_done,
                          st)) != hipSuccess)
    return e;
  if (gram_ev && (e = hipEventRecord(gram_ev[1], st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lr_trace, dim3(slot_grid(S)), dim3(256), 0, st, w.lrG, nb, sG, w.lrScal,
                     0, live);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int tn = (nb + 63) / 64;
  const int gtiles = tn * tn;
  const int rgx = (nb + 255) / 256;
  const int dgrid = (S + 255) / 256;
  {
    // zero-output certificate from the Gram matrix alone: the Collatz-Wielandt bound of
    // |G| (r = |G| 1, bound max_i (|G| r)_i / r_i); the slots it cannot settle go on
    // to the subspace iteration (fall[5 S ..], counts[5])
    if (!rows_done) {   // (else the Gram kernel wrote the per-tile |G| row sums)
      hipLaunchKernelGGL(k_lr_gabs_rowpart, dim3(gtiles, slot_grid(S, 8192 / gtiles + 1)),
                         dim3(256), 0, st, w.lrG, nb, w.lrRow, live);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_lr_rsum, dim3(rgx, slot_grid(S, 8192 / rgx + 1)), dim3(256), 0, st,
                       w.lrRow, nb, nullptr, live);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwy, dim3(gtiles, slot_grid(S, 8192 / gtiles + 1)), dim3(256), 0, st,
                       w.lrG, w.lrRow, nb, nullptr, live);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwmax, dim3(slot_grid(S)), dim3(256), 0, st, w.lrRow, nb, w.lrScal,
                       nullptr, live, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_gram_decide, dim3(dgrid), dim3(256), 0, st, live, S, w.lrScal,
                       w.lrSig, tau, w.pflag, cnt, w.lrFall, w.stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int* slist = w.lrFall + 5 * S;
  const int* scount = cnt + 5;
  auto orth = [&](const float* Yin, float* Xout) -> hipError_t {
    const int gw = slot_grid((S + 3) / 4);
    if (nb <= 128)
      hipLaunchKernelGGL((k_lr_orth_w<P, 2>), dim3(gw), dim3(256), 0, st, Yin, Xout, nb, sY,
                         scount, slist);
    else if (nb <= 256)
      hipLaunchKernelGGL((k_lr_orth_w<P, 4>), dim3(gw), dim3(256), 0, st, Yin, Xout, nb, sY,
                         scount, slist);
    else if (nb <= 512)
      hipLaunchKernelGGL((k_lr_orth_w<P, 8>), dim3(gw), dim3(256), 0, st, Yin, Xout, nb, sY,
                         scount, slist);
    else
      hipLaunchKernelGGL(k_lr_orth_cq<P>, dim3(slot_grid(S)), dim3(1024), 0, st, Yin, Xout, nb,
                         sY, scount, slist);
    return hipGetLastError();
  };
  // G X for the slots of a list: barrier-free when nb % 16 == 0
  const bool symx = nb % 16 == 0;
  auto gxl = [&](const float* X, int64_t sX, float* Y, const int* dcount, const int* sl) {
    if (symx) return launch_sym_x(w.lrG, sG, nb, X, sX, nb, Y, sY, dcount, S, sl, w.lrSplit, st);
    return launch_sk(SK_DENSE, false, w.lrG, sG, nb, nullptr, g, sh, list, X, sX, nb, nb, Y, sY,
                     dcount, 0, S, sl, w.lrSkPart, w.lrSkChunks, st);
  };
  auto gx = [&](const float* X, int64_t sX, float* Y) { return gxl(X, sX, Y, scount, slist); };
  // subspace iteration: X0 = orth(G Omega), then X <- orth(G (G X)) three times (seven
  // products by G in total; orthonormalising every second product keeps every
  // direction with sigma > tau / 2 representable while (2 sigma_1 / tau)^4 << 1/eps;
  // an insufficiently converged subspace shows up in the coupling test)
  if ((e = gx(w.lrOm, 0, w.lrY)) != hipSuccess) return e;
  if ((e = orth(w.lrY, w.lrX)) != hipSuccess) return e;
  for (int it = 1; it < 4; ++it) {
    if ((e = gx(w.lrX, sY, w.lrW)) != hipSuccess) return e;
    if ((e = gx(w.lrW, sY, w.lrY)) != hipSuccess) return e;
    if ((e = orth(w.lrY, w.lrX)) != hipSuccess) return e;
  }
  // SVD of the reduced block B X from W0 = G X: sigma, V_r = X W and the coupling
  // product T^T = G V_r (row-major, lrT), all without touching B again
  if ((e = gx(w.lrX, sY, w.lrW)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lr_reduced<P>, dim3(slot_grid(S)), dim3(256), 0, st, w.lrX, w.lrW, nb,
                     w.lrV, w.lrT, w.lrSig, scount, slist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  float* mask = w.lrSig + (size_t)S * P;       // second third of the sigma buffer
  float* dmask = w.lrSig + 2 * (size_t)S * P;  // last third
  hipLaunchKernelGGL(k_lr_coupling<P>, dim3(slot_grid(S)), dim3(256), 0, st, w.lrT, w.lrSig,
                     w.lrV, nb, tau, kCouplingTol, w.lrScal, mask, dmask, scount, slist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // stage -1: the trace bound on lambda_max(E^T E) needs no E^T E; the slots it leaves
  // undecided (fall[3 S ..], counts[2]) get E^T E and its finer bounds
  hipLaunchKernelGGL(k_lr_decide, dim3(dgrid), dim3(256), 0, st, live, S, w.lrScal, w.lrSig,
                     dmask, tau, w.pflag, cnt, w.lrFall, list, w.stats, -1, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, st, cnt + 1, cnt + 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, cnt + 1, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int* flist = w.lrFall + 3 * S;
  const int* fcount = cnt + 2;
  // workgroups per slot of the elementwise passes over E^T E (at most 1024, and the frob
  // partials of one slot must fit in its nb x P part of lrY)
  const int tiles = (int)std::min<int64_t>(std::min<int64_t>((sG + 255) / 256, 1024),
                                           (int64_t)nb * P);
  {
    // E^T E and its bounds: with W = G V_r (the coupling product, lrT), Q = W - V H / 2
    // with H = V^T W (lrY), E^T E = G - Q V^T - V Q^T (lrP, tile partials in lrQ)
    hipLaunchKernelGGL(k_lr_q<P>, dim3(slot_grid(S)), dim3(256), 0, st, w.lrT, w.lrV, dmask, w.lrY,
                       nb, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_lr_ge(w.lrG, w.lrY, w.lrV, w.lrP, nb, w.lrQ, w.lrRow, flist, fcount, S, st)) !=
        hipSuccess)
      return e;
    // stage 0: Frobenius and Collatz-Wielandt bounds of E^T E
    hipLaunchKernelGGL(k_lr_ge_reduce, dim3(slot_grid(S)), dim3(256), 0, st, w.lrQ, gtiles,
                       w.lrScal, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_rsum, dim3(rgx, slot_grid(S, 8192 / rgx + 1)), dim3(256), 0, st,
                       w.lrRow, nb, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwy, dim3(gtiles, slot_grid(S, 8192 / gtiles + 1)), dim3(256), 0, st,
                       w.lrP, w.lrRow, nb, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwmax, dim3(slot_grid(S)), dim3(256), 0, st, w.lrRow, nb, w.lrScal,
                       flist, fcount, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_decide, dim3(dgrid), dim3(256), 0, st, live, S, w.lrScal, w.lrSig,
                       dmask, tau, w.pflag, cnt, w.lrFall, list, w.stats, 0, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, st, cnt + 1, cnt + 3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    // stage 1: square of E^T E / tr(E^T E); stage 2: its fourth power (eighth in all),
    // on the slots still undecided (fall[2 S ..], counts[3]), gathered to compact
    // positions (lrQ, then lrP); every launch is empty when none is left
    const int* ulist = w.lrFall + 2 * S;
    const int* ucount = cnt + 3;
    hipLaunchKernelGGL(k_lr_gather_scale, dim3(tiles, slot_grid(S, 8192 / tiles + 1)), dim3(256),
                       0, st, w.lrP, w.lrQ, nb, ulist, ucount, w.lrScal);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* a = w.lrQ;
    float* b = w.lrP;
    int power = 1;
    for (int stage = 1; stage <= 2; ++stage) {
      const int nsq = stage == 1 ? 1 : 2;
      for (int s2 = 0; s2 < nsq; ++s2) {
        // the matrices are symmetric (E^T E / tr and its exactly symmetric powers), so
        // the square is the Gram a^T a: half the tiles
        if ((e = launch_syrk(nb, nb, a, nb, sG, b, nb, sG, ucount, 0, S, st)) != hipSuccess)
          return e;
        float* t = a;
        a = b;
        b = t;
        power *= 2;
      }
      // partials go to lrY (free after stage 0); lrT keeps A_f^T B for the polar route
      hipLaunchKernelGGL(k_lr_frob_part, dim3(tiles, slot_grid(S, 8192 / tiles + 1)), dim3(256), 0,
                         st, a, nb, w.lrY, ucount);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_lr_frob_reduce, dim3(slot_grid(S)), dim3(256), 0, st, w.lrY, tiles,
                         ucount, ulist, w.lrScal, 3);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, cnt + 1, 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_lr_decide, dim3(dgrid), dim3(256), 0, st, live, S, w.lrScal, w.lrSig,
                         dmask, tau, w.pflag, cnt, w.lrFall, list, w.stats, stage, power);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // A_f = B V_r (B gathered) for the slots that need it: a rebuild with a direction above
  // tau, or an exact fallback that deflates with it (listed at fall[4 S ..], counts[4])
  int* aflist = w.lrFall + 4 * S;
  int* afcount = cnt + 4;
  hipLaunchKernelGGL(k_lr_aflist<P>, dim3(dgrid), dim3(256), 0, st, live, w.pflag, w.lrSig, tau,
                     aflist, afcount);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // (blocks 1024 wide or more split the contraction over the nb columns in 256-column
  // chunks, blocks 768 to 1023 wide in 128-column chunks: functions of the shape alone)
  const bool gsplit = w.lrSplit && nb >= 1024;
  const int afsplit = gsplit ? (nb + 255) / 256 : w.lrSkChunks;
  float* afpart = gsplit ? w.lrSplit : w.lrSkPart;
  if ((e = launch_sk(SK_B, false, nullptr, 0, 0, Dout, g, sh, list, w.lrV, sY, mb, nb, w.lrC, sC,
                     afcount, 0, S, aflist, afpart, afsplit, st)) != hipSuccess)
    return e;
  // Z = sum_{l in L} (1 - tau / sigma_l) a_l v_l^T for certified slots (matrix cores),
  // scattered to the shifted coordinates with D' = 2 Z' - V
  return launch_mf_rebuild(g, sh, Zout, Dout, afcount, aflist, list, S, w.pflag, w.lrC, w.lrV,
                           w.lrSig, nullptr, tau, st);
}

}  // namespace msld
