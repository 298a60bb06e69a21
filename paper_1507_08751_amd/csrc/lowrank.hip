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
// in LDS, else the polar route (polar.hip). The plain matrix products (Gram, subspace
// products, squarings) are rocBLAS batched GEMMs; the orthonormalisation, the reduced
// SVD, the certificate and the rebuild are the kernels below.
#include <rocblas/rocblas.h>

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
                                                  float* scal, int which) {
  __shared__ float red[8];
  const int slot = blockIdx.x;
  const float* g = G + (int64_t)slot * strideG;
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += g[(int64_t)i * nb + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) scal[slot * 8 + which] = s;
}

// Orthonormalise the p columns of Y (nb x p, column-major) into X by classical
// Gram-Schmidt with re-orthogonalisation until a pass keeps at least half the norm
// (at most 4 passes); a column that stays numerically dependent is set to zero.
template <int P>
__global__ void __launch_bounds__(256) k_lr_orth(const float* Y, float* X, int nb,
                                                 int64_t stride) {
  extern __shared__ float sy[];  // P x nb
  __shared__ float red[4 * P];
  __shared__ float coef[P];
  const int slot = blockIdx.x;
  const float* y = Y + (int64_t)slot * stride;
  float* x = X + (int64_t)slot * stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < nb * P; e += blockDim.x) sy[e] = y[e];
  __syncthreads();
  for (int j = 0; j < P; ++j) {
    float* yj = sy + j * nb;
    // original norm
    float n0 = 0.f;
    for (int r = tid; r < nb; r += blockDim.x) n0 += yj[r] * yj[r];
    n0 = block_sum(n0, red);
    float nprev = n0;
    bool dependent = true;
    for (int pass = 0; pass < 4 && j > 0; ++pass) {
      float part[P];
#pragma unroll
      for (int i = 0; i < P; ++i) part[i] = 0.f;
      for (int r = tid; r < nb; r += blockDim.x) {
        const float v = yj[r];
#pragma unroll
        for (int i = 0; i < P; ++i)
          if (i < j) part[i] += sy[i * nb + r] * v;
      }
#pragma unroll
      for (int i = 0; i < P; ++i) {
        float v = part[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        part[i] = v;
      }
      __syncthreads();
      if (lane == 0)
        for (int i = 0; i < j; ++i) red[wv * P + i] = part[i];
      __syncthreads();
      if (tid < j) coef[tid] = red[tid] + red[P + tid] + red[2 * P + tid] + red[3 * P + tid];
      __syncthreads();
      for (int r = tid; r < nb; r += blockDim.x) {
        float v = yj[r];
        for (int i = 0; i < j; ++i) v -= coef[i] * sy[i * nb + r];
        yj[r] = v;
      }
      __syncthreads();
      float nn = 0.f;
      for (int r = tid; r < nb; r += blockDim.x) nn += yj[r] * yj[r];
      nn = block_sum(nn, red);
      if (nn >= 0.25f * nprev) {   // norm kept above 1/2: orthogonal to working precision
        dependent = false;
        nprev = nn;
        break;
      }
      nprev = nn;
    }
    if (j == 0) dependent = false;
    const float nrm = sqrtf(nprev);
    const bool keep = !dependent && nrm > 1e-30f && nprev > 1e-12f * n0;
    const float inv = keep ? 1.f / nrm : 0.f;
    for (int r = tid; r < nb; r += blockDim.x) yj[r] = yj[r] * inv;
    __syncthreads();
  }
  for (int e = tid; e < nb * P; e += blockDim.x) x[e] = sy[e];
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Orthonormalisation with one wave per slot and the columns held in registers
// (lane l owns rows l + 64 r, r < RPL): no LDS and no workgroup barriers. Classical
// Gram-Schmidt with exactly two projection passes ("twice is enough"); a column whose
// norm drops below half in both passes is numerically dependent and set to zero. The
// fixed pass count keeps every register index static.
template <int P, int RPL>
__global__ void __launch_bounds__(256) k_lr_orth_w(const float* Y, float* X, int nb,
                                                   int64_t stride, int count) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = blockIdx.x * 4 + wv;
  if (slot >= count) return;  // the whole wave leaves together
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

// Round-robin pair order of a cyclic Jacobi sweep over ncols (even) indices: ncols - 1
// rounds of ncols / 2 disjoint pairs (the same order as the tiers in kernels.hip, which
// is not visible from this translation unit).
__device__ __forceinline__ void lr_pair(int round, int k, int ncols, int* a, int* b) {
  const int n1 = ncols - 1;
  *a = (k == 0) ? 0 : 1 + (k - 1 + round) % n1;
  *b = 1 + (ncols - 2 - k + round) % n1;
}

// SVD of the reduced block C = B X (mb x p): the p x p Gram K = C^T C accumulated in
// float64 over row chunks and its eigen-decomposition K = W diag(lambda) W^T by cyclic
// two-sided Jacobi in float64 (parallel pair order): A_f = C W (orthogonal columns
// a_l = sigma_l u_l), sigma_l = sqrt(lambda_l), V_r = X W. The coupling test of the
// certificate bounds what the float32 product C W loses in orthogonality.
template <int P>
__global__ void __launch_bounds__(256) k_lr_gram64(const float* C, int mb, int rows,
                                                   double* part, int64_t part_stride) {
  static_assert(P * P == 256, "one Gram entry per thread");
  __shared__ float tile[64][P + 1];
  const int slot = blockIdx.y, ch = blockIdx.x;
  const float* c = C + (int64_t)slot * mb * P;
  const int r0 = ch * rows;
  const int r1 = min(mb, r0 + rows);
  const int tid = threadIdx.x;
  const int a = tid / P, b = tid - (tid / P) * P;
  double acc = 0.0;
  for (int t0 = r0; t0 < r1; t0 += 64) {
    for (int e = tid; e < 64 * P; e += 256) {
      const int j = e / 64, r = e - j * 64;
      tile[r][j] = (t0 + r < r1) ? c[(int64_t)j * mb + t0 + r] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 64; ++r) acc += (double)tile[r][a] * (double)tile[r][b];
    __syncthreads();
  }
  part[(int64_t)slot * part_stride + (int64_t)ch * 256 + tid] = acc;
}

template <int P>
__global__ void __launch_bounds__(256) k_lr_eig64(const double* part, int chunks,
                                                  int64_t part_stride, const float* X,
                                                  float* Vr, float* sig, float* Wf, int nb) {
  __shared__ double K[P][P + 1];
  __shared__ double V[P][P + 1];
  __shared__ double cs[P / 2], sn[P / 2];
  __shared__ int s_rot;
  const int slot = blockIdx.x, tid = threadIdx.x;
  const double* pp = part + (int64_t)slot * part_stride;
  if (tid < P * P) {
    double k = 0.0;
    for (int ch = 0; ch < chunks; ++ch) k += pp[(int64_t)ch * 256 + tid];
    K[tid / P][tid % P] = k;
    V[tid / P][tid % P] = (tid / P == tid % P) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sw = 0; sw < 40; ++sw) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rd = 0; rd < P - 1; ++rd) {
      if (tid < P / 2) {
        int p, q;
        lr_pair(rd, tid, P, &p, &q);
        const double app = K[p][p], aqq = K[q][q], apq = K[p][q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-14 * sqrt(fabs(app) * fabs(aqq))) {
          const double th = (aqq - app) / (2.0 * apq);
          const double t = fabs(th) > 1e150 ? 0.5 / th
                                            : copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          s_rot = 1;
        }
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      if (tid < (P / 2) * P) {   // K <- K J and V <- V J (columns p, q of every pair)
        const int k = tid / P, r = tid - (tid / P) * P;
        int p, q;
        lr_pair(rd, k, P, &p, &q);
        const double c = cs[k], s = sn[k];
        const double kp = K[r][p], kq = K[r][q];
        K[r][p] = c * kp - s * kq;
        K[r][q] = s * kp + c * kq;
        const double vp = V[r][p], vq = V[r][q];
        V[r][p] = c * vp - s * vq;
        V[r][q] = s * vp + c * vq;
      }
      __syncthreads();
      if (tid < (P / 2) * P) {   // K <- J^T K (rows p, q)
        const int k = tid / P, col = tid - (tid / P) * P;
        int p, q;
        lr_pair(rd, k, P, &p, &q);
        const double c = cs[k], s = sn[k];
        const double kp = K[p][col], kq = K[q][col];
        K[p][col] = c * kp - s * kq;
        K[q][col] = s * kp + c * kq;
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }
  if (tid < P) sig[slot * P + tid] = (float)sqrt(fmax(K[tid][tid], 0.0));
  float* wf = Wf + (int64_t)slot * P * P;
  if (tid < P * P) wf[tid] = (float)V[tid / P][tid % P];   // row j, column l: W_jl
  const float* x = X + (int64_t)slot * nb * P;
  float* vr = Vr + (int64_t)slot * nb * P;
  for (int e = tid; e < nb * P; e += blockDim.x) {
    const int l = e / nb, row = e - l * nb;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) v += (double)x[j * nb + row] * V[j][l];
    vr[e] = (float)v;
  }
}

// C <- C W per slot (A_f of the tall path), one row per thread.
template <int P>
__global__ void __launch_bounds__(256) k_lr_rot_c(float* C, const float* Wf, int mb) {
  __shared__ float w[P * P];
  const int slot = blockIdx.y;
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) w[e] = Wf[(int64_t)slot * P * P + e];
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mb) return;
  float* c = C + (int64_t)slot * mb * P;
  float v[P];
#pragma unroll
  for (int j = 0; j < P; ++j) v[j] = c[(int64_t)j * mb + r];
#pragma unroll
  for (int l = 0; l < P; ++l) {
    float o = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) o += v[j] * w[j * P + l];
    c[(int64_t)l * mb + r] = o;
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
                                                     float* dmask) {
  __shared__ float red[8];
  __shared__ float cl[P];
  const int slot = blockIdx.x;
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

// Q = W - V H / 2 over the columns the mask selects (others zero), with W = G V_r and
// H = V^T W (P x P, from a batched GEMM), so that E^T E = G - Q V^T - V Q^T for the
// remainder E = B (I - V V^T) of the masked columns V.
template <int P>
__global__ void __launch_bounds__(256) k_lr_q(const float* Wg, const float* Vr, const float* H,
                                              const float* mask, float* Qo, int nb) {
  __shared__ float h[P * P];
  __shared__ float mk[P];
  const int slot = blockIdx.x;
  const float* w = Wg + (int64_t)slot * nb * P;
  const float* v = Vr + (int64_t)slot * nb * P;
  float* q = Qo + (int64_t)slot * nb * P;
  if (threadIdx.x < P) mk[threadIdx.x] = mask[slot * P + threadIdx.x];
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) h[e] = H[(int64_t)slot * P * P + e];
  __syncthreads();
  for (int e = threadIdx.x; e < nb * P; e += blockDim.x) {
    const int k = e / nb, r = e - k * nb;
    float s = 0.f;
    if (mk[k] > 0.f) {
      float vh = 0.f;
#pragma unroll
      for (int l = 0; l < P; ++l)
        if (mk[l] > 0.f) vh += v[l * nb + r] * h[k * P + l];   // H symmetric: H[l][k]
      s = w[e] - 0.5f * vh;
    }
    q[e] = s;
  }
}

// E^T E = G - Q V^T - V Q^T (masked columns of V_r) on 64 x 64 tiles, to Pm, with
// per-tile partial trace and squared Frobenius norm. Q and V rows of the tile's row
// and column ranges are staged in LDS; each thread accumulates a 2 x 8 block (rows
// i0 + il + 32 a, columns j0 + jg + 8 b), so one LDS value feeds several FMAs, and
// each wave reads and writes 128-byte column segments of G and Pm.
template <int P>
__global__ void __launch_bounds__(256) k_lr_ge(const float* G, const float* Qm, const float* Vr,
                                               const float* mask, float* Pm, int nb,
                                               float* part, float* rowpart, const int* list,
                                               const int* lcount) {
  __shared__ float qi[64][P + 1], vi[64][P + 1], qj[64][P + 1], vj[64][P + 1];
  __shared__ float mk[P];
  __shared__ float red[8];
  __shared__ float rs[8][64];
  if (lcount && (int)blockIdx.y >= *lcount) return;
  const int slot = list ? list[blockIdx.y] : blockIdx.y;
  const int tn = (nb + 63) / 64;
  const int ti = blockIdx.x % tn, tj = blockIdx.x / tn;
  const int i0 = ti * 64, j0 = tj * 64;
  const float* g = G + (int64_t)slot * nb * nb;
  const float* q = Qm + (int64_t)slot * nb * P;
  const float* v = Vr + (int64_t)slot * nb * P;
  float* pm = Pm + (int64_t)slot * nb * nb;
  const int tid = threadIdx.x;
  if (tid < P) mk[tid] = mask[slot * P + tid];
  __syncthreads();
  for (int e = tid; e < 64 * P; e += 256) {
    const int l = e / 64, r = e - l * 64;
    const bool m = mk[l] > 0.f;
    const int ri = i0 + r, rj = j0 + r;
    qi[r][l] = ri < nb ? q[l * nb + ri] : 0.f;
    vi[r][l] = (m && ri < nb) ? v[l * nb + ri] : 0.f;
    qj[r][l] = rj < nb ? q[l * nb + rj] : 0.f;
    vj[r][l] = (m && rj < nb) ? v[l * nb + rj] : 0.f;
  }
  __syncthreads();
  const int il = tid & 31;
  const int jg = tid >> 5;
  float acc[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.f;
#pragma unroll 4
  for (int l = 0; l < P; ++l) {
    const float qa0 = qi[il][l], qa1 = qi[il + 32][l];
    const float va0 = vi[il][l], va1 = vi[il + 32][l];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const float qb = qj[jg + 8 * b][l], vb = vj[jg + 8 * b][l];
      acc[0][b] += qa0 * vb + va0 * qb;
      acc[1][b] += qa1 * vb + va1 * qb;
    }
  }
  float tr = 0.f, f2 = 0.f;
  float ra[2] = {0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = i0 + il + 32 * a;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int j = j0 + jg + 8 * b;
      if (i < nb && j < nb) {
        const float sv = g[(int64_t)j * nb + i] - acc[a][b];
        pm[(int64_t)j * nb + i] = sv;
        if (i == j) tr += sv;
        f2 += sv * sv;
        ra[a] += fabsf(sv);
      }
    }
  }
  rs[jg][il] = ra[0];
  rs[jg][il + 32] = ra[1];
  tr = block_sum(tr, red);   // its barriers also order the rs writes before the reads
  f2 = block_sum(f2, red);
  if (tid == 0) {
    part[((int64_t)slot * gridDim.x + blockIdx.x) * 2] = tr;
    part[((int64_t)slot * gridDim.x + blockIdx.x) * 2 + 1] = f2;
  }
  // partial row |.| sums of this tile column (rows i0.., columns j0..j0+63)
  if (tid < 64 && i0 + tid < nb) {
    float r = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) r += rs[k][tid];
    rowpart[(int64_t)slot * nb * (tn + 1) + (int64_t)tj * nb + i0 + tid] = r;
  }
}

// Collatz-Wielandt bound for the symmetric M = E^T E (in Pm): with r = |M| 1 and
// y = |M| r, lambda_max(M) <= rho(|M|) <= max_i y_i / r_i (a row with r_i = 0 is zero).
// Three small steps on the tile partials, all in a fixed summation order:
// k_lr_rsum: r_i = sum over tile columns of the row partials of k_lr_ge (slice tn);
// k_lr_cwy: per 64 x 64 tile, partial y_i over its columns (slices 0..tn-1);
// k_lr_cwmax: y_i, the ratio, its maximum; scal[4] = min(||M||_F, bound) / tr(M).
__global__ void __launch_bounds__(256) k_lr_rsum(float* rowpart, int nb, const int* list,
                                                 const int* lcount) {
  if (lcount && (int)blockIdx.y >= *lcount) return;
  const int slot = list ? list[blockIdx.y] : blockIdx.y;
  const int tn = (nb + 63) / 64;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
  float v = 0.f;
  for (int t = 0; t < tn; ++t) v += rp[(int64_t)t * nb + i];
  rp[(int64_t)tn * nb + i] = v;
}

__global__ void __launch_bounds__(256) k_lr_cwy(const float* Pm, float* rowpart, int nb,
                                                const int* list, const int* lcount) {
  __shared__ float rj[64];
  __shared__ float ys[4][64];
  if (lcount && (int)blockIdx.y >= *lcount) return;
  const int slot = list ? list[blockIdx.y] : blockIdx.y;
  const int tn = (nb + 63) / 64;
  const int ti = blockIdx.x % tn, tj = blockIdx.x / tn;
  const int i0 = ti * 64, j0 = tj * 64;
  float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
  const float* pm = Pm + (int64_t)slot * nb * nb;
  const int tid = threadIdx.x;
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

__global__ void __launch_bounds__(256) k_lr_cwmax(const float* rowpart, int nb, float* scal,
                                                  const int* list, const int* lcount) {
  __shared__ float red[8];
  if (lcount && (int)blockIdx.x >= *lcount) return;
  const int slot = list ? list[blockIdx.x] : blockIdx.x;
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
  if (lane == 0) red[wv] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = fmaxf(b, red[w]);
    const float tr = scal[slot * 8 + 2];
    if (tr > 0.f && isfinite(b)) scal[slot * 8 + 4] = fminf(scal[slot * 8 + 4], b / tr);
  }
}

// Reduce the per-tile partials of k_lr_ge in a fixed order: scal[2] = tr(E^T E),
// scal[4] = ||E^T E||_F / tr(E^T E) (stage-0 bound factor).
__global__ void k_lr_ge_reduce(const float* part, int tiles, int count, float* scal,
                               const int* list, const int* lcount) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count || (lcount && idx >= *lcount)) return;
  const int slot = list ? list[idx] : idx;
  float tr = 0.f, f2 = 0.f;
  for (int t = 0; t < tiles; ++t) {
    tr += part[((int64_t)slot * tiles + t) * 2];
    f2 += part[((int64_t)slot * tiles + t) * 2 + 1];
  }
  scal[slot * 8 + 2] = tr;
  scal[slot * 8 + 4] = tr > 0.f ? sqrtf(f2) / tr : 0.f;
}

// Gather the undecided slots' E^T E (slot-indexed Pm) into compact positions of Dst,
// scaled by 1 / tr(E^T E) (0 stays 0), so that the squarings only touch those slots.
__global__ void k_lr_gather_scale(const float* Pm, float* Dst, int nb, const int* list,
                                  const float* scal) {
  const int c = blockIdx.y;
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

// ||Pm||_F per slot from per-tile partials (fixed reduction order).
__global__ void __launch_bounds__(256) k_lr_frob_part(const float* Pm, int nb, float* part) {
  __shared__ float red[8];
  const int slot = blockIdx.y;
  const float* pm = Pm + (int64_t)slot * nb * nb;
  const int64_t total = (int64_t)nb * nb;
  float acc = 0.f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    acc += pm[e] * pm[e];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)slot * gridDim.x + blockIdx.x] = acc;
}

// Compact entry c belongs to slot list[c].
__global__ void k_lr_frob_reduce(const float* part, int tiles, int count, const int* list,
                                 float* scal, int which) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  float f2 = 0.f;
  for (int t = 0; t < tiles; ++t) f2 += part[(int64_t)c * tiles + t];
  scal[list[c] * 8 + which] = sqrtf(f2);
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
// on lambda_max(E^T E), or -1 when the coupling test failed (no deflation possible).
__device__ __forceinline__ void lr_fallback(int slot, int slots, int* pflag, int* counts,
                                            int* fall, const int* live_list, float* scal,
                                            float bound) {
  pflag[4 * slot + 2] = 0;
  scal[slot * 8 + 5] = bound;
  const int f = atomicAdd(&counts[0], 1);
  fall[f] = live_list[slot];
  fall[slots + f] = slot;
}

__global__ void k_lr_decide(int count, int slots, float* scal, const float* sig,
                            const float* dmask, float tau, int* pflag, int* counts, int* fall,
                            const int* live_list, unsigned long long* stats, int stage,
                            int power) {
  // stage -1 walks all slots and lists the undecided ones at fall[3 slots ..] (their
  // count ends in counts[2]); stage 0 walks that list and lists its undecided ones at
  // fall[2 slots ..]; later stages walk that second list
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count || (stage == 0 && idx >= counts[2])) return;
  const int slot = stage < 0 ? idx : stage == 0 ? fall[3 * slots + idx] : fall[2 * slots + idx];
  const float* sc = scal + slot * 8;
  const float trG = sc[0], c2 = sc[1], trE = sc[2];
  const float lim = tau * tau * (1.f - kCertMargin);
  if (stage < 0) {
    pflag[4 * slot + 3] = 0;
    const bool c_ok = c2 <= kCouplingTol * kCouplingTol * trG && isfinite(c2) && isfinite(trG);
    if (!c_ok) {
      lr_fallback(slot, slots, pflag, counts, fall, live_list, scal, -1.f);
      atomicAdd(&stats[4], 1ull);
      return;
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
    }
    return;
  }
  if (stage == 0) {
    pflag[4 * slot + 3] = 0;
    const bool c_ok = c2 <= kCouplingTol * kCouplingTol * trG && isfinite(c2) && isfinite(trE);
    if (!c_ok) {
      lr_fallback(slot, slots, pflag, counts, fall, live_list, scal, -1.f);
      atomicAdd(&stats[4], 1ull);
      return;
    }
    // lambda_max(E_L^T E_L) <= max(max_l' sigma_l'^2, lambda_max(E^T E)) + ||A'^T E||_2,
    // l' over the split-off directions, E the remainder after them and L, and
    // ||A'^T E||_F^2 <= sum sigma_l'^2 c_l'^2
    const float b0 = fmaxf(sc[7], trE > 0.f ? trE * sc[4] : 0.f) + sqrtf(sc[6]);
    if (b0 <= lim && isfinite(b0)) {
      lr_certify(slot, sig, tau, pflag, stats);
    } else {
      pflag[4 * slot + 3] = 1;
      const int u = atomicAdd(&counts[1], 1);
      fall[2 * slots + u] = slot;
    }
  } else {
    // sc[3] = ||(E^T E / tr)^power||_F, so lambda_max <= tr * sc[3]^(1/power)
    if (!pflag[4 * slot + 3]) return;
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

// Z = sum_{l in L} (1 - tau/sigma_l) a_l v_l^T for certified slots, scattered to the
// shifted block coordinates with the dual update D' = 2 Z' - V.
template <int P>
__global__ void __launch_bounds__(256) k_lr_rebuild(float* __restrict__ Zout,
                                                    float* __restrict__ Dout, ScaleGeom g,
                                                    ShiftSpec sh, const int* live_list,
                                                    const int* pflag, const float* Af,
                                                    const float* Vr, const float* sig,
                                                    float tau) {
  __shared__ float gl[P];
  __shared__ int s_any;
  const int N = g.N, m = g.m, n = g.n, Q = g.Q, mb = g.mb, nb = g.nb;
  const int slot = blockIdx.y;
  if (!pflag[4 * slot + 2]) return;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (threadIdx.x < P) {
    const float s = sig[slot * P + threadIdx.x];
    gl[threadIdx.x] = s > tau ? 1.f - tau / s : 0.f;
    if (s > tau) s_any = 1;
  }
  __syncthreads();
  if (!s_any) return;   // Z = 0: the stream pass already wrote Z' = 0, D' = -V
  const int blk = live_list[slot];
  const int p = blk / Q, q = blk - p * Q;
  int sr, sc;
  block_shift(sh, p / g.PI, m, n, &sr, &sc);
  const float* af = Af + (int64_t)slot * mb * P;
  const float* vr = Vr + (int64_t)slot * nb * P;
  const int tilesj = (n + 31) / 32;
  const int ti = blockIdx.x / tilesj, tj = blockIdx.x - (blockIdx.x / tilesj) * tilesj;
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int i = ti * 32 + (e >> 5), j = tj * 32 + (e & 31);
    if (i >= m || j >= n) continue;
    const int r = g.trans ? j : i;
    const int c = g.trans ? i : j;
    float z = 0.f;
#pragma unroll
    for (int l = 0; l < P; ++l)
      if (gl[l] > 0.f) z += gl[l] * af[l * mb + r] * vr[l * nb + c];
    const int64_t o = (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc);
    const float v = -Dout[o];
    Zout[o] = z;
    Dout[o] = 2.f * z - v;
  }
}

// ------------------------------------------------ split-K products of tall blocks
// C = A^T B for blocks with many more rows than columns (A: K x Ma, B: K x Nb, both
// column-major with leading dimension K, slot strides sa, sb), when too few output
// tiles exist to fill the chip: the rows are split into `chunks` ranges of KC rows,
// each workgroup forms one 64 x 64 output tile of one range, and a second kernel
// sums the ranges in a fixed order into C (leading dimension ldc, slot stride sc).
__global__ void __launch_bounds__(256) k_tall_atb_part(const float* __restrict__ A, int64_t sa,
                                                       int Ma, const float* __restrict__ B,
                                                       int64_t sb, int Nb, int K, int KC,
                                                       float* __restrict__ part, int chunks) {
  __shared__ float As[32][64 + 4];
  __shared__ float Bs[32][64 + 4];
  const int tilesN = (Nb + 63) / 64;
  const int ti = blockIdx.x / tilesN, tj = blockIdx.x - (blockIdx.x / tilesN) * tilesN;
  const int ch = blockIdx.y, slot = blockIdx.z;
  const float* a = A + (int64_t)slot * sa;
  const float* b = B + (int64_t)slot * sb;
  const int k0 = ch * KC, k1 = min(K, k0 + KC);
  const int t = threadIdx.x;
  const int ty = t / 16, tx = t - (t / 16) * 16;
  float acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.f;
  for (int kb = k0; kb < k1; kb += 32) {
    const int kk = t & 31;
    const int k = kb + kk;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = (t >> 5) + 8 * u;
      const int ia = ti * 64 + c, jb = tj * 64 + c;
      As[kk][c] = (k < k1 && ia < Ma) ? a[(int64_t)ia * K + k] : 0.f;
      Bs[kk][c] = (k < k1 && jb < Nb) ? b[(int64_t)jb * K + k] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int q = 0; q < 32; ++q) {
      const float4 x = *reinterpret_cast<const float4*>(&As[q][ty * 4]);
      const float4 y = *reinterpret_cast<const float4*>(&Bs[q][tx * 4]);
      const float xa[4] = {x.x, x.y, x.z, x.w}, yb[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += xa[u] * yb[v];
    }
    __syncthreads();
  }
  float* o = part + ((int64_t)slot * chunks + ch) * Ma * Nb;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 64 + ty * 4 + u, j = tj * 64 + tx * 4 + v;
      if (i < Ma && j < Nb) o[(int64_t)j * Ma + i] = acc[u][v];
    }
}

__global__ void __launch_bounds__(256) k_tall_atb_sum(const float* __restrict__ part, int Ma,
                                                      int Nb, int chunks, float* __restrict__ C,
                                                      int ldc, int64_t sc) {
  const int slot = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Ma * Nb) return;
  const int j = e / Ma, i = e - (e / Ma) * Ma;
  const float* pp = part + (int64_t)slot * chunks * Ma * Nb;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += pp[(int64_t)c * Ma * Nb + e];
  C[(int64_t)slot * sc + (int64_t)j * ldc + i] = s;
}

// Split-K A^T B when it pays (tall blocks, few output tiles, partials fit `cap`
// floats); returns false (nothing launched) otherwise.
static bool tall_atb(const float* A, int64_t sa, int Ma, const float* B, int64_t sb, int Nb,
                     int K, float* C, int ldc, int64_t sc, int count, float* part, size_t cap,
                     hipStream_t st, hipError_t* err) {
  *err = hipSuccess;
  if (!part || K < 4 * Nb) return false;
  const int tiles = ((Ma + 63) / 64) * ((Nb + 63) / 64);
  if ((int64_t)count * tiles >= 256) return false;
  int chunks = (K + 255) / 256;
  if (chunks > 64) chunks = 64;
  while (chunks > 1 && (size_t)count * chunks * Ma * Nb > cap) --chunks;
  if (chunks < 2) return false;
  int KC = (K + chunks - 1) / chunks;
  KC = (KC + 31) / 32 * 32;
  chunks = (K + KC - 1) / KC;
  hipLaunchKernelGGL(k_tall_atb_part, dim3(tiles, chunks, count), dim3(256), 0, st, A, sa, Ma, B,
                     sb, Nb, K, KC, part, chunks);
  if ((*err = hipGetLastError()) != hipSuccess) return true;
  hipLaunchKernelGGL(k_tall_atb_sum, dim3((Ma * Nb + 255) / 256, count), dim3(256), 0, st, part,
                     Ma, Nb, chunks, C, ldc, sc);
  *err = hipGetLastError();
  return true;
}

// ------------------------------------------------------------------ driver
hipError_t batched_sgemm(void* blas, bool ta, bool tb, int m, int n, int k, const float* A,
                         int lda, int64_t sa, const float* B, int ldb, int64_t sb, float* C,
                         int ldc, int64_t sc, int batch) {
  const float one = 1.f, zero = 0.f;
  rocblas_status s = rocblas_sgemm_strided_batched(
      reinterpret_cast<rocblas_handle>(blas), ta ? rocblas_operation_transpose : rocblas_operation_none,
      tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k, &one, A, lda, sa, B, ldb,
      sb, &zero, C, ldc, sc, batch);
  return s == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

static hipError_t gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m,
                       int n, int k, const float* A, int lda, int64_t sa, const float* B, int ldb,
                       int64_t sb, float* C, int ldc, int64_t sc, int batch) {
  return batched_sgemm(h, ta == rocblas_operation_transpose, tb == rocblas_operation_transpose,
                       m, n, k, A, lda, sa, B, ldb, sb, C, ldc, sc, batch);
}

hipError_t run_lowrank(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                       const ShiftSpec& sh, float jtol, int count, int* fallback_host,
                       hipStream_t st) {
  constexpr int P = 16;
  hipError_t e;
  rocblas_handle h = reinterpret_cast<rocblas_handle>(w.blas);
  const int mb = g.mb, nb = g.nb;
  const int64_t sB = (int64_t)w.nbp * mb;   // pA slot stride
  const int64_t sG = (int64_t)nb * nb;
  const int64_t sY = (int64_t)nb * P;
  const int64_t sC = (int64_t)mb * P;
  hipLaunchKernelGGL(k_lr_omega, dim3((nb * P + 255) / 256), dim3(256), 0, st, w.lrOm, nb, P);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, w.lrCount, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // G = B^T B (split-K for tall blocks)
  if (!tall_atb(w.pA, sB, nb, w.pA, sB, nb, mb, w.lrG, nb, sG, count, w.lrSplit, kSplitFloats,
                st, &e)) {
    if ((e = gemm(h, rocblas_operation_transpose, rocblas_operation_none, nb, nb, mb, w.pA, mb,
                  sB, w.pA, mb, sB, w.lrG, nb, sG, count)) != hipSuccess)
      return e;
  } else if (e != hipSuccess) {
    return e;
  }
  hipLaunchKernelGGL(k_lr_trace, dim3(count), dim3(256), 0, st, w.lrG, nb, sG, w.lrScal, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // subspace iteration: X0 = orth(G Omega), then X <- orth(G (G X)) three times
  // (seven products by G in total; orthonormalising every second product keeps every
  // direction with sigma > tau / 2 representable while (2 sigma_1 / tau)^4 << 1/eps;
  // an insufficiently converged subspace shows up in the coupling test)
  const int q = 4;
  for (int it = 0; it < q; ++it) {
    if (it == 0) {
      if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, nb, P, nb, w.lrG, nb, sG,
                    w.lrOm, nb, 0, w.lrY, nb, sY, count)) != hipSuccess)
        return e;
    } else {
      if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, nb, P, nb, w.lrG, nb, sG,
                    w.lrX, nb, sY, w.lrW, nb, sY, count)) != hipSuccess)
        return e;
      if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, nb, P, nb, w.lrG, nb, sG,
                    w.lrW, nb, sY, w.lrY, nb, sY, count)) != hipSuccess)
        return e;
    }
    if (nb <= 128)
      hipLaunchKernelGGL((k_lr_orth_w<P, 2>), dim3((count + 3) / 4), dim3(256), 0, st, w.lrY,
                         w.lrX, nb, sY, count);
    else if (nb <= 256)
      hipLaunchKernelGGL((k_lr_orth_w<P, 4>), dim3((count + 3) / 4), dim3(256), 0, st, w.lrY,
                         w.lrX, nb, sY, count);
    else if (nb <= 512)
      hipLaunchKernelGGL((k_lr_orth_w<P, 8>), dim3((count + 3) / 4), dim3(256), 0, st, w.lrY,
                         w.lrX, nb, sY, count);
    else
      hipLaunchKernelGGL(k_lr_orth<P>, dim3(count), dim3(256), (size_t)4 * nb * P, st, w.lrY,
                         w.lrX, nb, sY);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // C = B X, then its SVD: the float64 Gram C^T C in row chunks (partials in lrQ, free
  // here), its eigen-decomposition (rotation into lrP, free here), A_f = C W
  if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, mb, P, nb, w.pA, mb, sB,
                w.lrX, nb, sY, w.lrC, mb, sC, count)) != hipSuccess)
    return e;
  {
    (void)jtol;
    // partials: lrQ (nb^2 floats per slot) when it holds one chunk of p^2 doubles, else
    // the split-K buffer of tall blocks (free between the Gram and the coupling product)
    int64_t pstride = (int64_t)nb * nb / 2;   // doubles per slot
    double* part = reinterpret_cast<double*>(w.lrQ);
    if (pstride < 256) {
      if (!w.lrSplit || (int64_t)count * 256 > (int64_t)(kSplitFloats / 2))
        return hipErrorInvalidValue;   // the plan gives blocks this narrow a split buffer
      pstride = (int64_t)(kSplitFloats / 2) / count;
      part = reinterpret_cast<double*>(w.lrSplit);
    }
    int chunks = (mb + 511) / 512;
    if (chunks > pstride / 256) chunks = (int)(pstride / 256);
    const int rows = (mb + chunks - 1) / chunks;
    chunks = (mb + rows - 1) / rows;
    hipLaunchKernelGGL(k_lr_gram64<P>, dim3(chunks, count), dim3(256), 0, st, w.lrC, mb, rows,
                       part, pstride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_eig64<P>, dim3(count), dim3(256), 0, st, part, chunks, pstride,
                       w.lrX, w.lrV, w.lrSig, w.lrP, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_rot_c<P>, dim3((mb + 255) / 256, count), dim3(256), 0, st, w.lrC,
                       w.lrP, mb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // coupling: T = A_f^T B (p x nb)
  if (!tall_atb(w.lrC, sC, P, w.pA, sB, nb, mb, w.lrT, P, (int64_t)P * nb, count, w.lrSplit,
                kSplitFloats, st, &e)) {
    if ((e = gemm(h, rocblas_operation_transpose, rocblas_operation_none, P, nb, mb, w.lrC, mb,
                  sC, w.pA, mb, sB, w.lrT, P, (int64_t)P * nb, count)) != hipSuccess)
      return e;
  } else if (e != hipSuccess) {
    return e;
  }
  float* mask = w.lrSig + (size_t)w.slots * P;       // second third of the sigma buffer
  float* dmask = w.lrSig + 2 * (size_t)w.slots * P;  // last third
  hipLaunchKernelGGL(k_lr_coupling<P>, dim3(count), dim3(256), 0, st, w.lrT, w.lrSig, w.lrV, nb,
                     tau, kCouplingTol, w.lrScal, mask, dmask);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // stage -1: the trace bound on lambda_max(E^T E) needs no E^T E; the slots it leaves
  // undecided (listed at fall[3 slots ..], counted in counts[2]) get E^T E and its finer
  // bounds. The launches below cover every slot and return early past that count, so
  // the host does not wait for it.
  hipLaunchKernelGGL(k_lr_decide, dim3((count + 255) / 256), dim3(256), 0, st, count, w.slots,
                     w.lrScal, w.lrSig, dmask, tau, w.pflag, w.lrCount, w.lrFall, w.live_list,
                     w.stats, -1, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, st, w.lrCount + 1, w.lrCount + 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, w.lrCount + 1, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int* flist = w.lrFall + 3 * w.slots;
  const int* fcount = w.lrCount + 2;
  const int tiles = (int)((sG + 255) / 256 < 64 ? (sG + 255) / 256 : 64);
  {
    // E^T E and its power bound: W = G V_r, H = V_r^T W (into lrQ), Q = W - V H / 2
    // (into lrY), E^T E = G - Q V^T - V Q^T (into lrP, partials into lrQ)
    if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, nb, P, nb, w.lrG, nb, sG,
                  w.lrV, nb, sY, w.lrW, nb, sY, count)) != hipSuccess)
      return e;
    if ((e = gemm(h, rocblas_operation_transpose, rocblas_operation_none, P, P, nb, w.lrV, nb,
                  sY, w.lrW, nb, sY, w.lrQ, P, (int64_t)P * P, count)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_lr_q<P>, dim3(count), dim3(256), 0, st, w.lrW, w.lrV, w.lrQ, dmask,
                       w.lrY, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int gtiles = ((nb + 63) / 64) * ((nb + 63) / 64);
    hipLaunchKernelGGL(k_lr_ge<P>, dim3(gtiles, count), dim3(256), 0, st, w.lrG, w.lrY, w.lrV,
                       dmask, w.lrP, nb, w.lrQ, w.lrRow, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // stage 0: Frobenius and Collatz-Wielandt bounds of E^T E (partials were written to lrQ)
    hipLaunchKernelGGL(k_lr_ge_reduce, dim3((count + 255) / 256), dim3(256), 0, st, w.lrQ,
                       gtiles, count, w.lrScal, flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_rsum, dim3((nb + 255) / 256, count), dim3(256), 0, st, w.lrRow, nb,
                       flist, fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwy, dim3(gtiles, count), dim3(256), 0, st, w.lrP, w.lrRow, nb, flist,
                       fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_cwmax, dim3(count), dim3(256), 0, st, w.lrRow, nb, w.lrScal, flist,
                       fcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_decide, dim3((count + 255) / 256), dim3(256), 0, st, count, w.slots,
                       w.lrScal, w.lrSig, dmask, tau, w.pflag, w.lrCount, w.lrFall, w.live_list,
                       w.stats, 0, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(w.hostInts + 1, w.lrCount + 1, sizeof(int), hipMemcpyDeviceToHost,
                          st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const int und = w.hostInts[1];
  if (und > 0) {
    // stage 1: square of E^T E / tr(E^T E); stage 2: its fourth power (eighth in all),
    // on the undecided slots only, gathered to compact positions (lrQ, then lrP)
    const int* ulist = w.lrFall + 2 * w.slots;
    hipLaunchKernelGGL(k_lr_gather_scale, dim3(tiles, und), dim3(256), 0, st, w.lrP, w.lrQ, nb,
                       ulist, w.lrScal);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* a = w.lrQ;
    float* b = w.lrP;
    int power = 1;
    for (int stage = 1; stage <= 2; ++stage) {
      const int nsq = stage == 1 ? 1 : 2;
      for (int s2 = 0; s2 < nsq; ++s2) {
        if ((e = gemm(h, rocblas_operation_none, rocblas_operation_none, nb, nb, nb, a, nb, sG, a,
                      nb, sG, b, nb, sG, und)) != hipSuccess)
          return e;
        float* t = a;
        a = b;
        b = t;
        power *= 2;
      }
      const int ftiles = tiles;
      // partials go to lrY (free after stage 0); lrT keeps A_f^T B for the polar route
      hipLaunchKernelGGL(k_lr_frob_part, dim3(ftiles, und), dim3(256), 0, st, a, nb, w.lrY);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_lr_frob_reduce, dim3((und + 255) / 256), dim3(256), 0, st, w.lrY,
                         ftiles, und, ulist, w.lrScal, 3);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, w.lrCount + 1, 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_lr_decide, dim3((und + 255) / 256), dim3(256), 0, st, und,
                         w.slots, w.lrScal, w.lrSig, dmask, tau, w.pflag, w.lrCount, w.lrFall,
                         w.live_list, w.stats, stage, power);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (stage == 1) {
        if ((e = hipMemcpyAsync(w.hostInts + 1, w.lrCount + 1, sizeof(int),
                                hipMemcpyDeviceToHost, st)) != hipSuccess)
          return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (w.hostInts[1] == 0) break;
      }
    }
  }
  {
    const int tl = ((g.m + 31) / 32) * ((g.n + 31) / 32);
    hipLaunchKernelGGL(k_lr_rebuild<P>, dim3(tl, count), dim3(256), 0, st, Zout, Dout, g, sh,
                       w.live_list, w.pflag, w.lrC, w.lrV, w.lrSig, tau);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(w.hostInts + 1, w.lrCount, sizeof(int), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *fallback_host = w.hostInts[1];
  return hipSuccess;
}

}  // namespace msld
