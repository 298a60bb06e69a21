// Certified low-rank BlockSVT for blocks up to 64 x 128, fused into one kernel.
//
// The same certificate as the large-block path (lowrank.hip), but every step for one
// block runs inside one workgroup with the block and its Gram in LDS: no library
// calls and no round trips through HBM. For a live block B (logical mb x nb,
// mb >= nb, zero-padded to MB x NB):
//   G = B^T B; X0 = orth(G Omega); X <- orth(G (G X)) three times (seven products);
//   one-sided Jacobi on C = B X gives A_f = B V_r (columns a_l = sigma_l u_l);
//   coupling c_l = ||u_l^T B - sigma_l v_l^T||; deflation set L = live directions
//   (sigma > tau) plus near-live ones (tau/2 < sigma <= tau) with tiny coupling;
//   the remainder E_L = B (I - V_L V_L^T) is bounded through the remainder E after L and
//   the further well-converged directions K: lambda_max(E_L^T E_L) <= max(max_{l in K}
//   sigma_l^2, lambda_max(E^T E)) + (sum_{l in K} sigma_l^2 c_l^2)^(1/2), with
//   lambda_max(E^T E) <= min(||E^T E||_F, the Collatz-Wielandt bound of |E^T E| with its
//   row sums), then tr * ||(E^T E / tr)^k||_F^(1/k), k = 2, 8.
// Accepted blocks get Z = sum_{l in L, sigma_l > tau} (1 - tau / sigma_l) a_l v_l^T
// (the error is at most the tested coupling, by non-expansiveness of the prox of
// eq:svt); the others are listed for the LDS Jacobi tier, which runs right after.
#include "msld_internal.h"

namespace msld {

namespace {

constexpr float kSmallCertMargin = 2e-3f;    // relative margin on tau^2
constexpr float kSmallCouplingTol = 1e-5f;   // sum_L c_l^2 <= tol^2 ||B||_F^2

__device__ __forceinline__ float wsum(float v) { return wave_sum_dpp(v); }

template <int NT>
__device__ __forceinline__ float bsum(float v, float* red) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

template <int NT>
__device__ __forceinline__ float bmax(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s = fmaxf(s, red[w]);
  return s;
}

// C = A^T A for A with K rows and NB columns (column j at A + j * lda), C column-major
// with leading dimension ldc. Each of TG x TG threads owns a TI x TI tile of
// interleaved rows and columns (i = ti + TG a, j = tj + TG b).
template <int NB, int NT>
__device__ __forceinline__ void ata(const float* A, int lda, int K, float* C, int ldc) {
  constexpr int TG = NT == 256 ? 16 : 8;   // TG x TG threads, each a TI x TI tile
  constexpr int TI = NB / TG;
  const int ti = threadIdx.x % TG, tj = threadIdx.x / TG;
  float acc[TI][TI];
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TI; ++b) acc[a][b] = 0.f;
  for (int r = 0; r < K; ++r) {
    float x[TI], y[TI];
#pragma unroll
    for (int a = 0; a < TI; ++a) x[a] = A[(ti + TG * a) * lda + r];
#pragma unroll
    for (int b = 0; b < TI; ++b) y[b] = A[(tj + TG * b) * lda + r];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
      for (int b = 0; b < TI; ++b) acc[a][b] += x[a] * y[b];
  }
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TI; ++b) C[(tj + TG * b) * ldc + ti + TG * a] = acc[a][b];
}

// Y = M X for the symmetric NB x NB matrix M (ld ldm) and X (NB x P, ld NB).
template <int NB, int P, int NT>
__device__ __forceinline__ void sym_mul(const float* M, int ldm, const float* X, float* Y) {
  for (int o = threadIdx.x; o < NB * P; o += NT) {
    const int l = o / NB, i = o - l * NB;
    const float* mi = M + i * ldm;   // column i = row i (symmetric)
    const float* xl = X + l * NB;
    float s = 0.f;
#pragma unroll 8
    for (int k = 0; k < NB; ++k) s += mi[k] * xl[k];
    Y[o] = s;
  }
}

// Orthonormalise the P columns of X (NB x P, ld NB) in place by classical
// Gram-Schmidt with re-orthogonalisation (wave 0; rows lane + 64 r). A column that
// stays numerically dependent is set to zero.
template <int NB, int P>
__device__ __forceinline__ void orth_w0(float* X) {
  constexpr int R = (NB + 63) / 64;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    float v[P][R];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = lane + 64 * r;
        v[j][r] = row < NB ? X[j * NB + row] : 0.f;
      }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      float n0 = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) n0 += v[j][r] * v[j][r];
      n0 = wsum(n0);
      float nprev = n0;
      bool dependent = j > 0;
      if (j > 0) {
        for (int pass = 0; pass < 4; ++pass) {
          float c[P];
#pragma unroll
          for (int i = 0; i < P; ++i) {
            c[i] = 0.f;
            if (i < j) {
              float sdot = 0.f;
#pragma unroll
              for (int r = 0; r < R; ++r) sdot += v[i][r] * v[j][r];
              c[i] = wsum(sdot);
            }
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            float t = v[j][r];
#pragma unroll
            for (int i = 0; i < P; ++i)
              if (i < j) t -= c[i] * v[i][r];
            v[j][r] = t;
          }
          float nn = 0.f;
#pragma unroll
          for (int r = 0; r < R; ++r) nn += v[j][r] * v[j][r];
          nn = wsum(nn);
          const bool done = nn >= 0.25f * nprev;
          nprev = nn;
          if (done) {
            dependent = false;
            break;
          }
        }
      }
      const float nrm = sqrtf(nprev);
      const bool keep = !dependent && nrm > 1e-30f && nprev > 1e-12f * n0;
      const float inv = keep ? 1.f / nrm : 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) v[j][r] *= inv;
    }
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = lane + 64 * r;
        if (row < NB) X[j * NB + row] = v[j][r];
      }
  }
  __syncthreads();
}

// Frobenius norm squared of the NB x NB matrix M (ld ldm).
template <int NB, int NT>
__device__ __forceinline__ float frob2(const float* M, int ldm, float* red) {
  float s = 0.f;
  for (int o = threadIdx.x; o < NB * NB; o += NT) {
    const int j = o / NB, i = o - j * NB;
    const float v = M[j * ldm + i];
    s += v * v;
  }
  return bsum<NT>(s, red);
}

}  // namespace

template <int NB, int MB, int P, int NT>
__global__ void __launch_bounds__(NT) k_lr_small(float* __restrict__ Zout,
                                                  float* __restrict__ Dout, ScaleGeom g,
                                                  ShiftSpec sh, float tau,
                                                  const int* __restrict__ live_count,
                                                  const int* __restrict__ live_list,
                                                  int* __restrict__ fall_count,
                                                  int* __restrict__ fall_list,
                                                  unsigned long long* __restrict__ stats) {
  constexpr int LDB = MB + 1;   // B column stride; squarings reuse it with ld NB + 1
  constexpr int LDG = NB + 1;
  constexpr int LDC = MB + 1;
  constexpr int LDW = P + 1;
  extern __shared__ float sm[];
  float* Bs = sm;                   // NB x LDB
  float* Gs = Bs + NB * LDB;        // NB x LDG
  float* Xs = Gs + NB * LDG;        // NB x P: X, then T = A_f^T B, then Q
  float* Ws = Xs + NB * P;          // NB x P: G X, then V_r
  float* Cs = Ws + NB * P;          // P x LDC: B X, then A_f
  float* Rj = Cs + P * LDC;         // P x LDW Jacobi rotations
  __shared__ float red[NT / 64];
  __shared__ float sig[P], mask[P], dmask[P], cl[P], H[P * P];
  __shared__ float s_trG, s_omax, s_cross;
  __shared__ int s_state;
  const int N = g.N, m = g.m, n = g.n, Q = g.Q, mb = g.mb, nb = g.nb;
  const int tid = threadIdx.x;
  const int count = *live_count;
  const float lim = tau * tau * (1.f - kSmallCertMargin);
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const int blk = live_list[it];
    const int p = blk / Q, q = blk - p * Q;
    int sr, sc;
    block_shift(sh, p / g.PI, m, n, &sr, &sc);
    // B = V = -D' (written by the stream pass), logical column-major, zero-padded
    for (int e = tid; e < NB * LDB; e += NT) Bs[e] = 0.f;
    __syncthreads();
    for (int e = tid; e < m * n; e += NT) {
      const int i = e / n, j = e - i * n;
      const float v = -Dout[(int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc)];
      if (!g.trans) Bs[j * LDB + i] = v;
      else Bs[i * LDB + j] = v;
    }
    __syncthreads();
    ata<NB, NT>(Bs, LDB, MB, Gs, LDG);
    __syncthreads();
    {
      float t = 0.f;
      for (int i = tid; i < NB; i += NT) t += Gs[i * LDG + i];
      t = bsum<NT>(t, red);
      if (tid == 0) s_trG = t;
    }
    {
      // zero-output certificate from the Gram matrix alone: sigma_max(B)^2 is at most the
      // Collatz-Wielandt bound of |G| (r = |G| 1, max_i (|G| r)_i / r_i); below tau^2
      // (with the margin) the SVT is zero, which the stream pass already wrote. r goes
      // to Xs, free until the probe is drawn.
      for (int i = tid; i < NB; i += NT) {
        float r = 0.f;
        for (int j = 0; j < NB; ++j) r += fabsf(Gs[j * LDG + i]);
        Xs[i] = r;
      }
      __syncthreads();
      float best = 0.f;
      for (int i = tid; i < NB; i += NT) {
        float y = 0.f;
        for (int j = 0; j < NB; ++j) y += fabsf(Gs[j * LDG + i]) * Xs[j];
        const float ri = Xs[i];
        if (ri > 0.f) best = fmaxf(best, y / ri);
        else if (y > 0.f) best = __int_as_float(0x7f800000);
      }
      best = bmax<NT>(best, red);   // the same value in every thread
      if (best <= lim && isfinite(best)) {
        if (tid == 0) {
          atomicAdd(&stats[0], 1ull);
          atomicAdd(&stats[3], 1ull);
          atomicAdd(&stats[8], 1ull);
        }
        continue;
      }
    }
    // X0 = orth(G Omega), Omega = fixed +-1 probe
    for (int o = tid; o < NB * P; o += NT) {
      const uint64_t z = mix64(0x243F6A8885A308D3ull + (uint64_t)o);
      Xs[o] = (z >> 63) ? 1.f : -1.f;
    }
    __syncthreads();
    sym_mul<NB, P, NT>(Gs, LDG, Xs, Ws);
    __syncthreads();
    orth_w0<NB, P>(Ws);
    for (int o = tid; o < NB * P; o += NT) Xs[o] = Ws[o];
    __syncthreads();
    for (int rep = 0; rep < 3; ++rep) {
      sym_mul<NB, P, NT>(Gs, LDG, Xs, Ws);
      __syncthreads();
      sym_mul<NB, P, NT>(Gs, LDG, Ws, Xs);
      __syncthreads();
      orth_w0<NB, P>(Xs);
    }
    // C = B X
    for (int o = tid; o < MB * P; o += NT) {
      const int l = o / MB, r = o - l * MB;
      float s = 0.f;
#pragma unroll 8
      for (int k = 0; k < NB; ++k) s += Bs[k * LDB + r] * Xs[l * NB + k];
      Cs[l * LDC + r] = s;
    }
    for (int o = tid; o < P * LDW; o += NT) {
      const int j = o / LDW, r = o - j * LDW;
      Rj[o] = (j == r) ? 1.f : 0.f;
    }
    __syncthreads();
    // one-sided Jacobi on the P columns of C (one wave per column pair)
    {
      const float rr_tol = 5.9604645e-8f * sqrtf((float)mb);
      const int t = tid & 63;
      for (int sw = 0; sw < 40; ++sw) {
        int rotated = 0;
        for (int rd = 0; rd < P - 1; ++rd) {
          // pair group grp on wave grp mod (NT / 64)
          for (int grp = tid >> 6; grp < P / 2; grp += NT / 64) {
            const int n1 = P - 1;
            const int pa = (grp == 0) ? 0 : 1 + (grp - 1 + rd) % n1;
            const int pb = 1 + (P - 2 - grp + rd) % n1;
            float* ap = Cs + pa * LDC;
            float* aq = Cs + pb * LDC;
            float al = 0.f, be = 0.f, ga = 0.f;
            for (int r = t; r < MB; r += 64) {
              const float u = ap[r], v = aq[r];
              al += u * u;
              be += v * v;
              ga += u * v;
            }
            al = wsum(al);
            be = wsum(be);
            ga = wsum(ga);
            if (jacobi_rotates(ga, al, be, rr_tol)) {
              rotated = 1;
              float cs, sn;
              jacobi_cs(ga, al, be, &cs, &sn);
              for (int r = t; r < MB; r += 64) {
                const float u = ap[r], v = aq[r];
                ap[r] = cs * u - sn * v;
                aq[r] = sn * u + cs * v;
              }
              if (t < P) {
                float* wp = Rj + pa * LDW;
                float* wq = Rj + pb * LDW;
                const float u = wp[t], v = wq[t];
                wp[t] = cs * u - sn * v;
                wq[t] = sn * u + cs * v;
              }
            }
          }
          __syncthreads();
        }
        if (!__syncthreads_or(rotated)) break;
      }
    }
    // sigma_l = ||a_l||, V_r = X R (into Ws)
    for (int l = tid >> 6; l < P; l += NT / 64) {
      float s2 = 0.f;
      for (int r = tid & 63; r < MB; r += 64) s2 += Cs[l * LDC + r] * Cs[l * LDC + r];
      s2 = wsum(s2);
      if ((tid & 63) == 0) sig[l] = sqrtf(s2);
    }
    for (int o = tid; o < NB * P; o += NT) {
      const int l = o / NB, row = o - l * NB;
      float v = 0.f;
#pragma unroll
      for (int j = 0; j < P; ++j) v += Xs[j * NB + row] * Rj[l * LDW + j];
      Ws[o] = v;
    }
    __syncthreads();
    // T = A_f^T B (P x NB, T[c P + l]) into Xs
    for (int o = tid; o < NB * P; o += NT) {
      const int c = o / P, l = o - c * P;
      float s = 0.f;
#pragma unroll 8
      for (int r = 0; r < MB; ++r) s += Cs[l * LDC + r] * Bs[c * LDB + r];
      Xs[o] = s;
    }
    __syncthreads();
    // coupling per direction, deflation mask
    for (int l = tid >> 6; l < P; l += NT / 64) {
      const float s = sig[l];
      float acc = 0.f;
      if (s > 0.f) {
        const float inv = 1.f / s;
        for (int c = tid & 63; c < NB; c += 64) {
          const float d = Xs[c * P + l] * inv - s * Ws[l * NB + c];
          acc += d * d;
        }
        acc = wsum(acc);
      }
      if ((tid & 63) == 0) cl[l] = acc;
    }
    __syncthreads();
    if (tid == 0) {
      const float trG = s_trG;
      const float near_lim = 0.09f * kSmallCouplingTol * kSmallCouplingTol * trG;
      float c2 = 0.f, omax = 0.f, cross = 0.f;
      for (int l = 0; l < P; ++l) {
        const float s = sig[l];
        const bool live = s > tau;
        const bool near = !live && s > 0.5f * tau && cl[l] <= near_lim;
        const bool in = live || near;
        const float x = s * s * cl[l];
        const bool split = !in && s > 0.f && s * sqrtf(cl[l]) <= 1e-3f * tau * tau;
        mask[l] = in ? 1.f : 0.f;
        dmask[l] = (in || split) ? 1.f : 0.f;
        if (in) c2 += cl[l];
        if (split) {
          omax = fmaxf(omax, s * s);
          cross += x;
        }
      }
      s_omax = omax * (1.f + 1e-4f);
      s_cross = sqrtf(cross);
      const bool c_ok = c2 <= kSmallCouplingTol * kSmallCouplingTol * trG && isfinite(c2);
      s_state = c_ok ? 0 : -1;
    }
    __syncthreads();
    int state = s_state;   // 0 undecided, 1 certified, -1 coupling failure, -2 bound failure
    if (state == 0) {
      // Wg = G V_r into Xs; H = V_L^T Wg; Q = Wg - V_L H / 2 (in place, row by row)
      sym_mul<NB, P, NT>(Gs, LDG, Ws, Xs);
      __syncthreads();
      for (int o = tid; o < P * P; o += NT) {
        const int l = o / P, k = o - l * P;
        float s = 0.f;
        if (dmask[l] > 0.f && dmask[k] > 0.f)
          for (int i = 0; i < NB; ++i) s += Ws[l * NB + i] * Xs[k * NB + i];
        H[o] = s;
      }
      __syncthreads();
      for (int i = tid; i < NB; i += NT) {
        float q[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          float s = 0.f;
#pragma unroll
          for (int l = 0; l < P; ++l) s += Ws[l * NB + i] * H[l * P + k];
          q[k] = Xs[k * NB + i] - 0.5f * s;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) Xs[k * NB + i] = q[k];
      }
      __syncthreads();
      // E^T E = G - Q V_L^T - V_L Q^T in place, with its trace and Frobenius norm
      float tr = 0.f, f2 = 0.f;
      for (int o = tid; o < NB * NB; o += NT) {
        const int j = o / NB, i = o - j * NB;
        float s = Gs[j * LDG + i];
#pragma unroll
        for (int l = 0; l < P; ++l)
          if (dmask[l] > 0.f)
            s -= Xs[l * NB + i] * Ws[l * NB + j] + Ws[l * NB + i] * Xs[l * NB + j];
        Gs[j * LDG + i] = s;
        if (i == j) tr += s;
        f2 += s * s;
      }
      tr = bsum<NT>(tr, red);
      f2 = bsum<NT>(f2, red);
      // Collatz-Wielandt bound of |E^T E| with its row sums r: lambda_max <= max_i
      // (|E^T E| r)_i / r_i (r kept in Bs, free from here on)
      __syncthreads();
      for (int i = tid; i < NB; i += NT) {
        float v = 0.f;
        for (int j = 0; j < NB; ++j) v += fabsf(Gs[j * LDG + i]);
        Bs[i] = v;
      }
      __syncthreads();
      float cw = 0.f;
      for (int i = tid; i < NB; i += NT) {
        float y = 0.f;
        for (int j = 0; j < NB; ++j) y += fabsf(Gs[i * LDG + j]) * Bs[j];
        const float ri = Bs[i];
        if (ri > 0.f) cw = fmaxf(cw, y / ri);
        else if (y > 0.f) cw = __int_as_float(0x7f800000);
      }
      cw = bmax<NT>(cw, red);
      // lambda_max(E_L^T E_L) <= max(max_l' sigma_l'^2, lambda_max(E^T E)) + cross term,
      // l' the well-converged directions split off besides L, E the remainder after both
      const float omax = s_omax, cross = s_cross;
      const float b0 = fmaxf(omax, tr > 0.f ? fminf(sqrtf(f2), cw) : 0.f) + cross;
      if (b0 <= lim && isfinite(b0)) {
        state = 1;
      } else if (!(tr > 0.f) || !isfinite(tr)) {
        state = -2;
      } else {
        // stage 1: (E^T E / tr)^2; stage 2: its fourth power (eighth in all)
        const float inv = 1.f / tr;
        for (int o = tid; o < NB * NB; o += NT) {
          const int j = o / NB, i = o - j * NB;
          Gs[j * LDG + i] *= inv;
        }
        __syncthreads();
        ata<NB, NT>(Gs, LDG, NB, Bs, LDG);
        __syncthreads();
        const float s1 = sqrtf(sqrtf(frob2<NB, NT>(Bs, LDG, red)));
        const float b1 = fmaxf(omax, tr * s1) + cross;
        if (b1 <= lim && isfinite(b1)) {
          state = 1;
        } else {
          ata<NB, NT>(Bs, LDG, NB, Gs, LDG);
          __syncthreads();
          ata<NB, NT>(Gs, LDG, NB, Bs, LDG);
          __syncthreads();
          const float f8 = frob2<NB, NT>(Bs, LDG, red);
          const float b2 = fmaxf(omax, tr * powf(f8, 1.f / 16.f)) + cross;
          state = (b2 <= lim && isfinite(b2)) ? 1 : -2;
        }
      }
    }
    int nlive = 0;
#pragma unroll
    for (int l = 0; l < P; ++l) nlive += (mask[l] > 0.f && sig[l] > tau) ? 1 : 0;
    if (state == 1 && nlive > 0) {
      // Z = sum_L (1 - tau / sigma_l)_+ a_l v_l^T, scattered with D' = 2 Z' - V (with no
      // live direction the stream pass already wrote Z' = 0, D' = -V)
      for (int e = tid; e < m * n; e += NT) {
        const int i = e / n, j = e - i * n;
        const int r = g.trans ? j : i;
        const int c = g.trans ? i : j;
        float z = 0.f;
#pragma unroll
        for (int l = 0; l < P; ++l) {
          const float s = sig[l];
          if (mask[l] > 0.f && s > tau)
            z += (1.f - tau / s) * Cs[l * LDC + r] * Ws[l * NB + c];
        }
        const int64_t o = (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc);
        const float v = -Dout[o];
        Zout[o] = z;
        Dout[o] = 2.f * z - v;
      }
    }
    if (tid == 0) {
      if (state == 1) {
        atomicAdd(&stats[0], 1ull);
        atomicAdd(&stats[2], (unsigned long long)nlive);
        atomicAdd(&stats[3], 1ull);
      } else {
        atomicAdd(&stats[state == -1 ? 4 : 5], 1ull);
        const int f = atomicAdd(fall_count, 1);
        fall_list[f] = blk;
      }
    }
    __syncthreads();
  }
}

size_t lr_small_lds_bytes(int NB, int MB, int P) {
  return 4 * ((size_t)NB * (MB + 1) + (size_t)NB * (NB + 1) + 2 * (size_t)NB * P +
              (size_t)P * (MB + 1) + (size_t)P * (P + 1));
}

// (NB, MB) padded sizes the fused kernel is instantiated for, and the subspace width of
// its first pass (the retry pass on failures uses twice that); 0 when none fits.
int lr_small_shape(int mb, int nb, int* NB, int* MB, int* P) {
  // beyond 64 columns the batched-GEMM path is faster (its products keep the whole
  // chip busy, while this kernel holds one block per workgroup)
  auto up = [](int v) { return v <= 32 ? 32 : v <= 64 ? 64 : v <= 128 ? 128 : 0; };
  const int nbp = up(nb), mbp = up(mb);
  if (!nbp || !mbp || mbp < nbp || nbp > 64) return 0;
  *NB = nbp;
  *MB = mbp;
  *P = nbp == 32 ? 4 : 8;
  return 1;
}

// One pass of the fused kernel over (count, list); failures are appended to
// (fcount, flist). pass 0 uses the first subspace width, pass 1 (a retry on few blocks)
// and pass 2 (a first pass over all live blocks) twice that.
hipError_t launch_lr_small(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout,
                           float tau, const ShiftSpec& sh, int num_cus, int pass,
                           const int* count, const int* list, int* fcount, int* flist,
                           hipStream_t st) {
  int NB = 0, MB = 0, P = 0;
  if (!lr_small_shape(g.mb, g.nb, &NB, &MB, &P)) return hipErrorInvalidValue;
  if (pass) P *= 2;   // pass 1: retry of the failures, pass 2: wide first pass
  const size_t lds = lr_small_lds_bytes(NB, MB, P);
  // first passes over 32-wide blocks: one wave per workgroup (no barrier waits across
  // waves, more blocks in flight per CU); 64-wide blocks and the retry pass (twice the
  // column pairs): four waves
  const int NT = (NB == 32 && pass != 1) ? 64 : 256;
  int per_cu = (int)(160 * 1024 / (lds + 2048));
  const int cap = NT == 64 ? 16 : 8;
  if (per_cu > cap) per_cu = cap;
  if (pass == 1 && per_cu > 1) per_cu = 1;   // the retry list is short
  if (per_cu < 1) per_cu = 1;
  int grid = num_cus * per_cu;
  const int nblk = g.P * g.Q;
  if (grid > nblk) grid = nblk;
#define MSLD_LRS(nb_, mb_, p_, nt_)                                                             \
  if (NB == nb_ && MB == mb_ && P == p_ && NT == nt_)                                           \
    hipLaunchKernelGGL((k_lr_small<nb_, mb_, p_, nt_>), dim3(grid), dim3(nt_), lds, st, Zout,  \
                       Dout, g, sh, tau, count, list, fcount, flist, w.stats)
  MSLD_LRS(32, 32, 4, 64);
  else MSLD_LRS(32, 64, 4, 64);
  else MSLD_LRS(32, 128, 4, 64);
  else MSLD_LRS(32, 32, 8, 64);
  else MSLD_LRS(32, 64, 8, 64);
  else MSLD_LRS(32, 128, 8, 64);
  else MSLD_LRS(32, 32, 4, 256);
  else MSLD_LRS(32, 64, 4, 256);
  else MSLD_LRS(32, 128, 4, 256);
  else MSLD_LRS(32, 32, 8, 256);
  else MSLD_LRS(32, 64, 8, 256);
  else MSLD_LRS(32, 128, 8, 256);
  else MSLD_LRS(64, 64, 8, 256);
  else MSLD_LRS(64, 128, 8, 256);
  else MSLD_LRS(64, 64, 16, 256);
  else MSLD_LRS(64, 128, 16, 256);
  else return hipErrorInvalidValue;
#undef MSLD_LRS
  return hipGetLastError();
}

}  // namespace msld
