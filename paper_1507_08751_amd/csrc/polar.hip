// Exact BlockSVT for large blocks whose low-rank certificate failed.
//
// The soft-threshold of eq:svt through the polar decomposition: for a block E
// (logical mb x nb, mb >= nb) with E = Q H, Q with orthonormal columns on the range
// of E and H = (E^T E)^(1/2), SVT_tau(E) = Q (H - tau I)_+, and for the symmetric
// S = H - tau I, (S)_+ = S (I + sign S) / 2. Both the polar factor and the matrix
// sign come from the cubic Newton-Schulz map f(x) = x (3 - x^2) / 2 applied to the
// singular values (X <- X (3I - X^T X) / 2) or eigenvalues (Y <- Y (3I - Y^2) / 2),
// so the whole fallback is batched matrix products plus small elementwise kernels.
//
// Accuracy, per singular value sigma of E, with X0 = E / alpha (alpha >= sigma_max):
//  * singular values below tau land on negative eigenvalues of S whatever the polar
//    accuracy, so the K polar steps only need f_K(tau / alpha) >= 1 - 5e-8;
//  * an eigenvalue s of S with |s| <= alpha_S is mapped to s (1 + f_J(s / alpha_S)) / 2
//    instead of (s)_+, an error of at most alpha_S max_x x (1 - f_J(x)) / 2; only
//    singular values close to tau are affected, each by a fraction of its distance.
// K and J are chosen on the host from these scalar recursions, per failed block.
//
// Deflation: when the coupling test of the low-rank path passed, its live directions
// U_L (with singular values S_L, right vectors V_L) are split off first. With
// E' = (I - U_L U_L^T) B, the matrix B0 = U_L S_L V_L^T + E' is within ||U_L^T E||_F
// of B (the tested coupling), the two terms are orthogonal on both sides, so
// SVT(B0) = Z_L + SVT(E') and ||SVT(B) - SVT(B0)||_F <= ||U_L^T E||_F by
// non-expansiveness. The remainder bound of the failed certificate bounds sigma_max(E'),
// so alpha is within a small factor of tau and K is a handful of steps. Without a
// passed coupling test the whole block goes through the polar route (L empty), with
// alpha the smaller of ||B||_F and the square root of the Collatz-Wielandt bound of
// |B^T B| that the zero-output certificate computed (both bound sigma_max(B)).
#include <algorithm>
#include <cmath>

#include "msld_internal.h"

namespace msld {

// E' / alpha for each failed slot of the chunk, plus per-slot scalars
// (alpha, alpha_S, deflated flag, ||B||_F).
template <int P>
__global__ void __launch_bounds__(256) k_pl_prepare(const float* __restrict__ Dout, ScaleGeom g,
                                                    ShiftSpec sh,
                                                    const int* __restrict__ live_list,
                                                    const float* __restrict__ Af,
                                                    const float* __restrict__ T,
                                                    const float* __restrict__ sig,
                                                    const float* __restrict__ mask,
                                                    const float* __restrict__ scal,
                                                    const int* __restrict__ fslot, int c0, int mb,
                                                    int nb, float tau, float* __restrict__ X0,
                                                    float* __restrict__ plscal) {
  __shared__ float coef[P];
  __shared__ float inv_alpha;
  const int c = blockIdx.y;
  const int slot = fslot[c0 + c];
  const float* sc = scal + slot * 8;
  const float bound = sc[5];
  const bool defl = bound >= 0.f && isfinite(bound);
  if (threadIdx.x < P) {
    const float s = sig[slot * P + threadIdx.x];
    coef[threadIdx.x] =
        (defl && mask[slot * P + threadIdx.x] > 0.f && s > 0.f) ? 1.f / (s * s) : 0.f;
  }
  if (threadIdx.x == 0) {
    const float fro = sqrtf(fmaxf(sc[0], 0.f));
    // without deflation alpha bounds sigma_max(B): the smaller of ||B||_F and the
    // Collatz-Wielandt bound of the Gram matrix (stored negated), with a margin
    float alpha = defl ? 1.02f * sqrtf(bound) : 1.001f * fro;
    if (!defl && bound < 0.f && isfinite(bound)) alpha = fminf(alpha, 1.02f * sqrtf(-bound));
    if (!(alpha > 1e-30f)) alpha = 1e-30f;
    inv_alpha = 1.f / alpha;
    if (blockIdx.x == 0) {
      plscal[4 * c + 0] = alpha;
      plscal[4 * c + 1] = 1.02f * fmaxf(tau, alpha - tau);
      plscal[4 * c + 2] = defl ? 1.f : 0.f;
      plscal[4 * c + 3] = fro;
    }
  }
  __syncthreads();
  const int64_t elems = (int64_t)mb * nb;
  // the block is read from V = -D' at its shifted coordinates (logical B(r, col))
  const int blk = live_list[slot];
  const int p = blk / g.Q, q = blk - p * g.Q;
  int sr, scol;
  block_shift(sh, p / g.PI, g.m, g.n, &sr, &scol);
  const float* af = Af + (int64_t)slot * mb * P;
  const float* t = T + (int64_t)slot * P * nb;
  float* x = X0 + (int64_t)c * elems;
  const float ia = inv_alpha;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e / mb);
    const int r = (int)(e - (int64_t)col * mb);
    const int i = g.trans ? col : r, j = g.trans ? r : col;
    float v = -Dout[(int64_t)grow(g, p, i, sr) * g.N + gcol(g, q, j, scol)];
    if (defl) {
#pragma unroll
      for (int l = 0; l < P; ++l)
        if (coef[l] != 0.f) v -= af[l * mb + r] * (t[col * P + l] * coef[l]);
    }
    x[e] = v * ia;
  }
}

// M <- a I + b M for each nb x nb matrix of the chunk; with steps, a block whose own step
// count steps[2 c] is reached (k >= steps[2 c]) gets M = I instead, so the product that
// follows carries its iterate over unchanged (x 1 plus exact zeros).
__global__ void __launch_bounds__(256) k_pl_affine(float* M, int nb, float a, float b,
                                                   const int* __restrict__ steps, int k) {
  const int c = blockIdx.y;
  const bool frozen = steps != nullptr && k >= steps[2 * c];
  const int64_t elems = (int64_t)nb * nb;
  float* m = M + (int64_t)c * elems;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / nb);
    const int i = (int)(e - (int64_t)j * nb);
    m[e] = frozen ? (i == j ? 1.f : 0.f) : b * m[e] + (i == j ? a : 0.f);
  }
}

// The same, with M the in-order sum of the chunks partials left by a split product
// (chunk z of matrix c at part + (c chunks + z) nb^2), written to M.
__global__ void __launch_bounds__(256) k_pl_affine_part(const float* __restrict__ part,
                                                        int chunks, float* M, int nb, float a,
                                                        float b, const int* __restrict__ steps,
                                                        int k) {
  const int c = blockIdx.y;
  const bool frozen = steps != nullptr && k >= steps[2 * c];
  const int64_t elems = (int64_t)nb * nb;
  const float* p = part + (int64_t)c * chunks * elems;
  float* m = M + (int64_t)c * elems;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / nb);
    const int i = (int)(e - (int64_t)j * nb);
    float v = 0.f;
    if (!frozen)
      for (int z = 0; z < chunks; ++z) v += p[(int64_t)z * elems + e];
    m[e] = frozen ? (i == j ? 1.f : 0.f) : b * v + (i == j ? a : 0.f);
  }
}

// S = alpha (H + H^T) / 2 - tau I and Y0 = S / alpha_S, with H = Q^T X0.
__global__ void __launch_bounds__(256) k_pl_shift(const float* __restrict__ H,
                                                  float* __restrict__ S, float* __restrict__ Y,
                                                  int nb, float tau,
                                                  const float* __restrict__ plscal) {
  const int c = blockIdx.y;
  const float alpha = plscal[4 * c + 0];
  const float ias = 1.f / plscal[4 * c + 1];
  const int64_t elems = (int64_t)nb * nb;
  const float* h = H + (int64_t)c * elems;
  float* s = S + (int64_t)c * elems;
  float* y = Y + (int64_t)c * elems;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / nb);
    const int i = (int)(e - (int64_t)j * nb);
    float v = 0.5f * alpha * (h[e] + h[(int64_t)i * nb + j]);
    if (i == j) v -= tau;
    s[e] = v;
    y[e] = v * ias;
  }
}

// Z = Z_L + Ze scattered to the shifted block coordinates, with D' = 2 Z' - V
// (the stream pass left D' = -V for every live block).
template <int P>
__global__ void __launch_bounds__(256) k_pl_rebuild(float* __restrict__ Zout,
                                                    float* __restrict__ Dout, ScaleGeom g,
                                                    ShiftSpec sh, const int* __restrict__ live_list,
                                                    const int* __restrict__ fslot, int c0,
                                                    const float* __restrict__ Af,
                                                    const float* __restrict__ Vr,
                                                    const float* __restrict__ sig,
                                                    const float* __restrict__ mask, float tau,
                                                    const float* __restrict__ Ze,
                                                    const float* __restrict__ plscal) {
  __shared__ float gl[P];
  const int N = g.N, m = g.m, n = g.n, Q = g.Q, mb = g.mb, nb = g.nb;
  const int c = blockIdx.y;
  const int slot = fslot[c0 + c];
  const bool defl = plscal[4 * c + 2] > 0.f;
  if (threadIdx.x < P) {
    const float s = sig[slot * P + threadIdx.x];
    gl[threadIdx.x] =
        (defl && mask[slot * P + threadIdx.x] > 0.f && s > tau) ? 1.f - tau / s : 0.f;
  }
  __syncthreads();
  const int blk = live_list[slot];
  const int p = blk / Q, q = blk - p * Q;
  int sr, sc;
  block_shift(sh, p / g.PI, m, n, &sr, &sc);
  const float* af = Af + (int64_t)slot * mb * P;
  const float* vr = Vr + (int64_t)slot * nb * P;
  const float* ze = Ze + (int64_t)c * mb * nb;
  const int tilesj = (n + 31) / 32;
  const int ti = blockIdx.x / tilesj, tj = blockIdx.x - (blockIdx.x / tilesj) * tilesj;
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int i = ti * 32 + (e >> 5), j = tj * 32 + (e & 31);
    if (i >= m || j >= n) continue;
    const int r = g.trans ? j : i;
    const int col = g.trans ? i : j;
    float z = ze[(int64_t)col * mb + r];
#pragma unroll
    for (int l = 0; l < P; ++l)
      if (gl[l] > 0.f) z += gl[l] * af[l * mb + r] * vr[l * nb + col];
    const int64_t o = (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc);
    const float v = -Dout[o];
    Zout[o] = z;
    Dout[o] = 2.f * z - v;
  }
}

// ------------------------------------------------------------------ host side
namespace {

inline double ns_map(double x) { return 0.5 * x * (3.0 - x * x); }

// Polar steps that raise l to within 5e-8 of 1.
int polar_steps(double l) {
  if (!(l > 0.0)) return -1;
  if (l >= 1.0) l = 1.0;
  int k = 0;
  double x = l;
  while (1.0 - x > 5e-8 && k < 200) {
    x = ns_map(x);
    ++k;
  }
  return k;
}

// err[J] >= max over x in (0, 1] of x (1 - f_J(x)); a log grid of the scalar map with
// a 10 % allowance for the grid spacing (the maximiser moves by a factor 2/3 per step,
// far coarser than the grid).
struct SignTable {
  double err[96];
  SignTable() {
    constexpr int kPts = 4000;
    static double xs[kPts], fs[kPts];
    for (int i = 0; i < kPts; ++i) {
      xs[i] = std::pow(10.0, -14.0 + 14.0 * i / (kPts - 1));
      fs[i] = xs[i];
    }
    for (int j = 0; j < 96; ++j) {
      double mx = 0.0;
      for (int i = 0; i < kPts; ++i) {
        const double v = xs[i] * (1.0 - fs[i]);
        if (v > mx) mx = v;
      }
      err[j] = 1.1 * mx;
      for (int i = 0; i < kPts; ++i) fs[i] = ns_map(fs[i]);
    }
  }
};

const SignTable& sign_table() {
  static const SignTable t;
  return t;
}

// Sign steps so that the per-eigenvalue error alpha_S err[J] / 2 stays below
// 2e-7 ||B||_F.
int sign_steps(double alpha_s, double fro) {
  const SignTable& t = sign_table();
  const double target = 2e-7 * (fro > 0.0 ? fro : alpha_s);
  for (int j = 0; j < 96; ++j)
    if (0.5 * alpha_s * t.err[j] <= target) return j;
  return 95;
}

hipError_t last() { return hipGetLastError(); }

}  // namespace

int64_t polar_part_floats(int mb, int nb) {
  // the route's products: X^T X and Q^T X0 (nb x nb, contraction mb), X T and Q W
  // (mb x nb, contraction nb), Y Y, Y W and S Y (nb x nb, contraction nb)
  auto need = [](int M, int N, int K) -> int64_t {
    const int c = gemm_split(M, N, K, nullptr);
    return c > 1 ? (int64_t)c * M * N : 0;
  };
  return std::max(need(nb, nb, mb), std::max(need(mb, nb, nb), need(nb, nb, nb)));
}

hipError_t run_polar(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                     const ShiftSpec& sh, int nfall, hipStream_t st) {
  constexpr int P = 16;
  hipError_t e;
  const int mb = g.mb, nb = g.nb;
  const int64_t sX = (int64_t)mb * nb;
  const int64_t sN = (int64_t)nb * nb;
  const int* fslot = w.lrFall + w.slots;
  const float* mask = w.lrSig + (size_t)w.slots * P;
  const int tilesX = (int)std::min<int64_t>((sX + 1023) / 1024, 256);
  const int tilesN = (int)std::min<int64_t>((sN + 1023) / 1024, 256);
  const int tilesP = (int)std::min<int64_t>((sN + 255) / 256, 4096);
  const int tilesZ = ((g.m + 31) / 32) * ((g.n + 31) / 32);
  // split partial products of the GEMMs: room for every block of a chunk at the split
  // gemm_split gives each shape, so the split depends on the shapes alone
  float* part = w.plPart;
  const int64_t pfl = (int64_t)w.plCap * polar_part_floats(mb, nb);
  // Failed blocks in chunks of plCap. The step counts K and J are each block's own: the
  // chunk runs the largest, and a block past its own count multiplies by an exact
  // identity (k_pl_affine with steps), so its result is the one it gets alone, whatever
  // other blocks fail beside it (alone or in a batch).
  for (int c0 = 0; c0 < nfall; c0 += w.plCap) {
    const int cnt = std::min(w.plCap, nfall - c0);
    hipLaunchKernelGGL(k_pl_prepare<P>, dim3(tilesX, cnt), dim3(256), 0, st, Dout, g, sh,
                       w.live_list, w.lrC, w.lrT, w.lrSig, mask, w.lrScal, fslot, c0, mb, nb, tau, w.plX0,
                       w.plScal);
    if ((e = last()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(w.hostPl, w.plScal, sizeof(float) * 4 * cnt, hipMemcpyDeviceToHost,
                            st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    int K = 0, J = 0;
    for (int c = 0; c < cnt; ++c) {
      const double alpha = w.hostPl[4 * c + 0], alpha_s = w.hostPl[4 * c + 1];
      const int k = polar_steps((double)tau / alpha);
      const int j = sign_steps(alpha_s, w.hostPl[4 * c + 3]);
      if (k < 0 || !std::isfinite(alpha_s)) return hipErrorInvalidValue;
      w.hostSteps[2 * c + 0] = k;
      w.hostSteps[2 * c + 1] = j;
      K = std::max(K, k);
      J = std::max(J, j);
      w.stats_host[1] += k;
      w.stats_host[2] += j;
    }
    w.stats_host[0] += cnt;
    // (the next chunk overwrites the staging only after its own stream synchronisation)
    if ((e = hipMemcpyAsync(w.plSteps, w.hostSteps, sizeof(int) * 2 * cnt,
                            hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
    // M <- a I + b (product), from its unsummed split partials when ch > 1
    auto affine = [&](float* Mm, int ch, float a, float b, const int* steps, int step) {
      if (ch > 1)   // (one element per thread: the chunk reads are the latency)
        hipLaunchKernelGGL(k_pl_affine_part, dim3(tilesP, cnt), dim3(256), 0, st, part, ch, Mm,
                           nb, a, b, steps, step);
      else
        hipLaunchKernelGGL(k_pl_affine, dim3(tilesN, cnt), dim3(256), 0, st, Mm, nb, a, b,
                           steps, step);
      return last();
    };
    // polar factor of E' / alpha: X <- X (1.5 I - 0.5 X^T X)
    const float* X = w.plX0;
    float* Xn = w.plXa;
    for (int k = 0; k < K; ++k) {
      int ch = 0;
      if ((e = launch_gemm_sym(nb, mb, X, mb, sX, X, mb, sX, w.plT, nb, sN, cnt, st, part, pfl, &ch)) != hipSuccess)
        return e;
      if ((e = affine(w.plT, ch, 1.5f, -0.5f, w.plSteps, k)) != hipSuccess) return e;
      if ((e = launch_gemm(false, mb, nb, nb, X, mb, sX, w.plT, nb, sN, Xn, mb, sX, nullptr, cnt, cnt, st, part, pfl)) != hipSuccess)
        return e;
      X = Xn;
      Xn = (Xn == w.plXa) ? w.plXb : w.plXa;
    }
    // H = Q^T (E' / alpha); S = alpha sym(H) - tau I; Y0 = S / alpha_S
    if ((e = launch_gemm(true, nb, nb, mb, X, mb, sX, w.plX0, mb, sX, w.plT, nb, sN, nullptr, cnt, cnt, st, part, pfl)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_pl_shift, dim3(tilesN, cnt), dim3(256), 0, st, w.plT, w.plS, w.plY, nb,
                       tau, w.plScal);
    if ((e = last()) != hipSuccess) return e;
    // sign(S): Y <- Y (1.5 I - 0.5 Y^2)
    float* Y = w.plY;
    float* Yn = w.plT;
    for (int j = 0; j < J; ++j) {
      int ch = 0;
      if ((e = launch_gemm_sym(nb, nb, Y, nb, sN, Y, nb, sN, w.plW, nb, sN, cnt, st, part, pfl, &ch)) != hipSuccess)
        return e;
      if ((e = affine(w.plW, ch, 1.5f, -0.5f, w.plSteps + 1, j)) != hipSuccess) return e;
      if ((e = launch_gemm_sym(nb, nb, Y, nb, sN, w.plW, nb, sN, Yn, nb, sN, cnt, st, part, pfl)) != hipSuccess)
        return e;
      std::swap(Y, Yn);
    }
    // (S)_+ = S (I + Y) / 2, then Ze = Q (S)_+ into the X0 buffer
    hipLaunchKernelGGL(k_pl_affine, dim3(tilesN, cnt), dim3(256), 0, st, Y, nb, 0.5f, 0.5f,
                       (const int*)nullptr, 0);
    if ((e = last()) != hipSuccess) return e;
    if ((e = launch_gemm_sym(nb, nb, w.plS, nb, sN, Y, nb, sN, w.plW, nb, sN, cnt, st, part, pfl)) != hipSuccess)
      return e;
    if ((e = launch_gemm(false, mb, nb, nb, X, mb, sX, w.plW, nb, sN, Xn, mb, sX, nullptr, cnt, cnt, st, part, pfl)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_pl_rebuild<P>, dim3(tilesZ, cnt), dim3(256), 0, st, Zout, Dout, g, sh,
                       w.live_list, fslot, c0, w.lrC, w.lrV, w.lrSig, mask, tau, Xn, w.plScal);
    if ((e = last()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace msld
