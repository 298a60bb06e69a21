// HIP kernels for the ADMM / block-wise SVT iteration on gfx950 (wave64).
//
// State kept in "D form": with D_i = Z_i - U_i the iteration of Sec. 7 (eq:admm),
//   X_i = (Z_i - U_i) + (Y - sum_j (Z_j - U_j)) / L,  Z_i' = BSVT(X_i + U_i),
//   U_i' = U_i - (Z_i' - X_i),
// becomes, with R = (Y - sum_j D_j) / L and V_i = X_i + U_i = Z_i + R:
//   Z_i' = BSVT_{lambda_i/rho}(V_i),   D_i' = Z_i' - U_i' = 2 Z_i' - V_i,
// and the primal residual term is X_i - Z_i' = D_i + R - Z_i'.
// A pass reads R and Z_i and writes Z_i' and D_i'; no U plane is stored.
#include "msld_internal.h"

namespace msld {

static constexpr float kEps = 5.9604645e-8f;  // 2^-24, unit roundoff of float32

__device__ __forceinline__ int wrap_add(int base, int off, int mod) {
  int v = base + off;
  return v >= mod ? v - mod : v;
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(float* __restrict__ p, float v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill(float* p, float v, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

// ------------------------------------------------------ averaged cycle spinning
// Cycle spinning of Sec. 9 as a mean over a shift set S: the Z-step of a scale runs
// once per shift into a scratch plane, k_spin_acc sums the results, and k_spin_finish
// forms Z' = Acc / |S| and D' = 2 Z' - (Z + R) (the D form of the ADMM update).
// Rows of retired instances (iactive[z] == 0, z = row / IM) are left untouched.
__global__ void k_spin_acc(float* __restrict__ acc, const float* __restrict__ zs, size_t n,
                           size_t inst_elems, const int* __restrict__ iactive, bool vec4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec4) {
    for (; 4 * i < n; i += stride) {
      if (iactive && !iactive[4 * i / inst_elems]) continue;
      float4 a = reinterpret_cast<float4*>(acc)[i];
      const float4 b = reinterpret_cast<const float4*>(zs)[i];
      a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
      reinterpret_cast<float4*>(acc)[i] = a;
    }
  } else {
    for (; i < n; i += stride) {
      if (iactive && !iactive[i / inst_elems]) continue;
      acc[i] += zs[i];
    }
  }
}

__global__ void k_spin_finish(float* __restrict__ Z, float* __restrict__ D,
                              const float* __restrict__ R, const float* __restrict__ acc,
                              float inv, size_t n, size_t inst_elems,
                              const int* __restrict__ iactive, bool vec4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec4) {
    for (; 4 * i < n; i += stride) {
      if (iactive && !iactive[4 * i / inst_elems]) continue;
      const float4 z = reinterpret_cast<const float4*>(Z)[i];
      const float4 r = reinterpret_cast<const float4*>(R)[i];
      const float4 a = reinterpret_cast<const float4*>(acc)[i];
      float4 zn, d;
      zn.x = a.x * inv; zn.y = a.y * inv; zn.z = a.z * inv; zn.w = a.w * inv;
      d.x = 2.f * zn.x - (z.x + r.x);
      d.y = 2.f * zn.y - (z.y + r.y);
      d.z = 2.f * zn.z - (z.z + r.z);
      d.w = 2.f * zn.w - (z.w + r.w);
      reinterpret_cast<float4*>(Z)[i] = zn;
      reinterpret_cast<float4*>(D)[i] = d;
    }
  } else {
    for (; i < n; i += stride) {
      if (iactive && !iactive[i / inst_elems]) continue;
      const float zn = acc[i] * inv;
      D[i] = 2.f * zn - (Z[i] + R[i]);
      Z[i] = zn;
    }
  }
}

static unsigned spin_blocks(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 8192) b = 8192;
  return (unsigned)(b ? b : 1);
}

hipError_t launch_spin_acc(float* acc, const float* zs, size_t n, size_t inst_elems,
                           const int* iactive, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const bool vec4 = inst_elems % 4 == 0;
  hipLaunchKernelGGL(k_spin_acc, dim3(spin_blocks(vec4 ? n / 4 : n)), dim3(256), 0, st, acc, zs,
                     n, inst_elems, iactive, vec4);
  return hipGetLastError();
}

hipError_t launch_spin_finish(float* Z, float* D, const float* R, const float* acc, float inv,
                              size_t n, size_t inst_elems, const int* iactive, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const bool vec4 = inst_elems % 4 == 0;
  hipLaunchKernelGGL(k_spin_finish, dim3(spin_blocks(vec4 ? n / 4 : n)), dim3(256), 0, st, Z, D,
                     R, acc, inv, n, inst_elems, iactive, vec4);
  return hipGetLastError();
}

// ---------------------------------------------------------- consensus pass
// R = (Y - sum_j D_j) / L  (X-update of eq:admm), fused with every 1x1 scale:
// for 1x1 blocks the block-wise SVT is the entrywise soft-threshold (Sec. 7), so
// Z_i' = soft(Z_i + R, tau_i) and D_i' = 2 Z_i' - (Z_i + R) are produced here.
struct OneByOne {
  int idx[16];
  float tau[16];
  int n;
};

__device__ __forceinline__ float soft(float v, float t) {
  return v - fminf(fmaxf(v, -t), t);
}

__global__ void __launch_bounds__(256) k_consensus_v4(
    const float* __restrict__ Y, int64_t ldY, const float* __restrict__ Dcur,
    float* __restrict__ Dnext, float* __restrict__ Z, float* __restrict__ R, int M, int N,
    int L, float invL, OneByOne ob, int IM, const int* __restrict__ iactive,
    const uint8_t* __restrict__ mask, int64_t ldmask) {
  const int64_t MN = (int64_t)M * N;
  const int total4 = (int)(MN >> 2);
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total4; e += stride) {
    const int flat = e << 2;
    const int r = flat / N;
    const int c = flat - r * N;
    if (iactive && !iactive[r / IM]) continue;
    float4 y = *reinterpret_cast<const float4*>(Y + (int64_t)r * ldY + c);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int j = 0; j < L; ++j) {
      const float4 d = *reinterpret_cast<const float4*>(Dcur + j * MN + flat);
      s.x += d.x; s.y += d.y; s.z += d.z; s.w += d.w;
    }
    float4 rr;
    rr.x = (y.x - s.x) * invL; rr.y = (y.y - s.y) * invL;
    rr.z = (y.z - s.z) * invL; rr.w = (y.w - s.w) * invL;
    if (mask) {   // masked data consistency: no correction on unobserved entries
      const uint8_t* mk = mask + (int64_t)r * ldmask + c;
      if (!mk[0]) rr.x = 0.f;
      if (!mk[1]) rr.y = 0.f;
      if (!mk[2]) rr.z = 0.f;
      if (!mk[3]) rr.w = 0.f;
    }
    for (int t = 0; t < ob.n; ++t) {
      const int j = ob.idx[t];
      const float tau = ob.tau[t];
      float4* zp = reinterpret_cast<float4*>(Z + j * MN + flat);
      float4 z = *zp;
      float4 v;
      v.x = z.x + rr.x; v.y = z.y + rr.y; v.z = z.z + rr.z; v.w = z.w + rr.w;
      z.x = soft(v.x, tau); z.y = soft(v.y, tau); z.z = soft(v.z, tau); z.w = soft(v.w, tau);
      *zp = z;
      float4 d;
      d.x = 2.f * z.x - v.x; d.y = 2.f * z.y - v.y; d.z = 2.f * z.z - v.z; d.w = 2.f * z.w - v.w;
      *reinterpret_cast<float4*>(Dnext + j * MN + flat) = d;
    }
    *reinterpret_cast<float4*>(R + flat) = rr;
  }
}

__global__ void __launch_bounds__(256) k_consensus_s(
    const float* __restrict__ Y, int64_t ldY, const float* __restrict__ Dcur,
    float* __restrict__ Dnext, float* __restrict__ Z, float* __restrict__ R, int M, int N,
    int L, float invL, OneByOne ob, int IM, const int* __restrict__ iactive,
    const uint8_t* __restrict__ mask, int64_t ldmask) {
  const int64_t MN = (int64_t)M * N;
  const int total = (int)MN;
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int r = e / N;
    const int c = e - r * N;
    if (iactive && !iactive[r / IM]) continue;
    float s = 0.f;
    for (int j = 0; j < L; ++j) s += Dcur[j * MN + e];
    float rr = (Y[(int64_t)r * ldY + c] - s) * invL;
    if (mask && !mask[(int64_t)r * ldmask + c]) rr = 0.f;   // unobserved entry
    for (int t = 0; t < ob.n; ++t) {
      const int j = ob.idx[t];
      const float v = Z[j * MN + e] + rr;
      const float z = soft(v, ob.tau[t]);
      Z[j * MN + e] = z;
      Dnext[j * MN + e] = 2.f * z - v;
    }
    R[e] = rr;
  }
}

hipError_t launch_consensus(const float* Y, int64_t ldY, const float* Dcur, float* Dnext,
                            float* Z, float* R, int M, int N, int L, const int* scales1,
                            const float* taus1, int n1, int IM, const int* iactive,
                            const uint8_t* mask, int64_t ldmask, hipStream_t st) {
  OneByOne ob;
  ob.n = n1;
  for (int t = 0; t < 16; ++t) {
    ob.idx[t] = t < n1 ? scales1[t] : 0;
    ob.tau[t] = t < n1 ? taus1[t] : 0.f;
  }
  const int64_t MN = (int64_t)M * N;
  const float invL = 1.0f / (float)L;
  const bool vec = (N % 4 == 0) && (ldY % 4 == 0) &&
                   ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
  int64_t work = vec ? MN / 4 : MN;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  if (vec)
    hipLaunchKernelGGL(k_consensus_v4, dim3((unsigned)blocks), dim3(256), 0, st, Y, ldY,
                       Dcur, Dnext, Z, R, M, N, L, invL, ob, IM, iactive, mask, ldmask);
  else
    hipLaunchKernelGGL(k_consensus_s, dim3((unsigned)blocks), dim3(256), 0, st, Y, ldY,
                       Dcur, Dnext, Z, R, M, N, L, invL, ob, IM, iactive, mask, ldmask);
  return hipGetLastError();
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

__global__ void k_copy_count(const int* src, int* dst) {
  if (threadIdx.x == 0) *dst = *src;
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_fill_ints(int* p, int v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_set_int(int* p, int idx, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) p[idx] = v;
}

__global__ void k_set_u64(unsigned long long* p, int idx, unsigned long long v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) p[idx] = v;
}

// Per-instance iteration counters advance for the active instances only.
__global__ void k_inc_active(int* k, const int* active, int n) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < n && active[z]) k[z] += 1;
}

hipError_t launch_fill_ints(int* p, int v, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_ints, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int idx, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, idx, v);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long* p, int idx, unsigned long long v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, p, idx, v);
  return hipGetLastError();
}

hipError_t launch_inc_active(int* k, const int* active, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_inc_active, dim3((n + 255) / 256), dim3(256), 0, st, k, active, n);
  return hipGetLastError();
}

// Retirement of stacked instances on the device, after an iteration's residual sums
// (res[z], ||Y_z||^2 at res[n + z]) and iteration counters (ik[z], already advanced):
// an active instance stops when r = sqrt(res / ||Y||^2) is not finite, when tol > 0,
// ik % check_every == 0 and r <= tol, or when ik reaches max_iters. Its activity flag
// drops, so later iterations leave its state untouched, and out_iters / out_resid keep
// the count and residual it stopped with (the same as a check after every iteration).
__global__ void k_retire(const double* res, int n, float tol, int check_every, int max_iters,
                         const int* ik, int* active, int* out_iters, double* out_resid) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= n || !active[z]) return;
  const double ny2 = res[n + z] > 0.0 ? res[n + z] : 1.0;
  const double r = sqrt(res[z] / ny2);
  const int k = ik[z];
  out_iters[z] = k;
  out_resid[z] = r;
  if (!isfinite(r) || (tol > 0.f && k % check_every == 0 && r <= (double)tol) || k >= max_iters)
    active[z] = 0;
}

hipError_t launch_retire(const double* res, int n, float tol, int check_every, int max_iters,
                         const int* ik, int* active, int* out_iters, double* out_resid,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_retire, dim3((n + 255) / 256), dim3(256), 0, st, res, n, tol, check_every,
                     max_iters, ik, active, out_iters, out_resid);
  return hipGetLastError();
}

// ------------------------------------------------------- register tier (small blocks)
// Register tier, live blocks only: one lane per block of the live list built by the
// stream pass. The block's V (SM x SN as stored) is read back from D' = -V (written by
// the stream pass), decomposed by cyclic one-sided Jacobi in registers on the shorter
// side (LN columns of length LM: the block, or its transpose when SM < SN),
// thresholded (eq:svt) and written back with the dual update.
template <int SM, int SN>
__global__ void __launch_bounds__(256) k_tiny_live(
    float* __restrict__ Zout, float* __restrict__ Dout, ScaleGeom g, float tau,
    ShiftSpec sh, float jtol, int max_sweeps, const int* __restrict__ live_count,
    const int* __restrict__ live_list, unsigned long long* __restrict__ stats) {
  constexpr bool TR = SM < SN;
  constexpr int LM = TR ? SN : SM;
  constexpr int LN = TR ? SM : SN;
  const int N = g.N, Q = g.Q;
  const int count = *live_count;
  const int stride = gridDim.x * blockDim.x;
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < count; it += stride) {
    const int b = live_list[it];
    const int p = b / Q;
    const int q = b - p * Q;
    int sr, sc;
    block_shift(sh, p / g.PI, SM, SN, &sr, &sc);
    int rows[SM], cols[SN];
#pragma unroll
    for (int i = 0; i < SM; ++i) rows[i] = grow(g, p, i, sr);
#pragma unroll
    for (int j = 0; j < SN; ++j) cols[j] = gcol(g, q, j, sc);
    // a[i][j] (LM x LN) is the logical block: stored (i, j), or (j, i) when transposed
    float a[LM][LN], v0[LM][LN];
#pragma unroll
    for (int i = 0; i < LM; ++i)
#pragma unroll
      for (int j = 0; j < LN; ++j) {
        const int r = TR ? rows[j] : rows[i];
        const int c = TR ? cols[i] : cols[j];
        v0[i][j] = -Dout[(int64_t)r * N + c];
        a[i][j] = v0[i][j];
      }
    float w[LN][LN];
#pragma unroll
    for (int i = 0; i < LN; ++i)
#pragma unroll
      for (int j = 0; j < LN; ++j) w[i][j] = (i == j) ? 1.f : 0.f;
    int sweeps = 0;
    for (int swp = 0; swp < max_sweeps; ++swp) {
      bool rot = false;
#pragma unroll
      for (int pp = 0; pp < LN - 1; ++pp)
#pragma unroll
        for (int qq = pp + 1; qq < LN; ++qq) {
          float al = 0.f, be = 0.f, ga = 0.f;
#pragma unroll
          for (int i = 0; i < LM; ++i) {
            al += a[i][pp] * a[i][pp];
            be += a[i][qq] * a[i][qq];
            ga += a[i][pp] * a[i][qq];
          }
          if (jacobi_rotates(ga, al, be, jtol)) {
            rot = true;
            float c, s;
            jacobi_cs(ga, al, be, &c, &s);
#pragma unroll
            for (int i = 0; i < LM; ++i) {
              const float x = a[i][pp], y = a[i][qq];
              a[i][pp] = c * x - s * y;
              a[i][qq] = s * x + c * y;
            }
#pragma unroll
            for (int i = 0; i < LN; ++i) {
              const float u = w[i][pp], v = w[i][qq];
              w[i][pp] = c * u - s * v;
              w[i][qq] = s * u + c * v;
            }
          }
        }
      ++sweeps;
      if (!rot) break;
    }
    float gn[LN];
    int rank = 0;
#pragma unroll
    for (int j = 0; j < LN; ++j) {
      float s2 = 0.f;
#pragma unroll
      for (int i = 0; i < LM; ++i) s2 += a[i][j] * a[i][j];
      const float sig = sqrtf(s2);
      gn[j] = sig > tau ? 1.f - tau / sig : 0.f;
      rank += gn[j] > 0.f;
    }
    // rank 0: the stream pass already wrote Z' = 0, D' = -V
    if (rank > 0) {
#pragma unroll
      for (int i = 0; i < LM; ++i)
#pragma unroll
        for (int c2 = 0; c2 < LN; ++c2) {
          float z = 0.f;
#pragma unroll
          for (int j = 0; j < LN; ++j) z += gn[j] * a[i][j] * w[c2][j];
          const int r = TR ? rows[c2] : rows[i];
          const int c = TR ? cols[i] : cols[c2];
          const int64_t o = (int64_t)r * N + c;
          Zout[o] = z;
          Dout[o] = 2.f * z - v0[i][c2];
        }
    }
    atomicAdd(&stats[0], 1ull);
    atomicAdd(&stats[1], (unsigned long long)sweeps);
    atomicAdd(&stats[2], (unsigned long long)rank);
  }
}

template <int SM, int SN>
static bool tiny_launch(int blocks, const ScaleGeom& g, float* Zout, float* Dout, float tau,
                        const ShiftSpec& sh, float jtol, int max_sweeps, const ScaleWork& w,
                        hipStream_t st) {
  if (g.m != SM || g.n != SN) return false;
  hipLaunchKernelGGL((k_tiny_live<SM, SN>), dim3(blocks), dim3(256), 0, st, Zout, Dout, g, tau,
                     sh, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
  return true;
}

bool reg_tier_shape(int m, int n) {
  const int lo = m < n ? m : n, hi = m < n ? n : m;
  if (lo == hi) return lo == 2 || lo == 4 || lo == 8;
  return (lo == 2 && (hi == 4 || hi == 8 || hi == 16)) || (lo == 4 && (hi == 8 || hi == 16));
}

// ---------------------------------------------------------------- stream pass
// For one scale: gather V = Z + R over every (shifted) block, write the result the
// block would have if its SVT is zero (Z' = 0, D' = -V) and evaluate the bound of
// Sec. 8 (plus the Frobenius norm, another valid bound on sigma_max). Blocks whose
// bound exceeds tau enter the live list; the SVD pass later reads their V back
// from D' = -V and overwrites both outputs.
// A workgroup handles all m rows of one block row and a strip of `w` columns.
// One strip (item) of one scale; smem is the workgroup's dynamic LDS; NT threads.
template <int NT>
__device__ __forceinline__ void stream_strip(
    int item, const float* __restrict__ Zin, const float* __restrict__ R,
    float* __restrict__ Zout, float* __restrict__ Dout, const ScaleGeom& g,
    const StreamPlan& sp, const ShiftSpec& sh, float tau2lim, int* __restrict__ live_count,
    int* __restrict__ live_list, float* __restrict__ rowpart, float* __restrict__ fropart,
    float* smem) {
  const int N = g.N, m = g.m, n = g.n, Q = g.Q;
  const int p = item / sp.spr;
  const int j = item - p * sp.spr;
  if (!inst_active(sh, p / g.PI)) return;   // uniform: the strip lies in one instance
  int sr, sc;
  block_shift(sh, p / g.PI, m, n, &sr, &sc);
  int col0, w, q0 = 0, nq = 1, part = 0, rlo = 0, rhi = m;
  if (sp.whole) {
    q0 = j * sp.kb;
    nq = min(sp.kb, Q - q0);
    col0 = q0 * n;
    w = nq * n;
  } else {
    q0 = j / sp.spb;
    part = j - q0 * sp.spb;
    const int rpart = part / sp.cst, cpart = part - (part / sp.cst) * sp.cst;
    int start = cpart * sp.ws;
    if (sp.align) {
      // a = columns before the block's first 32-column boundary (global columns,
      // N a multiple of 32, so the boundaries survive the wrap)
      const int a = (32 - (q0 * n + sc) % 32) % 32;
      start = cpart == 0 ? 0 : (a == 0 ? cpart * sp.ws : a + (cpart - 1) * sp.ws);
      const int end = cpart == 0 ? (a == 0 ? sp.ws : a) : start + sp.ws;
      w = min(end, n) - start;
    } else {
      w = min(sp.ws, n - start);
    }
    col0 = q0 * n + start;
    rlo = rpart * sp.rch;
    rhi = min(m, rlo + sp.rch);
    if (w <= 0) {
      // empty strip (aligned layout): zero partials for the bound
      const int64_t blk = (int64_t)p * Q + q0;
      if (sp.rowbound)
        for (int r = threadIdx.x; r < m; r += NT) rowpart[(blk * sp.spb + part) * m + r] = 0.f;
      if (threadIdx.x == 0) fropart[blk * sp.spb + part] = 0.f;
      return;
    }
  }
  // The tile keeps |v| rounded up to bfloat16 (only the bound reads it, and a
  // rounded-up magnitude keeps it an upper bound); the column |.| and squared sums
  // are accumulated from the float values while they stream through.
  const int ldt = w + 1;
  unsigned short* tile = reinterpret_cast<unsigned short*>(smem);   // m x ldt
  float* pcs = smem + (sp.rowbound ? ((m * ldt + 1) >> 1) : 0);  // NT partial column |.| sums
  float* pcq = pcs + NT;                    // NT partial column squares
  float* cs = pcq + NT;                     // w column sums
  float* cq = cs + sp.ws + 1;               // w column squares
  unsigned* smax = reinterpret_cast<unsigned*>(cq + sp.ws + 1);  // nq row maxima
  const int tid = threadIdx.x;
  // strips are at most 256 columns wide (the plan caps them): thread (row group rq,
  // column c) walks rows rq, rq + rpp, ...; kU rows are loaded before any is stored,
  // so every thread keeps 2 kU loads in flight
  const int rpp = NT / w;
  {
    constexpr int kU = 8;
    const int c = tid % w;
    const int rq = tid / w;
    int gc = col0 + c + sc;
    if (gc >= N) gc -= N;
    const bool act = rq < rpp;
    const int z = p / g.PI;
    const int pl = p - z * g.PI;
    const int rbase = pl * m + sr;   // instance-local row of block row 0 (contiguous)
    const int64_t zoff = (int64_t)z * g.IM;
    float sabs = 0.f, ssq = 0.f;
    for (int r0 = rlo + rq; act && r0 < rhi; r0 += kU * rpp) {
      float v[kU];
      int64_t o[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int r = r0 + u * rpp;
        o[u] = -1;
        v[u] = 0.f;
        if (r < rhi) {
          int lr;
          if (g.pw) {
            lr = local_row(g, pl, r, sr);
          } else {
            lr = rbase + r;
            if (lr >= g.IM) lr -= g.IM;
          }
          o[u] = (zoff + lr) * N + gc;
          v[u] = Zin[o[u]] + (R ? R[o[u]] : 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (o[u] >= 0) {
          const float a = fabsf(v[u]);
          sabs += a;
          ssq += v[u] * v[u];
          // round the magnitude up to bfloat16 (beyond the largest finite bfloat16, and
          // for NaN, infinity: the block then always counts as live)
          const unsigned ab = __float_as_uint(a);
          const unsigned bits = ab > 0x7F7F0000u ? 0x7F80u : (ab + 0xFFFFu) >> 16;
          if (sp.rowbound) tile[(r0 + u * rpp) * ldt + c] = (unsigned short)bits;
          Zout[o[u]] = 0.f;
          Dout[o[u]] = -v[u];
        }
      }
    }
    if (act) {
      pcs[tid] = sabs;
      pcq[tid] = ssq;
    }
  }
  if (tid < nq) smax[tid] = 0u;
  __syncthreads();
  if (tid < w) {
    float s = 0.f, s2 = 0.f;
    for (int gq = 0; gq < rpp; ++gq) {
      s += pcs[gq * w + tid];
      s2 += pcq[gq * w + tid];
    }
    cs[tid] = s;
    cq[tid] = s2;
  }
  __syncthreads();
  // weighted row sums per (row, block segment)
  const int segw = sp.whole ? n : w;
  const int npairs = sp.rowbound ? m * nq : 0;
  for (int e = tid; e < npairs; e += NT) {
    const int s = e / m;
    const int r = e - s * m;
    const unsigned short* row = tile + r * ldt + s * segw;
    const float* csg = cs + s * segw;
    float acc = 0.f;
    for (int c = 0; c < segw; ++c) acc += __uint_as_float((unsigned)row[c] << 16) * csg[c];
    if (sp.whole) {
      atomicMax(&smax[s], __float_as_uint(acc));
    } else {
      const int64_t blk = (int64_t)p * Q + q0;
      rowpart[(blk * sp.spb + part) * m + r] = acc;
    }
  }
  __syncthreads();
  if (sp.whole) {
    if (tid < nq) {
      float fro = 0.f;
      for (int c = 0; c < n; ++c) fro += cq[tid * n + c];
      const float bnd = sp.rowbound ? __uint_as_float(smax[tid]) : fro;
      if (fminf(bnd, fro) > tau2lim) {
        const int slot = atomicAdd(live_count, 1);
        live_list[slot] = p * Q + q0 + tid;
      }
    }
  } else if (tid == 0) {
    float fro = 0.f;
    for (int c = 0; c < w; ++c) fro += cq[c];
    fropart[((int64_t)p * Q + q0) * sp.spb + part] = fro;
  }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_stream(
    const float* __restrict__ Zin, const float* __restrict__ R, float* __restrict__ Zout,
    float* __restrict__ Dout, ScaleGeom g, StreamPlan sp, ShiftSpec sh, float tau2lim,
    int* __restrict__ live_count, int* __restrict__ live_list, float* __restrict__ rowpart,
    float* __restrict__ fropart) {
  extern __shared__ float smem[];
  stream_strip<NT>(blockIdx.x, Zin, R, Zout, Dout, g, sp, sh, tau2lim, live_count, live_list,
               rowpart, fropart, smem);
}

// The stream pass of every decomposed scale in one launch: workgroup b takes item
// b - first[i] of the scale i whose item range holds b.
template <int NT>
__global__ void __launch_bounds__(NT) k_stream_all(StreamAll a, const float* __restrict__ Z,
                                                    const float* __restrict__ R,
                                                    float* __restrict__ D, ShiftSpec sh) {
  extern __shared__ float smem[];
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.first[i + 1]) ++i;
  const StreamScale& d = a.s[i];
  ShiftSpec shi = sh;
  shi.scale = d.scale;
  const size_t off = a.plane * (size_t)d.scale;
  stream_strip<NT>(b - a.first[i], Z + off, R, const_cast<float*>(Z) + off, D + off, d.g, d.sp, shi,
               d.tau2lim, d.live_count, d.live_list, d.rowpart, d.fropart, smem);
}

__global__ void k_zero_counts(StreamAll a) {
  if ((int)threadIdx.x < a.n) *a.s[threadIdx.x].live_count = 0;
}

size_t stream_lds_bytes(int m, const StreamPlan& sp);

// One launch per scale on the caller's stream, each with its own LDS size (a shared
// launch would reserve the largest tile for every workgroup and halve the occupancy
// of the small-block scales).
hipError_t launch_stream_all(const StreamAll& a, const float* Z, const float* R, float* D,
                             const ShiftSpec& sh, hipStream_t st, hipEvent_t* after_scale) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int i = 0; i < a.n; ++i) {
    StreamAll b = a;
    b.n = 1;
    b.s[0] = a.s[i];
    b.first[0] = 0;
    b.first[1] = a.first[i + 1] - a.first[i];
    const size_t lds = stream_lds_bytes(a.s[i].g.m, a.s[i].sp);
    if (a.s[i].sp.nt == 512)
      hipLaunchKernelGGL(k_stream_all<512>, dim3(b.first[1]), dim3(512), lds, st, b, Z, R, D, sh);
    else
      hipLaunchKernelGGL(k_stream_all<256>, dim3(b.first[1]), dim3(256), lds, st, b, Z, R, D, sh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the scale's own fork point: its BlockSVT needs no other scale's stream pass
    if (after_scale && after_scale[a.s[i].scale] &&
        (e = hipEventRecord(after_scale[a.s[i].scale], st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Completes the bound of blocks split over several strips (fixed summation order).
__global__ void __launch_bounds__(256) k_bound_reduce(ScaleGeom g, StreamPlan sp,
                                                      float tau2lim, int* live_count,
                                                      int* live_list, const float* rowpart,
                                                      const float* fropart, ShiftSpec sh) {
  __shared__ float red[256];
  const int blk = blockIdx.x;
  if (!inst_active(sh, (blk / g.Q) / g.PI)) return;
  const int m = g.m;
  float mx = 0.f;
  if (!sp.rowbound) mx = __int_as_float(0x7f800000);   // Frobenius bound alone
  for (int r = threadIdx.x; sp.rowbound && r < m; r += 256) {
    // the strip partials of one row, 8 loads in flight (the sum order is fixed)
    const float* rp = rowpart + (int64_t)blk * sp.spb * m + r;
    float s = 0.f;
    int t = 0;
    for (; t + 8 <= sp.spb; t += 8) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = rp[(int64_t)(t + u) * m];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; t < sp.spb; ++t) s += rp[(int64_t)t * m];
    mx = fmaxf(mx, s);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float fro = 0.f;
    for (int t = 0; t < sp.spb; ++t) fro += fropart[(int64_t)blk * sp.spb + t];
    if (fminf(red[0], fro) > tau2lim) {
      const int slot = atomicAdd(live_count, 1);
      live_list[slot] = blk;
    }
  }
}

// ------------------------------------------------------ one-sided Jacobi core
// Parallel (round-robin) ordering: ncols (even) columns, ncols-1 rounds of ncols/2
// disjoint pairs; over a sweep every pair meets once.
__device__ __forceinline__ void rr_pair(int round, int k, int ncols, int* a, int* b) {
  const int n1 = ncols - 1;
  *a = (k == 0) ? 0 : 1 + (k - 1 + round) % n1;
  *b = 1 + (ncols - 2 - k + round) % n1;
}

// Hestenes one-sided Jacobi on the columns of A (column j at A + j*lda, `arows`
// rows), accumulating the same rotations into W (column j at W + j*ldw, `wrows`
// rows). Each pair is handled by G consecutive lanes; lane t owns rows t + G*i,
// i < RPL (G * RPL >= arows, wrows), cached in registers for the step. The three
// inner products are reduced across the G lanes with xor shuffles. Returns the
// number of sweeps run; *any_rot tells whether any rotation was applied. All threads
// of the workgroup must call it. With SG > 0 the workgroup is one wavefront holding
// 64 / SG independent matrices, one per group of SG lanes (lanes of a disabled group,
// en == false, take part in the barriers only); the sweep loop then runs until every
// group has converged, and a converged group's extra sweeps rotate nothing, so each
// group's result and sweep count are those it would have alone.
template <int G, int RPL, int SG = 0>
__device__ int jacobi_sweeps(float* A, int lda, int arows, float* W, int ldw, int wrows,
                             int ncols, int max_sweeps, float tol, int* any_rot, bool en = true) {
  const int tid = SG ? (int)(threadIdx.x % SG) : (int)threadIdx.x;
  const int npairs = ncols >> 1;
  const int grp = tid / G;
  const int t = tid - grp * G;
  const bool act = en && grp < npairs;
  const int n1 = ncols - 1;
  // round-robin schedule: pa = 0 or 1 + (grp - 1 + rd) mod n1, pb = 1 + (ncols - 2 - grp + rd) mod n1
  const int ia = grp - 1;
  const int ib = ncols - 2 - grp;
  int sweeps = 0;
  [[maybe_unused]] bool done = false;
  *any_rot = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int rotated = 0;
    for (int rd = 0; rd < n1; ++rd) {
      float al = 0.f, be = 0.f, ga = 0.f;
      float x[RPL], y[RPL];
      int pa = 0, pb = 0;
      if (act) {
        int ta = ia + rd;
        if (ta >= n1) ta -= n1;
        int tb = ib + rd;
        if (tb >= n1) tb -= n1;
        pa = (grp == 0) ? 0 : 1 + ta;
        pb = 1 + tb;
        const float* ap = A + pa * lda;
        const float* aq = A + pb * lda;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = t + G * i;
          x[i] = r < arows ? ap[r] : 0.f;
          y[i] = r < arows ? aq[r] : 0.f;
          al += x[i] * x[i];
          be += y[i] * y[i];
          ga += x[i] * y[i];
        }
      }
#pragma unroll
      for (int o = G >> 1; o > 0; o >>= 1) {
        al += __shfl_xor(al, o);
        be += __shfl_xor(be, o);
        ga += __shfl_xor(ga, o);
      }
      if (act && jacobi_rotates(ga, al, be, tol)) {
        rotated = 1;
        float c, s;
        jacobi_cs(ga, al, be, &c, &s);
        float* ap = A + pa * lda;
        float* aq = A + pb * lda;
        float* wp = W + pa * ldw;
        float* wq = W + pb * ldw;
        float u[RPL], v[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = t + G * i;
          u[i] = r < wrows ? wp[r] : 0.f;
          v[i] = r < wrows ? wq[r] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = t + G * i;
          if (r < arows) {
            ap[r] = c * x[i] - s * y[i];
            aq[r] = s * x[i] + c * y[i];
          }
          if (r < wrows) {
            wp[r] = c * u[i] - s * v[i];
            wq[r] = s * u[i] + c * v[i];
          }
        }
      }
      __syncthreads();
    }
    if constexpr (SG == 0) {
      ++sweeps;
      if (!__syncthreads_or(rotated)) break;
      *any_rot = 1;
    } else {
      const unsigned long long bal = __ballot(rotated);
      const int sb = threadIdx.x / SG;
      const bool mine = ((bal >> (sb * SG)) & ((1ull << SG) - 1ull)) != 0ull;
      if (!done) {
        ++sweeps;
        if (mine) *any_rot = 1;
        else done = true;
      }
      if (!__syncthreads_or(!done)) break;
    }
  }
  return sweeps;
}

// ------------------------------------------------------------- LDS tier
// One workgroup per live block (persistent over the live list), or, for blocks whose
// pairs fill at most half a wavefront (BPW > 1), one wavefront of 64 lanes holding BPW
// blocks, one per group of 64 / BPW lanes. The logical block B (block or its
// transpose, mb >= nb) and the rotation matrix W live in LDS, one region per block.
template <int G, int RPL, int BPW>
__global__ void __launch_bounds__(1024) k_svd_lds(
    float* __restrict__ Zout, float* __restrict__ Dout, ScaleGeom g, ShiftSpec sh,
    float tau, float jtol, int max_sweeps, const int* __restrict__ live_count,
    const int* __restrict__ live_list, unsigned long long* __restrict__ stats) {
  extern __shared__ float smem[];
  const int N = g.N, m = g.m, n = g.n, Q = g.Q;
  const int mb = g.mb, nb = g.nb, trans = g.trans;
  const int nbp = (nb + 1) & ~1;
  const int lda = mb | 1;
  const int ldw = nb | 1;
  constexpr int SG = BPW > 1 ? 64 / BPW : 0;
  const int sb = BPW > 1 ? (int)threadIdx.x / SG : 0;
  float* A = smem + sb * (nbp * lda + nbp * ldw + 2 * nbp);
  float* W = A + nbp * lda;
  float* gain = W + nbp * ldw;
  int* lcols = reinterpret_cast<int*>(gain + nbp);
  __shared__ int s_k[BPW];
  const int count = *live_count;
  const int nt = BPW > 1 ? SG : (int)blockDim.x;
  const int tid = BPW > 1 ? (int)threadIdx.x - sb * SG : (int)threadIdx.x;
  for (int base = blockIdx.x * BPW; base < count; base += gridDim.x * BPW) {
    const int it = base + sb;
    const bool valid = it < count;
    const int blk = valid ? live_list[it] : 0;
    const int p = blk / Q;
    const int q = blk - p * Q;
    int sr, sc;
    block_shift(sh, p / g.PI, m, n, &sr, &sc);
    // gather V = -D' (written by the stream pass) into logical column-major B, four
    // loads in flight per lane
    const int tot = valid ? m * n : 0;
    for (int e0 = tid; e0 < tot; e0 += 4 * nt) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * nt;
        const int i = e / n, j = e - (e / n) * n;
        v[u] = e < tot ? -Dout[(int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc)] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * nt;
        if (e >= tot) break;
        const int i = e / n, j = e - (e / n) * n;
        if (!trans) A[j * lda + i] = v[u];
        else A[i * lda + j] = v[u];
      }
    }
    if (valid && nbp > nb)
      for (int r = tid; r < mb; r += nt) A[nb * lda + r] = 0.f;
    for (int e = tid; valid && e < nbp * nb; e += nt) {
      const int jj = e / nb;
      const int c = e - jj * nb;
      W[jj * ldw + c] = (jj == c) ? 1.f : 0.f;
    }
    __syncthreads();
    int any_rot;
    const int sweeps = jacobi_sweeps<G, RPL, SG>(A, lda, mb, W, ldw, nb, nbp, max_sweeps, jtol,
                                                 &any_rot, valid);
    // singular values sigma_j = ||B w_j||, gains max(1 - tau/sigma_j, 0)  (eq:svt)
    for (int jj = tid; valid && jj < nb; jj += nt) {
      float s2 = 0.f;
      for (int r = 0; r < mb; ++r) s2 += A[jj * lda + r] * A[jj * lda + r];
      const float sig = sqrtf(s2);
      gain[jj] = sig > tau ? 1.f - tau / sig : 0.f;
    }
    __syncthreads();
    if (valid && tid == 0) {
      int k = 0;
      for (int jj = 0; jj < nb; ++jj)
        if (gain[jj] > 0.f) lcols[k++] = jj;
      s_k[sb] = k;
      atomicAdd(&stats[0], 1ull);
      atomicAdd(&stats[1], (unsigned long long)sweeps);
      atomicAdd(&stats[2], (unsigned long long)k);
    }
    __syncthreads();
    const int k = valid ? s_k[sb] : 0;
    // rebuild B' = sum_j g_j (B w_j) w_j^T and scatter to the wrapped coordinates
    // (rank 0: the stream pass already wrote Z' = 0, D' = -V)
    const int totr = k > 0 ? m * n : 0;
    for (int e0 = tid; e0 < totr; e0 += 4 * nt) {
      int64_t o[4];
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * nt;
        const int i = e / n, j = e - (e / n) * n;
        o[u] = e < totr ? (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc) : 0;
        v[u] = e < totr ? -Dout[o[u]] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * nt;
        if (e >= totr) break;
        const int i = e / n, j = e - (e / n) * n;
        const int r = trans ? j : i;
        const int c = trans ? i : j;
        float z = 0.f;
        for (int t = 0; t < k; ++t) {
          const int l = lcols[t];
          z += gain[l] * A[l * lda + r] * W[l * ldw + c];
        }
        Zout[o[u]] = z;
        Dout[o[u]] = 2.f * z - v[u];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ panel tier
// Blocks too large for LDS: block one-sided Jacobi over column panels of width pw
// kept in HBM (column-major A, W per live block slot). Each round pairs panels
// round-robin; a workgroup orthogonalises the 2*pw columns of one panel pair in
// LDS (one inner sweep) and writes them back.
__global__ void __launch_bounds__(256) k_panel_load(const float* __restrict__ Dout, ScaleGeom g,
                                                    ShiftSpec sh, const int* live_count,
                                                    const int* live_list, float* pA, int nbp) {
  __shared__ float tile[32][33];
  const int N = g.N, m = g.m, n = g.n, Q = g.Q, mb = g.mb;
  const int count = *live_count;
  const int tilesj = (n + 31) / 32;
  const int ti = blockIdx.x / tilesj;
  const int tj = blockIdx.x - ti * tilesj;
  const int i0 = ti * 32, j0 = tj * 32;
  for (int it = blockIdx.y; it < count; it += gridDim.y) {
    const int blk = live_list[it];
    const int p = blk / Q;
    const int q = blk - p * Q;
    int sr, sc;
    block_shift(sh, p / g.PI, m, n, &sr, &sc);
    float* A = pA + (int64_t)it * nbp * mb;
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int ii = e >> 5, jj = e & 31;
      const int i = i0 + ii, j = j0 + jj;
      float v = 0.f;
      if (i < m && j < n) {
        const int64_t o = (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc);
        v = -Dout[o];
      }
      tile[ii][jj] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int a = e >> 5, b = e & 31;
      if (!g.trans) {
        // column j0+a of B, rows i0+b
        const int i = i0 + b, j = j0 + a;
        if (i < m && j < n) A[(int64_t)j * mb + i] = tile[b][a];
      } else {
        // B = block^T: column i0+a of B, rows j0+b
        const int i = i0 + a, j = j0 + b;
        if (i < m && j < n) A[(int64_t)i * mb + j] = tile[a][b];
      }
    }
    __syncthreads();
  }
}

__global__ void k_panel_init(ScaleGeom g, const int* live_count, float* pA, float* pW,
                             int* pflag, int nbp) {
  const int count = *live_count;
  const int mb = g.mb, nb = g.nb;
  for (int it = blockIdx.y; it < count; it += gridDim.y) {
    float* A = pA + (int64_t)it * nbp * mb;
    float* W = pW + (int64_t)it * nbp * nb;
    const int64_t wn = (int64_t)nbp * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < wn;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int jj = (int)(e / nb);
      const int c = (int)(e - (int64_t)jj * nb);
      W[e] = (jj == c) ? 1.f : 0.f;
    }
    const int64_t pad = (int64_t)(nbp - nb) * mb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < pad;
         e += (int64_t)gridDim.x * blockDim.x)
      A[(int64_t)nb * mb + e] = 0.f;
    if (blockIdx.x == 0 && threadIdx.x < 4) pflag[4 * it + threadIdx.x] = 0;
  }
}

template <int G, int PRPL>
__global__ void __launch_bounds__(256) k_panel_round(ScaleGeom g, const int* live_count,
                                                     float* pA, float* pW, int* pflag, int nbp,
                                                     int pw, int round, float jtol) {
  extern __shared__ float smem[];
  const int mb = g.mb, nb = g.nb;
  const int npan = nbp / pw;
  const int lda = mb | 1;
  const int ldw = nb | 1;
  float* A = smem;                 // 2pw x lda
  float* W = A + 2 * pw * lda;     // 2pw x ldw
  const int count = *live_count;
  int pa, pb;
  rr_pair(round, blockIdx.x, npan, &pa, &pb);
  for (int it = blockIdx.y; it < count; it += gridDim.y) {
    if (pflag[4 * it + 1]) continue;  // converged: uniform across the workgroup
    float* gA = pA + (int64_t)it * nbp * mb;
    float* gW = pW + (int64_t)it * nbp * nb;
    for (int e = threadIdx.x; e < 2 * pw * mb; e += blockDim.x) {
      const int jj = e / mb;
      const int r = e - jj * mb;
      const int col = (jj < pw) ? pa * pw + jj : pb * pw + (jj - pw);
      A[jj * lda + r] = gA[(int64_t)col * mb + r];
    }
    for (int e = threadIdx.x; e < 2 * pw * nb; e += blockDim.x) {
      const int jj = e / nb;
      const int r = e - jj * nb;
      const int col = (jj < pw) ? pa * pw + jj : pb * pw + (jj - pw);
      W[jj * ldw + r] = gW[(int64_t)col * nb + r];
    }
    __syncthreads();
    int any_rot;
    jacobi_sweeps<G, PRPL>(A, lda, mb, W, ldw, nb, 2 * pw, 1, jtol, &any_rot);
    if (any_rot && threadIdx.x == 0) atomicOr(&pflag[4 * it], 1);
    for (int e = threadIdx.x; e < 2 * pw * mb; e += blockDim.x) {
      const int jj = e / mb;
      const int r = e - jj * mb;
      const int col = (jj < pw) ? pa * pw + jj : pb * pw + (jj - pw);
      gA[(int64_t)col * mb + r] = A[jj * lda + r];
    }
    for (int e = threadIdx.x; e < 2 * pw * nb; e += blockDim.x) {
      const int jj = e / nb;
      const int r = e - jj * nb;
      const int col = (jj < pw) ? pa * pw + jj : pb * pw + (jj - pw);
      gW[(int64_t)col * nb + r] = W[jj * ldw + r];
    }
    __syncthreads();
  }
}

__global__ void k_panel_sweep_end(const int* live_count, int* pflag,
                                  unsigned long long* stats) {
  const int count = *live_count;
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < count;
       it += gridDim.x * blockDim.x) {
    if (pflag[4 * it + 1]) continue;
    atomicAdd(&stats[1], 1ull);                   // one more sweep ran on this block
    if (!pflag[4 * it]) pflag[4 * it + 1] = 1;   // no pair above tolerance: converged
    pflag[4 * it] = 0;
  }
}

__global__ void __launch_bounds__(256) k_panel_gain(ScaleGeom g, const int* live_count,
                                                    const float* pA, float* pg, int nbp,
                                                    float tau, unsigned long long* stats,
                                                    const int* pflag) {
  __shared__ int s_rank;
  const int mb = g.mb, nb = g.nb;
  const int count = *live_count;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    if (pflag[4 * it + 2]) continue;  // handled by the certified low-rank path
    if (threadIdx.x == 0) s_rank = 0;
    __syncthreads();
    const float* A = pA + (int64_t)it * nbp * mb;
    for (int jj = wv; jj < nb; jj += 4) {
      float s2 = 0.f;
      for (int r = lane; r < mb; r += 64) s2 += A[(int64_t)jj * mb + r] * A[(int64_t)jj * mb + r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
      if (lane == 0) {
        const float sig = sqrtf(s2);
        const float gj = sig > tau ? 1.f - tau / sig : 0.f;
        pg[(int64_t)it * nbp + jj] = gj;
        if (gj > 0.f) atomicAdd(&s_rank, 1);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicAdd(&stats[0], 1ull);
      atomicAdd(&stats[2], (unsigned long long)s_rank);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_panel_rebuild(float* __restrict__ Zout,
                                                       float* __restrict__ Dout, ScaleGeom g,
                                                       ShiftSpec sh, const int* live_count,
                                                       const int* live_list, const float* pA,
                                                       const float* pW, const float* pg,
                                                       int nbp, const int* pflag) {
  __shared__ int lcols[4096];
  __shared__ float lg[4096];
  __shared__ int s_k;
  const int N = g.N, m = g.m, n = g.n, Q = g.Q, mb = g.mb, nb = g.nb;
  const int count = *live_count;
  const int tilesj = (n + 31) / 32;
  const int ti = blockIdx.x / tilesj;
  const int tj = blockIdx.x - ti * tilesj;
  const int i0 = ti * 32, j0 = tj * 32;
  for (int it = blockIdx.y; it < count; it += gridDim.y) {
    if (pflag[4 * it + 2]) continue;  // handled by the certified low-rank path
    const int blk = live_list[it];
    const int p = blk / Q;
    const int q = blk - p * Q;
    int sr, sc;
    block_shift(sh, p / g.PI, m, n, &sr, &sc);
    const float* A = pA + (int64_t)it * nbp * mb;
    const float* W = pW + (int64_t)it * nbp * nb;
    const float* gg = pg + (int64_t)it * nbp;
    if (threadIdx.x == 0) {
      int k = 0;
      for (int l = 0; l < nb && k < 4096; ++l)
        if (gg[l] > 0.f) {
          lcols[k] = l;
          lg[k] = gg[l];
          ++k;
        }
      s_k = k;
    }
    __syncthreads();
    const int k = s_k;
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int ii = e >> 5, jj = e & 31;
      const int i = i0 + ii, j = j0 + jj;
      if (i >= m || j >= n) continue;
      const int r = g.trans ? j : i;
      const int c = g.trans ? i : j;
      float z = 0.f;
      for (int t = 0; t < k; ++t) {
        const int l = lcols[t];
        z += lg[t] * A[(int64_t)l * mb + r] * W[(int64_t)l * nb + c];
      }
      const int64_t o = (int64_t)grow(g, p, i, sr) * N + gcol(g, q, j, sc);
      const float v = -Dout[o];
      Zout[o] = z;
      Dout[o] = 2.f * z - v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------- scale dispatcher
template <int G>
static hipError_t launch_lds_g(int grid, int threads, size_t lds, float* Zout, float* Dout,
                               const ScaleGeom& g, const ShiftSpec& sh, float tau, float jtol,
                               int max_sweeps, ScaleWork& w, hipStream_t st, int bpw = 1) {
  // rows per lane: G * RPL >= mb
  const int need = (g.mb + G - 1) / G;
  if (bpw > 1) {
    // several blocks per wavefront: lds holds bpw block regions
    if constexpr (G <= 8) {
      if (need > 8 || threads != 64 || ((g.nb + 1) / 2) * G > 64 / bpw) return hipErrorInvalidValue;
      if (bpw == 2)
        hipLaunchKernelGGL((k_svd_lds<G, 8, 2>), dim3(grid), dim3(64), lds, st, Zout, Dout, g,
                           sh, tau, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
      else if (bpw == 4)
        hipLaunchKernelGGL((k_svd_lds<G, 8, 4>), dim3(grid), dim3(64), lds, st, Zout, Dout, g,
                           sh, tau, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
      else if (bpw == 8)
        hipLaunchKernelGGL((k_svd_lds<G, 8, 8>), dim3(grid), dim3(64), lds, st, Zout, Dout, g,
                           sh, tau, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
      else
        return hipErrorInvalidValue;
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (need <= 8)
    hipLaunchKernelGGL((k_svd_lds<G, 8, 1>), dim3(grid), dim3(threads), lds, st, Zout, Dout, g,
                       sh, tau, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
  else if (need <= 32)
    hipLaunchKernelGGL((k_svd_lds<G, 32, 1>), dim3(grid), dim3(threads), lds, st, Zout, Dout, g,
                       sh, tau, jtol, max_sweeps, w.live_count, w.live_list, w.stats);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int G>
static hipError_t launch_round_g(dim3 grid, size_t lds, const ScaleGeom& g, ScaleWork& w,
                                 int round, float jtol, hipStream_t st) {
  // rows per lane for the panel pair: G * PRPL >= max(mb, nb)
  const int need = (g.mb + G - 1) / G;
  if (need <= 8)
    hipLaunchKernelGGL((k_panel_round<G, 8>), grid, dim3(256), lds, st, g, w.live_count, w.pA,
                       w.pW, w.pflag, w.nbp, w.pw, round, jtol);
  else if (need <= 32)
    hipLaunchKernelGGL((k_panel_round<G, 32>), grid, dim3(256), lds, st, g, w.live_count, w.pA,
                       w.pW, w.pflag, w.nbp, w.pw, round, jtol);
  else if (need <= 128)
    hipLaunchKernelGGL((k_panel_round<G, 128>), grid, dim3(256), lds, st, g, w.live_count, w.pA,
                       w.pW, w.pflag, w.nbp, w.pw, round, jtol);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int lds_tier_threads(int nb, int mb, int* G) {
  const int pairs = (nb + 1) / 2;
  int gg = 1;
  while (gg * 8 < mb && gg < 32) gg *= 2;   // rows per lane stay <= 8
  *G = gg;
  int threads = pairs * gg;
  threads = ((threads + 63) / 64) * 64;
  return threads;   // the plan only uses the LDS tier when this is <= 1024
}

static int lds_tier_pack(int nb, int mb) {
  // blocks per wavefront: pairs * G lanes rounded up to a power of two (at least 8)
  int G = 1;
  const int threads = lds_tier_threads(nb, mb, &G);
  const int lanes = ((nb + 1) / 2) * G;
  if (threads != 64 || G > 8 || lanes > 32) return 1;
  int sg = 8;
  while (sg < lanes) sg *= 2;
  return 64 / sg;
}

size_t lds_tier_bytes(int mb, int nb) {
  const int nbp = (nb + 1) & ~1;
  return (size_t)4 * ((size_t)nbp * (mb | 1) + (size_t)nbp * (nb | 1) + nbp) + 4 * (size_t)nbp;
}

size_t stream_lds_bytes(int m, const StreamPlan& sp) {
  // bfloat16 tile (m x (ws + 1), only for the row bound), then 2 nt + 2 (ws + 1) + ws + 1
  // floats
  const size_t tile = sp.rowbound ? ((size_t)m * (sp.ws + 1) + 1) / 2 : 0;
  return (size_t)4 * (tile + 2 * (size_t)sp.nt + 2 * (sp.ws + 1) + sp.ws + 1);
}

#define MSLD_EV(i)                                                    \
  do {                                                                \
    if (ev) {                                                         \
      hipError_t ee_ = hipEventRecord(ev[(i)], st);                   \
      if (ee_ != hipSuccess) return ee_;                              \
    }                                                                 \
  } while (0)

// ------------------------------------------------------------ noise scale
// The noise scale of Sec. 2 reshapes the whole (instance) matrix to an MN x 1 vector;
// the SVT of eq:svt on it is z = v max(1 - tau / ||v||_F, 0) with v = Z + R. Three
// steps: per-instance partial sums of squares (fixed order), the gain, the update with
// the fused dual D' = 2 Z' - V.
__global__ void __launch_bounds__(256) k_fro_norm(const float* __restrict__ Zin,
                                                  const float* __restrict__ R,
                                                  int64_t inst_elems,
                                                  const int* __restrict__ iactive,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int z = blockIdx.y;
  double acc = 0.0;
  if (!iactive || iactive[z]) {
    const int64_t base = (int64_t)z * inst_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < inst_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
      const float v = Zin[base + e] + (R ? R[base + e] : 0.f);
      acc += (double)v * (double)v;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)z * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_fro_gain(const double* __restrict__ part, int parts, int ninst, float tau,
                           const int* __restrict__ iactive, float* __restrict__ gain,
                           unsigned long long* __restrict__ stats) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= ninst) return;
  if (iactive && !iactive[z]) return;
  double ss = 0.0;
  for (int b = 0; b < parts; ++b) ss += part[(int64_t)z * parts + b];
  const double nv = sqrt(ss);
  const float g = nv > (double)tau ? (float)(1.0 - (double)tau / nv) : 0.f;
  gain[z] = g;
  atomicAdd(&stats[0], 1ull);
  if (g > 0.f) atomicAdd(&stats[2], 1ull);
}

__global__ void __launch_bounds__(256) k_fro_apply(const float* __restrict__ Zin,
                                                   const float* __restrict__ R,
                                                   float* __restrict__ Zout,
                                                   float* __restrict__ Dout, int64_t inst_elems,
                                                   int ninst, const int* __restrict__ iactive,
                                                   const float* __restrict__ gain) {
  const int64_t total = inst_elems * ninst;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(e / inst_elems);
    if (iactive && !iactive[z]) continue;
    const float v = Zin[e] + (R ? R[e] : 0.f);
    const float zz = gain[z] * v;
    Zout[e] = zz;
    Dout[e] = 2.f * zz - v;
  }
}

static hipError_t launch_noise(const ScaleGeom& g, ScaleWork& w, const float* Zin,
                               const float* R, float* Zout, float* Dout, float tau,
                               const ShiftSpec& sh, hipStream_t st) {
  const int64_t inst = (int64_t)g.IM * g.N;
  hipLaunchKernelGGL(k_fro_norm, dim3(kFroParts, g.NI), dim3(256), 0, st, Zin, R, inst,
                     sh.iactive, w.froPart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fro_gain, dim3((g.NI + 255) / 256), dim3(256), 0, st, w.froPart,
                     kFroParts, g.NI, tau, sh.iactive, w.froGain, w.stats);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t blocks = (inst * g.NI + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fro_apply, dim3((unsigned)blocks), dim3(256), 0, st, Zin, R, Zout, Dout,
                     inst, g.NI, sh.iactive, w.froGain);
  return hipGetLastError();
}

float stream_tau2lim(const ScaleGeom& g, float tau) {
  // skip only if the bound is below tau^2 by more than its rounding error
  const double tl = (double)tau * (double)tau *
                    (1.0 - 2.0 * (double)(g.m + g.n + 4) * (double)kEps);
  return (float)tl;
}

hipError_t finish_fallback(const ScaleGeom& g, ScaleWork& w, float* Zout, float* Dout, float tau,
                           const ShiftSpec& sh, hipStream_t st) {
  hipError_t e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const int fallback = w.hostInts[1];
  if (fallback > 0) return run_polar(g, w, Zout, Dout, tau, sh, fallback, st);
  return hipSuccess;
}

hipError_t launch_scale(const ScaleGeom& g, int tier, const StreamPlan& sp, ScaleWork& w,
                        const float* Zin, const float* R, float* Zout, float* Dout, float tau,
                        const ShiftSpec& sh, float jtol, int max_sweeps, int panel_sweeps,
                        int num_cus, hipStream_t st, hipEvent_t* ev, int* round_launches,
                        bool stream_done, int* deferred) {
  hipError_t e;
  if (deferred) *deferred = 0;
  if (tier == TIER_FRO) {
    MSLD_EV(0); MSLD_EV(1); MSLD_EV(2);
    if ((e = launch_noise(g, w, Zin, R, Zout, Dout, tau, sh, st)) != hipSuccess) return e;
    MSLD_EV(3); MSLD_EV(4);
    return hipSuccess;
  }
  const float tau2lim = stream_tau2lim(g, tau);
  const int nblk = g.P * g.Q;
  // stream pass: speculative zero-output write + bound + live list (unless the caller
  // ran it for all scales at once)
  {
    MSLD_EV(0);   // events 0-1 bracket the stream kernel alone
    if (!stream_done) {
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, w.live_count);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const size_t lds = stream_lds_bytes(g.m, sp);
      if (sp.nt == 512)
        hipLaunchKernelGGL(k_stream<512>, dim3(g.P * sp.spr), dim3(512), lds, st, Zin, R, Zout,
                           Dout, g, sp, sh, tau2lim, w.live_count, w.live_list, w.rowpart,
                           w.fropart);
      else
        hipLaunchKernelGGL(k_stream<256>, dim3(g.P * sp.spr), dim3(256), lds, st, Zin, R, Zout,
                           Dout, g, sp, sh, tau2lim, w.live_count, w.live_list, w.rowpart,
                           w.fropart);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    MSLD_EV(1);
    if (!sp.whole) {
      hipLaunchKernelGGL(k_bound_reduce, dim3(nblk), dim3(256), 0, st, g, sp, tau2lim,
                         w.live_count, w.live_list, w.rowpart, w.fropart, sh);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (tier == TIER_REG) {
    MSLD_EV(2);
    int blocks = num_cus * 8;
    if (blocks * 256 > nblk) blocks = (nblk + 255) / 256;
    const bool ok =
        tiny_launch<2, 2>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<4, 4>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<8, 8>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<4, 2>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<2, 4>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<8, 2>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<2, 8>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<16, 2>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<2, 16>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<8, 4>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<4, 8>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<16, 4>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st) ||
        tiny_launch<4, 16>(blocks, g, Zout, Dout, tau, sh, jtol, max_sweeps, w, st);
    if (!ok) return hipErrorInvalidValue;   // the plan only picks shapes listed here
    if ((e = hipGetLastError()) != hipSuccess) return e;
    MSLD_EV(3); MSLD_EV(4);
    return hipSuccess;
  }
  if (tier == TIER_LRS) {
    // fused certified low-rank kernel; its failures get a retry with a twice wider
    // subspace (unless the first pass already used it), and what still fails goes to
    // the LDS Jacobi tier
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, w.lrCount, 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    MSLD_EV(2);
    if ((e = launch_lr_small(g, w, Zout, Dout, tau, sh, num_cus, w.lrs_wide ? 2 : 0,
                             w.live_count, w.live_list, w.lrCount, w.lrFall, st)) != hipSuccess)
      return e;
    MSLD_EV(3);
    if (w.lrs_wide) {
      // the failures of the wide pass are the fallback list
      hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, st, w.lrCount, w.lrCount + 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = launch_lr_small(g, w, Zout, Dout, tau, sh, num_cus, 1, w.lrCount, w.lrFall,
                                    w.lrCount + 1, w.lrFall + nblk, st)) != hipSuccess) {
      return e;
    }
    int G = 1;
    const int threads = lds_tier_threads(g.nb, g.mb, &G);
    const size_t ldsb = lds_tier_bytes(g.mb, g.nb);
    // failures are rare and counted on the device: a small grid walks the list
    int grid = 64;
    if (grid > nblk) grid = nblk;
    ScaleWork fw = w;
    fw.live_count = w.lrCount + 1;
    fw.live_list = w.lrs_wide ? w.lrFall : w.lrFall + nblk;
    switch (G) {
      case 1: e = launch_lds_g<1>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      case 2: e = launch_lds_g<2>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      case 4: e = launch_lds_g<4>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      case 8: e = launch_lds_g<8>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      case 16: e = launch_lds_g<16>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      default: e = launch_lds_g<32>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
    }
    if (e != hipSuccess) return e;
    MSLD_EV(4);
    return hipSuccess;
  }
  if (tier == TIER_LDS) {
    MSLD_EV(2);
    int G = 1;
    const int threads = lds_tier_threads(g.nb, g.mb, &G);
    const int bpw = lds_tier_pack(g.nb, g.mb);
    const size_t lds = lds_tier_bytes(g.mb, g.nb) * bpw;
    int per_cu = (int)(160 * 1024 / (lds + 1024));
    const int by_waves = 32 / ((threads + 63) / 64);
    if (per_cu > by_waves) per_cu = by_waves;
    if (per_cu < 1) per_cu = 1;
    if (w.lds_cap > 0 && per_cu > w.lds_cap) per_cu = w.lds_cap;   // autotuned
    int grid = num_cus * per_cu;
    const int units = (nblk + bpw - 1) / bpw;
    if (grid > units) grid = units;
    switch (G) {
      case 1: e = launch_lds_g<1>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st, bpw); break;
      case 2: e = launch_lds_g<2>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st, bpw); break;
      case 4: e = launch_lds_g<4>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st, bpw); break;
      case 8: e = launch_lds_g<8>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st, bpw); break;
      case 16: e = launch_lds_g<16>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st); break;
      default: e = launch_lds_g<32>(grid, threads, lds, Zout, Dout, g, sh, tau, jtol, max_sweeps, w, st); break;
    }
    if (e != hipSuccess) return e;
    MSLD_EV(3); MSLD_EV(4);
    return hipSuccess;
  }
  if (w.use_lr) {
    // certified low-rank path: every launch walks the live count on the device
    MSLD_EV(2);
    if ((e = run_lowrank(g, w, Zout, Dout, tau, sh, st, ev ? ev + 5 : nullptr)) != hipSuccess)
      return e;
    MSLD_EV(3);
    if (w.lds_fallback) {
      // blocks that failed the certificate and fit in LDS: one-sided Jacobi LDS tier
      // over the fallback list (its count on the device; empty in the common case)
      int G = 1;
      const int threads = lds_tier_threads(g.nb, g.mb, &G);
      const size_t ldsb = lds_tier_bytes(g.mb, g.nb);
      // failures are rare and their count is only known on the device: a small grid
      // that walks the list (a full-chip grid of LDS-hungry workgroups would wait for
      // the concurrent scales' kernels to drain before it could even retire empty)
      int grid = 32;
      if (grid > nblk) grid = nblk;
      ScaleWork fw = w;
      fw.live_count = w.lrCount;
      fw.live_list = w.lrFall;
      switch (G) {
        case 1: e = launch_lds_g<1>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
        case 2: e = launch_lds_g<2>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
        case 4: e = launch_lds_g<4>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
        case 8: e = launch_lds_g<8>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
        case 16: e = launch_lds_g<16>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
        default: e = launch_lds_g<32>(grid, threads, ldsb, Zout, Dout, g, sh, tau, jtol, max_sweeps, fw, st); break;
      }
      if (e != hipSuccess) return e;
      MSLD_EV(4);
      return hipSuccess;
    }
    // failed certificates of blocks beyond the LDS tier: exact polar-route SVT, whose
    // step counts are chosen on the host: the one read-back of this path. With
    // `deferred`, the count is only copied back here and finish_fallback (after the
    // caller has issued its other work) waits for it and runs the polar route.
    if ((e = hipMemcpyAsync(w.hostInts + 1, w.lrCount, sizeof(int), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return e;
    if (deferred) {
      *deferred = 1;
      return hipSuccess;
    }
    if ((e = finish_fallback(g, w, Zout, Dout, tau, sh, st)) != hipSuccess) return e;
    MSLD_EV(4);
    return hipSuccess;
  }
  // panel tier
  const int slots_y = w.slots < 65535 ? w.slots : 65535;
  {
    const int tiles = ((g.m + 31) / 32) * ((g.n + 31) / 32);
    hipLaunchKernelGGL(k_panel_load, dim3(tiles, slots_y), dim3(256), 0, st, Dout, g, sh,
                       w.live_count, w.live_list, w.pA, w.nbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // rotation accumulators and padding for the panel rounds
    hipLaunchKernelGGL(k_panel_init, dim3(64, slots_y), dim3(256), 0, st, g, w.live_count, w.pA,
                       w.pW, w.pflag, w.nbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  MSLD_EV(2);
  MSLD_EV(3);
  const int npan = w.nbp / w.pw;
  const int G = 256 / w.pw;
  const size_t lds = (size_t)4 * 2 * w.pw * ((g.mb | 1) + (g.nb | 1));
  for (int sweep = 0; sweep < panel_sweeps; ++sweep) {
    for (int rd = 0; rd < npan - 1; ++rd) {
      const dim3 grid(npan / 2, slots_y);
      switch (G) {
        case 1: e = launch_round_g<1>(grid, lds, g, w, rd, jtol, st); break;
        case 2: e = launch_round_g<2>(grid, lds, g, w, rd, jtol, st); break;
        case 4: e = launch_round_g<4>(grid, lds, g, w, rd, jtol, st); break;
        case 8: e = launch_round_g<8>(grid, lds, g, w, rd, jtol, st); break;
        case 16: e = launch_round_g<16>(grid, lds, g, w, rd, jtol, st); break;
        case 32: e = launch_round_g<32>(grid, lds, g, w, rd, jtol, st); break;
        default: e = launch_round_g<64>(grid, lds, g, w, rd, jtol, st); break;
      }
      if (e != hipSuccess) return e;
      if (round_launches) ++*round_launches;
    }
    hipLaunchKernelGGL(k_panel_sweep_end, dim3((w.slots + 255) / 256), dim3(256), 0, st,
                       w.live_count, w.pflag, w.stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_panel_gain, dim3(slots_y), dim3(256), 0, st, g, w.live_count, w.pA, w.pg,
                     w.nbp, tau, w.stats, w.pflag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    const int tiles = ((g.m + 31) / 32) * ((g.n + 31) / 32);
    hipLaunchKernelGGL(k_panel_rebuild, dim3(tiles, slots_y), dim3(256), 0, st, Zout, Dout, g,
                       sh, w.live_count, w.live_list, w.pA, w.pW, w.pg, w.nbp, w.pflag);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  MSLD_EV(4);
  return hipSuccess;
}

// ------------------------------------------------------------------ residual
// sum_i ||D_i + R - Z_i'||^2 (= sum_i ||X_i - Z_i'||^2) per instance, with
// per-workgroup partials reduced in a fixed order (independent of scheduling).
// Instance z owns rows [z IM, (z+1) IM) of every plane; grid = (parts, NI).
// Per-instance sums of the primal residual sum_i ||X_i - Z_i'||^2 (X_i = D_i + R in D
// form) and, into partial + NI * gridDim.x, of the dual residual sum_i ||Z_i' - Z_i||^2:
// with V_i = Z_i + R and D_i' = 2 Z_i' - V_i, the previous iterate is
// Z_i = 2 Z_i' - D_i' - R, so Z_i' - Z_i = D_i' + R - Z_i'.
__global__ void __launch_bounds__(256) k_resid(const float* __restrict__ Dold,
                                               const float* __restrict__ Dnew,
                                               const float* __restrict__ R,
                                               const float* __restrict__ Z, int64_t MN, int L,
                                               int64_t inst_elems, double* __restrict__ partial) {
  __shared__ double red[2][256];
  const int z = blockIdx.y;
  double acc = 0.0, accd = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)z * inst_elems;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < inst_elems;
       e0 += stride) {
    const int64_t e = base + e0;
    const float r = R[e];
    float s = 0.f, sd = 0.f;
    for (int i = 0; i < L; ++i) {
      const float zi = Z[i * MN + e];
      const float d = Dold[i * MN + e] + r - zi;
      const float dd = Dnew[i * MN + e] + r - zi;
      s += d * d;
      sd += dd * dd;
    }
    acc += (double)s;
    accd += (double)sd;
  }
  red[0][threadIdx.x] = acc;
  red[1][threadIdx.x] = accd;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[(int64_t)z * gridDim.x + blockIdx.x] = red[0][0];
    partial[((int64_t)gridDim.y + z) * gridDim.x + blockIdx.x] = red[1][0];
  }
}

__global__ void __launch_bounds__(256) k_sumsq(const float* __restrict__ Y, int64_t ldY, int IM,
                                               int N, const uint8_t* __restrict__ mask,
                                               int64_t ldmask, double* __restrict__ partial) {
  __shared__ double red[256];
  const int z = blockIdx.y;
  double acc = 0.0;
  const int64_t total = (int64_t)IM * N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / N;
    const int64_t c = e - r * N;
    const float y = Y[((int64_t)z * IM + r) * ldY + c];
    if (mask && !mask[((int64_t)z * IM + r) * ldmask + c]) continue;   // unobserved
    acc += (double)y * (double)y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)z * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_final_sum(const double* partial, int nparts, int NI, double* out) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= NI) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += partial[(int64_t)z * nparts + i];
  out[z] = s;
}

hipError_t launch_resid(const float* Dold, const float* Dnew, const float* R, const float* Z,
                        int M, int N, int L, int IM, int NI, double* partial, int nparts,
                        double* out, double* out_dual, hipStream_t st) {
  hipLaunchKernelGGL(k_resid, dim3(nparts, NI), dim3(256), 0, st, Dold, Dnew, R, Z,
                     (int64_t)M * N, L, (int64_t)IM * N, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final_sum, dim3((NI + 63) / 64), dim3(64), 0, st, partial, nparts, NI, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_final_sum, dim3((NI + 63) / 64), dim3(64), 0, st,
                     partial + (size_t)nparts * NI, nparts, NI, out_dual);
  return hipGetLastError();
}

hipError_t launch_sumsq(const float* Y, int64_t ldY, int IM, int N, int NI, const uint8_t* mask,
                        int64_t ldmask, double* partial, int nparts, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(nparts, NI), dim3(256), 0, st, Y, ldY, IM, N, mask, ldmask,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final_sum, dim3((NI + 63) / 64), dim3(64), 0, st, partial, nparts, NI, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- shift probe
struct Ladder16 {
  int m[16], n[16];
};

__global__ void k_device_shifts(uint64_t seed, int k0, int count, int L, Ladder16 lad,
                                int* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * L) return;
  const int kk = t / L;
  const int i = t - kk * L;
  ShiftSpec sh;
  sh.seed = seed;
  sh.k = k0 + kk;
  sh.scale = i;
  sh.mode = 1;
  sh.sr = sh.sc = 0;
  sh.iseed = nullptr;
  sh.ik = nullptr;
  sh.iactive = nullptr;
  int sr, sc;
  block_shift(sh, 0, lad.m[i], lad.n[i], &sr, &sc);
  out[2 * t] = sr;
  out[2 * t + 1] = sc;
}

hipError_t launch_device_shifts(uint64_t seed, int k0, int count, int L, const int* bm,
                                const int* bn, int* out, hipStream_t st) {
  Ladder16 lad;
  for (int i = 0; i < 16; ++i) {
    lad.m[i] = i < L ? bm[i] : 1;
    lad.n[i] = i < L ? bn[i] : 1;
  }
  const int total = count * L;
  hipLaunchKernelGGL(k_device_shifts, dim3((total + 255) / 256), dim3(256), 0, st, seed, k0,
                     count, L, lad, out);
  return hipGetLastError();
}

}  // namespace msld
