// FP32 matrix-core (MFMA) kernels of the certified low-rank BlockSVT (eq:svt on blocks
// of 32 columns and more): the Gram matrix B^T B of every live block, the skinny
// products of the subspace iteration and the certificate, the squarings of the
// remainder bound, the products of the polar fallback, and the rebuild
// Z = A_f diag(g) V_r^T with its scatter.
//
// The block B (logical mb x nb, mb >= nb) is never copied out of the iterate: every
// loader reads V = -D' (the stream pass left D' = -V at every live block) at the
// block's shifted, wrapped coordinates (R_b and Shift_s of eq:bsvt and Sec. 9), so
// the gather is fused into the products.
//
// Lane layouts of the two FP32 matrix instructions (wave of 64 lanes, lane l):
//   v_mfma_f32_32x32x2f32: A operand A(i = l % 32, k = l / 32), B operand
//     B(k = l / 32, j = l % 32); the 16 accumulators hold D(8 (r / 4) + 4 (l / 32)
//     + r % 4, l % 32), r < 16.
//   v_mfma_f32_16x16x4f32: A(i = l % 16, k = l / 16), B(k = l / 16, j = l % 16);
//     the 4 accumulators hold D(4 (l / 16) + r, l % 16), r < 4.
// Every launch covers a fixed grid sized for the most blocks a scale can have and
// walks the live slots up to a count read on the device, so no launch depends on a
// count read back to the host.
#include <cstdlib>

#include "msld_internal.h"

namespace msld {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Where block slot `slot` lives: block row p (instance z, block row pl inside it),
// block column q, shift (sr, sc).
struct BlockAt {
  int p, q, sr, sc, z, pl;
};
__device__ __forceinline__ BlockAt block_at(const ScaleGeom& g, const ShiftSpec& sh,
                                            const int* live_list, int slot) {
  BlockAt b;
  const int blk = live_list[slot];
  b.p = blk / g.Q;
  b.q = blk - b.p * g.Q;
  b.z = b.p / g.PI;
  b.pl = b.p - b.z * g.PI;
  block_shift(sh, b.z, g.m, g.n, &b.sr, &b.sc);
  return b;
}
// Offset of stored block row i (0 <= i < m) and of stored block column j (0 <= j < n):
// grow / gcol of the block, with its instance split off once.
__device__ __forceinline__ int64_t row_off(const ScaleGeom& g, const BlockAt& b, int i) {
  return ((int64_t)b.z * g.IM + local_row(g, b.pl, i, b.sr)) * g.N;
}
__device__ __forceinline__ int col_off(const ScaleGeom& g, const BlockAt& b, int j) {
  return gcol(g, b.q, j, b.sc);
}

__device__ __forceinline__ int dev_count(const int* dcount, int hcount) {
  return dcount ? *dcount : hcount;
}

// ------------------------------------------------------------------ Gram B^T B
// 64 x 64 tiles of G (column-major nb x nb per slot, slot stride sG); only tiles with
// ti <= tj are formed (blockIdx.x enumerates the upper triangle) and written to both
// (ti, tj) and (tj, ti). The rows of B (the contraction) are split into gridDim.z
// chunks of KC rows: with one chunk the tile goes to G, else chunk c writes its partial
// tile to part + (slot * chunks + c) * nb * nb and k_gram_sum adds the chunks in a
// fixed order. Four waves, each a 32 x 32 quarter of the tile.
constexpr int kGLd = 65;   // LDS row pitch of the staged slabs (conflict-free transposes)

// Workgroup w of the launch is dispatched to XCD w mod 8 (the chip hands workgroups
// to its eight XCDs in turn); every tile of one (slot, row chunk) unit is given ids of
// one residue, so the unit's rows are fetched into one XCD's L2 once and shared by all
// its tiles.
// TM x TM tiles, four waves each owning a quarter as (TM / 64)^2 blocks of 32 x 32
// accumulators (every operand value read from LDS feeds TM / 64 matrix instructions);
// slabs of KS rows, the next one loaded into registers while the matrix cores work on
// the current one.
// TR: the block is stored transposed (g.trans), a template argument so that each
// orientation's loader keeps only its own registers.
template <int TM, int KS, int TR>
__global__ void __launch_bounds__(256) k_mf_gram(const float* __restrict__ Dout, ScaleGeom g,
                                                 ShiftSpec sh, const int* __restrict__ live_count,
                                                 const int* __restrict__ live_list,
                                                 float* __restrict__ G, int64_t sG,
                                                 float* __restrict__ part, int KC, int chunks,
                                                 float* __restrict__ rowpart) {
  constexpr int LD = TM + 1;           // LDS pitch
  constexpr int QB = TM / 64;          // 32 x 32 blocks per wave and dimension
  constexpr int NL = KS * TM / 256;    // staged elements per thread and operand
  __shared__ float sm[2 * KS * LD];    // As[k][i], Bs[k][j]; output staging at the end
  static_assert(2 * KS * LD >= 64 * LD, "output staging");
  float* As = sm;
  float* Bs = sm + KS * LD;
  const int nb = g.nb, mb = g.mb;
  const int tn = (nb + TM - 1) / TM;
  const int tri = tn * (tn + 1) / 2;
  const int id = blockIdx.x;
  const int xcd = id & 7, kq = id >> 3;
  // unit = (slot, row chunk); every tile of a unit runs on one XCD, and consecutive
  // units on consecutive XCDs (a single wide block's chunks spread over the chip)
  const int unit = (kq / tri) * 8 + xcd;
  const int slot = unit / chunks, ch = unit - (unit / chunks) * chunks;
  const int count = *live_count;
  if (slot >= count) return;
  int t = kq % tri;
  int ti = 0;
  while (t >= tn - ti) {
    t -= tn - ti;
    ++ti;
  }
  const int tj = ti + t;
  const bool diag = ti == tj;
  const int i0 = ti * TM, j0 = tj * TM;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv & 1, wj = wv >> 1;   // wave quarter: rows wi TM/2.., cols wj TM/2..
  const int k0 = ch * KC, k1 = min(mb, k0 + KC);
  const BlockAt b = block_at(g, sh, live_list, slot);
  f32x16 acc[QB][QB];
#pragma unroll
  for (int x = 0; x < QB; ++x)
#pragma unroll
    for (int y = 0; y < QB; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
  float pa[NL], pb[NL];
  int sidx[NL];
  auto compute = [&](const float* Bv) {
#pragma unroll
    for (int kk = 0; kk < KS; kk += 2) {
      const int row = (kk + (lane >> 5)) * LD;
      float av[QB], bv[QB];
#pragma unroll
      for (int x = 0; x < QB; ++x) av[x] = As[row + wi * (TM / 2) + x * 32 + (lane & 31)];
#pragma unroll
      for (int y = 0; y < QB; ++y) bv[y] = Bv[row + wj * (TM / 2) + y * 32 + (lane & 31)];
#pragma unroll
      for (int x = 0; x < QB; ++x)
#pragma unroll
        for (int y = 0; y < QB; ++y) acc[x][y] = mfma32(av[x], bv[y], acc[x][y]);
    }
  };
  if constexpr (!TR) {
    // B(r, c) = stored (r, c): a slab row is contiguous along c; thread column
    // cc = tid % TM, rows tid / TM + (256 / TM) u
    constexpr int RS = 256 / TM;
    const int cc = tid % TM;
    const int ca = i0 + cc, cb = j0 + cc;
    const int oa = ca < nb ? col_off(g, b, ca) : -1;
    const int ob = (!diag && cb < nb) ? col_off(g, b, cb) : -1;
#pragma unroll
    for (int u = 0; u < NL; ++u) sidx[u] = (tid / TM + RS * u) * LD + cc;
    auto load = [&](int kb) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int r = kb + tid / TM + RS * u;
        pa[u] = pb[u] = 0.f;
        if (r < k1) {
          const int64_t ro = row_off(g, b, r);
          if (oa >= 0) pa[u] = -Dout[ro + oa];
          if (ob >= 0) pb[u] = -Dout[ro + ob];
        }
      }
    };
    load(k0);
    for (int kb = k0; kb < k1; kb += KS) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        As[sidx[u]] = pa[u];
        if (!diag) Bs[sidx[u]] = pb[u];
      }
      __syncthreads();
      if (kb + KS < k1) load(kb + KS);
      compute(diag ? As : Bs);
      __syncthreads();
    }
  } else {
    // B(r, c) = stored (c, r): stored rows are the tile's columns, contiguous along r;
    // thread row kk = tid % KS, columns tid / KS + (256 / KS) u
    constexpr int CS = 256 / KS;
    const int kk = tid % KS;
    int64_t ra[NL], rb[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int c = tid / KS + CS * u;
      ra[u] = i0 + c < nb ? row_off(g, b, i0 + c) : -1;
      rb[u] = (!diag && j0 + c < nb) ? row_off(g, b, j0 + c) : -1;
      sidx[u] = kk * LD + c;
    }
    auto load = [&](int kb) {
      const int r = kb + kk;
      const int co = r < k1 ? col_off(g, b, r) : 0;
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        pa[u] = (r < k1 && ra[u] >= 0) ? -Dout[ra[u] + co] : 0.f;
        pb[u] = (r < k1 && rb[u] >= 0) ? -Dout[rb[u] + co] : 0.f;
      }
    };
    load(k0);
    for (int kb = k0; kb < k1; kb += KS) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        As[sidx[u]] = pa[u];
        if (!diag) Bs[sidx[u]] = pb[u];
      }
      __syncthreads();
      if (kb + KS < k1) load(kb + KS);
      compute(diag ? As : Bs);
      __syncthreads();
    }
  }
  // write the tile (and its mirror) through LDS, 64 rows at a time: T[ii][jj] for rows
  // h 64 .. h 64 + 63 of the tile (held by the waves whose quarter contains them)
  float* dst = chunks == 1 ? G + (int64_t)slot * sG
                           : part + ((int64_t)slot * chunks + ch) * (int64_t)nb * nb;
  float* T = sm;   // 64 x LD floats
  for (int h = 0; h < TM / 64; ++h) {
#pragma unroll
    for (int x = 0; x < QB; ++x) {
      // rows of block x of this wave: wi TM/2 + x 32 .. + 31; they lie in half h when
      // (wi TM/2 + x 32) / 64 == h
      if ((wi * (TM / 2) + x * 32) / 64 != h) continue;
#pragma unroll
      for (int y = 0; y < QB; ++y)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int ii = (wi * (TM / 2) + x * 32) % 64 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int jj = wj * (TM / 2) + y * 32 + (lane & 31);
          T[ii * LD + jj] = acc[x][y][r];
        }
    }
    __syncthreads();
    const int ib = i0 + h * 64;
    if (rowpart && TM == 64) {
      // |G| row sums of this tile (slice tj, rows ib..) and, for an off-diagonal tile, of
      // its mirror (column sums: slice ti, rows j0..), for the Gram bound of the low-rank
      // path; fixed summation order
      const int tn = (nb + 63) / 64;
      float* rp = rowpart + (int64_t)slot * nb * (tn + 1);
      if (tid < 64 && ib + tid < nb) {
        float a = 0.f;
        for (int jj = 0; jj < 64; ++jj) a += fabsf(T[tid * LD + jj]);
        rp[(int64_t)tj * nb + ib + tid] = a;
      } else if (!diag && tid >= 64 && tid < 128 && j0 + tid - 64 < nb) {
        const int cc = tid - 64;
        float a = 0.f;
        for (int ii = 0; ii < 64; ++ii) a += fabsf(T[ii * LD + cc]);
        rp[(int64_t)ti * nb + j0 + cc] = a;
      }
    }
    for (int e = tid; e < 64 * TM; e += 256) {
      const int jj = e >> 6, ii = e & 63;   // element (ib + ii, j0 + jj)
      if (ib + ii < nb && j0 + jj < nb) dst[(int64_t)(j0 + jj) * nb + ib + ii] = T[ii * LD + jj];
    }
    if (!diag) {
      // mirror: element (j0 + jj, ib + ii) = T[ii][jj], coalesced along jj
      for (int e = tid; e < 64 * TM; e += 256) {
        const int ii = e / TM, jj = e % TM;
        if (ib + ii < nb && j0 + jj < nb) dst[(int64_t)(ib + ii) * nb + j0 + jj] = T[ii * LD + jj];
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_gram_sum(const float* __restrict__ part, int chunks,
                                                  int nb, const int* __restrict__ live_count,
                                                  float* __restrict__ G, int64_t sG) {
  const int count = *live_count;
  const int64_t nn = (int64_t)nb * nb;
  for (int slot = blockIdx.y; slot < count; slot += gridDim.y)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
      const float* p = part + (int64_t)slot * chunks * nn + e;
      float s = 0.f;
      for (int c = 0; c < chunks; ++c) s += p[(int64_t)c * nn];
      G[(int64_t)slot * sG + e] = s;
    }
}

// ------------------------------------------------------ skinny products C = A X
// C (M x 16) = A (M x K) X (K x 16) per slot, X column-major (X[l K + k], slot stride
// sX; 0 shares one X), C column-major (C[l M + i]) or row-major (C[i 16 + l]).
// A is one of
//   SK_DENSE: a column-major matrix (A[k lda + i], slot stride sA);
//   SK_B:     the block B (M = mb, K = nb), gathered from V = -D';
//   SK_BT:    its transpose B^T (M = nb, K = mb).
// 64 rows per workgroup, 16 rows per wave on v_mfma_f32_16x16x4f32, slabs of 64 along
// K staged in LDS. gridDim.z > 1 splits K into chunks of KC: chunk c writes its partial
// product (row-major, M x 16) to part + (slot * chunks + c) * M * 16, summed by k_sk_sum.
// Slot c of the walk is slot_list[c] when a list is given (slots of the undecided
// list), else c.
template <int MODE, int ROWMAJ, int TR>
__global__ void __launch_bounds__(256) k_sk(const float* __restrict__ A, int64_t sA, int lda,
                                            const float* __restrict__ Dout, ScaleGeom g,
                                            ShiftSpec sh, const int* __restrict__ live_list,
                                            const float* __restrict__ X, int64_t sX, int M,
                                            int K, float* __restrict__ C, int64_t sC,
                                            const int* __restrict__ dcount, int hcount,
                                            const int* __restrict__ slot_list,
                                            float* __restrict__ part, int KC) {
  __shared__ float As[64 * kGLd];   // As[k][i]
  __shared__ float Xs[64 * 17];     // Xs[k][l]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = blockIdx.x * 64;
  const int chunks = gridDim.z, ch = blockIdx.z;
  const int k0 = ch * KC, k1 = min(K, k0 + KC);
  const int count = dev_count(dcount, hcount);
  // which index of the A tile runs along memory: "k-major" loads map lanes to k
  // (TR = g.trans, a template argument so that each orientation keeps its own registers)
  constexpr bool kmajor = MODE == SK_B ? !TR : MODE == SK_BT ? (TR != 0) : false;
  for (int cidx = blockIdx.y; cidx < count; cidx += gridDim.y) {
    const int slot = slot_list ? slot_list[cidx] : cidx;
    BlockAt b;
    if (MODE != SK_DENSE) b = block_at(g, sh, live_list, slot);
    const float* a = A + (int64_t)slot * sA;
    const float* x = X + (int64_t)slot * sX;
    // stored-row offsets that stay fixed over the K loop (k-major gathers: the tile's
    // rows i0 + (tid >> 6) + 4u are stored rows), and the fixed stored column of the
    // i-major gathers (the tile's row i0 + (tid & 63))
    int64_t ro[16];
    int cfix = 0;
    if (MODE != SK_DENSE) {
      if constexpr (kmajor) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + (tid >> 6) + 4 * u;
          ro[u] = i < M ? row_off(g, b, i) : -1;
        }
      } else {
        const int i = i0 + (tid & 63);
        cfix = i < M ? col_off(g, b, i) : -1;
      }
    }
    f32x4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = 0.f;
    for (int kb = k0; kb < k1; kb += 64) {
      if constexpr (MODE == SK_DENSE || !kmajor) {
        // lanes along i: column-major dense A, or gathers whose stored rows are k
        const int ii = tid & 63;
        const int i = i0 + ii;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int kk = (tid >> 6) + 4 * u;
          const int k = kb + kk;
          float v = 0.f;
          if (i < M && k < k1) {
            if (MODE == SK_DENSE) v = a[(int64_t)k * lda + i];
            else v = -Dout[row_off(g, b, k) + cfix];
          }
          As[kk * kGLd + ii] = v;
        }
      } else {
        // lanes along k: gathers whose stored rows are the tile's rows i
        const int kk = tid & 63;
        const int k = kb + kk;
        const int co = k < k1 ? col_off(g, b, k) : 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int ii = (tid >> 6) + 4 * u;
          As[kk * kGLd + ii] = (k < k1 && ro[u] >= 0) ? -Dout[ro[u] + co] : 0.f;
        }
      }
      for (int e = tid; e < 64 * 16; e += 256) {
        const int l = e >> 6, kk = e & 63;
        const int k = kb + kk;
        Xs[kk * 17 + l] = k < k1 ? x[(int64_t)l * K + k] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 64; kk += 4) {
        const float av = As[(kk + (lane >> 4)) * kGLd + wv * 16 + (lane & 15)];
        const float xv = Xs[(kk + (lane >> 4)) * 17 + (lane & 15)];
        acc = mfma16(av, xv, acc);
      }
      __syncthreads();
    }
    const int l = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wv * 16 + 4 * (lane >> 4) + r;
      if (i >= M) continue;
      if (chunks > 1)
        part[((int64_t)slot * chunks + ch) * (int64_t)M * 16 + (int64_t)i * 16 + l] = acc[r];
      else if (ROWMAJ)
        C[(int64_t)slot * sC + (int64_t)i * 16 + l] = acc[r];
      else
        C[(int64_t)slot * sC + (int64_t)l * M + i] = acc[r];
    }
  }
}

// Y (M x 16, column-major) = A X for a symmetric A (column-major, so A[i lda + k] is
// A(i, k) along contiguous k) and X (M x 16, column-major): the products of the subspace
// iteration by the Gram matrix. No LDS and no barrier: each wave owns 16 rows and reads
// its operands straight into registers, four contraction indices per lane and load.
// Within each group of 16 contraction indices, lane l (row l % 16, q = l / 16) holds
// A(i, k0 + 4 q + j) and X(k0 + 4 q + j, l % 16) for j < 4 as one 16-byte load each,
// and matrix instruction j contracts over {k0 + 4 q + j : q < 4}; the four
// instructions together cover the 16 indices once (a permutation of the sum).
// Requires M % 16 == 0 and 16-byte aligned rows (lda % 4 == 0). With gridDim.z > 1 the
// contraction is split into chunks of KC (a multiple of 16) and chunk z writes its
// partial product to part + (slot * chunks + z) * M * 16 (row-major), summed by
// k_sk_sum.
__global__ void __launch_bounds__(256) k_sym_x(const float* __restrict__ A, int64_t sA, int lda,
                                               const float* __restrict__ X, int64_t sX, int M,
                                               float* __restrict__ Y, int64_t sY,
                                               const int* __restrict__ dcount,
                                               const int* __restrict__ slot_list,
                                               float* __restrict__ part, int KC) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int count = *dcount;
  const int rows_per = gridDim.x * 64;
  const int chunks = gridDim.z, ch = blockIdx.z;
  const int kb = ch * KC, ke = min(M, kb + KC);
  for (int cidx = blockIdx.y; cidx < count; cidx += gridDim.y) {
    const int slot = slot_list ? slot_list[cidx] : cidx;
    for (int i0 = blockIdx.x * 64 + wv * 16; i0 < M; i0 += rows_per) {
      const float* arow = A + (int64_t)slot * sA + (int64_t)(i0 + c) * lda + 4 * q;
      const float* xcol = X + (int64_t)slot * sX + (int64_t)c * M + 4 * q;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int k0 = kb; k0 < ke; k0 += 16) {
        const float4 av = *reinterpret_cast<const float4*>(arow + k0);
        const float4 xv = *reinterpret_cast<const float4*>(xcol + k0);
        acc = mfma16(av.x, xv.x, acc);
        acc = mfma16(av.y, xv.y, acc);
        acc = mfma16(av.z, xv.z, acc);
        acc = mfma16(av.w, xv.w, acc);
      }
      if (chunks > 1) {
        float* pp = part + ((int64_t)slot * chunks + ch) * M * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) pp[(int64_t)(i0 + 4 * q + r) * 16 + c] = acc[r];
      } else {
        float* y = Y + (int64_t)slot * sY + (int64_t)c * M + i0 + 4 * q;
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = acc[r];
      }
    }
  }
}

// The same products with A the gathered block B (SK_B: A(i, k) = B(i, k)) or its
// transpose (SK_BT: A(i, k) = B(k, i)), barrier-free in the lane layout of k_sym_x:
// lane l provides A(i0 + l % 16, k0 + 4 (l / 16) + j) as four single loads and
// X(k0 + 4 (l / 16) + j, l % 16) as one 16-byte load. When a fixed A row runs along a
// stored row (KROW) a lane walks one stored row and its column offsets; otherwise the
// 16 lanes of a group read 16 consecutive stored columns of one stored row (64 bytes).
// gridDim.z > 1 splits K into chunks of KC (partial products, row-major, to `part`).
// Requires K % 16 == 0.
template <int MODE, int ROWMAJ>
__global__ void __launch_bounds__(256) k_skg(const float* __restrict__ Dout, ScaleGeom g,
                                             ShiftSpec sh, const int* __restrict__ live_list,
                                             const float* __restrict__ X, int64_t sX, int M,
                                             int K, float* __restrict__ C, int64_t sC,
                                             const int* __restrict__ dcount,
                                             float* __restrict__ part, int KC) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int chunks = gridDim.z, ch = blockIdx.z;
  const int kb0 = ch * KC, kb1 = min(K, kb0 + KC);
  const bool krow = (MODE == SK_B) != (g.trans != 0);
  const int count = *dcount;
  const int rows_per = gridDim.x * 64;
  for (int slot = blockIdx.y; slot < count; slot += gridDim.y) {
    const BlockAt b = block_at(g, sh, live_list, slot);
    const int cbase = b.q * g.n + b.sc;   // stored column 0 before the wrap
    for (int i0 = blockIdx.x * 64 + wv * 16; i0 < M; i0 += rows_per) {
      const int i = i0 + c;
      const bool iv = i < M;
      // the lane's fixed stored row (krow) or stored column (otherwise)
      int64_t ro = 0;
      int co = 0;
      if (iv) {
        if (krow) ro = row_off(g, b, i);
        else {
          co = cbase + i;
          if (co >= g.N) co -= g.N;
        }
      }
      const float* xcol = X + (int64_t)slot * sX + (int64_t)c * K + 4 * q;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int k0 = kb0; k0 < kb1; k0 += 16) {
        const float4 xv = *reinterpret_cast<const float4*>(xcol + k0);
        float av[4];
        const int kq = k0 + 4 * q;
        if (krow) {
          int col = cbase + kq;
          if (col >= g.N) col -= g.N;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            int cj = col + j;
            if (cj >= g.N) cj -= g.N;
            av[j] = iv ? -Dout[ro + cj] : 0.f;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) av[j] = iv ? -Dout[row_off(g, b, kq + j) + co] : 0.f;
        }
        acc = mfma16(av[0], xv.x, acc);
        acc = mfma16(av[1], xv.y, acc);
        acc = mfma16(av[2], xv.z, acc);
        acc = mfma16(av[3], xv.w, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * q + r;
        if (row >= M) continue;
        if (chunks > 1)
          part[((int64_t)slot * chunks + ch) * (int64_t)M * 16 + (int64_t)row * 16 + c] = acc[r];
        else if (ROWMAJ)
          C[(int64_t)slot * sC + (int64_t)row * 16 + c] = acc[r];
        else
          C[(int64_t)slot * sC + (int64_t)c * M + row] = acc[r];
      }
    }
  }
}

template <int ROWMAJ>
__global__ void __launch_bounds__(256) k_sk_sum(const float* __restrict__ part, int chunks, int M,
                                                float* __restrict__ C, int64_t sC,
                                                const int* __restrict__ dcount, int hcount,
                                                const int* __restrict__ slot_list) {
  const int count = dev_count(dcount, hcount);
  const int64_t n = (int64_t)M * 16;
  for (int cidx = blockIdx.y; cidx < count; cidx += gridDim.y) {
    const int slot = slot_list ? slot_list[cidx] : cidx;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
      const float* p = part + (int64_t)slot * chunks * n + e;
      float s = 0.f;
      for (int c = 0; c < chunks; ++c) s += p[(int64_t)c * n];
      const int i = (int)(e >> 4), l = (int)(e & 15);
      if (ROWMAJ) C[(int64_t)slot * sC + e] = s;
      else C[(int64_t)slot * sC + (int64_t)l * M + i] = s;
    }
  }
}

// ------------------------------------------------------------ general GEMM
// C (M x N) = op(A) B, column-major, one problem per batch entry c < count (pointer
// strides sa, sb, sc); op(A) = A (TA = 0, A[k lda + i]) or A^T (TA = 1, A[i lda + k]).
// 64 x 64 tiles, slabs of 32 along K, four waves on v_mfma_f32_32x32x2f32.
// SYM (with TA = 1, M = N, for products A^T B known to be symmetric: A^T A, or A^T B with
// A and B symmetric and commuting): only the tiles with i0 <= j0 are formed (blockIdx.x
// enumerates the upper triangle), each also written mirrored and the diagonal tiles from
// their upper triangle, so C is exactly symmetric. With gridDim.z > 1 the contraction is
// split into chunks of KC and chunk z writes its partial product to part + (c chunks + z)
// M N (column-major, ld M), summed by k_gemm_sum.
template <int TA, int SYM = 0>
__global__ void __launch_bounds__(256) k_gemm(const float* __restrict__ A, int lda, int64_t sa,
                                              const float* __restrict__ B, int ldb, int64_t sb,
                                              float* __restrict__ C, int ldc, int64_t sc, int M,
                                              int N, int K, const int* __restrict__ dcount,
                                              int hcount, float* __restrict__ part, int KC) {
  __shared__ float sm[64 * kGLd];   // As[k][i] then Bs[k][j]; the output tile at the end
  float* As = sm;
  float* Bs = sm + 32 * kGLd;
  const int tiles_m = (M + 63) / 64;
  int ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
  if (SYM) {
    int t = blockIdx.x;
    ti = 0;
    while (t >= tiles_m - ti) {
      t -= tiles_m - ti;
      ++ti;
    }
    tj = ti + t;
  }
  const int i0 = ti * 64, j0 = tj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv & 1, wj = wv >> 1;
  const int count = dev_count(dcount, hcount);
  const int chunks = gridDim.z, ch = blockIdx.z;
  const int k0 = ch * KC, k1 = min(K, k0 + KC);
  for (int c = blockIdx.y; c < count; c += gridDim.y) {
    const float* a = A + (int64_t)c * sa;
    const float* b = B + (int64_t)c * sb;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // 32-deep slabs of A and B staged through LDS; the next slab's global loads are
    // issued into registers before the current slab's products, so they are in flight
    // while the matrix cores run
    float ra[8], rb[8];
    auto load = [&](int kb) {
      if (!TA) {
        const int ii = tid & 63;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int kk = (tid >> 6) + 4 * u;
          const int i = i0 + ii, k = kb + kk;
          ra[u] = (i < M && k < k1) ? a[(int64_t)k * lda + i] : 0.f;
        }
      } else {
        const int kk = tid & 31;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int ii = (tid >> 5) + 8 * u;
          const int i = i0 + ii, k = kb + kk;
          ra[u] = (i < M && k < k1) ? a[(int64_t)i * lda + k] : 0.f;
        }
      }
      const int kk = tid & 31;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jj = (tid >> 5) + 8 * u;
        const int j = j0 + jj, k = kb + kk;
        rb[u] = (j < N && k < k1) ? b[(int64_t)j * ldb + k] : 0.f;
      }
    };
    if (k0 < k1) load(k0);
    for (int kb = k0; kb < k1; kb += 32) {
      if (!TA) {
#pragma unroll
        for (int u = 0; u < 8; ++u) As[((tid >> 6) + 4 * u) * kGLd + (tid & 63)] = ra[u];
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) As[(tid & 31) * kGLd + (tid >> 5) + 8 * u] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[(tid & 31) * kGLd + (tid >> 5) + 8 * u] = rb[u];
      __syncthreads();
      if (kb + 32 < k1) load(kb + 32);
#pragma unroll
      for (int kk = 0; kk < 32; kk += 2) {
        const float av = As[(kk + (lane >> 5)) * kGLd + wi * 32 + (lane & 31)];
        const float bv = Bs[(kk + (lane >> 5)) * kGLd + wj * 32 + (lane & 31)];
        acc = mfma32(av, bv, acc);
      }
      __syncthreads();
    }
    float* T = sm;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ii = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int jj = wj * 32 + (lane & 31);
      T[ii * kGLd + jj] = acc[r];
    }
    __syncthreads();
    float* cc = chunks > 1 ? part + ((int64_t)c * chunks + ch) * M * N : C + (int64_t)c * sc;
    const int ldo = chunks > 1 ? M : ldc;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int jj = e >> 6, ii = e & 63;
      // (a diagonal tile of a symmetric product takes its upper triangle on both sides)
      const float v = (SYM && i0 == j0 && ii > jj) ? T[jj * kGLd + ii] : T[ii * kGLd + jj];
      if (i0 + ii < M && j0 + jj < N) cc[(int64_t)(j0 + jj) * ldo + i0 + ii] = v;
    }
    if (SYM && i0 != j0)
      for (int e = tid; e < 64 * 64; e += 256) {
        const int ii = e >> 6, jj = e & 63;   // element (j0 + jj, i0 + ii), along jj
        if (i0 + ii < M && j0 + jj < N) cc[(int64_t)(i0 + ii) * ldo + j0 + jj] = T[ii * kGLd + jj];
      }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ rebuild
// Z = sum_{l in L, sigma_l > tau} (1 - tau / sigma_l) a_l v_l^T (A_f: mb x P column-major
// per slot, V_r: nb x P) for the slots whose certificate passed (pflag[4 slot + 2]),
// scattered to the block's shifted coordinates with the dual update D' = 2 Z' - V
// (V = -D' as left by the stream pass). 64 x 64 stored-block tiles, four waves on
// v_mfma_f32_32x32x2f32 with K = P: D(i, j) = sum_l U(i, l) W(j, l) with U(i, l) the
// factor of stored row i and W(j, l) that of stored column j; an accumulator's lanes
// run along stored columns, so each write is a contiguous row segment.
template <int P, int TR>
__global__ void __launch_bounds__(256) k_mf_rebuild(float* __restrict__ Zout,
                                                    float* __restrict__ Dout, ScaleGeom g,
                                                    ShiftSpec sh, const int* __restrict__ count_p,
                                                    const int* __restrict__ slot_list,
                                                    const int* __restrict__ live_list,
                                                    const int* __restrict__ pflag,
                                                    const float* __restrict__ Af,
                                                    const float* __restrict__ Vr,
                                                    const float* __restrict__ sig,
                                                    const float* __restrict__ mask, float tau) {
  __shared__ float gl[P];
  __shared__ int s_any;
  const int m = g.m, n = g.n, mb = g.mb, nb = g.nb;
  const int tiles_j = (n + 63) / 64;
  const int i0 = (blockIdx.x / tiles_j) * 64, j0 = (blockIdx.x % tiles_j) * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv & 1, wj = wv >> 1;   // wave's 32 x 32 quarter: stored rows wi, cols wj
  const int count = *count_p;
  for (int cidx = blockIdx.y; cidx < count; cidx += gridDim.y) {
    const int slot = slot_list ? slot_list[cidx] : cidx;
    if (!pflag[4 * slot + 2]) continue;   // uniform: failed certificates go elsewhere
    __syncthreads();
    if (tid == 0) s_any = 0;
    __syncthreads();
    if (tid < P) {
      const float s = sig[slot * P + tid];
      const bool on = (mask == nullptr || mask[slot * P + tid] > 0.f) && s > tau;
      gl[tid] = on ? 1.f - tau / s : 0.f;
      if (on) s_any = 1;
    }
    __syncthreads();
    if (!s_any) continue;   // Z = 0: the stream pass already wrote Z' = 0, D' = -V
    const BlockAt b = block_at(g, sh, live_list, slot);
    const float* af = Af + (int64_t)slot * mb * P;
    const float* vr = Vr + (int64_t)slot * nb * P;
    // factors by orientation: B = block (U = a_l g_l, W = v_l) or B = block^T (U = v_l,
    // W = a_l g_l)
    const int i = i0 + wi * 32 + (lane & 31);   // stored row of this lane's A operand
    const int j = j0 + wj * 32 + (lane & 31);   // stored column of this lane's B operand
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int kk = 0; kk < P; kk += 2) {
      const int l = kk + (lane >> 5);
      float urow = 0.f, wcol = 0.f;
      if (i < m) urow = TR ? vr[(int64_t)l * nb + i] : af[(int64_t)l * mb + i] * gl[l];
      if (j < n) wcol = TR ? af[(int64_t)l * mb + j] * gl[l] : vr[(int64_t)l * nb + j];
      acc = mfma32(urow, wcol, acc);
    }
    // accumulator r: stored row i0 + wi 32 + 8 (r / 4) + 4 (lane / 32) + r % 4, stored
    // column j0 + wj 32 + lane % 32
    const int jc = j0 + wj * 32 + (lane & 31);
    if (jc < n) {
      const int co = col_off(g, b, jc);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ir = i0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (ir >= m) continue;
        const int64_t o = row_off(g, b, ir) + co;
        const float z = acc[r];
        const float v = -Dout[o];
        Zout[o] = z;
        Dout[o] = 2.f * z - v;
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
static int grid_slots(int slots, int per_slot) {
  // enough workgroups to fill the chip several times over, never more than slots
  int y = (8192 + per_slot - 1) / per_slot;
  if (y < 1) y = 1;
  if (y > slots) y = slots;
  if (y > 65535) y = 65535;
  return y;
}

int split_chunks(int mb, int nb) {
  // tall blocks split their rows (the contraction of B^T B and B^T A_f) into chunks of
  // about 512 rows, and blocks 768 wide or more into chunks of 256 rows, so that few
  // blocks still fill the chip; a function of the block shape alone, so that a block's
  // result does not depend on how many others run
  int c = 1;
  if (nb >= 768)
    c = (mb + 255) / 256;
  else if (mb >= 4 * nb)
    c = (mb + 511) / 512;
  return c > 64 ? 64 : c;
}

int gram_tile() {
  // Gram tile variant: 0 = 64 x 64 with 32-row slabs, 1 = 64 x 64 with 64-row slabs,
  // 2 = 128 x 128 with 32-row slabs (MSLD_GRAM_TILE overrides the default)
  static int v = [] {
    const char* e = std::getenv("MSLD_GRAM_TILE");
    const int x = e ? std::atoi(e) : 0;
    return (x >= 0 && x <= 2) ? x : 0;
  }();
  return v;
}

hipError_t launch_mf_gram(const ScaleGeom& g, const ShiftSpec& sh, const float* Dout,
                          const int* live_count, const int* live_list, int slots, float* G,
                          float* part, float* rowpart, bool* rows_done, hipStream_t st) {
  const int nb = g.nb, mb = g.mb;
  const int var = gram_tile();
  const int TM = var == 2 ? 128 : 64, KS = var == 1 ? 64 : 32;
  const int tn = (nb + TM - 1) / TM;
  const int tri = tn * (tn + 1) / 2;
  int chunks = part ? split_chunks(mb, nb) : 1;
  int KC = (mb + chunks - 1) / chunks;
  KC = (KC + KS - 1) / KS * KS;
  chunks = (mb + KC - 1) / KC;
  // one workgroup per (slot, chunk, tile), ids grouped so that a (slot, chunk) unit
  // stays on one XCD
  const int64_t groups = ((int64_t)slots * chunks + 7) / 8;
  const int64_t nwg = groups * 8 * tri;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t sG = (int64_t)nb * nb;
  // the |G| row sums come with the tiles when the tiles are final (no split) and 64 wide
  float* rp = (chunks == 1 && TM == 64) ? rowpart : nullptr;
  if (rows_done) *rows_done = rp != nullptr;
#define MSLD_GRAM(tm, ks, rpp)                                                                \
  do {                                                                                        \
    if (g.trans)                                                                              \
      hipLaunchKernelGGL((k_mf_gram<tm, ks, 1>), dim3((unsigned)nwg), dim3(256), 0, st, Dout, \
                         g, sh, live_count, live_list, G, sG, part, KC, chunks, rpp);         \
    else                                                                                      \
      hipLaunchKernelGGL((k_mf_gram<tm, ks, 0>), dim3((unsigned)nwg), dim3(256), 0, st, Dout, \
                         g, sh, live_count, live_list, G, sG, part, KC, chunks, rpp);         \
  } while (0)
  if (var == 0)
    MSLD_GRAM(64, 32, rp);
  else if (var == 1)
    MSLD_GRAM(64, 64, rp);
  else
    MSLD_GRAM(128, 32, nullptr);
#undef MSLD_GRAM
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  const int gx = (int)std::min<int64_t>((sG + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gram_sum, dim3(gx, grid_slots(slots, gx)), dim3(256), 0, st, part, chunks,
                     nb, live_count, G, sG);
  return hipGetLastError();
}

hipError_t launch_sk(int mode, bool rowmaj, const float* A, int64_t sA, int lda,
                     const float* Dout, const ScaleGeom& g, const ShiftSpec& sh,
                     const int* live_list, const float* X, int64_t sX, int M, int K, float* C,
                     int64_t sC, const int* dcount, int hcount, int slots, const int* slot_list,
                     float* part, int split, hipStream_t st) {
  const int tm = (M + 63) / 64;
  // split the contraction into `split` chunks (partial sums indexed by slot)
  int chunks = (part && split > 1) ? split : 1;
  int KC = (K + chunks - 1) / chunks;
  KC = (KC + 63) / 64 * 64;
  chunks = (K + KC - 1) / KC;
  const dim3 grid(tm, grid_slots(slots, tm * chunks), chunks);
  // the barrier-free gathered kernel where its lanes read contiguous stored columns
  // (A = B^T of a row-major stored block, or A = B of a transposed one); a lane walking
  // one stored row touches 16 rows per load, slower than the LDS-staged kernel
  const bool colwise = (mode == SK_BT) != (g.trans != 0);
  if (mode != SK_DENSE && colwise && K % 16 == 0 && !slot_list && dcount) {
    const int kc16 = (KC + 15) / 16 * 16;
    const int ch16 = (K + kc16 - 1) / kc16;
    const dim3 gg(tm, grid_slots(slots, tm * ch16), ch16);
    if (mode == SK_B) {
      if (rowmaj) hipLaunchKernelGGL((k_skg<SK_B, 1>), gg, dim3(256), 0, st, Dout, g, sh, live_list, X, sX, M, K, C, sC, dcount, part, kc16);
      else hipLaunchKernelGGL((k_skg<SK_B, 0>), gg, dim3(256), 0, st, Dout, g, sh, live_list, X, sX, M, K, C, sC, dcount, part, kc16);
    } else {
      if (rowmaj) hipLaunchKernelGGL((k_skg<SK_BT, 1>), gg, dim3(256), 0, st, Dout, g, sh, live_list, X, sX, M, K, C, sC, dcount, part, kc16);
      else hipLaunchKernelGGL((k_skg<SK_BT, 0>), gg, dim3(256), 0, st, Dout, g, sh, live_list, X, sX, M, K, C, sC, dcount, part, kc16);
    }
    chunks = ch16;
  } else {
#define MSLD_SK(md, rm)                                                                         \
  do {                                                                                          \
    if (md != SK_DENSE && g.trans)                                                              \
      hipLaunchKernelGGL((k_sk<md, rm, 1>), grid, dim3(256), 0, st, A, sA, lda, Dout, g, sh,     \
                         live_list, X, sX, M, K, C, sC, dcount, hcount, slot_list, part, KC);   \
    else                                                                                        \
      hipLaunchKernelGGL((k_sk<md, rm, 0>), grid, dim3(256), 0, st, A, sA, lda, Dout, g, sh,     \
                         live_list, X, sX, M, K, C, sC, dcount, hcount, slot_list, part, KC);   \
  } while (0)
  if (mode == SK_DENSE) {
    if (rowmaj) MSLD_SK(SK_DENSE, 1); else MSLD_SK(SK_DENSE, 0);
  } else if (mode == SK_B) {
    if (rowmaj) MSLD_SK(SK_B, 1); else MSLD_SK(SK_B, 0);
  } else {
    if (rowmaj) MSLD_SK(SK_BT, 1); else MSLD_SK(SK_BT, 0);
  }
#undef MSLD_SK
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  const int64_t n = (int64_t)M * 16;
  const int gx = (int)std::min<int64_t>((n + 255) / 256, 64);
  if (rowmaj)
    hipLaunchKernelGGL(k_sk_sum<1>, dim3(gx, grid_slots(slots, gx)), dim3(256), 0, st, part,
                       chunks, M, C, sC, dcount, hcount, slot_list);
  else
    hipLaunchKernelGGL(k_sk_sum<0>, dim3(gx, grid_slots(slots, gx)), dim3(256), 0, st, part,
                       chunks, M, C, sC, dcount, hcount, slot_list);
  return hipGetLastError();
}

hipError_t launch_sym_x(const float* A, int64_t sA, int lda, const float* X, int64_t sX, int M,
                        float* Y, int64_t sY, const int* dcount, int slots, const int* slot_list,
                        float* part, hipStream_t st) {
  const int gx = (M + 63) / 64;
  // matrices 1024 wide or more split the contraction into 256-column chunks (a function
  // of M alone, so a product's rounding does not depend on the slot count)
  const int chunks = (part && M >= 1024) ? (M + 255) / 256 : 1;
  const int KC = chunks > 1 ? 256 : M;
  hipLaunchKernelGGL(k_sym_x, dim3(gx, grid_slots(slots, gx * chunks), chunks), dim3(256), 0, st,
                     A, sA, lda, X, sX, M, Y, sY, dcount, slot_list, part, KC);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  const int64_t n = (int64_t)M * 16;
  const int sx = (int)std::min<int64_t>((n + 255) / 256, 64);
  hipLaunchKernelGGL(k_sk_sum<0>, dim3(sx, grid_slots(slots, sx)), dim3(256), 0, st, part, chunks,
                     M, Y, sY, dcount, 0, slot_list);
  return hipGetLastError();
}

hipError_t launch_syrk(int M, int K, const float* A, int lda, int64_t sa, float* C, int ldc,
                       int64_t sc, const int* dcount, int hcount, int max_count, hipStream_t st) {
  if (max_count <= 0) return hipSuccess;
  const int tm = (M + 63) / 64;
  const int tiles = tm * (tm + 1) / 2;
  const dim3 grid(tiles, grid_slots(max_count, tiles));
  hipLaunchKernelGGL((k_gemm<1, 1>), grid, dim3(256), 0, st, A, lda, sa, A, lda, sa, C, ldc, sc, M,
                     M, K, dcount, hcount, nullptr, K);
  return hipGetLastError();
}

// C[c] (column-major, ldc) = sum over the chunks of k_gemm's partial products, in order.
__global__ void __launch_bounds__(256) k_gemm_sum(const float* __restrict__ part, int chunks,
                                                  int M, int N, float* __restrict__ C, int ldc,
                                                  int64_t sc, const int* __restrict__ dcount,
                                                  int hcount) {
  const int count = dev_count(dcount, hcount);
  const int64_t n = (int64_t)M * N;
  for (int c = blockIdx.y; c < count; c += gridDim.y)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
      const float* p = part + (int64_t)c * chunks * n + e;
      float s = 0.f;
      for (int ch = 0; ch < chunks; ++ch) s += p[(int64_t)ch * n];
      const int64_t j = e / M, i = e - (e / M) * M;
      C[(int64_t)c * sc + j * ldc + i] = s;
    }
}

int gemm_split(int M, int N, int K, int* kc) {
  // few output tiles and a long contraction: chunks of 128 or more, 32-aligned
  // (about 1024 workgroups: the chip's 256 compute units each run several)
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int chunks = (tiles < 512 && K >= 256) ? std::max(1, std::min(1024 / tiles, std::min(K / 128, 8))) : 1;
  int KC = (K + chunks - 1) / chunks;
  KC = (KC + 31) / 32 * 32;
  if (kc) *kc = KC;
  return (K + KC - 1) / KC;
}

hipError_t launch_gemm(bool ta, int M, int N, int K, const float* A, int lda, int64_t sa,
                       const float* B, int ldb, int64_t sb, float* C, int ldc, int64_t sc,
                       const int* dcount, int hcount, int max_count, hipStream_t st, float* part,
                       int64_t part_floats) {
  if (max_count <= 0) return hipSuccess;
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  // the split is a function of the shape alone (gemm_split); a part too small for it
  // means no split
  int KC = (K + 31) / 32 * 32, chunks = 1;
  if (part) {
    int kc = 0;
    const int c = gemm_split(M, N, K, &kc);
    if (c > 1 && (int64_t)c * M * N * max_count <= part_floats) {
      chunks = c;
      KC = kc;
    }
  }
  const dim3 grid(tiles, grid_slots(max_count, tiles * chunks), chunks);
  if (ta)
    hipLaunchKernelGGL(k_gemm<1>, grid, dim3(256), 0, st, A, lda, sa, B, ldb, sb, C, ldc, sc, M,
                       N, K, dcount, hcount, part, KC);
  else
    hipLaunchKernelGGL(k_gemm<0>, grid, dim3(256), 0, st, A, lda, sa, B, ldb, sb, C, ldc, sc, M,
                       N, K, dcount, hcount, part, KC);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  const int64_t n = (int64_t)M * N;
  const int gx = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gemm_sum, dim3(gx, grid_slots(max_count, gx)), dim3(256), 0, st, part,
                     chunks, M, N, C, ldc, sc, dcount, hcount);
  return hipGetLastError();
}

hipError_t launch_gemm_sym(int M, int K, const float* A, int lda, int64_t sa, const float* B,
                           int ldb, int64_t sb, float* C, int ldc, int64_t sc, int count,
                           hipStream_t st, float* part, int64_t part_floats, int* unsummed) {
  if (unsummed) *unsummed = 0;
  if (count <= 0) return hipSuccess;
  const int tm = (M + 63) / 64;
  const int tiles = tm * (tm + 1) / 2;
  // the split of the full M x M product (gemm_split), so that part is sized alike
  int KC = (K + 31) / 32 * 32, chunks = 1;
  if (part) {
    int kc = 0;
    const int c = gemm_split(M, M, K, &kc);
    if (c > 1 && (int64_t)c * M * M * count <= part_floats) {
      chunks = c;
      KC = kc;
    }
  }
  const dim3 grid(tiles, grid_slots(count, tiles * chunks), chunks);
  hipLaunchKernelGGL((k_gemm<1, 1>), grid, dim3(256), 0, st, A, lda, sa, B, ldb, sb, C, ldc, sc,
                     M, M, K, nullptr, count, part, KC);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  if (unsummed) {
    *unsummed = chunks;   // the caller's next kernel sums the partials
    return hipSuccess;
  }
  const int64_t n = (int64_t)M * M;
  const int gx = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gemm_sum, dim3(gx, grid_slots(count, gx)), dim3(256), 0, st, part, chunks,
                     M, M, C, ldc, sc, nullptr, count);
  return hipGetLastError();
}

// E^T E = G - Q V^T - V Q^T for the undecided slots of the certificate (Q is zero outside
// the masked columns, so V needs no mask), written to Pm with per-tile partial trace and
// squared Frobenius norm (part) and per-row partial |.| sums of each 64-column tile
// column (rowpart, slices 0 .. tn-1). 64 x 64 tiles, one 32 x 32 quadrant per wave on
// v_mfma_f32_32x32x2f32 with K = 2P: A = [Q | V] at the quadrant's column indices j,
// B = [V | Q] at its row indices i, so the accumulators hold D(j, i) with i = lane % 32
// and each store of a column of Pm is a 128-byte segment. Q, V and the G tile are read
// straight into registers in the accumulator layout.
template <int P>
__global__ void __launch_bounds__(256) k_mf_lr_ge(const float* G, const float* Qm,
                                                  const float* Vr, float* Pm, int nb,
                                                  float* part, float* rowpart, const int* list,
                                                  const int* lcount) {
  static_assert(P % 2 == 0, "K pairs");
  __shared__ float red[2][4];
  __shared__ float rs[2][64];
  const int cnt = *lcount;
  const int tn = (nb + 63) / 64;
  const int ti = blockIdx.x % tn, tj = blockIdx.x / tn;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int i = ti * 64 + (wv & 1) * 32 + li;   // B operand row, accumulator column
  const int jb = tj * 64 + (wv >> 1) * 32;      // first D row of the quadrant
  const int ja = jb + li;                       // A operand row
  const bool iok = i < nb, jok = ja < nb;
  for (int cidx = blockIdx.y; cidx < cnt; cidx += gridDim.y) {
    const int slot = list[cidx];
    const float* g = G + (int64_t)slot * nb * nb;
    const float* q = Qm + (int64_t)slot * nb * P;
    const float* v = Vr + (int64_t)slot * nb * P;
    float* pm = Pm + (int64_t)slot * nb * nb;
    float gv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = jb + 8 * (r >> 2) + 4 * lk + (r & 3);
      gv[r] = (iok && j < nb) ? g[(int64_t)j * nb + i] : 0.f;
    }
    float qa[P / 2], va[P / 2], qb[P / 2], vb[P / 2];
#pragma unroll
    for (int s = 0; s < P / 2; ++s) {
      const int64_t l = 2 * s + lk;
      qa[s] = jok ? q[l * nb + ja] : 0.f;
      va[s] = jok ? v[l * nb + ja] : 0.f;
      qb[s] = iok ? q[l * nb + i] : 0.f;
      vb[s] = iok ? v[l * nb + i] : 0.f;
    }
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int s = 0; s < P / 2; ++s) acc = mfma32(qa[s], vb[s], acc);
#pragma unroll
    for (int s = 0; s < P / 2; ++s) acc = mfma32(va[s], qb[s], acc);
    float tr = 0.f, f2 = 0.f, ra = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = jb + 8 * (r >> 2) + 4 * lk + (r & 3);
      if (iok && j < nb) {
        const float sv = gv[r] - acc[r];
        pm[(int64_t)j * nb + i] = sv;
        if (i == j) tr += sv;
        f2 += sv * sv;
        ra += fabsf(sv);
      }
    }
    ra += __shfl_xor(ra, 32);   // the quadrant's other 16 columns
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      tr += __shfl_xor(tr, o);
      f2 += __shfl_xor(f2, o);
    }
    __syncthreads();   // the previous slot's reads of rs and red are done
    if (lk == 0) rs[wv >> 1][(wv & 1) * 32 + li] = ra;
    if (lane == 0) {
      red[0][wv] = tr;
      red[1][wv] = f2;
    }
    __syncthreads();
    if (tid == 0) {
      float* pp = part + ((int64_t)slot * gridDim.x + blockIdx.x) * 2;
      pp[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      pp[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
    if (tid < 64 && ti * 64 + tid < nb)
      rowpart[(int64_t)slot * nb * (tn + 1) + (int64_t)tj * nb + ti * 64 + tid] =
          rs[0][tid] + rs[1][tid];
  }
}

hipError_t launch_lr_ge(const float* G, const float* Q, const float* V, float* Pm, int nb,
                        float* part, float* rowpart, const int* list, const int* lcount,
                        int slots, hipStream_t st) {
  const int tn = (nb + 63) / 64;
  const int tiles = tn * tn;
  hipLaunchKernelGGL(k_mf_lr_ge<16>, dim3(tiles, grid_slots(slots, tiles)), dim3(256), 0, st, G,
                     Q, V, Pm, nb, part, rowpart, list, lcount);
  return hipGetLastError();
}

hipError_t launch_mf_rebuild(const ScaleGeom& g, const ShiftSpec& sh, float* Zout, float* Dout,
                             const int* count, const int* slot_list, const int* live_list,
                             int slots, const int* pflag, const float* Af, const float* Vr,
                             const float* sig, const float* mask, float tau, hipStream_t st) {
  const int tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
  if (g.trans)
    hipLaunchKernelGGL((k_mf_rebuild<16, 1>), dim3(tiles, grid_slots(slots, tiles)), dim3(256), 0,
                       st, Zout, Dout, g, sh, count, slot_list, live_list, pflag, Af, Vr, sig,
                       mask, tau);
  else
    hipLaunchKernelGGL((k_mf_rebuild<16, 0>), dim3(tiles, grid_slots(slots, tiles)), dim3(256), 0,
                       st, Zout, Dout, g, sh, count, slot_list, live_list, pflag, Af, Vr, sig,
                       mask, tau);
  return hipGetLastError();
}

}  // namespace msld
