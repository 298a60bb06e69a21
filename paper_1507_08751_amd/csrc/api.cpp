// C-ABI runtime: parameter validation, per-scale planning, workspace arena, the ADMM
// driver loop (Sec. 7 eq:admm with the random cycle spinning of Sec. 9) and batched
// solves of many independent instances grouped by shape.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace msld;

namespace msld {

namespace {

constexpr int kResidPartsMax = 1024;
// profiling events per scale and iteration: 0-4 bracket the phases, 5-6 the Gram kernel
// of a low-rank tier
constexpr int kEvPerScale = 7;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

}  // namespace

// A block fits the LDS Jacobi tier if B and W fit the LDS budget, one workgroup
// covers all column pairs, and G lanes x 32 rows per lane cover the rows.
bool lds_fits(int mb, int nb) {
  int G = 1;
  const int threads = lds_tier_threads(nb, mb, &G);
  return lds_tier_bytes(mb, nb) <= kLdsTierMax && threads <= 1024 && G * 32 >= mb;
}

double lambda_default(int M, int N, int m, int n) {
  return std::sqrt((double)m) + std::sqrt((double)n) +
         std::sqrt(std::log((double)M * (double)N / (double)(m > n ? m : n)));
}

msld_status validate_params(const msld_params* p) {
  if (!p) return MSLD_EINVAL;
  if (p->M < 1 || p->N < 1 || p->M > (1 << 20) || p->N > (1 << 20)) return MSLD_EINVAL;
  if ((int64_t)p->M * p->N >= ((int64_t)1 << 31)) return MSLD_EINVAL;
  if (p->L < 1 || p->L > MSLD_MAX_SCALES) return MSLD_EINVAL;
  if (!(p->rho > 0.f) || !std::isfinite(p->rho)) return MSLD_EINVAL;
  if (p->max_iters < 1) return MSLD_EINVAL;
  if (!(p->tol >= 0.f) || !std::isfinite(p->tol)) return MSLD_EINVAL;
  if (p->check_every < 1) return MSLD_EINVAL;
  if (p->cycle_spin != 0 && p->cycle_spin != 1) return MSLD_EINVAL;
  if (p->spin_count < 0) return MSLD_EINVAL;
  if (p->fork_mode < 0 || p->fork_mode > 3) return MSLD_EINVAL;
  if (p->image_w < 0 || (p->image_w > 0 && p->M % p->image_w)) return MSLD_EINVAL;
  for (int i = 0; i < p->L; ++i) {
    const int m = p->block_m[i], n = p->block_n[i];
    if (m < 1 || n < 1 || p->M % m || p->N % n) return MSLD_EINVAL;
    if (!std::isfinite(p->lambda[i])) return MSLD_EINVAL;
    if (p->kind[i] != MSLD_KIND_BLOCK && p->kind[i] != MSLD_KIND_NOISE &&
        p->kind[i] != MSLD_KIND_SPATIAL)
      return MSLD_EINVAL;
    if (p->kind[i] == MSLD_KIND_NOISE && (m != p->M || n != p->N)) return MSLD_EINVAL;
    if (p->kind[i] == MSLD_KIND_SPATIAL) {
      // ph x pw patches tile the H x W image, bt = n frames tile the columns
      const int pw = p->patch_w[i];
      if (p->image_w == 0 || pw < 1 || m % pw || p->image_w % pw) return MSLD_EINVAL;
      if ((p->M / p->image_w) % (m / pw)) return MSLD_EINVAL;
    }
  }
  return MSLD_OK;
}

// Two parameter sets can share stacked launches when everything but the shift seed
// agrees (the seed is per instance).
bool host_waits(const Plan& pl, int i) {
  return pl.use_lr[i] && !lds_fits(pl.geom[i].mb, pl.geom[i].nb);
}

bool same_class(const msld_params& a, const msld_params& b) {
  if (a.M != b.M || a.N != b.N || a.L != b.L || a.rho != b.rho || a.max_iters != b.max_iters ||
      a.tol != b.tol || a.check_every != b.check_every || a.cycle_spin != b.cycle_spin ||
      a.lowrank_min != b.lowrank_min || a.spin_count != b.spin_count ||
      a.image_w != b.image_w || a.fork_mode != b.fork_mode)
    return false;
  for (int i = 0; i < a.L; ++i)
    if (a.block_m[i] != b.block_m[i] || a.block_n[i] != b.block_n[i] ||
        a.lambda[i] != b.lambda[i] || a.kind[i] != b.kind[i] ||
        (a.kind[i] == MSLD_KIND_SPATIAL && a.patch_w[i] != b.patch_w[i]))
      return false;
  return true;
}

msld_status make_plan(const msld_params* p, int ninst, Plan* pl) {
  msld_status st = validate_params(p);
  if (st != MSLD_OK) return st;
  if (ninst < 1 || (int64_t)ninst * p->M * p->N >= ((int64_t)1 << 31)) return MSLD_EINVAL;
  std::memset(pl, 0, sizeof(*pl));
  const int IM = p->M, N = p->N, L = p->L;
  const int M = IM * ninst;
  const size_t MN = (size_t)M * N;
  pl->ninst = ninst;
  int parts = (int)(((size_t)IM * N + 4095) / 4096);
  if (parts > kResidPartsMax) parts = kResidPartsMax;
  if (parts < 1) parts = 1;
  pl->resid_parts = parts;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + (bytes ? bytes : 1), 256);
    return o;
  };
  pl->off_R = take(4 * MN);
  pl->off_D = take(4 * MN * (size_t)L * 2);
  pl->off_part = take(8 * 2 * (size_t)parts * ninst);
  pl->off_res = take(8 * 3 * (size_t)ninst);   // primal sums, ||Y||^2, dual sums
  pl->off_shift = take(4 * 2 * (size_t)L * 1024);
  pl->off_inst = take(8 * (size_t)ninst + 4 * 2 * (size_t)ninst);
  for (int i = 0; i < L; ++i) {
    const int m = p->block_m[i], n = p->block_n[i];
    ScaleGeom& g = pl->geom[i];
    g.M = M; g.N = N; g.m = m; g.n = n;
    g.IM = IM; g.PI = IM / m; g.NI = ninst;
    g.P = g.PI * ninst; g.Q = N / n;
    g.trans = m < n ? 1 : 0;
    g.mb = m < n ? n : m;
    g.nb = m < n ? m : n;
    if (p->kind[i] == MSLD_KIND_SPATIAL) {
      g.pw = p->patch_w[i];
      g.ph = m / g.pw;
      g.iw = p->image_w;
      g.ih = IM / p->image_w;
    }
    const bool noise = p->kind[i] == MSLD_KIND_NOISE;
    const double lam = p->lambda[i] > 0.f ? (double)p->lambda[i]
                       : noise ? lambda_default(IM, N, IM * N, 1)   // the MN x 1 block
                               : lambda_default(IM, N, m, n);
    pl->tau_default[i] = (float)(lam / (double)p->rho);
    const int nblk = g.P * g.Q;
    if (noise) {
      // Frobenius prox: per-instance partial sums of squares and gains
      pl->tier[i] = TIER_FRO;
      pl->off_stats[i] = take(8 * kStatsWords);
      pl->off_lr[i] = take(8 * (size_t)kFroParts * ninst + 4 * (size_t)ninst);
      continue;
    }
    // certified low-rank paths: fused per-block kernel up to 64 x 128 (falls back to
    // the LDS tier), batched-GEMM path beyond (falls back to the polar route)
    const int lr_min = p->lowrank_min == 0 ? 32 : p->lowrank_min;
    int sNB, sMB, sP;
    const bool lrs = lr_min > 0 && g.nb >= lr_min && lr_small_shape(g.mb, g.nb, &sNB, &sMB, &sP) &&
                     lds_fits(g.mb, g.nb) && lr_small_lds_bytes(sNB, sMB, sP) <= kLdsTierMax;
    // (narrower blocks take it only when the alternative would be the HBM panel tier)
    // (the orthonormalisation keeps p columns of nb in LDS: nb <= 2048)
    // (tall blocks of 16..31 columns that fit neither LDS nor the panel tier take it too)
    const bool panel_fits =
        kLdsTierMax / 4 / (2 * ((size_t)(g.mb | 1) + (size_t)(g.nb | 1))) >= 4;
    bool lr = !lrs && lr_min > 0 && g.nb <= 2048 &&
              ((g.nb >= lr_min &&
                (g.nb >= 4 * kLRP || (g.nb >= 2 * kLRP && !lds_fits(g.mb, g.nb)))) ||
               (g.nb >= kLRP && !lds_fits(g.mb, g.nb) && !panel_fits));
    int tier;
    if (m == 1 && n == 1) tier = TIER_1X1;
    else if (reg_tier_shape(m, n)) tier = TIER_REG;
    else if (lrs) tier = TIER_LRS;
    else if (!lr && lds_fits(g.mb, g.nb)) tier = TIER_LDS;
    else tier = TIER_PANEL;
    // an autotuned choice for this block size (msld_autotune), where it applies
    TuneCfg tc;
    if (tier != TIER_1X1 && tune_lookup(m, n, &tc)) {
      if (tc.tier == TIER_REG && reg_tier_shape(m, n)) {
        tier = TIER_REG;
        lr = false;
      } else if (tc.tier == TIER_LRS && lrs) {
        tier = TIER_LRS;
        lr = false;
        pl->lrs_wide[i] = tc.lrs_wide;
      } else if (tc.tier == TIER_LDS && lds_fits(g.mb, g.nb)) {
        tier = TIER_LDS;
        lr = false;
        pl->lds_cap[i] = tc.lds_cap;
      } else if (tc.tier == kTierLowRank && lr_min > 0 && g.nb >= lr_min && g.nb <= 2048) {
        tier = TIER_PANEL;
        lr = true;
      }
    }
    pl->use_lr[i] = lr ? 1 : 0;
    pl->tier[i] = tier;
    pl->off_stats[i] = take(8 * kStatsWords);
    if (tier == TIER_1X1) continue;
    // averaged cycle spinning: a cyclic shift along an axis the block spans whole
    // permutes rows (columns) inside each block, which its SVT follows exactly, so
    // that axis has one distinct shift; a scale with a single one keeps the plain step
    const int64_t mr = m == IM ? 1 : m, nc = n == N ? 1 : n;
    if (p->cycle_spin && p->spin_count > 1 && mr * nc > 1) {
      pl->spin_full[i] = p->spin_count >= mr * nc ? 1 : 0;
      pl->spin[i] = (int)(pl->spin_full[i] ? mr * nc : p->spin_count);
      pl->off_spin[i] = take(4 * MN * 2);
    }
    // stream plan
    StreamPlan& sp = pl->sp[i];
    int ws = kStreamFloats / m;
    if (ws > 256) ws = 256;
    if (ws < 1) ws = 1;
    ws = pow2_floor(ws);
    if (n <= ws) {
      sp.whole = 1;
      sp.kb = ws / n;
      sp.ws = sp.kb * n;
      sp.spb = 1;
      sp.spr = (g.Q + sp.kb - 1) / sp.kb;
    } else {
      sp.whole = 0;
      sp.ws = ws;
      sp.kb = 1;
      sp.spb = (n + ws - 1) / ws;
      sp.spr = g.Q * sp.spb;
    }
    sp.rowbound = (sp.whole || sp.ws >= 8) ? 1 : 0;
    sp.cst = sp.spb;
    sp.rch = m;
    sp.align = 0;
    if (!sp.whole && sp.rowbound && N % 32 == 0 && sp.ws % 32 == 0) {
      sp.align = 1;
      sp.cst = (n + sp.ws - 1) / sp.ws + 1;
      sp.spb = sp.cst;
      sp.spr = g.Q * sp.spb;
    }
    if (!sp.rowbound) {
      // Frobenius bound only: strips of up to 256 columns and 128 rows (coalesced rows,
      // and enough strips per block to spread a tall block over the chip)
      sp.ws = n < 256 ? n : 256;
      sp.cst = (n + sp.ws - 1) / sp.ws;
      sp.rch = 128;
      sp.spb = sp.cst * ((m + sp.rch - 1) / sp.rch);
      sp.spr = g.Q * sp.spb;
    }
    // a bfloat16 tile of 16 KiB or more leaves room for few workgroups per compute unit:
    // 512 threads each then keep twice the loads in flight for the same LDS
    sp.nt = (sp.rowbound && (size_t)m * (sp.ws + 1) * 2 >= 16384) ? 512 : 256;
    if (stream_lds_bytes(m, sp) > kLdsTierMax) return MSLD_EINVAL;
    pl->off_count[i] = take(4);
    pl->off_list[i] = take(4 * (size_t)nblk);
    if (!sp.whole) {
      if (sp.rowbound) pl->off_rowp[i] = take(4 * (size_t)nblk * sp.spb * m);
      pl->off_frop[i] = take(4 * (size_t)nblk * sp.spb);
    }
    if (tier == TIER_LRS) pl->off_lr[i] = take(4 * (64 + 2 * (size_t)nblk));   // fallback lists
    if (tier == TIER_PANEL) {
      // panel width: two panels of A (mb rows) and W (nb rows) in LDS; 4 <= pw <= 64
      // (the low-rank path only uses the panel layout, padded to a multiple of 8)
      int pw = lr ? 4 : (int)(kLdsTierMax / 4 / (2 * ((size_t)(g.mb | 1) + (size_t)(g.nb | 1))));
      if (pw > 64) pw = 64;
      pw = pow2_floor(pw < 1 ? 1 : pw);
      while (pw > 4 && 2 * pw > g.nb) pw >>= 1;
      if (pw < 4 || g.nb > 4096) return MSLD_EINVAL;  // beyond the panel tier's limits
      const int nbp = (g.nb + 2 * pw - 1) / (2 * pw) * (2 * pw);
      pl->pw[i] = pw;
      pl->nbp[i] = nbp;
      if (!lr) {
        // HBM panels of the block one-sided Jacobi (the low-rank path reads every block
        // straight from the iterate and needs only the per-slot flags)
        pl->off_pA[i] = take(4 * (size_t)nblk * nbp * g.mb);
        pl->off_pW[i] = take(4 * (size_t)nblk * nbp * g.nb);
        pl->off_pg[i] = take(4 * (size_t)nblk * nbp);
      }
      pl->off_pflag[i] = take(4 * 4 * (size_t)nblk);
      if (lr) {
        const size_t nb2 = (size_t)g.nb * g.nb;
        const size_t tn = ((size_t)g.nb + 63) / 64;
        const size_t per = 3 * nb2 + 4 * (size_t)g.nb * kLRP + (size_t)g.mb * kLRP +
                           (size_t)kLRP * g.nb + 3 * kLRP + 8 + (size_t)g.nb * (tn + 1);
        pl->off_lr[i] = take(4 * ((size_t)nblk * per + (size_t)g.nb * kLRP + 64 + 6 * nblk));
        // split partials of the Gram matrix of tall or wide blocks, sized by the block
        // shape and the slot count
        const int ch = split_chunks(g.mb, g.nb);
        if (ch > 1) pl->off_split[i] = take(4 * (size_t)nblk * ch * nb2);
        // a single wide block would leave its skinny products to a handful of
        // workgroups: their contractions split too
        if (g.nb >= 768)
          pl->off_skpart[i] = take(4 * (size_t)nblk * sk_chunks(g.nb) *
                                   (size_t)std::max(g.mb, g.nb) * kLRP);
        if (!lds_fits(g.mb, g.nb)) {
          // polar fallback buffers for a chunk of failed certificates (<= 256 MiB): per
          // block its iterates, scalars and step counts, and the split partial products
          // of its GEMMs at the split the shapes alone give
          const size_t pper = 3 * (size_t)g.mb * g.nb + 4 * nb2 + 6 +
                              (size_t)polar_part_floats(g.mb, g.nb);
          size_t cap = ((size_t)256 << 20) / (4 * pper);
          if (cap < 1) cap = 1;
          if (cap > (size_t)nblk) cap = (size_t)nblk;
          pl->pl_cap[i] = (int)cap;
          pl->off_pl[i] = take(4 * cap * pper);
        }
      }
    }
  }
  pl->bytes = off;
  return MSLD_OK;
}

msld_status dev_err(msld_solver* s, hipError_t e) {
  if (e == hipSuccess) return MSLD_OK;
  if (s) s->failed = true;
  return MSLD_EDEVICE;
}

size_t plane_elems(const msld_solver* s) { return (size_t)s->p.M * s->ninst * s->p.N; }

float* plane_R(msld_solver* s) { return reinterpret_cast<float*>(s->arena + s->plan.off_R); }

float* plane_D(msld_solver* s, int which) {
  return reinterpret_cast<float*>(s->arena + s->plan.off_D) +
         (size_t)which * plane_elems(s) * s->p.L;
}

double* dev_res(msld_solver* s) { return reinterpret_cast<double*>(s->arena + s->plan.off_res); }

static void drop_graphs(msld_solver* s) {
  for (auto& g : s->gx)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

static void destroy_solver(msld_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  drop_graphs(s);
  if (s->prof_ev) {
    for (size_t e = 0; e < (4 + kEvPerScale * (size_t)s->p.L) * (size_t)s->prof_cap; ++e)
      (void)hipEventDestroy(s->prof_ev[e]);
    std::free(s->prof_ev);
  }
  for (int i = 0; i < MSLD_MAX_SCALES; ++i) {
    if (s->sst[i]) {
      (void)hipStreamSynchronize(s->sst[i]);
      (void)hipStreamDestroy(s->sst[i]);
    }
    if (s->ev_join[i]) (void)hipEventDestroy(s->ev_join[i]);
    if (s->ev_sfork[i]) (void)hipEventDestroy(s->ev_sfork[i]);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->cst) (void)hipStreamDestroy(s->cst);
  if (s->arena) (void)hipFree(s->arena);
  if (s->host_res) (void)hipHostFree(s->host_res);
  if (s->host_ints) (void)hipHostFree(s->host_ints);
  if (s->host_pl) (void)hipHostFree(s->host_pl);
  delete s;
}

msld_status create_solver(const msld_params* p, int ninst, hipStream_t stream,
                          msld_solver** out) {
  if (!out) return MSLD_EINVAL;
  *out = nullptr;
  msld_solver* s = new (std::nothrow) msld_solver();
  if (!s) return MSLD_ENOMEM;
  msld_status st = make_plan(p, ninst, &s->plan);
  if (st != MSLD_OK) {
    delete s;
    return st;
  }
  s->p = *p;
  s->ninst = ninst;
  s->st = stream;
  s->failed = false;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return MSLD_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) {
    delete s;
    return MSLD_EDEVICE;
  }
  s->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (hipMalloc(&s->arena, s->plan.bytes) != hipSuccess) {
    s->arena = nullptr;
    destroy_solver(s);
    return MSLD_ENOMEM;
  }
  if (hipHostMalloc(&s->host_res, 3 * (size_t)ninst * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(&s->host_ints, 2 * MSLD_MAX_SCALES * sizeof(int), hipHostMallocDefault) !=
          hipSuccess) {
    destroy_solver(s);
    return MSLD_ENOMEM;
  }
  {
    // scales run concurrently: each low-rank scale gets its own slice
    int cap = 0;
    for (int i = 0; i < p->L; ++i) cap += s->plan.pl_cap[i];
    if (cap > 0 && hipHostMalloc(&s->host_pl, 6 * (size_t)cap * sizeof(float),
                                 hipHostMallocDefault) != hipSuccess) {
      destroy_solver(s);
      return MSLD_ENOMEM;
    }
  }
  const Plan& pl = s->plan;
  s->d_seed = reinterpret_cast<unsigned long long*>(s->arena + pl.off_inst);
  s->d_k = reinterpret_cast<int*>(s->d_seed + ninst);
  s->d_active = s->d_k + ninst;
  // an iteration can be captured once no scale's driver waits on the host (only a
  // low-rank scale whose blocks exceed the LDS tier reads its fallback count back, to
  // size the polar route); such solvers keep the shift seed and iteration counter on
  // the device, so a replay needs no host values
  s->graphable = true;
  for (int i = 0; i < p->L; ++i)
    if (host_waits(pl, i)) s->graphable = false;
  s->graph_on = s->graphable;
  if (s->graphable && hipStreamCreateWithFlags(&s->cst, hipStreamNonBlocking) != hipSuccess) {
    s->cst = nullptr;
    destroy_solver(s);
    return MSLD_EDEVICE;
  }
  if (ninst == 1) {
    const unsigned long long seed = p->shift_seed;
    if (hipMemcpy(s->d_seed, &seed, sizeof(seed), hipMemcpyHostToDevice) != hipSuccess) {
      destroy_solver(s);
      return MSLD_EDEVICE;
    }
  }
  if (hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess) {
    s->ev_fork = nullptr;
    destroy_solver(s);
    return MSLD_EDEVICE;
  }
  // Stream creation order. Once a process holds all its hardware queues (HIP reads the
  // count from GPU_MAX_HW_QUEUES, default 4), HIP attaches a new stream to the least
  // used one. When the scale streams outnumber the queues left beside the caller's, the
  // low-rank scales' streams come first, so their long chains get queues of their own
  // and the short scales share what is left; otherwise scale order (measured faster
  // when every stream has a queue of its own).
  int hwq = 4;
  if (const char* q = std::getenv("GPU_MAX_HW_QUEUES")) {
    const int v = std::atoi(q);
    if (v > 0) hwq = v;
  }
  int nst = 0;
  for (int i = 0; i < p->L; ++i)
    if (pl.tier[i] != TIER_1X1) ++nst;
  const bool scarce = nst + 1 > hwq;
  int corder[MSLD_MAX_SCALES];
  int nco = 0;
  if (scarce) {
    for (int i = p->L - 1; i >= 0; --i)
      if (pl.use_lr[i]) corder[nco++] = i;
    for (int i = 0; i < p->L; ++i)
      if (!pl.use_lr[i]) corder[nco++] = i;
  } else {
    for (int i = 0; i < p->L; ++i) corder[nco++] = i;
  }
  for (int ci = 0; ci < nco; ++ci) {
    const int i = corder[ci];
    if (pl.tier[i] == TIER_1X1) continue;   // fused in the consensus pass
    if (hipStreamCreateWithFlags(&s->sst[i], hipStreamNonBlocking) != hipSuccess) {
      s->sst[i] = nullptr;
      destroy_solver(s);
      return MSLD_EDEVICE;
    }
    if (hipEventCreateWithFlags(&s->ev_join[i], hipEventDisableTiming) != hipSuccess) {
      s->ev_join[i] = nullptr;
      destroy_solver(s);
      return MSLD_EDEVICE;
    }
    if (hipEventCreateWithFlags(&s->ev_sfork[i], hipEventDisableTiming) != hipSuccess) {
      s->ev_sfork[i] = nullptr;
      destroy_solver(s);
      return MSLD_EDEVICE;
    }
  }
  for (int i = 0; i < p->L; ++i) {
    ScaleWork& w = s->work[i];
    std::memset(&w, 0, sizeof(w));
    w.stats = reinterpret_cast<unsigned long long*>(s->arena + pl.off_stats[i]);
    w.lds_cap = pl.lds_cap[i];
    w.lrs_wide = pl.lrs_wide[i];
    if (pl.spin[i]) {
      w.spinAcc = reinterpret_cast<float*>(s->arena + pl.off_spin[i]);
      w.spinTmp = w.spinAcc + plane_elems(s);
    }
    w.hostInts = s->host_ints + 2 * i;
    if (pl.tier[i] == TIER_FRO) {
      w.froPart = reinterpret_cast<double*>(s->arena + pl.off_lr[i]);
      w.froGain = reinterpret_cast<float*>(w.froPart + (size_t)kFroParts * ninst);
      continue;
    }
    if (pl.tier[i] != TIER_1X1) {
      w.live_count = reinterpret_cast<int*>(s->arena + pl.off_count[i]);
      w.live_list = reinterpret_cast<int*>(s->arena + pl.off_list[i]);
      if (!pl.sp[i].whole) {
        w.rowpart = pl.sp[i].rowbound ? reinterpret_cast<float*>(s->arena + pl.off_rowp[i])
                                      : nullptr;
        w.fropart = reinterpret_cast<float*>(s->arena + pl.off_frop[i]);
      }
    }
    if (pl.tier[i] == TIER_LRS) {
      w.lrCount = reinterpret_cast<int*>(s->arena + pl.off_lr[i]);
      w.lrFall = w.lrCount + 64;
    }
    if (pl.tier[i] == TIER_PANEL) {
      const ScaleGeom& g = pl.geom[i];
      if (!pl.use_lr[i]) {
        w.pA = reinterpret_cast<float*>(s->arena + pl.off_pA[i]);
        w.pW = reinterpret_cast<float*>(s->arena + pl.off_pW[i]);
        w.pg = reinterpret_cast<float*>(s->arena + pl.off_pg[i]);
      }
      w.pflag = reinterpret_cast<int*>(s->arena + pl.off_pflag[i]);
      w.slots = g.P * g.Q;
      w.nbp = pl.nbp[i];
      w.pw = pl.pw[i];
      if (pl.use_lr[i]) {
        const size_t nb2 = (size_t)g.nb * g.nb;
        const size_t slots = (size_t)w.slots;
        float* f = reinterpret_cast<float*>(s->arena + pl.off_lr[i]);
        w.use_lr = 1;
        w.lrG = f; f += slots * nb2;
        w.lrP = f; f += slots * nb2;
        w.lrQ = f; f += slots * nb2;
        w.lrY = f; f += slots * g.nb * kLRP;
        w.lrX = f; f += slots * g.nb * kLRP;
        w.lrW = f; f += slots * g.nb * kLRP;
        w.lrV = f; f += slots * g.nb * kLRP;
        w.lrC = f; f += slots * g.mb * kLRP;
        w.lrT = f; f += slots * kLRP * g.nb;
        w.lrSig = f; f += 3 * slots * kLRP;   // sigma, deflation mask, bound mask
        w.lrScal = f; f += slots * 8;
        w.lrRow = f; f += slots * (size_t)g.nb * (((size_t)g.nb + 63) / 64 + 1);
        w.lrOm = f; f += (size_t)g.nb * kLRP;
        w.lrSplit = pl.off_split[i] ? reinterpret_cast<float*>(s->arena + pl.off_split[i])
                                    : nullptr;
        w.lrChunks = w.lrSplit ? split_chunks(g.mb, g.nb) : 1;
        w.lrSkPart = pl.off_skpart[i] ? reinterpret_cast<float*>(s->arena + pl.off_skpart[i])
                                      : nullptr;
        w.lrSkChunks = w.lrSkPart ? sk_chunks(g.nb) : 1;
        w.lrCount = reinterpret_cast<int*>(f);
        w.lrFall = w.lrCount + 64;
        w.lds_fallback = lds_fits(g.mb, g.nb) ? 1 : 0;
        if (pl.pl_cap[i] > 0) {
          const size_t cap = (size_t)pl.pl_cap[i];
          const size_t x = (size_t)g.mb * g.nb;
          float* q = reinterpret_cast<float*>(s->arena + pl.off_pl[i]);
          w.plCap = pl.pl_cap[i];
          w.plX0 = q; q += cap * x;
          w.plXa = q; q += cap * x;
          w.plXb = q; q += cap * x;
          w.plT = q; q += cap * nb2;
          w.plS = q; q += cap * nb2;
          w.plY = q; q += cap * nb2;
          w.plW = q; q += cap * nb2;
          w.plScal = q; q += 4 * cap;
          w.plSteps = reinterpret_cast<int*>(q); q += 2 * cap;
          w.plPart = q;
          // pinned host slice: 4 scalars and 2 step counts per block
          size_t hoff = 0;
          for (int i2 = 0; i2 < i; ++i2) hoff += 6 * (size_t)pl.pl_cap[i2];
          w.hostPl = s->host_pl + hoff;
          w.hostSteps = reinterpret_cast<int*>(w.hostPl + 4 * cap);
        }
      }
    }
  }
  // fused stream-pass descriptor
  // Early forks: each scale's BlockSVT starts right after its own stream pass (low-rank
  // scales' passes first, largest first) instead of after all of them. The started
  // chains then share the chip with the remaining passes, which pays while the passes
  // are short: planes of up to 2^24 elements (video stand-in +5.7%, batches +3%). At
  // 8192^2 the iteration gained 1.3% but the HBM-bound passes ran 2.4x slower, so large
  // planes keep them uncontended. The caller can force either schedule (fork_mode).
  s->serial = p->fork_mode == 3;
  s->early_fork = p->fork_mode == 1                        ? 1
                  : (p->fork_mode == 2 || p->fork_mode == 3) ? 0
                                                             : (plane_elems(s) <= ((size_t)1 << 24) ? 1 : 0);
  {
    StreamAll& a = s->sall;
    std::memset(&a, 0, sizeof(a));
    a.plane = plane_elems(s);
    int sorder[MSLD_MAX_SCALES], nso = 0;
    if (s->early_fork) {
      for (int i = p->L - 1; i >= 0; --i)
        if (pl.use_lr[i]) sorder[nso++] = i;
      for (int i = 0; i < p->L; ++i)
        if (!pl.use_lr[i]) sorder[nso++] = i;
    } else {
      for (int i = 0; i < p->L; ++i) sorder[nso++] = i;
    }
    for (int si = 0; si < nso; ++si) {
      const int i = sorder[si];
      // (averaged scales run their own stream pass per shift)
      if (pl.tier[i] == TIER_1X1 || pl.tier[i] == TIER_FRO || pl.spin[i]) continue;
      StreamScale& d = a.s[a.n];
      d.g = pl.geom[i];
      d.sp = pl.sp[i];
      d.scale = i;
      d.tau2lim = stream_tau2lim(pl.geom[i], pl.tau_default[i]);
      d.live_count = s->work[i].live_count;
      d.live_list = s->work[i].live_list;
      d.rowpart = s->work[i].rowpart;
      d.fropart = s->work[i].fropart;
      a.first[a.n + 1] = a.first[a.n] + pl.geom[i].P * pl.sp[i].spr;
      ++a.n;
    }
  }
  *out = s;
  return MSLD_OK;
}

static float jacobi_tol(int mb) { return jacobi_tolerance(mb); }

// Scale i's BlockSVT on its own stream; the caller forks it from s->st (after the
// consensus) and joins it back.
static msld_status run_scale(msld_solver* s, int i, const float* Zin, const float* R, float* Zout,
                             float* Dout, float tau, const ShiftSpec& sh, hipEvent_t* ev,
                             bool stream_done) {
  const Plan& pl = s->plan;
  const ScaleGeom& g = pl.geom[i];
  int rl = 0;
  MSLD_TRY(s, launch_scale(g, pl.tier[i], pl.sp[i], s->work[i], Zin, R, Zout, Dout, tau, sh,
                           jacobi_tol(g.mb), 40, 20, s->num_cus, s->sst[i], ev, &rl,
                           stream_done));
  if (ev) s->round_launches[i] += rl;
  return MSLD_OK;
}

static msld_status fork_scale(msld_solver* s, int i, bool own = false) {
  MSLD_TRY(s, hipStreamWaitEvent(s->sst[i], own ? s->ev_sfork[i] : s->ev_fork, 0));
  return MSLD_OK;
}

static msld_status join_scale(msld_solver* s, int i) {
  MSLD_TRY(s, hipEventRecord(s->ev_join[i], s->sst[i]));
  MSLD_TRY(s, hipStreamWaitEvent(s->st, s->ev_join[i], 0));
  return MSLD_OK;
}

// The stream scale i's BlockSVT runs on inside an iteration: its own, or the handle's
// stream when the scales run one after another (fork_mode 3).
static hipStream_t scale_stream(const msld_solver* s, int i) {
  return s->serial ? s->st : s->sst[i];
}

static msld_status zero_stats(msld_solver* s) {
  for (int i = 0; i < s->p.L; ++i) {
    MSLD_TRY(s, hipMemsetAsync(s->work[i].stats, 0, 8 * kStatsWords, s->st));
    for (long long& v : s->work[i].stats_host) v = 0;
  }
  return MSLD_OK;
}

msld_status iterate_once(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                         bool want_res) {
  const msld_params& p = s->p;
  const Plan& pl = s->plan;
  const int IM = p.M, N = p.N, L = p.L;
  const int M = IM * s->ninst;
  const size_t MN = plane_elems(s);
  // per-instance device seeds, iteration counters and activity flags: stacked instances,
  // and single solves that may be captured into a graph
  const bool stacked = s->ninst > 1 || s->graphable || s->per_instance;
  float* R = plane_R(s);
  float* Dc = plane_D(s, s->cur);
  float* Dn = plane_D(s, 1 - s->cur);
  int scales1[16];
  float taus1[16];
  int n1 = 0;
  for (int i = 0; i < L; ++i)
    if (pl.tier[i] == TIER_1X1) {
      scales1[n1] = i;
      taus1[n1] = pl.tau_default[i];
      ++n1;
    }
  hipEvent_t* ev = nullptr;
  if (s->prof_ev && s->prof_n < s->prof_cap) {
    ev = s->prof_ev + (size_t)s->prof_n * (4 + kEvPerScale * L);
    ++s->prof_n;
    MSLD_TRY(s, hipEventRecord(ev[0], s->st));
  }
  MSLD_TRY(s, launch_consensus(d_Y, ldY, Dc, Dn, d_Z, R, M, N, L, scales1, taus1, n1, IM,
                               stacked ? s->d_active : nullptr, s->mask, s->ldmask, s->st));
  if (ev) MSLD_TRY(s, hipEventRecord(ev[1], s->st));
  {
    // stream pass of every decomposed scale in one launch
    ShiftSpec sh;
    sh.seed = p.shift_seed;
    sh.k = s->k;
    sh.scale = 0;
    sh.mode = p.cycle_spin ? 1 : 0;
    sh.sr = sh.sc = 0;
    sh.iseed = stacked ? s->d_seed : nullptr;
    sh.ik = stacked ? s->d_k : nullptr;
    sh.iactive = stacked ? s->d_active : nullptr;
    if (ev) MSLD_TRY(s, hipEventRecord(ev[2], s->st));
    if (s->sall.n > 0)
      MSLD_TRY(s, launch_stream_all(s->sall, d_Z, R, Dn, sh, s->st,
                                    s->early_fork ? s->ev_sfork : nullptr));
    if (ev) MSLD_TRY(s, hipEventRecord(ev[3], s->st));
  }
  MSLD_TRY(s, hipEventRecord(s->ev_fork, s->st));
  // issue order: the scales with the largest blocks first (their BlockSVT chains are the
  // longest, so the critical path is queued earliest); every scale's work is enqueued
  // from this thread: a low-rank scale whose fallback is the polar route defers its one
  // read-back (finish_fallback) until all scales are queued
  int order[MSLD_MAX_SCALES], no = 0;
  for (int i = 0; i < L; ++i)
    if (pl.tier[i] != TIER_1X1) order[no++] = i;
  std::stable_sort(order, order + no, [&](int x, int y) {
    return (int64_t)pl.geom[x].m * pl.geom[x].n > (int64_t)pl.geom[y].m * pl.geom[y].n;
  });
  ShiftSpec shs[MSLD_MAX_SCALES];
  for (int oi = 0; oi < no; ++oi) {
    const int i = order[oi];
    // with early forks, a scale of the stream-pass descriptor waits for its own pass only
    bool own = false;
    if (s->early_fork)
      for (int k = 0; k < s->sall.n; ++k)
        if (s->sall.s[k].scale == i) own = true;
    if (!s->serial) {
      msld_status fs = fork_scale(s, i, own);
      if (fs != MSLD_OK) return fs;
    }
    ShiftSpec& sh = shs[i];
    sh.seed = p.shift_seed;
    sh.k = s->k;
    sh.scale = i;
    sh.mode = p.cycle_spin ? 1 : 0;
    sh.sr = sh.sc = 0;
    sh.iseed = stacked ? s->d_seed : nullptr;
    sh.ik = stacked ? s->d_k : nullptr;
    sh.iactive = stacked ? s->d_active : nullptr;
  }
  hipError_t herr[MSLD_MAX_SCALES];
  int rls[MSLD_MAX_SCALES];
  int deferred[MSLD_MAX_SCALES];
  auto issue = [&](int i) {
    float* Zi = d_Z + MN * i;
    rls[i] = 0;
    deferred[i] = 0;
    if (!pl.spin[i]) {
      herr[i] = launch_scale(pl.geom[i], pl.tier[i], pl.sp[i], s->work[i], Zi, R, Zi,
                             Dn + MN * i, pl.tau_default[i], shs[i], jacobi_tol(pl.geom[i].mb),
                             40, 20, s->num_cus, scale_stream(s, i),
                             ev ? ev + 4 + kEvPerScale * i : nullptr,
                             &rls[i], true, s->serial ? nullptr : &deferred[i]);
      return;
    }
    // averaged cycle spinning: Z_i stays the input of every shift's Z-step until the
    // finish kernel replaces it by the mean (phase timings cover the first shift); each
    // shift's fallback completes before its Z-step is accumulated
    const ScaleWork& w = s->work[i];
    const int nc = pl.geom[i].n == N ? 1 : pl.geom[i].n;
    const int* act = stacked ? s->d_active : nullptr;
    const size_t inst = (size_t)IM * N;
    hipError_t e = hipSuccess;
    for (int j = 0; j < pl.spin[i] && e == hipSuccess; ++j) {
      ShiftSpec sj = shs[i];
      if (pl.spin_full[i]) {
        sj.mode = 2;
        sj.sr = j / nc;
        sj.sc = j % nc;
      } else {
        sj.seed_add = (uint64_t)j;
      }
      float* out = j == 0 ? w.spinAcc : w.spinTmp;
      int rl = 0;
      e = launch_scale(pl.geom[i], pl.tier[i], pl.sp[i], s->work[i], Zi, R, out, Dn + MN * i,
                       pl.tau_default[i], sj, jacobi_tol(pl.geom[i].mb), 40, 20, s->num_cus,
                       scale_stream(s, i), (ev && j == 0) ? ev + 4 + kEvPerScale * i : nullptr, &rl,
                       false);
      rls[i] += rl;
      if (e == hipSuccess && j > 0)
        e = launch_spin_acc(w.spinAcc, w.spinTmp, MN, inst, act, scale_stream(s, i));
    }
    if (e == hipSuccess)
      e = launch_spin_finish(Zi, Dn + MN * i, R, w.spinAcc, 1.0f / (float)pl.spin[i], MN, inst,
                             act, scale_stream(s, i));
    herr[i] = e;
  };
  for (int oi = 0; oi < no; ++oi) issue(order[oi]);
  for (int oi = 0; oi < no; ++oi) {
    const int i = order[oi];
    if (herr[i] != hipSuccess || !deferred[i]) continue;
    herr[i] = finish_fallback(pl.geom[i], s->work[i], d_Z + MN * i, Dn + MN * i,
                              pl.tau_default[i], shs[i], scale_stream(s, i));
    if (herr[i] == hipSuccess && ev)
      herr[i] = hipEventRecord(ev[4 + kEvPerScale * i + 4], scale_stream(s, i));
  }
  for (int oi = 0; oi < no; ++oi) {
    const int i = order[oi];
    if (herr[i] != hipSuccess) return dev_err(s, herr[i]);
    if (ev) s->round_launches[i] += rls[i];
    if (s->serial) continue;
    msld_status rs = join_scale(s, i);
    if (rs != MSLD_OK) return rs;
  }
  if (want_res) {
    double* part = reinterpret_cast<double*>(s->arena + pl.off_part);
    MSLD_TRY(s, launch_resid(Dc, Dn, R, d_Z, M, N, L, IM, s->ninst, part, pl.resid_parts,
                             dev_res(s), dev_res(s) + 2 * s->ninst, s->st));
  }
  if (stacked) MSLD_TRY(s, launch_inc_active(s->d_k, s->d_active, s->ninst, s->st));
  s->k += 1;
  s->cur = 1 - s->cur;
  return MSLD_OK;
}

msld_status step_iteration(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                           bool want_res) {
  if (want_res || !s->graph_on || s->prof_ev) return iterate_once(s, d_Y, ldY, d_Z, want_res);
  if (s->gY != d_Y || s->gZ != d_Z || s->gldY != ldY) {
    drop_graphs(s);
    s->gY = d_Y;
    s->gZ = d_Z;
    s->gldY = ldY;
  }
  const int c = s->cur;
  if (!s->gx[c]) {
    // captured on the solver's own stream (the null stream cannot be captured); the
    // graph is then launched on the caller's stream
    const int k0 = s->k;
    hipStream_t st0 = s->st;
    hipGraph_t g = nullptr;
    MSLD_TRY(s, hipStreamBeginCapture(s->cst, hipStreamCaptureModeThreadLocal));
    s->st = s->cst;
    const msld_status st = iterate_once(s, d_Y, ldY, d_Z, false);
    const hipError_t ec = hipStreamEndCapture(s->cst, &g);
    s->st = st0;
    s->k = k0;
    s->cur = c;
    if (st != MSLD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess || !g) return dev_err(s, ec != hipSuccess ? ec : hipErrorUnknown);
    const hipError_t ei = hipGraphInstantiate(&s->gx[c], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      s->gx[c] = nullptr;
      return dev_err(s, ei);
    }
  }
  MSLD_TRY(s, hipGraphLaunch(s->gx[c], s->st));
  s->k += 1;
  s->cur = 1 - s->cur;
  return MSLD_OK;
}

// ||Y_z||^2 of every instance into dres[ninst + z].
msld_status launch_ynorms(msld_solver* s, const float* d_Y, int64_t ldY) {
  double* part = reinterpret_cast<double*>(s->arena + s->plan.off_part);
  MSLD_TRY(s, launch_sumsq(d_Y, ldY, s->p.M, s->p.N, s->ninst, s->mask, s->ldmask, part,
                           s->plan.resid_parts, dev_res(s) + s->ninst, s->st));
  return MSLD_OK;
}

static msld_status reset_state(msld_solver* s, float* d_Z) {
  const size_t MN = plane_elems(s);
  MSLD_TRY(s, launch_fill(d_Z, 0.f, MN * s->p.L, s->st));
  MSLD_TRY(s, launch_fill(plane_D(s, 0), 0.f, MN * s->p.L, s->st));
  MSLD_TRY(s, launch_fill_ints(s->d_k, 0, (size_t)s->ninst, s->st));
  MSLD_TRY(s, launch_fill_ints(s->d_active, 1, (size_t)s->ninst, s->st));
  s->k = 0;
  s->cur = 0;
  return zero_stats(s);
}

// residuals of instance 0 after an iterate_once(..., want_res = true): the primal
// r_k = sqrt(sum_i ||X_i - Z_i'||^2) / ||Y||_F and the dual rho ||Z' - Z|| / ||Y||_F
static msld_status read_resid(msld_solver* s, const float* d_Y, int64_t ldY, double* out,
                              double* dual = nullptr) {
  msld_status st = launch_ynorms(s, d_Y, ldY);
  if (st != MSLD_OK) return st;
  const int n = s->ninst;
  MSLD_TRY(s, hipMemcpyAsync(s->host_res, dev_res(s), 24 * (size_t)n, hipMemcpyDeviceToHost,
                             s->st));
  MSLD_TRY(s, hipStreamSynchronize(s->st));
  const double ny2 = s->host_res[n] > 0 ? s->host_res[n] : 1.0;
  *out = std::sqrt(s->host_res[0] / ny2);
  if (dual) *dual = (double)s->p.rho * std::sqrt(s->host_res[2 * n] / ny2);
  return std::isfinite(*out) ? MSLD_OK : MSLD_ENUMERIC;
}

// ||Y||_F^2 of instance 0 must be finite: a NaN or Inf in Y is reported before any
// iteration runs (MSLD_ENUMERIC)
static msld_status check_y_finite(msld_solver* s, const float* d_Y, int64_t ldY) {
  msld_status st = launch_ynorms(s, d_Y, ldY);
  if (st != MSLD_OK) return st;
  MSLD_TRY(s, hipMemcpyAsync(s->host_res + s->ninst, dev_res(s) + s->ninst, 8,
                             hipMemcpyDeviceToHost, s->st));
  MSLD_TRY(s, hipStreamSynchronize(s->st));
  return std::isfinite(s->host_res[s->ninst]) ? MSLD_OK : MSLD_ENUMERIC;
}

static msld_status fill_stats(msld_solver* s, msld_result* info) {
  std::memset(info, 0, sizeof(*info));
  info->iters = s->k;
  info->primal_resid = -1.0;
  for (int i = 0; i < s->p.L; ++i) {
    unsigned long long st8[kStatsWords];
    MSLD_TRY(s, hipMemcpyAsync(st8, s->work[i].stats, sizeof(st8), hipMemcpyDeviceToHost, s->st));
    MSLD_TRY(s, hipStreamSynchronize(s->st));
    info->live[i] = st8[0];
    info->sweeps[i] = st8[1];
    info->rank[i] = st8[2];
    info->certified[i] = st8[3];
    info->fail_coupling[i] = st8[4];
    info->fail_bound[i] = st8[5];
    info->polar[i] = (uint64_t)s->work[i].stats_host[0];
    info->polar_steps[i] = (uint64_t)(s->work[i].stats_host[1] + s->work[i].stats_host[2]);
    info->undecided[i] = st8[6];
    info->cw_certified[i] = st8[7];
    info->gram_certified[i] = st8[8];
  }
  return MSLD_OK;
}

}  // namespace msld

extern "C" {

const char* msld_status_string(int32_t status) {
  switch (status) {
    case MSLD_OK: return "MSLD_OK";
    case MSLD_EINVAL: return "MSLD_EINVAL: invalid argument";
    case MSLD_ENOMEM: return "MSLD_ENOMEM: allocation failed";
    case MSLD_EDEVICE: return "MSLD_EDEVICE: HIP runtime error";
    case MSLD_ENUMERIC: return "MSLD_ENUMERIC: non-finite iterate";
    case MSLD_EBUSY: return "MSLD_EBUSY: busy";
    case MSLD_ETOOLARGE: return "MSLD_ETOOLARGE: beyond the fixed workspace of msld_bsvt_noalloc";
    default: return "MSLD_UNKNOWN";
  }
}

msld_status msld_default_lambda(int32_t M, int32_t N, int32_t m, int32_t n, float* out) {
  if (!out || M < 1 || N < 1 || m < 1 || n < 1 || m > M || n > N) return MSLD_EINVAL;
  *out = (float)lambda_default(M, N, m, n);
  return MSLD_OK;
}

msld_status msld_cycle_shift(uint64_t seed, int32_t k, int32_t i, int32_t m, int32_t n,
                             int32_t* sr, int32_t* sc) {
  if (!sr || !sc || k < 0 || i < 0 || i >= 16 || m < 1 || n < 1) return MSLD_EINVAL;
  int a, b;
  cycle_shift(seed, k, i, m, n, &a, &b);
  *sr = a;
  *sc = b;
  return MSLD_OK;
}

size_t msld_workspace_bytes(const msld_params* p) {
  Plan pl;
  if (make_plan(p, 1, &pl) != MSLD_OK) return 0;
  return pl.bytes;
}

msld_status msld_create(const msld_params* p, void* hip_stream, msld_solver** out) {
  return create_solver(p, 1, reinterpret_cast<hipStream_t>(hip_stream), out);
}

void msld_free(msld_solver* s) { destroy_solver(s); }

int32_t msld_scale_tier(const msld_solver* s, int32_t scale) {
  if (!s || scale < 0 || scale >= s->p.L) return -1;
  return s->plan.use_lr[scale] ? 4 : s->plan.tier[scale];
}

msld_status msld_reset(msld_solver* s, float* d_Z) {
  if (!s || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  return reset_state(s, d_Z);
}

msld_status msld_step(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z, int32_t count,
                      double* resid) {
  if (!s || !d_Y || !d_Z || count < 1) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (ldY < s->p.N) return MSLD_EINVAL;
  for (int c = 0; c < count; ++c) {
    msld_status st = step_iteration(s, d_Y, ldY, d_Z, resid != nullptr && c == count - 1);
    if (st != MSLD_OK) return st;
  }
  if (resid) return read_resid(s, d_Y, ldY, resid);
  return MSLD_OK;
}

msld_status msld_stats(msld_solver* s, msld_result* info) {
  if (!s || !info) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  return fill_stats(s, info);
}

msld_status msld_solve(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                       msld_result* info) {
  if (!s || !d_Y || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  const msld_params& p = s->p;
  if (ldY < p.N) return MSLD_EINVAL;
  msld_status st = reset_state(s, d_Z);
  if (st != MSLD_OK) return st;
  double resid = -1.0, dual = -1.0;
  msld_status result = check_y_finite(s, d_Y, ldY);
  for (int k = 0; k < p.max_iters && result == MSLD_OK; ++k) {
    const int iters = k + 1;
    const bool check = p.tol > 0.f && (iters % p.check_every == 0);
    const bool last = iters == p.max_iters;
    const bool want = check || (last && info);
    st = step_iteration(s, d_Y, ldY, d_Z, want);
    if (st != MSLD_OK) return st;
    if (want) {
      result = read_resid(s, d_Y, ldY, &resid, &dual);
      if (result != MSLD_OK) break;
      if (check && resid <= (double)p.tol) break;
    }
  }
  if (result == MSLD_EDEVICE) return result;
  if (info) {
    st = fill_stats(s, info);
    if (st != MSLD_OK) return st;
    info->primal_resid = resid;
    info->dual_resid = dual;
    info->status = result;
  }
  return result;
}

msld_status msld_profile_begin(msld_solver* s, int32_t max_iters) {
  if (!s || max_iters < 1) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (s->prof_ev) return MSLD_EINVAL;
  const size_t per = 4 + kEvPerScale * (size_t)s->p.L;
  const size_t n = per * (size_t)max_iters;
  s->prof_ev = static_cast<hipEvent_t*>(std::calloc(n, sizeof(hipEvent_t)));
  if (!s->prof_ev) return MSLD_ENOMEM;
  for (size_t e = 0; e < n; ++e)
    if (hipEventCreate(&s->prof_ev[e]) != hipSuccess) {
      for (size_t f = 0; f < e; ++f) (void)hipEventDestroy(s->prof_ev[f]);
      std::free(s->prof_ev);
      s->prof_ev = nullptr;
      return MSLD_EDEVICE;
    }
  s->prof_cap = max_iters;
  s->prof_n = 0;
  for (int i = 0; i < MSLD_MAX_SCALES; ++i) s->round_launches[i] = 0;
  return MSLD_OK;
}

msld_status msld_profile_end(msld_solver* s, double* ms, int64_t* round_launches,
                             int32_t* iters_recorded) {
  if (!s || !ms || !round_launches || !iters_recorded) return MSLD_EINVAL;
  if (!s->prof_ev) return MSLD_EINVAL;
  const int L = s->p.L;
  const size_t per = 4 + kEvPerScale * (size_t)L;
  msld_status result = MSLD_OK;
  if (hipStreamSynchronize(s->st) != hipSuccess) result = dev_err(s, hipErrorUnknown);
  for (int i = 0; i < 4 * (L + 1) + L; ++i) ms[i] = 0.0;
  for (int it = 0; it < s->prof_n && result == MSLD_OK; ++it) {
    hipEvent_t* ev = s->prof_ev + (size_t)it * per;
    float t;
    if (hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) ms[4 * L] += t;
    if (s->sall.n > 0 && hipEventElapsedTime(&t, ev[2], ev[3]) == hipSuccess) ms[4 * L + 1] += t;
    for (int i = 0; i < L; ++i) {
      if (s->plan.tier[i] == TIER_1X1) continue;
      hipEvent_t* e5 = ev + 4 + kEvPerScale * i;
      for (int j = 0; j < 4; ++j)
        if (hipEventElapsedTime(&t, e5[j], e5[j + 1]) == hipSuccess) ms[4 * i + j] += t;
      // the Gram kernel of a low-rank tier (events 5 and 6; never recorded otherwise)
      if (s->work[i].use_lr && hipEventElapsedTime(&t, e5[5], e5[6]) == hipSuccess)
        ms[4 * (L + 1) + i] += t;
    }
  }
  for (int i = 0; i < L; ++i) round_launches[i] = s->round_launches[i];
  *iters_recorded = s->prof_n;
  for (size_t e = 0; e < per * (size_t)s->prof_cap; ++e) (void)hipEventDestroy(s->prof_ev[e]);
  std::free(s->prof_ev);
  s->prof_ev = nullptr;
  s->prof_cap = s->prof_n = 0;
  return result;
}

msld_status msld_set_mask(msld_solver* s, const uint8_t* d_mask, int64_t ldmask) {
  if (!s) return MSLD_EINVAL;
  if (s->ninst != 1) return MSLD_EINVAL;
  if (d_mask && ldmask < s->p.N) return MSLD_EINVAL;
  s->mask = d_mask;
  s->ldmask = d_mask ? ldmask : 0;
  drop_graphs(s);   // captured iterations hold the previous mask
  return MSLD_OK;
}

int32_t msld_set_graph(msld_solver* s, int32_t enable) {
  if (!s) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (hipStreamSynchronize(s->st) != hipSuccess) return dev_err(s, hipErrorUnknown);
  drop_graphs(s);
  s->graph_on = s->graphable && enable != 0;
  return s->graph_on ? 1 : 0;
}

msld_status msld_bsvt(msld_solver* s, int32_t scale, const float* d_V, float* d_Z, float tau,
                      int32_t sr, int32_t sc) {
  if (!s || !d_V || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (s->ninst != 1 || scale < 0 || scale >= s->p.L) return MSLD_EINVAL;
  const ScaleGeom& g = s->plan.geom[scale];
  if (sr < 0 || sr >= g.m || sc < 0 || sc >= g.n) return MSLD_EINVAL;
  if (!(tau >= 0.f) || !std::isfinite(tau)) return MSLD_EINVAL;
  const size_t MN = (size_t)g.M * g.N;
  float* Dws = plane_D(s, 0) + MN * scale;
  ShiftSpec sh;
  std::memset(&sh, 0, sizeof(sh));
  sh.scale = scale;
  sh.mode = 2;
  sh.sr = sr;
  sh.sc = sc;
  if (s->plan.tier[scale] == TIER_1X1) {
    // 1x1 blocks: the entrywise soft-threshold of the consensus kernel, run with
    // L = 1, Y = V, an all-zero D plane and an all-zero Z plane: R = V and
    // Z' = soft(R, tau). The second D buffer serves as the Z plane.
    float* Zp = plane_D(s, 1);
    int idx0 = 0;
    float t0 = tau;
    MSLD_TRY(s, launch_fill(Dws, 0.f, MN, s->st));
    MSLD_TRY(s, launch_fill(Zp, 0.f, MN, s->st));
    MSLD_TRY(s, launch_consensus(d_V, g.N, Dws, Dws, Zp, plane_R(s), g.M, g.N, 1, &idx0, &t0, 1,
                                 g.M, nullptr, nullptr, 0, s->st));
    MSLD_TRY(s, hipMemcpyAsync(d_Z, Zp, MN * 4, hipMemcpyDeviceToDevice, s->st));
    return MSLD_OK;
  }
  msld_status zs = zero_stats(s);
  if (zs != MSLD_OK) return zs;
  MSLD_TRY(s, hipEventRecord(s->ev_fork, s->st));
  msld_status rs = fork_scale(s, scale);
  if (rs == MSLD_OK) rs = run_scale(s, scale, d_V, nullptr, d_Z, Dws, tau, sh, nullptr, false);
  if (rs == MSLD_OK) rs = join_scale(s, scale);
  return rs;
}

msld_status msld_device_shifts(msld_solver* s, int32_t k0, int32_t count, int32_t* out) {
  if (!s || !out || count < 1 || count > 1024 || k0 < 0) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  int* d = reinterpret_cast<int*>(s->arena + s->plan.off_shift);
  MSLD_TRY(s, launch_device_shifts(s->p.shift_seed, k0, count, s->p.L, s->p.block_m,
                                   s->p.block_n, d, s->st));
  MSLD_TRY(s, hipMemcpyAsync(out, d, sizeof(int) * 2 * s->p.L * count, hipMemcpyDeviceToHost,
                             s->st));
  MSLD_TRY(s, hipStreamSynchronize(s->st));
  return MSLD_OK;
}

// ------------------------------------------------------------------ batches
// Many independent decompositions solved together: instances whose parameters agree
// except for the shift seed form a class and are stacked along the rows of one set
// of planes, so every kernel of an iteration is launched once per class for all of
// its instances (and the Gram / power GEMMs of the low-rank path are batched across
// instances). Each instance keeps its own seed, iteration counter and residual.
struct msld_batch {
  struct Cls {
    msld_params p;
    std::vector<int> members;   // instance ids in slot order
    msld_solver* s;
    float* Y;                   // stacked Y (members x M x N)
    float* Z;                   // stacked Z (L planes)
    hipStream_t st;             // the class's own stream (classes run concurrently)
    hipEvent_t done;            // end of the class's work in a solve
  };
  int n;
  hipStream_t st;
  hipEvent_t ev_in = nullptr;   // the caller's stream position at the start of a solve
  std::vector<Cls> cls;
  std::vector<int> cls_of, slot_of;
};

static void batch_destroy(msld_batch* b) {
  if (!b) return;
  for (auto& c : b->cls) {
    if (c.s) destroy_solver(c.s);
    if (c.Y) (void)hipFree(c.Y);
    if (c.Z) (void)hipFree(c.Z);
    if (c.done) (void)hipEventDestroy(c.done);
    if (c.st) (void)hipStreamDestroy(c.st);
  }
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  delete b;
}

}  // extern "C"

// One class of a batch solve, on the class's stream: gather its instances, iterate,
// scatter the components, fill the instances' results. MSLD_ENUMERIC when an instance
// ended with a non-finite residual (the others still finish).
static msld_status batch_solve_class(msld_batch* b, size_t ci, const float* const* d_Y,
                                     const int64_t* ldY, float* const* d_Z, msld_result* info) {
  auto& c = b->cls[ci];
  msld_solver* s = c.s;
  const msld_params& p = c.p;
  const int ni = (int)c.members.size();
  const size_t inst = (size_t)p.M * p.N;
  const size_t MN = inst * ni;
  MSLD_TRY(s, hipSetDevice(s->device));   // the calling thread may be a fresh worker
  MSLD_TRY(s, hipStreamWaitEvent(c.st, b->ev_in, 0));
  for (int z = 0; z < ni; ++z) {
    const int i = c.members[z];
    MSLD_TRY(s, hipMemcpy2DAsync(c.Y + inst * z, 4 * (size_t)p.N, d_Y[i], 4 * (size_t)ldY[i],
                                 4 * (size_t)p.N, p.M, hipMemcpyDeviceToDevice, c.st));
  }
  msld_status st = reset_state(s, c.Z);
  if (st != MSLD_OK) return st;
  st = launch_ynorms(s, c.Y, p.N);
  if (st != MSLD_OK) return st;
  std::vector<int> active(ni, 1), iters(ni, 0);
  std::vector<double> resid(ni, -1.0);
  std::vector<int32_t> status(ni, MSLD_OK);
  int n_active = ni;
  for (int k = 0; k < p.max_iters && n_active > 0; ++k) {
    const bool check = (p.tol > 0.f && (k + 1) % p.check_every == 0) || k + 1 == p.max_iters;
    st = step_iteration(s, c.Y, p.N, c.Z, check);
    if (st != MSLD_OK) return st;
    for (int z = 0; z < ni; ++z)
      if (active[z]) iters[z] = k + 1;
    if (!check) continue;
    MSLD_TRY(s, hipMemcpyAsync(s->host_res, dev_res(s), 16 * (size_t)ni, hipMemcpyDeviceToHost,
                               c.st));
    MSLD_TRY(s, hipStreamSynchronize(c.st));
    for (int z = 0; z < ni; ++z) {
      if (!active[z]) continue;
      const double ny2 = s->host_res[ni + z] > 0 ? s->host_res[ni + z] : 1.0;
      resid[z] = std::sqrt(s->host_res[z] / ny2);
      const bool bad = !std::isfinite(resid[z]);
      if (bad || (p.tol > 0.f && resid[z] <= (double)p.tol)) {
        if (bad) status[z] = MSLD_ENUMERIC;
        active[z] = 0;
        --n_active;
        MSLD_TRY(s, launch_set_int(s->d_active, z, 0, c.st));
      }
    }
  }
  msld_status result = MSLD_OK;
  for (int z = 0; z < ni; ++z) {
    const int i = c.members[z];
    for (int l = 0; l < p.L; ++l)
      MSLD_TRY(s, hipMemcpyAsync(d_Z[i] + inst * l, c.Z + MN * l + inst * z, 4 * inst,
                                 hipMemcpyDeviceToDevice, c.st));
    if (status[z] != MSLD_OK) result = (msld_status)status[z];
  }
  if (info) {
    msld_result cls_info;
    st = fill_stats(s, &cls_info);
    if (st != MSLD_OK) return st;
    for (int z = 0; z < ni; ++z) {
      msld_result& r = info[c.members[z]];
      r = cls_info;   // per-class kernel counters (shared by the class's instances)
      r.iters = iters[z];
      r.primal_resid = resid[z];
      r.status = status[z];
    }
  }
  return result;
}

extern "C" {

msld_status msld_batch_create(int32_t n, const msld_params* params, void* hip_stream,
                              msld_batch** out) {
  if (!out || n < 1 || !params) return MSLD_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (validate_params(&params[i]) != MSLD_OK) return MSLD_EINVAL;
  msld_batch* b = new (std::nothrow) msld_batch();
  if (!b) return MSLD_ENOMEM;
  b->n = n;
  b->st = reinterpret_cast<hipStream_t>(hip_stream);
  b->cls_of.assign(n, -1);
  b->slot_of.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    int c = -1;
    for (size_t j = 0; j < b->cls.size(); ++j)
      if (same_class(b->cls[j].p, params[i])) {
        c = (int)j;
        break;
      }
    if (c < 0) {
      msld_batch::Cls nc;
      nc.p = params[i];
      nc.s = nullptr;
      nc.Y = nc.Z = nullptr;
      nc.st = nullptr;
      nc.done = nullptr;
      b->cls.push_back(nc);
      c = (int)b->cls.size() - 1;
    }
    b->cls_of[i] = c;
    b->slot_of[i] = (int)b->cls[c].members.size();
    b->cls[c].members.push_back(i);
  }
  if (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess) {
    b->ev_in = nullptr;
    batch_destroy(b);
    return MSLD_EDEVICE;
  }
  for (auto& c : b->cls) {
    const int ni = (int)c.members.size();
    if (hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) {
      batch_destroy(b);
      return MSLD_EDEVICE;
    }
    msld_status st = create_solver(&c.p, ni, c.st, &c.s);
    if (st != MSLD_OK) {
      batch_destroy(b);
      return st;
    }
    const size_t MN = (size_t)c.p.M * c.p.N * ni;
    if (hipMalloc(&c.Y, 4 * MN) != hipSuccess || hipMalloc(&c.Z, 4 * MN * c.p.L) != hipSuccess) {
      batch_destroy(b);
      return MSLD_ENOMEM;
    }
    std::vector<unsigned long long> seeds(ni);
    for (int z = 0; z < ni; ++z) seeds[z] = params[c.members[z]].shift_seed;
    if (hipMemcpy(c.s->d_seed, seeds.data(), 8 * (size_t)ni, hipMemcpyHostToDevice) !=
        hipSuccess) {
      batch_destroy(b);
      return MSLD_EDEVICE;
    }
  }
  *out = b;
  return MSLD_OK;
}

int32_t msld_batch_classes(const msld_batch* b) { return b ? (int32_t)b->cls.size() : -1; }

msld_status msld_batch_solve(msld_batch* b, const float* const* d_Y, const int64_t* ldY,
                             float* const* d_Z, msld_result* info) {
  if (!b || !d_Y || !ldY || !d_Z) return MSLD_EINVAL;
  for (int i = 0; i < b->n; ++i) {
    const msld_params& p = b->cls[b->cls_of[i]].p;
    if (!d_Y[i] || !d_Z[i] || ldY[i] < p.N) return MSLD_EINVAL;
  }
  if (info) std::memset(info, 0, sizeof(msld_result) * b->n);
  // every class starts after the caller's prior work on its stream, runs on its own
  // stream from its own host thread (a class's host waits do not hold back the others),
  // and the caller's stream waits for all of them at the end
  if (hipEventRecord(b->ev_in, b->st) != hipSuccess) return MSLD_EDEVICE;
  std::vector<msld_status> cres(b->cls.size(), MSLD_OK);
  auto run_class = [&](size_t ci) { cres[ci] = batch_solve_class(b, ci, d_Y, ldY, d_Z, info); };
  std::vector<std::thread> workers;
  for (size_t ci = 1; ci < b->cls.size(); ++ci) {
    try {
      workers.emplace_back(run_class, ci);
    } catch (...) {
      run_class(ci);   // no thread available: run it here
    }
  }
  if (!b->cls.empty()) run_class(0);
  for (auto& t : workers) t.join();
  msld_status result = MSLD_OK;
  for (size_t ci = 0; ci < b->cls.size(); ++ci) {
    auto& c = b->cls[ci];
    if (cres[ci] != MSLD_OK && (result == MSLD_OK || result == MSLD_ENUMERIC)) result = cres[ci];
    if (hipEventRecord(c.done, c.st) != hipSuccess ||
        hipStreamWaitEvent(b->st, c.done, 0) != hipSuccess)
      result = MSLD_EDEVICE;
  }
  if (hipStreamSynchronize(b->st) != hipSuccess) return MSLD_EDEVICE;
  return result;
}

void msld_batch_free(msld_batch* b) { batch_destroy(b); }

}  // extern "C"
