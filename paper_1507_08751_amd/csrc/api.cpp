// C-ABI runtime: parameter validation, per-scale planning, workspace arena and the
// ADMM driver loop (Sec. 7 eq:admm with the random cycle spinning of Sec. 9).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/msld.h"
#include "msld_internal.h"

using namespace msld;

namespace msld {
int lds_tier_threads(int nb, int mb, int* G);
size_t lds_tier_bytes(int mb, int nb);
size_t stream_lds_bytes(int m, const StreamPlan& sp);
}  // namespace msld

namespace {

constexpr size_t kLdsTierMax = 150 * 1024;   // LDS budget of one workgroup (160 KiB per CU)
constexpr int kStreamFloats = 16384;         // stream-pass tile budget (floats)
constexpr int kResidParts = 1024;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

struct Plan {
  ScaleGeom geom[MSLD_MAX_SCALES];
  StreamPlan sp[MSLD_MAX_SCALES];
  int tier[MSLD_MAX_SCALES];
  int pw[MSLD_MAX_SCALES];
  int nbp[MSLD_MAX_SCALES];
  float tau_default[MSLD_MAX_SCALES];
  size_t bytes;
  // byte offsets inside the arena
  size_t off_R, off_D, off_part, off_res, off_shift;
  size_t off_count[MSLD_MAX_SCALES], off_list[MSLD_MAX_SCALES], off_rowp[MSLD_MAX_SCALES],
      off_frop[MSLD_MAX_SCALES], off_stats[MSLD_MAX_SCALES], off_pA[MSLD_MAX_SCALES],
      off_pW[MSLD_MAX_SCALES], off_pflag[MSLD_MAX_SCALES], off_pg[MSLD_MAX_SCALES];
  int use_lr[MSLD_MAX_SCALES];
  size_t off_lr[MSLD_MAX_SCALES];   // start of the low-rank buffers of the scale
};

constexpr int kLRP = 16;  // subspace width of the certified low-rank path

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

msld_status validate(const msld_params* p) {
  if (!p) return MSLD_EINVAL;
  if (p->M < 1 || p->N < 1 || p->M > (1 << 20) || p->N > (1 << 20)) return MSLD_EINVAL;
  if ((int64_t)p->M * p->N >= ((int64_t)1 << 31)) return MSLD_EINVAL;
  if (p->L < 1 || p->L > MSLD_MAX_SCALES) return MSLD_EINVAL;
  if (!(p->rho > 0.f) || !std::isfinite(p->rho)) return MSLD_EINVAL;
  if (p->max_iters < 1) return MSLD_EINVAL;
  if (!(p->tol >= 0.f) || !std::isfinite(p->tol)) return MSLD_EINVAL;
  if (p->check_every < 1) return MSLD_EINVAL;
  if (p->cycle_spin != 0 && p->cycle_spin != 1) return MSLD_EINVAL;
  for (int i = 0; i < p->L; ++i) {
    const int m = p->block_m[i], n = p->block_n[i];
    if (m < 1 || n < 1 || p->M % m || p->N % n) return MSLD_EINVAL;
    if (!std::isfinite(p->lambda[i])) return MSLD_EINVAL;
  }
  return MSLD_OK;
}

msld_status make_plan(const msld_params* p, Plan* pl) {
  msld_status st = validate(p);
  if (st != MSLD_OK) return st;
  std::memset(pl, 0, sizeof(*pl));
  const int M = p->M, N = p->N, L = p->L;
  const size_t MN = (size_t)M * N;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + (bytes ? bytes : 1), 256);
    return o;
  };
  pl->off_R = take(4 * MN);
  pl->off_D = take(4 * MN * (size_t)L * 2);
  pl->off_part = take(8 * (size_t)kResidParts);
  pl->off_res = take(8 * 4);
  pl->off_shift = take(4 * 2 * (size_t)L * 1024);
  for (int i = 0; i < L; ++i) {
    const int m = p->block_m[i], n = p->block_n[i];
    ScaleGeom& g = pl->geom[i];
    g.M = M; g.N = N; g.m = m; g.n = n; g.P = M / m; g.Q = N / n;
    g.trans = m < n ? 1 : 0;
    g.mb = m < n ? n : m;
    g.nb = m < n ? m : n;
    const double lam = p->lambda[i] > 0.f ? (double)p->lambda[i] : lambda_default(M, N, m, n);
    pl->tau_default[i] = (float)(lam / (double)p->rho);
    const int nblk = g.P * g.Q;
    const int lr_min = p->lowrank_min == 0 ? 128 : p->lowrank_min;
    const bool lr = lr_min > 0 && g.nb >= lr_min && g.nb >= 4 * kLRP;
    int tier;
    if (m == 1 && n == 1) tier = TIER_1X1;
    else if (m == n && (m == 2 || m == 4 || m == 8)) tier = TIER_REG;
    else if (!lr && lds_fits(g.mb, g.nb)) tier = TIER_LDS;
    else tier = TIER_PANEL;
    pl->use_lr[i] = lr ? 1 : 0;
    pl->tier[i] = tier;
    pl->off_stats[i] = take(8 * 8);
    if (tier == TIER_1X1) continue;
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
    if (stream_lds_bytes(m, sp) > kLdsTierMax) return MSLD_EINVAL;
    pl->off_count[i] = take(4);
    pl->off_list[i] = take(4 * (size_t)nblk);
    if (!sp.whole) {
      pl->off_rowp[i] = take(4 * (size_t)nblk * sp.spb * m);
      pl->off_frop[i] = take(4 * (size_t)nblk * sp.spb);
    }
    if (tier == TIER_PANEL) {
      // panel width: two panels of A (mb rows) and W (nb rows) in LDS; 4 <= pw <= 64
      int pw = (int)(kLdsTierMax / 4 / (2 * ((size_t)(g.mb | 1) + (size_t)(g.nb | 1))));
      if (pw > 64) pw = 64;
      pw = pow2_floor(pw < 1 ? 1 : pw);
      while (pw > 4 && 2 * pw > g.nb) pw >>= 1;
      if (pw < 4 || g.nb > 4096) return MSLD_EINVAL;  // beyond the panel tier's limits
      const int nbp = (g.nb + 2 * pw - 1) / (2 * pw) * (2 * pw);
      pl->pw[i] = pw;
      pl->nbp[i] = nbp;
      pl->off_pA[i] = take(4 * (size_t)nblk * nbp * g.mb);
      pl->off_pW[i] = take(4 * (size_t)nblk * nbp * g.nb);
      pl->off_pflag[i] = take(4 * 4 * (size_t)nblk);
      pl->off_pg[i] = take(4 * (size_t)nblk * nbp);
      if (lr) {
        const size_t nb2 = (size_t)g.nb * g.nb;
        const size_t per = 3 * nb2 + 4 * (size_t)g.nb * kLRP + (size_t)g.mb * kLRP +
                           (size_t)kLRP * g.nb + 2 * kLRP + 8;
        pl->off_lr[i] = take(4 * ((size_t)nblk * per + (size_t)g.nb * kLRP + 64 + nblk));
      }
    }
  }
  pl->bytes = off;
  return MSLD_OK;
}

}  // namespace

struct msld_solver {
  msld_params p;
  Plan plan;
  hipStream_t st;
  int device;
  int num_cus;
  bool failed;
  char* arena;
  double* host_res;  // pinned, 4 doubles
  int* host_ints;    // pinned, 2 per scale
  rocblas_handle blas;
  ScaleWork work[MSLD_MAX_SCALES];
  int k;              // next iteration index (drives the cycle-spin shifts)
  int cur;            // which D buffer holds the current D_i
  // profiling: per iteration 2 consensus events + 5 events per scale
  int prof_cap, prof_n;
  hipEvent_t* prof_ev;
  int64_t round_launches[MSLD_MAX_SCALES];
};

namespace {

msld_status dev_err(msld_solver* s, hipError_t e) {
  if (e == hipSuccess) return MSLD_OK;
  if (s) s->failed = true;
  return MSLD_EDEVICE;
}

#define MSLD_TRY(s, call)                              \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return dev_err((s), e_);     \
  } while (0)

float jacobi_tol(int mb) { return 4.0f * 5.9604645e-8f * std::sqrt((float)mb); }

msld_status run_scale(msld_solver* s, int i, const float* Zin, const float* R, float* Zout,
                      float* Dout, float tau, const ShiftSpec& sh, hipEvent_t* ev) {
  const Plan& pl = s->plan;
  const ScaleGeom& g = pl.geom[i];
  int rl = 0;
  MSLD_TRY(s, launch_scale(g, pl.tier[i], pl.sp[i], s->work[i], Zin, R, Zout, Dout, tau, sh,
                           jacobi_tol(g.mb), 40, 20, s->num_cus, s->st, ev, &rl));
  if (ev) s->round_launches[i] += rl;
  return MSLD_OK;
}

}  // namespace

extern "C" {

const char* msld_status_string(int32_t status) {
  switch (status) {
    case MSLD_OK: return "MSLD_OK";
    case MSLD_EINVAL: return "MSLD_EINVAL: invalid argument";
    case MSLD_ENOMEM: return "MSLD_ENOMEM: allocation failed";
    case MSLD_EDEVICE: return "MSLD_EDEVICE: HIP runtime error";
    case MSLD_ENUMERIC: return "MSLD_ENUMERIC: non-finite iterate";
    case MSLD_EBUSY: return "MSLD_EBUSY: busy";
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
  if (make_plan(p, &pl) != MSLD_OK) return 0;
  return pl.bytes;
}

msld_status msld_create(const msld_params* p, void* hip_stream, msld_solver** out) {
  if (!out) return MSLD_EINVAL;
  *out = nullptr;
  msld_solver* s = new (std::nothrow) msld_solver();
  if (!s) return MSLD_ENOMEM;
  msld_status st = make_plan(p, &s->plan);
  if (st != MSLD_OK) {
    delete s;
    return st;
  }
  s->p = *p;
  s->st = reinterpret_cast<hipStream_t>(hip_stream);
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
    delete s;
    return MSLD_ENOMEM;
  }
  if (hipHostMalloc(&s->host_res, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(s->arena);
    delete s;
    return MSLD_ENOMEM;
  }
  if (hipHostMalloc(&s->host_ints, 2 * MSLD_MAX_SCALES * sizeof(int), hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipHostFree(s->host_res);
    (void)hipFree(s->arena);
    delete s;
    return MSLD_ENOMEM;
  }
  bool need_blas = false;
  for (int i = 0; i < p->L; ++i) need_blas = need_blas || s->plan.use_lr[i];
  s->blas = nullptr;
  if (need_blas) {
    if (rocblas_create_handle(&s->blas) != rocblas_status_success ||
        rocblas_set_stream(s->blas, s->st) != rocblas_status_success ||
        rocblas_set_atomics_mode(s->blas, rocblas_atomics_not_allowed) != rocblas_status_success) {
      if (s->blas) (void)rocblas_destroy_handle(s->blas);
      (void)hipHostFree(s->host_ints);
      (void)hipHostFree(s->host_res);
      (void)hipFree(s->arena);
      delete s;
      return MSLD_EDEVICE;
    }
  }
  const Plan& pl = s->plan;
  for (int i = 0; i < p->L; ++i) {
    ScaleWork& w = s->work[i];
    std::memset(&w, 0, sizeof(w));
    w.stats = reinterpret_cast<unsigned long long*>(s->arena + pl.off_stats[i]);
    if (pl.tier[i] != TIER_1X1) {
      w.live_count = reinterpret_cast<int*>(s->arena + pl.off_count[i]);
      w.live_list = reinterpret_cast<int*>(s->arena + pl.off_list[i]);
      if (!pl.sp[i].whole) {
        w.rowpart = reinterpret_cast<float*>(s->arena + pl.off_rowp[i]);
        w.fropart = reinterpret_cast<float*>(s->arena + pl.off_frop[i]);
      }
    }
    if (pl.tier[i] == TIER_PANEL) {
      w.pA = reinterpret_cast<float*>(s->arena + pl.off_pA[i]);
      w.pW = reinterpret_cast<float*>(s->arena + pl.off_pW[i]);
      w.pflag = reinterpret_cast<int*>(s->arena + pl.off_pflag[i]);
      w.pg = reinterpret_cast<float*>(s->arena + pl.off_pg[i]);
      w.slots = pl.geom[i].P * pl.geom[i].Q;
      w.nbp = pl.nbp[i];
      w.pw = pl.pw[i];
      w.hostInts = s->host_ints + 2 * i;
      if (pl.use_lr[i]) {
        const ScaleGeom& g = pl.geom[i];
        const size_t nb2 = (size_t)g.nb * g.nb;
        const size_t slots = (size_t)w.slots;
        float* f = reinterpret_cast<float*>(s->arena + pl.off_lr[i]);
        w.use_lr = 1;
        w.blas = s->blas;
        w.lrG = f; f += slots * nb2;
        w.lrP = f; f += slots * nb2;
        w.lrQ = f; f += slots * nb2;
        w.lrY = f; f += slots * g.nb * kLRP;
        w.lrX = f; f += slots * g.nb * kLRP;
        w.lrW = f; f += slots * g.nb * kLRP;
        w.lrV = f; f += slots * g.nb * kLRP;
        w.lrC = f; f += slots * g.mb * kLRP;
        w.lrT = f; f += slots * kLRP * g.nb;
        w.lrSig = f; f += 2 * slots * kLRP;   // sigma, then the deflation mask
        w.lrScal = f; f += slots * 8;
        w.lrOm = f; f += (size_t)g.nb * kLRP;
        w.lrCount = reinterpret_cast<int*>(f);
        w.lrFall = w.lrCount + 64;
        w.lds_fallback = lds_fits(g.mb, g.nb) ? 1 : 0;
      }
    }
  }
  *out = s;
  return MSLD_OK;
}

void msld_free(msld_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  if (s->prof_ev) {
    for (size_t e = 0; e < (2 + 5 * (size_t)s->p.L) * (size_t)s->prof_cap; ++e)
      (void)hipEventDestroy(s->prof_ev[e]);
    std::free(s->prof_ev);
  }
  if (s->blas) (void)rocblas_destroy_handle(s->blas);
  if (s->arena) (void)hipFree(s->arena);
  if (s->host_res) (void)hipHostFree(s->host_res);
  if (s->host_ints) (void)hipHostFree(s->host_ints);
  delete s;
}

int32_t msld_scale_tier(const msld_solver* s, int32_t scale) {
  if (!s || scale < 0 || scale >= s->p.L) return -1;
  return s->plan.use_lr[scale] ? 4 : s->plan.tier[scale];
}

static msld_status zero_stats(msld_solver* s) {
  for (int i = 0; i < s->p.L; ++i)
    MSLD_TRY(s, hipMemsetAsync(s->work[i].stats, 0, 8 * 8, s->st));
  return MSLD_OK;
}

static float* plane_R(msld_solver* s) {
  return reinterpret_cast<float*>(s->arena + s->plan.off_R);
}

static float* plane_D(msld_solver* s, int which) {
  const size_t MN = (size_t)s->p.M * s->p.N;
  return reinterpret_cast<float*>(s->arena + s->plan.off_D) + (size_t)which * MN * s->p.L;
}

msld_status msld_reset(msld_solver* s, float* d_Z) {
  if (!s || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  const size_t MN = (size_t)s->p.M * s->p.N;
  MSLD_TRY(s, launch_fill(d_Z, 0.f, MN * s->p.L, s->st));
  MSLD_TRY(s, launch_fill(plane_D(s, 0), 0.f, MN * s->p.L, s->st));
  s->k = 0;
  s->cur = 0;
  return zero_stats(s);
}

// One ADMM iteration k = s->k (eq:admm), D buffers ping-pong; when want_res the
// residual r_k is computed on device into dres[0].
static msld_status iterate_once(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                                bool want_res) {
  const msld_params& p = s->p;
  const Plan& pl = s->plan;
  const int M = p.M, N = p.N, L = p.L;
  const size_t MN = (size_t)M * N;
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
    ev = s->prof_ev + (size_t)s->prof_n * (2 + 5 * L);
    ++s->prof_n;
    MSLD_TRY(s, hipEventRecord(ev[0], s->st));
  }
  MSLD_TRY(s, launch_consensus(d_Y, ldY, Dc, Dn, d_Z, R, M, N, L, scales1, taus1, n1, s->st));
  if (ev) MSLD_TRY(s, hipEventRecord(ev[1], s->st));
  for (int i = 0; i < L; ++i) {
    if (pl.tier[i] == TIER_1X1) continue;
    ShiftSpec sh;
    sh.seed = p.shift_seed;
    sh.k = s->k;
    sh.scale = i;
    sh.mode = p.cycle_spin ? 1 : 0;
    sh.sr = sh.sc = 0;
    float* Zi = d_Z + MN * i;
    msld_status rs = run_scale(s, i, Zi, R, Zi, Dn + MN * i, pl.tau_default[i], sh,
                               ev ? ev + 2 + 5 * i : nullptr);
    if (rs != MSLD_OK) return rs;
  }
  if (want_res) {
    double* part = reinterpret_cast<double*>(s->arena + pl.off_part);
    double* dres = reinterpret_cast<double*>(s->arena + pl.off_res);
    MSLD_TRY(s, launch_resid(Dc, R, d_Z, M, N, L, part, kResidParts, dres, s->st));
  }
  s->k += 1;
  s->cur = 1 - s->cur;
  return MSLD_OK;
}

static msld_status read_resid(msld_solver* s, const float* d_Y, int64_t ldY, double* out) {
  const Plan& pl = s->plan;
  double* part = reinterpret_cast<double*>(s->arena + pl.off_part);
  double* dres = reinterpret_cast<double*>(s->arena + pl.off_res);
  MSLD_TRY(s, launch_sumsq(d_Y, ldY, s->p.M, s->p.N, part, kResidParts, dres + 1, s->st));
  MSLD_TRY(s, hipMemcpyAsync(s->host_res, dres, 16, hipMemcpyDeviceToHost, s->st));
  MSLD_TRY(s, hipStreamSynchronize(s->st));
  const double ny2 = s->host_res[1] > 0 ? s->host_res[1] : 1.0;
  *out = std::sqrt(s->host_res[0] / ny2);
  return std::isfinite(*out) ? MSLD_OK : MSLD_ENUMERIC;
}

msld_status msld_step(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z, int32_t count,
                      double* resid) {
  if (!s || !d_Y || !d_Z || count < 1) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (ldY < s->p.N) return MSLD_EINVAL;
  for (int c = 0; c < count; ++c) {
    msld_status st = iterate_once(s, d_Y, ldY, d_Z, resid != nullptr && c == count - 1);
    if (st != MSLD_OK) return st;
  }
  if (resid) return read_resid(s, d_Y, ldY, resid);
  return MSLD_OK;
}

msld_status msld_stats(msld_solver* s, msld_result* info) {
  if (!s || !info) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  std::memset(info, 0, sizeof(*info));
  info->iters = s->k;
  info->primal_resid = -1.0;
  for (int i = 0; i < s->p.L; ++i) {
    unsigned long long st8[8];
    MSLD_TRY(s, hipMemcpyAsync(st8, s->work[i].stats, sizeof(st8), hipMemcpyDeviceToHost, s->st));
    MSLD_TRY(s, hipStreamSynchronize(s->st));
    info->live[i] = st8[0];
    info->sweeps[i] = st8[1];
    info->rank[i] = st8[2];
    info->certified[i] = st8[3];
    info->fail_coupling[i] = st8[4];
    info->fail_bound[i] = st8[5];
  }
  return MSLD_OK;
}

msld_status msld_solve(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                       msld_result* info) {
  if (!s || !d_Y || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  const msld_params& p = s->p;
  if (ldY < p.N) return MSLD_EINVAL;
  msld_status st = msld_reset(s, d_Z);
  if (st != MSLD_OK) return st;
  double resid = -1.0;
  msld_status result = MSLD_OK;
  for (int k = 0; k < p.max_iters; ++k) {
    const int iters = k + 1;
    const bool check = p.tol > 0.f && (iters % p.check_every == 0);
    const bool last = iters == p.max_iters;
    const bool want = check || (last && info);
    st = iterate_once(s, d_Y, ldY, d_Z, want);
    if (st != MSLD_OK) return st;
    if (want) {
      result = read_resid(s, d_Y, ldY, &resid);
      if (result != MSLD_OK) break;
      if (check && resid <= (double)p.tol) break;
    }
  }
  if (info) {
    st = msld_stats(s, info);
    if (st != MSLD_OK) return st;
    info->primal_resid = resid;
    info->status = result;
  }
  return result;
}

msld_status msld_profile_begin(msld_solver* s, int32_t max_iters) {
  if (!s || max_iters < 1) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (s->prof_ev) return MSLD_EINVAL;
  const size_t per = 2 + 5 * (size_t)s->p.L;
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
  const size_t per = 2 + 5 * (size_t)L;
  msld_status result = MSLD_OK;
  if (hipStreamSynchronize(s->st) != hipSuccess) result = dev_err(s, hipErrorUnknown);
  for (int i = 0; i < 4 * (L + 1); ++i) ms[i] = 0.0;
  for (int it = 0; it < s->prof_n && result == MSLD_OK; ++it) {
    hipEvent_t* ev = s->prof_ev + (size_t)it * per;
    float t;
    if (hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) ms[4 * L] += t;
    for (int i = 0; i < L; ++i) {
      if (s->plan.tier[i] == TIER_1X1) continue;
      hipEvent_t* e5 = ev + 2 + 5 * i;
      for (int j = 0; j < 4; ++j)
        if (hipEventElapsedTime(&t, e5[j], e5[j + 1]) == hipSuccess) ms[4 * i + j] += t;
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

msld_status msld_bsvt(msld_solver* s, int32_t scale, const float* d_V, float* d_Z, float tau,
                      int32_t sr, int32_t sc) {
  if (!s || !d_V || !d_Z) return MSLD_EINVAL;
  if (s->failed) return MSLD_EDEVICE;
  if (scale < 0 || scale >= s->p.L) return MSLD_EINVAL;
  const ScaleGeom& g = s->plan.geom[scale];
  if (sr < 0 || sr >= g.m || sc < 0 || sc >= g.n) return MSLD_EINVAL;
  if (!(tau >= 0.f) || !std::isfinite(tau)) return MSLD_EINVAL;
  const size_t MN = (size_t)g.M * g.N;
  float* Dws = reinterpret_cast<float*>(s->arena + s->plan.off_D) + MN * scale;
  ShiftSpec sh;
  sh.seed = 0;
  sh.k = 0;
  sh.scale = scale;
  sh.mode = 2;
  sh.sr = sr;
  sh.sc = sc;
  if (s->plan.tier[scale] == TIER_1X1) {
    // 1x1 blocks: the entrywise soft-threshold of the consensus kernel, run with
    // L = 1, Y = V, an all-zero D plane and an all-zero Z plane: R = V and
    // Z' = soft(R, tau). The second D buffer serves as the Z plane.
    float* Rws = reinterpret_cast<float*>(s->arena + s->plan.off_R);
    float* Zp = reinterpret_cast<float*>(s->arena + s->plan.off_D) + MN * s->p.L;
    int idx0 = 0;
    float t0 = tau;
    MSLD_TRY(s, launch_fill(Dws, 0.f, MN, s->st));
    MSLD_TRY(s, launch_fill(Zp, 0.f, MN, s->st));
    MSLD_TRY(s, launch_consensus(d_V, g.N, Dws, Dws, Zp, Rws, g.M, g.N, 1, &idx0, &t0, 1, s->st));
    MSLD_TRY(s, hipMemcpyAsync(d_Z, Zp, MN * 4, hipMemcpyDeviceToDevice, s->st));
    return MSLD_OK;
  }
  msld_status zs = zero_stats(s);
  if (zs != MSLD_OK) return zs;
  return run_scale(s, scale, d_V, nullptr, d_Z, Dws, tau, sh, nullptr);
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

}  // extern "C"
