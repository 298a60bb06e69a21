// One block-wise SVT call (eq:bsvt with the Shift of Sec. 9) that allocates nothing:
// for callers that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid it). Its workspace (the speculative dual plane
// of the stream pass, the live-block list and count, the bound partials, the counters)
// lives in the file-scope device array `scratch` below; the register and LDS tiers of
// the solver run on it unchanged.
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace msld {
namespace {

constexpr size_t kNoAllocScratch = (size_t)32 << 20;   // bytes per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kNoAllocScratch];

// Device address of `scratch` on each device, taken once per device (with that device
// current): the array's name in host code is a host-side stand-in, never a device
// address, so every kernel argument below comes from this table.
void* g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_ptr(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return hipSuccess;
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace msld

using namespace msld;

extern "C" msld_status msld_bsvt_noalloc(int32_t M, int32_t N, int32_t m, int32_t n,
                                         const float* d_V, float* d_Z, float tau, int32_t sr,
                                         int32_t sc, void* hip_stream) {
  if (!d_V || !d_Z) return MSLD_EINVAL;
  if (M < 1 || N < 1 || m < 1 || n < 1 || M % m || N % n) return MSLD_EINVAL;
  if (sr < 0 || sr >= m || sc < 0 || sc >= n) return MSLD_EINVAL;
  if (!(tau >= 0.f) || !std::isfinite(tau)) return MSLD_EINVAL;
  if ((int64_t)M * N >= ((int64_t)1 << 31)) return MSLD_EINVAL;
  // the plan of a one-scale problem with the low-rank paths off: register or LDS tier
  msld_params p;
  std::memset(&p, 0, sizeof(p));
  p.M = M;
  p.N = N;
  p.L = 1;
  p.block_m[0] = m;
  p.block_n[0] = n;
  p.lambda[0] = 1.f;
  p.rho = 1.f;
  p.max_iters = 1;
  p.check_every = 1;
  p.lowrank_min = -1;
  Plan pl;
  const msld_status ps = make_plan(&p, 1, &pl);
  if (ps != MSLD_OK) return ps;
  const int tier = pl.tier[0];
  if (tier != TIER_REG && tier != TIER_LDS) return MSLD_EINVAL;   // 1 x 1 or panel blocks
  const ScaleGeom& g = pl.geom[0];
  const StreamPlan& sp = pl.sp[0];
  const size_t nblk = (size_t)g.P * g.Q;
  // workspace layout inside the scratch array
  size_t off = 0;
  const size_t o_dual = off;
  off = up256(off + 4 * (size_t)M * N);
  const size_t o_count = off;
  off = up256(off + 4);
  const size_t o_list = off;
  off = up256(off + 4 * nblk);
  size_t o_rowp = 0, o_frop = 0;
  if (!sp.whole) {
    if (sp.rowbound) {
      o_rowp = off;
      off = up256(off + 4 * nblk * sp.spb * (size_t)m);
    }
    o_frop = off;
    off = up256(off + 4 * nblk * sp.spb);
  }
  const size_t o_stats = off;
  off = up256(off + 8 * kStatsWords);
  if (off > kNoAllocScratch) return MSLD_ETOOLARGE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MSLD_EDEVICE;
  char* base = nullptr;
  if (scratch_ptr(dev, &base) != hipSuccess) return MSLD_EDEVICE;
  int num_cus = 0;
  if (hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return MSLD_EDEVICE;
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ScaleWork w;
  std::memset(&w, 0, sizeof(w));
  w.live_count = reinterpret_cast<int*>(base + o_count);
  w.live_list = reinterpret_cast<int*>(base + o_list);
  w.rowpart = (!sp.whole && sp.rowbound) ? reinterpret_cast<float*>(base + o_rowp) : nullptr;
  w.fropart = !sp.whole ? reinterpret_cast<float*>(base + o_frop) : nullptr;
  w.stats = reinterpret_cast<unsigned long long*>(base + o_stats);
  w.lds_cap = pl.lds_cap[0];
  w.slots = (int)nblk;
  float* dual = reinterpret_cast<float*>(base + o_dual);
  // the counters start at zero (a fill kernel; the live count is cleared by the stream
  // pass launch itself)
  if (launch_fill_ints(reinterpret_cast<int*>(w.stats), 0, 2 * kStatsWords, st) != hipSuccess)
    return MSLD_EDEVICE;
  ShiftSpec sh;
  std::memset(&sh, 0, sizeof(sh));
  sh.mode = 2;
  sh.sr = sr;
  sh.sc = sc;
  const float jtol = jacobi_tolerance(g.mb);
  const hipError_t e = launch_scale(g, tier, sp, w, d_V, nullptr, d_Z, dual, tau, sh, jtol, 40, 20,
                                    num_cus, st, nullptr, nullptr, false);
  return e == hipSuccess ? MSLD_OK : MSLD_EDEVICE;
}
