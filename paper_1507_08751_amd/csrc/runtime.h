// Host-side runtime shared by the C-ABI entry points (api.cpp) and the serving loop
// (server.cpp): per-scale plans, the solver object and the ADMM iteration driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../include/msld.h"
#include "msld_internal.h"

namespace msld {

constexpr size_t kLdsTierMax = 150 * 1024;   // LDS budget of one workgroup (160 KiB per CU)
constexpr int kStreamFloats = 16384;         // stream-pass tile budget (elements)
constexpr int kLRP = 16;                     // subspace width of the certified low-rank path

// Stopping threshold of the float32 one-sided Jacobi tiers: pair (p, q) is rotated while
// |b_p . b_q| > tol ||b_p|| ||b_q||. Those inner products over mb rows carry rounding
// noise of order mb 2^-24, and a threshold at that level lets a block keep rotating on
// noise up to the sweep cap (the slowest block sets a launch's time), so small blocks
// get 2 mb 2^-24 (at most 64 2^-24) and larger ones 4 sqrt(mb) 2^-24.
inline float jacobi_tolerance(int mb) {
  const float a = 4.0f * std::sqrt((float)mb);
  const float b = std::fmin(2.0f * (float)mb, 64.0f);
  return 5.9604645e-8f * std::fmax(a, b);
}
int lds_tier_threads(int nb, int mb, int* G);
size_t lds_tier_bytes(int mb, int nb);
size_t stream_lds_bytes(int m, const StreamPlan& sp);
hipError_t launch_fill_ints(int* p, int v, size_t count, hipStream_t st);
hipError_t launch_set_int(int* p, int idx, int v, hipStream_t st);
hipError_t launch_inc_active(int* k, const int* active, int n, hipStream_t st);
// Device-side retirement of stacked instances after an iteration (see kernels.hip).
hipError_t launch_retire(const double* res, int n, float tol, int check_every, int max_iters,
                         const int* ik, int* active, int* out_iters, double* out_resid,
                         hipStream_t st);

// Plan of one problem shape, for ninst instances stacked along the rows.
struct Plan {
  ScaleGeom geom[MSLD_MAX_SCALES];
  StreamPlan sp[MSLD_MAX_SCALES];
  int tier[MSLD_MAX_SCALES];
  int pw[MSLD_MAX_SCALES];
  int nbp[MSLD_MAX_SCALES];
  int use_lr[MSLD_MAX_SCALES];
  float tau_default[MSLD_MAX_SCALES];
  int ninst;
  int resid_parts;
  size_t bytes;
  // byte offsets inside the arena
  size_t off_R, off_D, off_part, off_res, off_shift, off_inst;
  size_t off_count[MSLD_MAX_SCALES], off_list[MSLD_MAX_SCALES], off_rowp[MSLD_MAX_SCALES],
      off_frop[MSLD_MAX_SCALES], off_stats[MSLD_MAX_SCALES], off_pA[MSLD_MAX_SCALES],
      off_pW[MSLD_MAX_SCALES], off_pflag[MSLD_MAX_SCALES], off_pg[MSLD_MAX_SCALES],
      off_lr[MSLD_MAX_SCALES], off_pl[MSLD_MAX_SCALES];
  int pl_cap[MSLD_MAX_SCALES];   // polar fallback chunk (0: none)
  size_t off_split[MSLD_MAX_SCALES];   // split partials (tall low-rank blocks; 0: none)
  size_t off_skpart[MSLD_MAX_SCALES];  // skinny-product split partials (wide blocks; 0: none)
  int lds_cap[MSLD_MAX_SCALES];    // LDS tier: workgroups per CU cap (0: as many as fit)
  int lrs_wide[MSLD_MAX_SCALES];   // fused low-rank kernel: first pass with 2p
  // averaged cycle spinning: shifts per iteration (0: one random shift), whether the
  // set is every shift, and the accumulator + scratch planes
  int spin[MSLD_MAX_SCALES];
  int spin_full[MSLD_MAX_SCALES];
  size_t off_spin[MSLD_MAX_SCALES];
};

// Autotuned launch choice of one block size (tune.cpp); tier in msld_scale_tier
// numbering (kTierLowRank for the batched low-rank path).
constexpr int kTierLowRank = 4;
struct TuneCfg {
  int tier;
  int lds_cap;
  int lrs_wide;
};
bool tune_lookup(int m, int n, TuneCfg* out);
bool lds_fits(int mb, int nb);
double lambda_default(int M, int N, int m, int n);

msld_status validate_params(const msld_params* p);
msld_status make_plan(const msld_params* p, int ninst, Plan* pl);
bool same_class(const msld_params& a, const msld_params& b);
// scale i's driver reads a count back from the device every iteration (a low-rank
// scale whose blocks exceed the LDS tier: its polar fallback is sized on the host)
bool host_waits(const Plan& pl, int i);

}  // namespace msld

// The solver: workspace and state of ninst stacked instances of one shape.
struct msld_solver {
  msld_params p;
  msld::Plan plan;
  hipStream_t st;
  int device;
  int num_cus;
  bool failed;
  char* arena;
  double* host_res;   // pinned: [0, ninst) residual sums, [ninst, 2 ninst) ||Y||^2
  int* host_ints;     // pinned, 2 per scale
  float* host_pl;     // pinned, per polar chunk slot 4 scalars and 2 step counts, one slice per scale
  // scales are independent between two consensus passes: each runs on its own
  // stream (forked from st after the consensus, joined before the residual)
  hipStream_t sst[MSLD_MAX_SCALES];
  hipEvent_t ev_fork;
  hipEvent_t ev_join[MSLD_MAX_SCALES];
  hipEvent_t ev_sfork[MSLD_MAX_SCALES];   // after scale i's stream pass (its own fork point)
  int early_fork;   // scales fork after their own stream pass (planes <= 2^24 elements)
  int serial;       // every scale's BlockSVT on the handle's stream, one after another
  int per_instance; // per-instance seeds, counters and activity flags even for one
                    // instance that is not replayed from graphs (the serving loop's
                    // device-side retirement needs the flags)
  msld::ScaleWork work[MSLD_MAX_SCALES];
  msld::StreamAll sall;   // the stream pass of all decomposed scales (one launch)
  const uint8_t* mask;    // observed-entry mask (caller-owned, device) or null
  int64_t ldmask;
  int ninst;
  int k;              // next iteration (single instance; stacked instances use d_k)
  int cur;            // which D buffer holds the current D_i
  unsigned long long* d_seed;   // [ninst] per-instance shift seeds (stacked only)
  int* d_k;                     // [ninst] per-instance iteration counters
  int* d_active;                // [ninst] active flags
  // profiling: per iteration 2 consensus events, 2 for the fused stream pass, 5 per scale
  int prof_cap, prof_n;
  hipEvent_t* prof_ev;
  int64_t round_launches[MSLD_MAX_SCALES];
  // HIP graphs of one iteration (one per D-buffer parity) for plans whose iteration
  // never waits on the host; keyed by the Y / Z buffers they were captured with
  bool graphable;
  bool graph_on;
  hipStream_t cst;   // capture stream (the caller's stream may be the null stream)
  hipGraphExec_t gx[2];
  const float* gY;
  int64_t gldY;
  float* gZ;
};

namespace msld {

msld_status create_solver(const msld_params* p, int ninst, hipStream_t st, msld_solver** out);
msld_status dev_err(msld_solver* s, hipError_t e);
float* plane_R(msld_solver* s);
float* plane_D(msld_solver* s, int which);
size_t plane_elems(const msld_solver* s);   // elements of one stacked plane
// One ADMM iteration on all active instances; with want_res the per-instance
// residual sums land in device memory (dres[z]).
msld_status iterate_once(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                         bool want_res);
// iterate_once, replayed from a captured HIP graph when the plan allows it and no
// residual is wanted
msld_status step_iteration(msld_solver* s, const float* d_Y, int64_t ldY, float* d_Z,
                           bool want_res);
double* dev_res(msld_solver* s);
msld_status launch_ynorms(msld_solver* s, const float* d_Y, int64_t ldY);

}  // namespace msld

#define MSLD_TRY(s, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return msld::dev_err((s), e_);    \
  } while (0)
