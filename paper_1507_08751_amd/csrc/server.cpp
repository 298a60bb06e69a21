// Serving loop: continuous batching of independent decompositions.
//
// Requests wait in a FIFO queue. A request is admitted into a free slot of a
// "class" -- a stacked solver for one problem shape (all parameters but the shift
// seed equal) with a fixed number of instance slots -- creating the class if the HBM
// budget allows (idle classes are released first when it does not). Every class
// advances on its own: a worker thread runs a batch of ADMM iterations for all of the
// class's active slots (one set of launches per iteration, on the class's stream) while
// the other classes run theirs, and each iteration ends with the residual check of
// every slot on the device: a slot that reaches its tolerance or iteration cap drops
// its activity flag, so the rest of the batch leaves it untouched (the outcome of a
// check after every iteration, without a host round trip per iteration). Between
// batches the server retires the slots that stopped (their Z planes are copied to the
// request's buffer), admits waiting requests into free slots and starts the next batch,
// sized so that a batch takes a few milliseconds. Slots are independent instances of
// deterministic kernels, so a request's result does not depend on which other requests
// share its class or run beside it.
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace msld;

namespace msld {
hipError_t launch_set_u64(unsigned long long* p, int idx, unsigned long long v, hipStream_t st);
}

namespace {
constexpr int kBatchMax = 64;
// wall time aimed at per batch of a class (MSLD_SERVE_BATCH_MS overrides the default)
double batch_target_ms() {
  static const double v = [] {
    const char* e = std::getenv("MSLD_SERVE_BATCH_MS");
    const double x = e ? std::atof(e) : 0.0;
    return (x > 0.0 && x <= 1000.0) ? x : 8.0;
  }();
  return v;
}
}  // namespace

struct msld_server {
  struct Req {
    msld_params p;
    const float* Y;
    int64_t ldY;
    float* Z;
    int64_t id;
  };
  struct Done {
    int64_t id;
    int32_t iters;
    int32_t status;
    double resid;
  };
  struct Cls {
    msld_params p;
    int slots;
    msld_solver* s;
    float* Y;
    float* Z;
    int* d_iters;       // [slots] iterations a slot ran when it stopped (device)
    double* d_resid;    // [slots] its residual then
    int* h_iters;       // pinned copies, read after a batch
    int* h_active;
    double* h_resid;
    size_t footprint;
    hipStream_t st;
    std::vector<int> used;
    std::vector<Req> req;
    std::vector<int> issued;   // iterations issued since the slot's admission
    int nactive;
    bool ynorms_stale;         // slots admitted since the last batch
    // batch in flight: started by the server (in_batch), run by a worker thread, which
    // clears `running` when done; the server then collects it
    std::thread worker;
    bool in_batch;
    std::atomic<int> running;
    int batch_iters;
    msld_status batch_status;
    double ms_per_iter;        // measured, sizes the next batch
  };
  int max_active;
  int slots_per_class;
  size_t budget;
  size_t used_bytes;
  int active_total;
  std::vector<hipStream_t> streams;
  int next_stream;
  std::deque<Req> queue;
  std::vector<Cls*> cls;
  std::deque<Done> done;
  std::mutex mu;                 // with cv: workers signal finished batches
  std::condition_variable cv;
  int finished;                  // batches finished and not yet collected
};

static void cls_destroy(msld_server* sv, msld_server::Cls* c) {
  if (!c) return;
  if (c->worker.joinable()) c->worker.join();
  if (c->s) msld_free(c->s);
  if (c->Y) (void)hipFree(c->Y);
  if (c->Z) (void)hipFree(c->Z);
  if (c->d_iters) (void)hipFree(c->d_iters);
  if (c->h_iters) (void)hipHostFree(c->h_iters);
  sv->used_bytes -= c->footprint;
  delete c;
}

static size_t cls_footprint(const msld_params& p, int slots) {
  Plan pl;
  if (make_plan(&p, slots, &pl) != MSLD_OK) return 0;
  return pl.bytes + (size_t)4 * p.M * p.N * slots * (size_t)(p.L + 1) + (size_t)16 * slots;
}

static msld_status cls_create(msld_server* sv, const msld_params& p, msld_server::Cls** out) {
  *out = nullptr;
  const size_t fp = cls_footprint(p, sv->slots_per_class);
  if (fp == 0) return MSLD_EINVAL;
  msld_server::Cls* c = new (std::nothrow) msld_server::Cls();
  if (!c) return MSLD_ENOMEM;
  c->p = p;
  c->slots = sv->slots_per_class;
  c->s = nullptr;
  c->Y = c->Z = nullptr;
  c->d_iters = nullptr;
  c->d_resid = nullptr;
  c->h_iters = nullptr;
  c->h_active = nullptr;
  c->h_resid = nullptr;
  c->footprint = 0;
  c->in_batch = false;
  c->running.store(0);
  c->batch_iters = 0;
  c->batch_status = MSLD_OK;
  c->ms_per_iter = 0.0;
  c->st = sv->streams[sv->next_stream];
  sv->next_stream = (sv->next_stream + 1) % (int)sv->streams.size();
  msld_status st = create_solver(&p, c->slots, c->st, &c->s);
  if (st == MSLD_OK) c->s->per_instance = 1;   // retirement drops per-slot activity flags
  const size_t MN = (size_t)p.M * p.N * c->slots;
  const size_t n = (size_t)c->slots;
  const size_t n2 = (n + 1) & ~(size_t)1;   // ints before the doubles, 8-byte aligned
  if (st == MSLD_OK &&
      (hipMalloc(&c->Y, 4 * MN) != hipSuccess || hipMalloc(&c->Z, 4 * MN * p.L) != hipSuccess))
    st = MSLD_ENOMEM;
  // device: iters (int), then resid (double); host (pinned): iters, active flags, resid
  if (st == MSLD_OK && hipMalloc(&c->d_iters, 4 * n2 + 8 * n) != hipSuccess) st = MSLD_ENOMEM;
  if (st == MSLD_OK) c->d_resid = reinterpret_cast<double*>(c->d_iters + n2);
  void* hp = nullptr;
  if (st == MSLD_OK && hipHostMalloc(&hp, 8 * n2 + 8 * n, hipHostMallocDefault) != hipSuccess)
    st = MSLD_ENOMEM;
  if (st == MSLD_OK) {
    c->h_iters = static_cast<int*>(hp);
    c->h_active = c->h_iters + n2;
    c->h_resid = reinterpret_cast<double*>(c->h_iters + 2 * n2);
  }
  c->footprint = fp;
  sv->used_bytes += fp;
  if (st != MSLD_OK) {
    cls_destroy(sv, c);
    return st;
  }
  c->used.assign(c->slots, 0);
  c->req.resize(c->slots);
  c->issued.assign(c->slots, 0);
  c->nactive = 0;
  c->ynorms_stale = false;
  // every slot starts inactive: kernels skip its rows until a request is admitted
  if (launch_fill_ints(c->s->d_active, 0, (size_t)c->slots, c->st) != hipSuccess ||
      launch_fill_ints(c->s->d_k, 0, (size_t)c->slots, c->st) != hipSuccess) {
    cls_destroy(sv, c);
    return MSLD_EDEVICE;
  }
  *out = c;
  return MSLD_OK;
}

// Put request r into free slot z of idle class c (all work on the class stream).
static msld_status slot_admit(msld_server::Cls* c, int z, const msld_server::Req& r) {
  msld_solver* s = c->s;
  const msld_params& p = c->p;
  const size_t inst = (size_t)p.M * p.N;
  const size_t MN = inst * c->slots;
  MSLD_TRY(s, hipMemcpy2DAsync(c->Y + inst * z, 4 * (size_t)p.N, r.Y, 4 * (size_t)r.ldY,
                               4 * (size_t)p.N, p.M, hipMemcpyDeviceToDevice, c->st));
  float* Dc = plane_D(s, s->cur);
  for (int l = 0; l < p.L; ++l) {
    MSLD_TRY(s, launch_fill(c->Z + MN * l + inst * z, 0.f, inst, c->st));
    MSLD_TRY(s, launch_fill(Dc + MN * l + inst * z, 0.f, inst, c->st));
  }
  MSLD_TRY(s, launch_set_u64(s->d_seed, z, (unsigned long long)r.p.shift_seed, c->st));
  MSLD_TRY(s, launch_set_int(s->d_k, z, 0, c->st));
  MSLD_TRY(s, launch_set_int(s->d_active, z, 1, c->st));
  c->used[z] = 1;
  c->req[z] = r;
  c->issued[z] = 0;
  c->nactive += 1;
  c->ynorms_stale = true;
  return MSLD_OK;
}

// Worker: `iters` iterations of class c, each followed by the device-side residual check
// of every active slot; then the slots' counters, flags and residuals are copied to the
// pinned host arrays and the class stream is drained.
static void run_batch(msld_server* sv, msld_server::Cls* c, int iters) {
  const auto t0 = std::chrono::steady_clock::now();
  msld_solver* s = c->s;
  const msld_params& p = c->p;
  const int n = c->slots;
  msld_status st = hipSetDevice(s->device) == hipSuccess ? MSLD_OK : MSLD_EDEVICE;
  for (int it = 0; it < iters && st == MSLD_OK; ++it) {
    st = iterate_once(s, c->Y, p.N, c->Z, true);
    if (st == MSLD_OK &&
        launch_retire(dev_res(s), n, p.tol, p.check_every, p.max_iters, s->d_k, s->d_active,
                      c->d_iters, c->d_resid, c->st) != hipSuccess)
      st = MSLD_EDEVICE;
  }
  if (st == MSLD_OK &&
      (hipMemcpyAsync(c->h_iters, c->d_iters, 4 * (size_t)n, hipMemcpyDeviceToHost, c->st) !=
           hipSuccess ||
       hipMemcpyAsync(c->h_resid, c->d_resid, 8 * (size_t)n, hipMemcpyDeviceToHost, c->st) !=
           hipSuccess ||
       hipMemcpyAsync(c->h_active, s->d_active, 4 * (size_t)n, hipMemcpyDeviceToHost, c->st) !=
           hipSuccess))
    st = MSLD_EDEVICE;
  if (hipStreamSynchronize(c->st) != hipSuccess && st == MSLD_OK) st = MSLD_EDEVICE;
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->batch_status = st;
  c->ms_per_iter = ms / (iters > 0 ? iters : 1);
  {
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->finished += 1;
    c->running.store(0);
  }
  sv->cv.notify_all();
}

// Collect the finished batch of class c: retire the slots that stopped (or all of them
// after a device error), copying their Z planes out.
static void collect(msld_server* sv, msld_server::Cls* c) {
  if (c->worker.joinable()) c->worker.join();
  c->in_batch = false;
  const msld_params& p = c->p;
  const size_t inst = (size_t)p.M * p.N;
  const size_t MN = inst * c->slots;
  const bool ok = c->batch_status == MSLD_OK;
  bool retired = false;
  for (int z = 0; z < c->slots; ++z) {
    if (!c->used[z]) continue;
    c->issued[z] += c->batch_iters;
    if (ok && c->h_active[z]) continue;
    int32_t status = ok ? MSLD_OK : c->batch_status;
    const double r = ok ? c->h_resid[z] : -1.0;
    if (ok && !std::isfinite(r)) status = MSLD_ENUMERIC;
    const msld_server::Req& rq = c->req[z];
    if (ok)
      for (int l = 0; l < p.L; ++l)
        if (hipMemcpyAsync(rq.Z + inst * l, c->Z + MN * l + inst * z, 4 * inst,
                           hipMemcpyDeviceToDevice, c->st) != hipSuccess)
          status = MSLD_EDEVICE;
    if (!ok && launch_set_int(c->s->d_active, z, 0, c->st) != hipSuccess) status = MSLD_EDEVICE;
    c->used[z] = 0;
    c->nactive -= 1;
    sv->active_total -= 1;
    msld_server::Done d;
    d.id = rq.id;
    d.iters = ok ? c->h_iters[z] : c->issued[z];
    d.status = status;
    d.resid = r;
    sv->done.push_back(d);
    retired = true;
  }
  if (retired) (void)hipStreamSynchronize(c->st);   // outputs complete before reporting
}

// Start the next batch of an idle class with active slots.
static msld_status start_batch(msld_server* sv, msld_server::Cls* c) {
  if (c->ynorms_stale) {
    msld_status st = launch_ynorms(c->s, c->Y, c->p.N);
    if (st != MSLD_OK) return st;
    c->ynorms_stale = false;
  }
  // about batch_target_ms() of work, never past the furthest iteration cap of the slots
  int k = c->ms_per_iter > 0.0 ? (int)(batch_target_ms() / c->ms_per_iter) : 2;
  if (k < 1) k = 1;
  if (k > kBatchMax) k = kBatchMax;
  int left = 0;
  for (int z = 0; z < c->slots; ++z)
    if (c->used[z] && c->p.max_iters - c->issued[z] > left) left = c->p.max_iters - c->issued[z];
  if (k > left) k = left > 0 ? left : 1;
  c->batch_iters = k;
  c->in_batch = true;
  c->running.store(1);
  try {
    c->worker = std::thread(run_batch, sv, c, k);
  } catch (...) {
    run_batch(sv, c, k);   // no thread available: run it here
  }
  return MSLD_OK;
}

extern "C" {

msld_status msld_server_create(int32_t max_active, size_t hbm_budget_bytes, int32_t num_streams,
                               msld_server** out) {
  if (!out || max_active < 1 || num_streams < 1 || num_streams > 64 || hbm_budget_bytes == 0)
    return MSLD_EINVAL;
  *out = nullptr;
  msld_server* sv = new (std::nothrow) msld_server();
  if (!sv) return MSLD_ENOMEM;
  sv->max_active = max_active;
  sv->slots_per_class = max_active < 8 ? max_active : 8;
  sv->budget = hbm_budget_bytes;
  sv->used_bytes = 0;
  sv->active_total = 0;
  sv->next_stream = 0;
  sv->finished = 0;
  for (int i = 0; i < num_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
      delete sv;
      return MSLD_EDEVICE;
    }
    sv->streams.push_back(st);
  }
  *out = sv;
  return MSLD_OK;
}

msld_status msld_server_submit(msld_server* sv, const msld_params* p, const float* d_Y,
                               int64_t ldY, float* d_Z, int64_t request_id) {
  if (!sv || !p || !d_Y || !d_Z) return MSLD_EINVAL;
  if (validate_params(p) != MSLD_OK || ldY < p->N) return MSLD_EINVAL;
  const size_t fp = cls_footprint(*p, sv->slots_per_class);
  if (fp == 0 || fp > sv->budget) return MSLD_EINVAL;   // could never be admitted
  msld_server::Req r;
  r.p = *p;
  r.Y = d_Y;
  r.ldY = ldY;
  r.Z = d_Z;
  r.id = request_id;
  sv->queue.push_back(r);
  return MSLD_OK;
}

// Admit the queue head if possible (into an idle class of its shape with a free slot,
// else into a new class if the budget allows after releasing idle empty classes);
// returns false when the head has to wait.
static bool admit_head(msld_server* sv) {
  if (sv->queue.empty() || sv->active_total >= sv->max_active) return false;
  const msld_server::Req& r = sv->queue.front();
  msld_server::Cls* target = nullptr;
  int slot = -1;
  for (msld_server::Cls* c : sv->cls) {
    if (c->in_batch || !same_class(c->p, r.p)) continue;   // a batch not yet collected
    for (int z = 0; z < c->slots; ++z)
      if (!c->used[z]) {
        target = c;
        slot = z;
        break;
      }
    if (target) break;
  }
  if (!target) {
    const size_t fp = cls_footprint(r.p, sv->slots_per_class);
    for (size_t i = 0; i < sv->cls.size() && sv->used_bytes + fp > sv->budget;) {
      if (sv->cls[i]->nactive == 0 && !sv->cls[i]->in_batch) {
        cls_destroy(sv, sv->cls[i]);
        sv->cls.erase(sv->cls.begin() + (long)i);
      } else {
        ++i;
      }
    }
    if (sv->used_bytes + fp > sv->budget) return false;
    msld_server::Cls* c = nullptr;
    msld_status st = cls_create(sv, r.p, &c);
    if (st == MSLD_ENOMEM) return false;
    if (st != MSLD_OK) {
      msld_server::Done d;
      d.id = r.id;
      d.iters = 0;
      d.status = st;
      d.resid = -1.0;
      sv->done.push_back(d);
      sv->queue.pop_front();
      return true;
    }
    sv->cls.push_back(c);
    target = c;
    slot = 0;
  }
  msld_status st = slot_admit(target, slot, r);
  msld_server::Req rr = r;
  sv->queue.pop_front();
  if (st != MSLD_OK) {
    msld_server::Done d;
    d.id = rr.id;
    d.iters = 0;
    d.status = st;
    d.resid = -1.0;
    sv->done.push_back(d);
    return true;
  }
  sv->active_total += 1;
  return true;
}

msld_status msld_server_step(msld_server* sv, int64_t* done_ids, int32_t* done_iters,
                             double* done_resid, int32_t* done_status, int32_t max_out,
                             int32_t* n_done, int32_t* n_active, int32_t* n_queued) {
  if (!sv || !n_done || max_out < 0 || (max_out > 0 && (!done_ids || !done_iters || !done_resid ||
                                                        !done_status)))
    return MSLD_EINVAL;
  // when every class with work is mid-batch and nothing is left to report, wait (at
  // most 50 ms) for a batch to finish rather than return empty-handed
  bool running = false, ready = false;
  for (msld_server::Cls* c : sv->cls) {
    if (c->running.load()) running = true;
    else if (c->in_batch || c->nactive > 0) ready = true;
  }
  const bool admittable = !sv->queue.empty() && sv->active_total < sv->max_active;
  if (running && !ready && !admittable && sv->done.empty()) {
    std::unique_lock<std::mutex> lock(sv->mu);
    sv->cv.wait_for(lock, std::chrono::milliseconds(50), [&] { return sv->finished > 0; });
  }
  // 1. collect finished batches: retire the slots that stopped
  for (msld_server::Cls* c : sv->cls)
    if (c->in_batch && !c->running.load()) {
      collect(sv, c);
      std::lock_guard<std::mutex> lock(sv->mu);
      sv->finished -= 1;
    }
  // 2. admission, first come first served
  while (admit_head(sv)) {
  }
  // 3. the next batch of every collected class with active slots (a batch that ended
  // after the collection above waits for the next step)
  for (msld_server::Cls* c : sv->cls)
    if (!c->in_batch && c->nactive > 0) {
      msld_status st = start_batch(sv, c);
      if (st != MSLD_OK) return st;
    }
  // 4. report
  int32_t k = 0;
  while (k < max_out && !sv->done.empty()) {
    const msld_server::Done& d = sv->done.front();
    done_ids[k] = d.id;
    done_iters[k] = d.iters;
    done_resid[k] = d.resid;
    done_status[k] = d.status;
    sv->done.pop_front();
    ++k;
  }
  *n_done = k;
  if (n_active) *n_active = sv->active_total;
  if (n_queued) *n_queued = (int32_t)(sv->queue.size() + sv->done.size());
  return MSLD_OK;
}

msld_status msld_server_class_bytes(const msld_params* p, int32_t max_active, size_t* out) {
  if (!p || !out || max_active < 1) return MSLD_EINVAL;
  *out = 0;
  if (validate_params(p) != MSLD_OK) return MSLD_EINVAL;
  const size_t fp = cls_footprint(*p, max_active < 8 ? max_active : 8);
  if (fp == 0) return MSLD_EINVAL;
  *out = fp;
  return MSLD_OK;
}

void msld_server_free(msld_server* sv) {
  if (!sv) return;
  for (msld_server::Cls* c : sv->cls) cls_destroy(sv, c);
  for (hipStream_t st : sv->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete sv;
}

}  // extern "C"
