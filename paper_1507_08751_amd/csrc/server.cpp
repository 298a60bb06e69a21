// Serving loop: continuous batching of independent decompositions.
//
// Requests wait in a FIFO queue. A request is admitted into a free slot of a
// "class" -- a stacked solver for one problem shape (all parameters but the shift
// seed equal) with a fixed number of instance slots -- creating the class if the HBM
// budget allows (idle classes are released first when it does not). Every
// msld_server_step runs one ADMM iteration for all active slots of every class with
// a single set of launches per class (classes run on different streams), reads the
// per-slot residuals back, and retires finished slots: their Z planes are copied to
// the request's buffer and the slot is freed for the next request. Slots are
// independent instances of the stacked kernels, so a request's result does not
// depend on which other requests share its class.
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace msld;

namespace msld {
hipError_t launch_set_u64(unsigned long long* p, int idx, unsigned long long v, hipStream_t st);
}

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
    size_t footprint;
    hipStream_t st;
    std::vector<int> used;
    std::vector<Req> req;
    std::vector<int> iters;
    int nactive;
    bool stepped;
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
};

static void cls_destroy(msld_server* sv, msld_server::Cls* c) {
  if (!c) return;
  if (c->s) msld_free(c->s);
  if (c->Y) (void)hipFree(c->Y);
  if (c->Z) (void)hipFree(c->Z);
  sv->used_bytes -= c->footprint;
  delete c;
}

static size_t cls_footprint(const msld_params& p, int slots) {
  Plan pl;
  if (make_plan(&p, slots, &pl) != MSLD_OK) return 0;
  return pl.bytes + (size_t)4 * p.M * p.N * slots * (size_t)(p.L + 1);
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
  c->footprint = 0;
  c->st = sv->streams[sv->next_stream];
  sv->next_stream = (sv->next_stream + 1) % (int)sv->streams.size();
  msld_status st = create_solver(&p, c->slots, c->st, &c->s);
  const size_t MN = (size_t)p.M * p.N * c->slots;
  if (st == MSLD_OK &&
      (hipMalloc(&c->Y, 4 * MN) != hipSuccess || hipMalloc(&c->Z, 4 * MN * p.L) != hipSuccess))
    st = MSLD_ENOMEM;
  c->footprint = fp;
  sv->used_bytes += fp;
  if (st != MSLD_OK) {
    cls_destroy(sv, c);
    return st;
  }
  c->used.assign(c->slots, 0);
  c->req.resize(c->slots);
  c->iters.assign(c->slots, 0);
  c->nactive = 0;
  c->stepped = false;
  // every slot starts inactive: kernels skip its rows until a request is admitted
  if (launch_fill_ints(c->s->d_active, 0, (size_t)c->slots, c->st) != hipSuccess ||
      launch_fill_ints(c->s->d_k, 0, (size_t)c->slots, c->st) != hipSuccess) {
    cls_destroy(sv, c);
    return MSLD_EDEVICE;
  }
  *out = c;
  return MSLD_OK;
}

// Put request r into free slot z of class c (all work on the class stream).
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
  c->iters[z] = 0;
  c->nactive += 1;
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

// Admit the queue head if possible; returns false when the head has to wait.
static bool admit_head(msld_server* sv) {
  if (sv->queue.empty() || sv->active_total >= sv->max_active) return false;
  const msld_server::Req& r = sv->queue.front();
  msld_server::Cls* target = nullptr;
  int slot = -1;
  for (msld_server::Cls* c : sv->cls) {
    if (!same_class(c->p, r.p)) continue;
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
    // release idle classes of other shapes until the new class fits
    for (size_t i = 0; i < sv->cls.size() && sv->used_bytes + fp > sv->budget;) {
      if (sv->cls[i]->nactive == 0) {
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
  target->stepped = false;
  sv->active_total += 1;
  return true;
}

msld_status msld_server_step(msld_server* sv, int64_t* done_ids, int32_t* done_iters,
                             double* done_resid, int32_t* done_status, int32_t max_out,
                             int32_t* n_done, int32_t* n_active, int32_t* n_queued) {
  if (!sv || !n_done || max_out < 0 || (max_out > 0 && (!done_ids || !done_iters || !done_resid ||
                                                        !done_status)))
    return MSLD_EINVAL;
  // 1. admission, first come first served
  std::vector<msld_server::Cls*> touched;
  while (admit_head(sv)) {
  }
  // refresh ||Y||^2 of classes that admitted requests (slots' Y changed)
  for (msld_server::Cls* c : sv->cls)
    if (c->nactive > 0 && !c->stepped) {
      if (launch_ynorms(c->s, c->Y, c->p.N) != MSLD_OK) return MSLD_EDEVICE;
      c->stepped = true;
    }
  // 2. one iteration for every class with active slots, enqueued before any wait
  // (classes whose iteration waits on the host run from worker threads, so that those
  // waits do not delay the other classes' launches)
  std::vector<int32_t> failed(sv->cls.size(), MSLD_OK);
  auto issue = [&](size_t i) {
    msld_server::Cls* c = sv->cls[i];
    msld_status st = hipSetDevice(c->s->device) == hipSuccess ? MSLD_OK : MSLD_EDEVICE;
    if (st == MSLD_OK) st = iterate_once(c->s, c->Y, c->p.N, c->Z, true);
    if (st == MSLD_OK &&
        hipMemcpyAsync(c->s->host_res, dev_res(c->s), 16 * (size_t)c->slots,
                       hipMemcpyDeviceToHost, c->st) != hipSuccess)
      st = MSLD_EDEVICE;
    failed[i] = st;
  };
  std::vector<std::thread> workers;
  for (size_t i = 0; i < sv->cls.size(); ++i) {
    msld_server::Cls* c = sv->cls[i];
    if (c->nactive == 0) continue;
    if (c->s->graphable) {   // no host waits: issue from this thread
      issue(i);
      continue;
    }
    try {
      workers.emplace_back(issue, i);
    } catch (...) {
      issue(i);
    }
  }
  for (auto& t : workers) t.join();
  // 3. residuals, retirement
  for (size_t i = 0; i < sv->cls.size(); ++i) {
    msld_server::Cls* c = sv->cls[i];
    if (c->nactive == 0) continue;
    const msld_params& p = c->p;
    const size_t inst = (size_t)p.M * p.N;
    const size_t MN = inst * c->slots;
    bool sync_ok = failed[i] == MSLD_OK && hipStreamSynchronize(c->st) == hipSuccess;
    bool retired = false;
    for (int z = 0; z < c->slots; ++z) {
      if (!c->used[z]) continue;
      c->iters[z] += 1;
      int32_t status = MSLD_OK;
      double r = -1.0;
      bool finish = false;
      if (!sync_ok) {
        status = failed[i] != MSLD_OK ? failed[i] : MSLD_EDEVICE;
        finish = true;
      } else {
        const double ny2 = c->s->host_res[c->slots + z] > 0 ? c->s->host_res[c->slots + z] : 1.0;
        r = std::sqrt(c->s->host_res[z] / ny2);
        if (!std::isfinite(r)) {
          status = MSLD_ENUMERIC;
          finish = true;
        } else if ((p.tol > 0.f && c->iters[z] % p.check_every == 0 && r <= (double)p.tol) ||
                   c->iters[z] >= p.max_iters) {
          finish = true;
        }
      }
      if (!finish) continue;
      const msld_server::Req& rq = c->req[z];
      if (sync_ok)
        for (int l = 0; l < p.L; ++l)
          if (hipMemcpyAsync(rq.Z + inst * l, c->Z + MN * l + inst * z, 4 * inst,
                             hipMemcpyDeviceToDevice, c->st) != hipSuccess)
            status = MSLD_EDEVICE;
      if (launch_set_int(c->s->d_active, z, 0, c->st) != hipSuccess) status = MSLD_EDEVICE;
      c->used[z] = 0;
      c->nactive -= 1;
      sv->active_total -= 1;
      msld_server::Done d;
      d.id = rq.id;
      d.iters = c->iters[z];
      d.status = status;
      d.resid = r;
      sv->done.push_back(d);
      retired = true;
    }
    if (retired) (void)hipStreamSynchronize(c->st);   // outputs complete before reporting
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
