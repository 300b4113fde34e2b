// em_server.cpp -- serving loop of libem.so: continuous batching of
// deconvolution jobs (each one EM run of Eq. (2), arXiv:2302.05804, Sec. 2).
//
//  * em_submit copies a job's host inputs and queues it (non-blocking): into
//    the server's pinned host staging area when it has room (the upload at
//    admission is then a DMA that does not hold up the worker), else into
//    pageable host memory.
//  * A worker thread admits queued jobs in arrival order while a slot and
//    enough of the HBM budget are free.  The budget is one device arena
//    allocated at em_server_create; every job's inputs, iterate and workspace
//    are first-fit sub-allocations of it (only the small per-round descriptor
//    tables are allocated separately, when they grow).
//  * All active jobs advance together in rounds of one EM iteration.  A round
//    is one batched launch per kernel family (forward, then adjoint with the
//    fused update) whose work items are the (job, tile, frame group) items of
//    every active job; the round is captured in a HIP graph and replayed until
//    the set of active jobs changes (a job finishes or one is admitted).
//  * A finished job's final log-likelihood and iterate are copied to host
//    memory and its device memory is returned to the arena immediately, so a
//    queued job can take its place in the next round.
// Every served job uses the serving plan (one frame group in the adjoint,
// fixed kernel variants), which depends on the job's shape only: its result
// is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "em.h"
#include "em_internal.h"

using namespace em;

namespace {

enum JobState { J_QUEUED, J_ACTIVE, J_DONE, J_FAILED, J_CANCELED };

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Job {
  em_job_id id = 0;
  em_problem prob{};
  Geometry g{};
  int n_iter = 0, done_iter = 0;
  std::vector<float> y, v, psf;   // host copies until admission (y and v
                                  // only when not staged in pinned memory)
  float *hy = nullptr, *hv = nullptr;   // y and v in the pinned staging area
  size_t pin_off = 0, pin_len = 0;      // its range there (pin_len 0: none)
  std::vector<float> x_out;       // result
  double loglik = 0.0;
  JobState state = J_QUEUED;
  int err = EM_OK;
  std::string errmsg;
  bool cancel = false;
  int waiters = 0;                // em_wait calls blocked on this job (em_release
                                  // keeps the job while any is)
  size_t off = 0, bytes = 0;      // arena range
  em_ctx* ctx = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // device views into the arena
  float *dy = nullptr, *dv = nullptr, *dpsf = nullptr, *dx = nullptr;
  void* dws = nullptr;
  size_t ws_bytes = 0;
};

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }

 private:
  std::map<size_t, size_t> free_;
};

// Device-side descriptor table of one kernel family for the current round.
struct Family {
  int kind = 0;       // 0 = FP32 direct, 1 = matrix core
  int sr = 1, KT = 43, precision = EM_FP32, fvar = 0, avar = 0;
  bool robust = false;  // Student-t noise: E-step weights in the forward, numerator adjoint
  bool r16 = false;     // FP16 split, Gaussian (sr = 1, or sr = 2 with frames in N): binary16 r planes
  bool m2n = false;     // FP16 split, sr = 2: forward with the frames in the N dimension
  std::vector<FwdLaunch> fwd32;
  std::vector<AdjLaunch> adj32, adjB32;
  std::vector<MfmaLaunch> fwdmf, adjmf, adjBmf;
  std::vector<int4> fitems, aitems;
  // device copies
  void* d_fdesc = nullptr;
  void* d_adesc = nullptr;
  void* d_bdesc = nullptr;   // numerator adjoints (Student-t), same items as the adjoint
  int4* d_fitems = nullptr;
  int4* d_aitems = nullptr;
  size_t cap_fdesc = 0, cap_adesc = 0, cap_bdesc = 0, cap_fitems = 0, cap_aitems = 0;
};

// job bytes: inputs, iterate and workspace under the serving plan
bool job_layout(const Geometry& g, size_t* total, size_t* o_y, size_t* o_v, size_t* o_psf,
                size_t* o_x, size_t* o_ws, size_t* ws_bytes) {
  const Plan pl = make_serving_plan(g);
  const Layout L = make_layout(g, pl);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al256(b);
    return o;
  };
  const size_t fb = (size_t)g.n * g.Nf * sizeof(float);
  *o_y = take(fb);
  *o_v = take(fb);
  *o_psf = take((size_t)g.n * g.K * g.K * sizeof(float));
  *o_x = take((size_t)g.Nl * sizeof(float));
  *o_ws = take(L.total);
  *ws_bytes = L.total;
  *total = off;
  return true;
}

}  // namespace

struct em_server {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // admissions (input upload, set-up) and finishing run on a second stream,
  // so that jobs can be admitted while the rounds of the others run
  hipStream_t side = nullptr;
  char* arena_base = nullptr;
  size_t budget = 0;
  Arena arena;
  // pinned host staging of queued jobs' y and v (a quarter of the budget, at
  // most 2 GiB; none if the allocation fails)
  char* pin_base = nullptr;
  size_t pin_bytes = 0;
  Arena pin_arena;
  int64_t staged_pinned = 0, staged_pageable = 0;
  int max_slots = 1;
  int round_chunk = 8;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::map<em_job_id, Job*> jobs;
  em_job_id next_id = 1;
  bool stop = false;
  std::thread worker;
  // round state
  std::vector<Family> fams;
  std::vector<R16Job> r16jobs;     // scale step of the r16 jobs of the round
  void* d_r16jobs = nullptr;
  size_t cap_r16jobs = 0;
  bool dirty = true;
  hipGraphExec_t graph{};
  bool graph_ok = false;
  int64_t rounds = 0, graphs_built = 0;
  // worker seconds per phase: admission (input upload, em_init), round
  // rebuilds (descriptors, graph capture), rounds (launch to completion),
  // finishing (final loglik, result copy)
  double sec_admit = 0, sec_build = 0, sec_rounds = 0, sec_finish = 0;
  std::string worker_error;
};

namespace {

template <class T>
int upload(em_server* S, void** dptr, size_t* cap, const std::vector<T>& v) {
  const size_t need = v.size() * sizeof(T);
  if (need == 0) return EM_OK;
  if (*cap < need) {
    if (*dptr) (void)hipFree(*dptr);
    *dptr = nullptr;
    *cap = 0;
    if (hipMalloc(dptr, need * 2) != hipSuccess) return fail(EM_EDEVICE, "descriptor allocation");
    *cap = need * 2;
  }
  if (hipMemcpyAsync(*dptr, v.data(), need, hipMemcpyHostToDevice, S->stream) != hipSuccess)
    return fail(EM_EDEVICE, "descriptor upload");
  return EM_OK;
}

// Work items of one job, ordered so that the longest items come first in the
// family's list (the persistent workgroups take items round-robin).
void add_items(std::vector<int4>& items, int desc, int tiles, int groups) {
  for (int gidx = 0; gidx < groups; ++gidx)
    for (int t = 0; t < tiles; ++t) items.push_back(make_int4(desc, t, gidx, 0));
}

int build_round(em_server* S) {
  // keep device buffers of existing families, rebuild their contents
  std::vector<Family> old;
  old.swap(S->fams);
  auto family_of = [&](const em_ctx* c) -> Family& {
    const int kind = uses_mfma(c->g) ? 1 : 0;
    const bool robust = c->g.weight_mode == EM_W_STUDENT_T;
    const bool r16 = uses_r16(c->g);
    const bool m2n = uses_m2n(c->g);
    for (auto& f : S->fams)
      if (f.kind == kind && f.sr == c->g.sr && f.KT == c->g.KT && f.precision == c->g.precision &&
          f.fvar == c->pl.fwd_variant && f.avar == c->pl.adj_variant && f.robust == robust &&
          f.r16 == r16 && f.m2n == m2n)
        return f;
    Family f;
    f.kind = kind;
    f.robust = robust;
    f.r16 = r16;
    f.m2n = m2n;
    f.sr = c->g.sr;
    f.KT = c->g.KT;
    f.precision = c->g.precision;
    f.fvar = c->pl.fwd_variant;
    f.avar = c->pl.adj_variant;
    // reuse device buffers of an old family slot if there is one
    if (!old.empty()) {
      Family& o = old.back();
      f.d_fdesc = o.d_fdesc; f.cap_fdesc = o.cap_fdesc;
      f.d_adesc = o.d_adesc; f.cap_adesc = o.cap_adesc;
      f.d_bdesc = o.d_bdesc; f.cap_bdesc = o.cap_bdesc;
      f.d_fitems = o.d_fitems; f.cap_fitems = o.cap_fitems;
      f.d_aitems = o.d_aitems; f.cap_aitems = o.cap_aitems;
      old.pop_back();
    }
    S->fams.push_back(f);
    return S->fams.back();
  };
  // longest jobs (frames x pixels) first
  std::vector<Job*> order = S->active;
  std::stable_sort(order.begin(), order.end(), [](const Job* a, const Job* b) {
    return (double)a->g.n * a->g.Nl > (double)b->g.n * b->g.Nl;
  });
  S->r16jobs.clear();
  for (Job* j : order) {
    Family& f = family_of(j->ctx);
    const em_ctx* c = j->ctx;
    // every descriptor is checked against its grid on the host before upload
    const double lcst = f.robust ? student_t_lcst((double)c->g.nu) : 0.0;
    if (f.kind == 1) {
      MfmaLaunch m;
      fill_forward_mfma(c, &m, true, false);
      if (f.robust) {
        m.out_y = c->ry;
        m.nu = c->g.nu;
        m.lcst = lcst;
      }
      if (f.r16) {
        apply_r16(c, &m, 0);
        S->r16jobs.push_back(R16Job{c->x, c->g.Nl, c->r16_xpart, c->r16_umax, c->r16_fsum,
                                    c->r16_e, c->g.n});
      }
      if (!mfma_desc_ok(c->g, 0, c->pl.fwd_tiles, c->pl.fwd_groups, m))
        return fail(EM_EDEVICE, "inconsistent forward descriptor");
      add_items(f.fitems, (int)f.fwdmf.size(), c->pl.fwd_tiles, c->pl.fwd_groups);
      f.fwdmf.push_back(m);
      fill_adjoint_mfma(c, &m, nullptr);
      if (f.r16) apply_r16(c, &m, 1);
      if (!mfma_desc_ok(c->g, 1, c->pl.adj_tiles, 1, m) || m.fused != 1)
        return fail(EM_EDEVICE, "inconsistent adjoint descriptor");
      add_items(f.aitems, (int)f.adjmf.size(), c->pl.adj_tiles, 1);
      f.adjmf.push_back(m);
      if (f.robust) {
        // numerator of the iteration: sum_t F_t^T (u w y) into B
        m.in = c->ry;
        m.fused = 0;
        m.plane = c->B;
        f.adjBmf.push_back(m);
      }
    } else {
      FwdLaunch fl;
      fill_forward_fp32(c, &fl, true, false);
      if (f.robust) {
        fl.out_y = c->ry;
        fl.nu = c->g.nu;
        fl.lcst = lcst;
      }
      if (!forward_desc_ok(c->g, c->pl.fwd_tiles, c->pl.fwd_groups, fl))
        return fail(EM_EDEVICE, "inconsistent forward descriptor");
      add_items(f.fitems, (int)f.fwd32.size(), c->pl.fwd_tiles, c->pl.fwd_groups);
      f.fwd32.push_back(fl);
      AdjLaunch al;
      fill_adjoint_fp32(c, &al, nullptr);
      if (!adjoint_desc_ok(c->g, c->pl.adj_tiles, 1, al) || al.fused != 1)
        return fail(EM_EDEVICE, "inconsistent adjoint descriptor");
      add_items(f.aitems, (int)f.adj32.size(), c->pl.adj_tiles, 1);
      f.adj32.push_back(al);
      if (f.robust) {
        al.in = c->ry;
        al.fused = 0;
        al.plane = c->B;
        f.adjB32.push_back(al);
      }
    }
  }
  for (auto& o : old) {
    if (o.d_fdesc) (void)hipFree(o.d_fdesc);
    if (o.d_adesc) (void)hipFree(o.d_adesc);
    if (o.d_bdesc) (void)hipFree(o.d_bdesc);
    if (o.d_fitems) (void)hipFree(o.d_fitems);
    if (o.d_aitems) (void)hipFree(o.d_aitems);
  }
  int rc;
  for (auto& f : S->fams) {
    if (f.kind == 1) {
      if ((rc = upload(S, &f.d_fdesc, &f.cap_fdesc, f.fwdmf))) return rc;
      if ((rc = upload(S, &f.d_adesc, &f.cap_adesc, f.adjmf))) return rc;
      if ((rc = upload(S, &f.d_bdesc, &f.cap_bdesc, f.adjBmf))) return rc;
    } else {
      if ((rc = upload(S, &f.d_fdesc, &f.cap_fdesc, f.fwd32))) return rc;
      if ((rc = upload(S, &f.d_adesc, &f.cap_adesc, f.adj32))) return rc;
      if ((rc = upload(S, &f.d_bdesc, &f.cap_bdesc, f.adjB32))) return rc;
    }
    if ((rc = upload(S, reinterpret_cast<void**>(&f.d_fitems), &f.cap_fitems, f.fitems))) return rc;
    if ((rc = upload(S, reinterpret_cast<void**>(&f.d_aitems), &f.cap_aitems, f.aitems))) return rc;
  }
  if ((rc = upload(S, &S->d_r16jobs, &S->cap_r16jobs, S->r16jobs))) return rc;
  if (hipStreamSynchronize(S->stream) != hipSuccess) return fail(EM_EDEVICE, "upload sync");
  // capture one round
  if (S->graph_ok) (void)hipGraphExecDestroy(S->graph);
  S->graph_ok = false;
  hipGraph_t gr = nullptr;
  if (hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(EM_EDEVICE, "graph capture");
  // the binary16 scales of every r16 job, from its current iterate
  hipError_t e = launch_r16_scale_batched(static_cast<const R16Job*>(S->d_r16jobs),
                                          (int)S->r16jobs.size(), S->stream);
  for (auto& f : S->fams) {
    if (e != hipSuccess) break;
    const int n = (int)f.fitems.size();
    if (f.kind == 1 && f.sr == 2) {
      e = launch_mfma2_batched(f.precision, 0, f.fvar, static_cast<const MfmaLaunch*>(f.d_fdesc),
                               f.d_fitems, n, std::min(n, 512), S->stream, f.robust, f.m2n);
    } else if (f.kind == 1) {
      e = launch_mfma_batched(f.KT, f.precision, 0, f.fvar,
                              static_cast<const MfmaLaunch*>(f.d_fdesc), f.d_fitems, n,
                              std::min(n, 512), S->stream, f.robust, f.r16);
    } else {
      e = launch_forward_batched(f.sr, f.KT, static_cast<const FwdLaunch*>(f.d_fdesc),
                                 f.d_fitems, n, std::min(n, 1024), S->stream);
    }
    if (e != hipSuccess) break;
  }
  // Student-t families: the numerator of this iteration, before any update
  for (auto& f : S->fams) {
    if (e != hipSuccess) break;
    if (!f.robust) continue;
    const int n = (int)f.aitems.size();
    if (f.kind == 1 && f.sr == 2) {
      e = launch_mfma2_batched(f.precision, 1, f.avar, static_cast<const MfmaLaunch*>(f.d_bdesc),
                               f.d_aitems, n, std::min(n, 1024), S->stream);
    } else if (f.kind == 1) {
      e = launch_mfma_batched(f.KT, f.precision, 1, f.avar,
                              static_cast<const MfmaLaunch*>(f.d_bdesc), f.d_aitems, n,
                              std::min(n, 512), S->stream);
    } else {
      e = launch_adjoint_batched(f.sr, f.KT, static_cast<const AdjLaunch*>(f.d_bdesc),
                                 f.d_aitems, n, std::min(n, 1024), S->stream);
    }
  }
  for (auto& f : S->fams) {
    if (e != hipSuccess) break;
    const int n = (int)f.aitems.size();
    if (f.kind == 1 && f.sr == 2) {
      e = launch_mfma2_batched(f.precision, 1, f.avar, static_cast<const MfmaLaunch*>(f.d_adesc),
                               f.d_aitems, n, std::min(n, 1024), S->stream, false, false, f.r16);
    } else if (f.kind == 1) {
      e = launch_mfma_batched(f.KT, f.precision, 1, f.avar,
                              static_cast<const MfmaLaunch*>(f.d_adesc), f.d_aitems, n,
                              std::min(n, 512), S->stream, false, f.r16);
    } else {
      e = launch_adjoint_batched(f.sr, f.KT, static_cast<const AdjLaunch*>(f.d_adesc),
                                 f.d_aitems, n, std::min(n, 1024), S->stream);
    }
  }
  const hipError_t e2 = hipStreamEndCapture(S->stream, &gr);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return fail(EM_EDEVICE, "round capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&S->graph, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return fail(EM_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  S->graph_ok = true;
  S->graphs_built++;
  S->dirty = false;
  return EM_OK;
}

// The job's pinned staging range back to the staging area (lock held).
void release_job_pinned(em_server* S, Job* j) {
  if (j->pin_len) {
    S->pin_arena.release(j->pin_off, j->pin_len);
    j->pin_len = 0;
    j->hy = j->hv = nullptr;
  }
}

void release_job_device(em_server* S, Job* j) {
  if (j->ctx) {
    em_destroy(j->ctx);
    j->ctx = nullptr;
  }
  if (j->bytes) {
    S->arena.release(j->off, j->bytes);
    j->bytes = 0;
  }
}

// Admission of one job (worker thread, lock not held): inputs to the device,
// em_init with the serving plan.
int admit(em_server* S, Job* j) {
  size_t total, oy, ov, opsf, ox, ows, wsb;
  job_layout(j->g, &total, &oy, &ov, &opsf, &ox, &ows, &wsb);
  char* base = S->arena_base + j->off;
  j->dy = reinterpret_cast<float*>(base + oy);
  j->dv = reinterpret_cast<float*>(base + ov);
  j->dpsf = reinterpret_cast<float*>(base + opsf);
  j->dx = reinterpret_cast<float*>(base + ox);
  j->dws = base + ows;
  j->ws_bytes = wsb;
  const size_t fb = (size_t)j->g.n * j->g.Nf * sizeof(float);
  const float* hy = j->pin_len ? j->hy : j->y.data();
  const float* hv = j->pin_len ? j->hv : j->v.data();
  if (hipMemcpyAsync(j->dy, hy, fb, hipMemcpyHostToDevice, S->side) != hipSuccess ||
      hipMemcpyAsync(j->dv, hv, fb, hipMemcpyHostToDevice, S->side) != hipSuccess ||
      hipMemcpyAsync(j->dpsf, j->psf.data(), j->psf.size() * sizeof(float),
                     hipMemcpyHostToDevice, S->side) != hipSuccess) {
    (void)hipStreamSynchronize(S->side);
    return fail(EM_EDEVICE, "input upload");
  }
  // set-up on the side stream (synchronised inside); the job's rounds start
  // on the round stream after this returns
  const int rc = init_ctx(&j->ctx, &j->prob, j->dy, j->dv, j->dpsf, nullptr, j->dx, j->dws,
                          j->ws_bytes, S->side, true);
  // every copy from the host buffers has completed (also when the set-up
  // stopped early) before they, or the job's arena range, are reused
  if (hipStreamSynchronize(S->side) != hipSuccess && rc == EM_OK)
    return fail(EM_EDEVICE, "input upload: %s", hipGetErrorString(hipGetLastError()));
  std::vector<float>().swap(j->y);
  std::vector<float>().swap(j->v);
  return rc;
}

int finish(em_server* S, Job* j) {
  double ll = 0.0;
  int rc = em_loglik(j->ctx, &ll);
  if (rc) return rc;
  j->x_out.resize((size_t)j->g.Nl);
  if (hipMemcpyAsync(j->x_out.data(), j->dx, (size_t)j->g.Nl * sizeof(float),
                     hipMemcpyDeviceToHost, S->side) != hipSuccess ||
      hipStreamSynchronize(S->side) != hipSuccess)
    return fail(EM_EDEVICE, "result copy");
  j->loglik = ll;
  return EM_OK;
}

// Admission in arrival order while a slot (counting `extra` jobs admitted but
// not yet active) and arena space are free; called with the lock held, which
// it releases around each job's upload and set-up.  Admitted jobs with work
// to do are appended to `admitted`.
void admit_queued(em_server* S, std::unique_lock<std::mutex>& lk, std::vector<Job*>& admitted) {
  while (!S->queue.empty() && (int)(S->active.size() + admitted.size()) < S->max_slots) {
    Job* j = S->queue.front();
    size_t off;
    if (!S->arena.alloc(j->bytes, &off)) break;
    S->queue.pop_front();
    j->off = off;
    j->state = J_ACTIVE;
    j->t_admit = now_s();
    lk.unlock();
    const double ta = now_s();
    const int rc = admit(S, j);
    S->sec_admit += now_s() - ta;
    lk.lock();
    release_job_pinned(S, j);
    if (rc != EM_OK) {
      j->err = rc;
      j->errmsg = em_last_error();
      release_job_device(S, j);
      j->state = J_FAILED;
      j->t_done = now_s();
      S->cv_done.notify_all();
      continue;
    }
    if (j->n_iter == 0) {  // nothing to iterate: finish at once
      lk.unlock();
      const int frc = finish(S, j);
      lk.lock();
      j->err = frc;
      if (frc) j->errmsg = em_last_error();
      release_job_device(S, j);
      j->state = frc ? J_FAILED : J_DONE;
      j->t_done = now_s();
      S->cv_done.notify_all();
      continue;
    }
    admitted.push_back(j);
  }
}

void worker_main(em_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
    if (S->stop) break;
    // --- remove cancelled active jobs
    for (size_t i = 0; i < S->active.size();) {
      Job* j = S->active[i];
      if (j->cancel) {
        release_job_device(S, j);
        j->state = J_CANCELED;
        j->t_done = now_s();
        S->active.erase(S->active.begin() + i);
        S->dirty = true;
        S->cv_done.notify_all();
      } else {
        ++i;
      }
    }
    // --- admission (arrival order, while a slot and arena space are free);
    // with nothing running it goes first, else it overlaps the rounds below
    std::vector<Job*> admitted;
    if (S->active.empty()) {
      admit_queued(S, lk, admitted);
      for (Job* j : admitted) S->active.push_back(j);
      if (!admitted.empty()) S->dirty = true;
      admitted.clear();
    }
    if (S->active.empty()) continue;
    // --- rounds until the first job finishes (at most round_chunk)
    int k = S->round_chunk;
    for (Job* j : S->active) k = std::min(k, j->n_iter - j->done_iter);
    lk.unlock();
    int rc = EM_OK;
    const double tb = now_s();
    if (S->dirty) rc = build_round(S);
    const double tr = now_s();
    if (rc == EM_OK) {
      for (int i = 0; i < k && rc == EM_OK; ++i)
        if (hipGraphLaunch(S->graph, S->stream) != hipSuccess) rc = fail(EM_EDEVICE, "round launch");
    }
    lk.lock();
    // queued jobs are uploaded and set up on the side stream while the rounds run
    if (rc == EM_OK) admit_queued(S, lk, admitted);
    lk.unlock();
    const double tw = now_s();
    if (rc == EM_OK && hipStreamSynchronize(S->stream) != hipSuccess)
      rc = fail(EM_EDEVICE, "round sync: %s", hipGetErrorString(hipGetLastError()));
    lk.lock();
    S->sec_build += tr - tb;
    S->sec_rounds += now_s() - tw;
    for (Job* j : admitted) S->active.push_back(j);
    if (!admitted.empty()) S->dirty = true;
    if (rc != EM_OK) {
      // a device failure ends every active job
      S->worker_error = em_last_error();
      for (Job* j : S->active) {
        j->err = rc;
        j->errmsg = S->worker_error;
        release_job_device(S, j);
        j->state = J_FAILED;
        j->t_done = now_s();
      }
      S->active.clear();
      S->dirty = true;
      S->cv_done.notify_all();
      continue;
    }
    S->rounds += k;
    for (Job* j : S->active)
      if (std::find(admitted.begin(), admitted.end(), j) == admitted.end()) j->done_iter += k;
    for (size_t i = 0; i < S->active.size();) {
      Job* j = S->active[i];
      if (j->done_iter < j->n_iter) {
        ++i;
        continue;
      }
      lk.unlock();
      const double tf = now_s();
      const int frc = finish(S, j);
      lk.lock();
      S->sec_finish += now_s() - tf;
      j->err = frc;
      if (frc) j->errmsg = em_last_error();
      release_job_device(S, j);
      j->state = frc ? J_FAILED : J_DONE;
      j->t_done = now_s();
      S->active.erase(S->active.begin() + i);
      S->dirty = true;
      S->cv_done.notify_all();
    }
  }
  // shutdown: cancel whatever is left
  for (Job* j : S->active) {
    release_job_device(S, j);
    j->state = J_CANCELED;
  }
  S->active.clear();
  for (Job* j : S->queue) {
    release_job_pinned(S, j);
    j->state = J_CANCELED;
  }
  S->queue.clear();
  S->cv_done.notify_all();
}

int job_result(Job* j, float* x_host_out, double* loglik_out) {
  if (j->state == J_DONE) {
    if (x_host_out) std::memcpy(x_host_out, j->x_out.data(), j->x_out.size() * sizeof(float));
    if (loglik_out) *loglik_out = j->loglik;
    return EM_OK;
  }
  if (j->state == J_FAILED) return fail(j->err ? j->err : EM_EDEVICE, "job %lld failed: %s",
                                        (long long)j->id, j->errmsg.c_str());
  if (j->state == J_CANCELED) return fail(EM_ECANCELED, "job %lld was cancelled", (long long)j->id);
  return EM_EAGAIN;
}

}  // namespace

extern "C" {

int em_server_create(em_server** out, size_t hbm_budget, int32_t max_slots, void* stream) {
  if (!out) return fail(EM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return fail(EM_EINVAL, "max_slots must be in [1, 4096]");
  if (hbm_budget < (1u << 20)) return fail(EM_EINVAL, "hbm_budget below 1 MiB");
  em_server* S = new (std::nothrow) em_server();
  if (!S) return fail(EM_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&S->device);
  S->stream = static_cast<hipStream_t>(stream);
  if (S->stream == nullptr) {
    // a created stream (default priority) so that rounds can be graph-captured
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
      delete S;
      return fail(EM_EDEVICE, "stream creation failed");
    }
    S->own_stream = true;
  }
  if (hipMalloc(reinterpret_cast<void**>(&S->arena_base), hbm_budget) != hipSuccess) {
    (void)hipGetLastError();
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(EM_ENOMEM, "cannot allocate an HBM budget of %zu bytes", hbm_budget);
  }
  if (hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(S->arena_base);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(EM_EDEVICE, "stream creation failed");
  }
  S->budget = hbm_budget;
  S->arena.reset(hbm_budget);
  S->pin_bytes = std::min(hbm_budget / 4, (size_t)2 << 30) & ~(size_t)255;
  if (hipHostMalloc(reinterpret_cast<void**>(&S->pin_base), S->pin_bytes,
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    S->pin_base = nullptr;
    S->pin_bytes = 0;
  }
  S->pin_arena.reset(S->pin_bytes);
  S->max_slots = max_slots;
  S->round_chunk = 8;
  S->worker = std::thread(worker_main, S);
  *out = S;
  return EM_OK;
}

int em_server_destroy(em_server* S) {
  if (!S) return EM_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (S->graph_ok) (void)hipGraphExecDestroy(S->graph);
  for (auto& f : S->fams) {
    if (f.d_fdesc) (void)hipFree(f.d_fdesc);
    if (f.d_adesc) (void)hipFree(f.d_adesc);
    if (f.d_bdesc) (void)hipFree(f.d_bdesc);
    if (f.d_fitems) (void)hipFree(f.d_fitems);
    if (f.d_aitems) (void)hipFree(f.d_aitems);
  }
  (void)hipStreamSynchronize(S->stream);
  if (S->d_r16jobs) (void)hipFree(S->d_r16jobs);
  (void)hipStreamSynchronize(S->side);
  (void)hipFree(S->arena_base);
  if (S->pin_base) (void)hipHostFree(S->pin_base);
  (void)hipStreamDestroy(S->side);
  if (S->own_stream) (void)hipStreamDestroy(S->stream);
  for (auto& kv : S->jobs) delete kv.second;
  delete S;
  return EM_OK;
}

int em_submit(em_server* S, const em_problem* p, const float* y_host, const float* v_host,
              const float* psf_host, int32_t n_iter, em_job_id* out) {
  if (!S || !out) return fail(EM_EINVAL, "NULL argument");
  if (!y_host || !v_host || !psf_host) return fail(EM_EINVAL, "NULL input");
  if (n_iter < 0) return fail(EM_EINVAL, "n_iter < 0");
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return fail(EM_EINVAL, "invalid problem: %s", why);
  if (g.weight_mode == EM_W_LITERAL) return fail(EM_ENOTSUP, "weight mode not provided");
  size_t total, a, b, c2, d, e, wsb;
  job_layout(g, &total, &a, &b, &c2, &d, &e, &wsb);
  if (total > S->budget)
    return fail(EM_ENOMEM, "job needs %zu bytes of HBM, the budget is %zu", total, S->budget);
  Job* j = new (std::nothrow) Job();
  if (!j) return fail(EM_ENOMEM, "host allocation failed");
  const size_t nf = (size_t)g.n * g.Nf;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    size_t off;
    if (S->pin_base && S->pin_arena.alloc(al256(2 * nf * sizeof(float)), &off)) {
      j->pin_off = off;
      j->pin_len = al256(2 * nf * sizeof(float));
      S->staged_pinned++;
    } else {
      S->staged_pageable++;
    }
  }
  try {
    if (j->pin_len) {
      // the range is this job's alone until it is queued below
      j->hy = reinterpret_cast<float*>(S->pin_base + j->pin_off);
      j->hv = j->hy + nf;
      std::memcpy(j->hy, y_host, nf * sizeof(float));
      std::memcpy(j->hv, v_host, nf * sizeof(float));
    } else {
      j->y.assign(y_host, y_host + nf);
      j->v.assign(v_host, v_host + nf);
    }
    j->psf.assign(psf_host, psf_host + (size_t)g.n * g.K * g.K);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      release_job_pinned(S, j);
    }
    delete j;
    return fail(EM_ENOMEM, "host copy of the inputs failed");
  }
  j->prob = *p;
  j->g = g;
  j->n_iter = n_iter;
  j->bytes = total;
  j->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    j->id = S->next_id++;
    S->jobs[j->id] = j;
    S->queue.push_back(j);
    *out = j->id;
  }
  S->cv_work.notify_all();
  return EM_OK;
}

int em_poll(em_server* S, em_job_id id, float* x_host_out, double* loglik_out) {
  if (!S) return fail(EM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(EM_EINVAL, "unknown job %lld", (long long)id);
  return job_result(it->second, x_host_out, loglik_out);
}

int em_wait(em_server* S, em_job_id id, float* x_host_out, double* loglik_out) {
  if (!S) return fail(EM_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(EM_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  // the waiter count keeps em_release from freeing the job while this thread
  // sleeps (the predicate reads it after every wake-up)
  ++j->waiters;
  S->cv_done.wait(lk, [&] {
    return j->state == J_DONE || j->state == J_FAILED || j->state == J_CANCELED;
  });
  const int rc = job_result(j, x_host_out, loglik_out);
  --j->waiters;
  return rc;
}

int em_cancel(em_server* S, em_job_id id) {
  if (!S) return fail(EM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(EM_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  if (j->state == J_QUEUED) {
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), j));
    release_job_pinned(S, j);
    j->state = J_CANCELED;
    j->t_done = now_s();
    S->cv_done.notify_all();
  } else if (j->state == J_ACTIVE) {
    j->cancel = true;
    S->cv_work.notify_all();
  }
  return EM_OK;
}

int em_release(em_server* S, em_job_id id) {
  if (!S) return fail(EM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(EM_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  if (j->state == J_QUEUED || j->state == J_ACTIVE)
    return fail(EM_EAGAIN, "job %lld is still pending", (long long)id);
  if (j->waiters > 0)
    return fail(EM_EAGAIN, "job %lld: another thread is still in em_wait", (long long)id);
  S->jobs.erase(it);
  delete j;
  return EM_OK;
}

int em_job_times(em_server* S, em_job_id id, double* t_submit, double* t_admit, double* t_done) {
  if (!S) return fail(EM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(EM_EINVAL, "unknown job %lld", (long long)id);
  const Job* j = it->second;
  if (t_submit) *t_submit = j->t_submit;
  if (t_admit) *t_admit = j->t_admit;
  if (t_done) *t_done = j->t_done;
  return EM_OK;
}

int em_server_stats(em_server* S, int64_t* stats) {
  if (!S || !stats) return fail(EM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t done = 0, failed = 0, canceled = 0;
  for (auto& kv : S->jobs) {
    done += kv.second->state == J_DONE;
    failed += kv.second->state == J_FAILED;
    canceled += kv.second->state == J_CANCELED;
  }
  stats[0] = (int64_t)S->queue.size();
  stats[1] = (int64_t)S->active.size();
  stats[2] = done;
  stats[3] = failed;
  stats[4] = canceled;
  stats[5] = S->rounds;
  stats[6] = S->graphs_built;
  stats[7] = (int64_t)(S->budget - S->arena.free_bytes());
  return EM_OK;
}

int em_server_phase_seconds(em_server* S, double* sec) {
  if (!S || !sec) return fail(EM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  sec[0] = S->sec_admit;
  sec[1] = S->sec_build;
  sec[2] = S->sec_rounds;
  sec[3] = S->sec_finish;
  return EM_OK;
}

int em_server_staging(em_server* S, int64_t* out) {
  if (!S || !out) return fail(EM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = (int64_t)S->pin_bytes;
  out[1] = S->staged_pinned;
  out[2] = S->staged_pageable;
  return EM_OK;
}

size_t em_job_bytes(const em_problem* p) {
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return 0;
  size_t total, a, b, c, d, e, w;
  job_layout(g, &total, &a, &b, &c, &d, &e, &w);
  return total;
}

}  // extern "C"
