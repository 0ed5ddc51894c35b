// Request server of libhmlik (hm_server_* in include/hmlik.h): evaluations of
// eq. (4) of Section 3.1, the calls a likelihood maximiser issues, for a
// stream of (dataset, theta, accuracy) requests on resident datasets, with
// continuous batching at the granularity of one dependency level of the
// H-Cholesky task graph (Section 3.2).
//
// One worker thread owns the context's device work.  Each step it
//   1. retires requests whose factorisation or forward solve has finished,
//   2. admits queued requests into free batch slots (assembly of C~(theta),
//      Section 2.1 and Remark 2.4, enqueued at once),
//   3. launches one batched level kernel that advances every admitted
//      factorisation by one level of its own schedule, and waits for it.
// A finished factorisation's forward solve and log-determinant run on a
// second stream with a workspace slot of their own, beside the next steps.
// The tasks, their inputs and their order within each dataset are those of
// a single evaluation, so every result is bitwise that of hm_loglik.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hm_internal.h"

using namespace hm;
using namespace hm_int;

namespace {

using Clock = std::chrono::steady_clock;

enum class RState { QUEUED, ACTIVE, SOLVING, DONE };

struct Request {
  uint64_t ticket = 0;
  hm_dataset* ds = nullptr;
  hm_theta th{};
  hm_approx ap{};
  int32_t r = 0;
  RState state = RState::QUEUED;
  bool cancel = false;
  int slot = -1;
  int32_t level = 0;   // next level of the dataset's schedule to run
  int32_t max_rank = 0;
  hm_status status = HM_OK;
  std::vector<hm_result> res;
  hm_request_stats stats{};
  Clock::time_point t_submit;
};

// Host records of one batch slot, written by asynchronous copies on the
// streams (pinned memory), and the events that say when they are complete.
struct Slot {
  Request* req = nullptr;
  bool factor_pending = false;   // last level launched; breakdown record being copied
  hipEvent_t ev_fac = nullptr, ev_sol0 = nullptr, ev_sol1 = nullptr;
  int32_t* h_abort = nullptr;
  unsigned long long* h_key = nullptr;
  int32_t* h_rank = nullptr;     // rank of every block (max_nblocks entries)
  double* h_out = nullptr;       // log-det and v^T v per column (1 + max_r entries)
};

double seconds_since(Clock::time_point t) {
  return std::chrono::duration<double>(Clock::now() - t).count();
}

}  // namespace

struct hm_server {
  hm_ctx* ctx = nullptr;
  int32_t max_active = 0;
  int64_t budget = 0;
  hipStream_t st = nullptr, st_solve = nullptr;
  DevData* dD = nullptr;     // device: one dataset descriptor per slot
  int32_t* dseg = nullptr;   // device: the step's task range per slot
  DevData* hD = nullptr;     // pinned staging of dD
  int32_t* hseg = nullptr;   // pinned staging of dseg
  char* pinned = nullptr;    // the slots' host records, one pinned allocation
  double* solve_ws = nullptr;
  int64_t max_nblocks = 0;
  int32_t max_r = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> reqs;   // every request not yet retired by a poll
  uint64_t next_ticket = 1;
  bool stop = false;
  hm_status failed = HM_OK;
  std::map<hm_dataset*, uint64_t> last_use;
  uint64_t use_clock = 0;
  std::thread worker;
};

namespace {

// Marks q finished with `status` (results already filled when the solve ran;
// otherwise r entries carrying the status and NaN values) and frees its slot.
void complete(hm_server* sv, Request* q, hm_status status) {
  if (q->res.empty()) {
    q->res.resize(q->r);
    for (hm_result& o : q->res) {
      std::memset(&o, 0, sizeof(o));
      o.loglik = o.logdet = o.quadform = NAN;
      o.fail_block = -1;
      o.fail_pivot = -1;
    }
  }
  for (hm_result& o : q->res) o.status = status;
  q->status = status;
  q->state = RState::DONE;
  if (q->slot >= 0) {
    sv->slots[q->slot].req = nullptr;
    sv->slots[q->slot].factor_pending = false;
    q->slot = -1;
  }
  q->stats.t_latency = seconds_since(q->t_submit);
  sv->cv_done.notify_all();
}

bool dataset_in_use(const hm_server* sv, const hm_dataset* ds) {
  for (const Slot& s : sv->slots)
    if (s.req && s.req->ds == ds) return true;
  return false;
}

int64_t attached_bytes(const hm_ctx* ctx) {
  int64_t b = 0;
  for (const hm_dataset* d : ctx->datasets)
    if (d->store) b += (int64_t)d->store_bytes;
  return b;
}

// Makes room for `need` more bytes of factor storage by releasing the storage
// of datasets no admitted request uses, least recently used first.
bool make_room(hm_server* sv, const hm_dataset* keep, int64_t need) {
  if (sv->budget <= 0) return true;
  while (attached_bytes(sv->ctx) + need > sv->budget) {
    hm_dataset* victim = nullptr;
    uint64_t oldest = ~0ull;
    for (hm_dataset* d : sv->ctx->datasets) {
      if (!d->store || d == keep || dataset_in_use(sv, d)) continue;
      auto it = sv->last_use.find(d);
      const uint64_t u = it == sv->last_use.end() ? 0 : it->second;
      if (u < oldest) {
        oldest = u;
        victim = d;
      }
    }
    if (!victim) return false;
    release_store(victim);
  }
  return true;
}

// Enqueues, after a factorisation's last level, the copies of its breakdown
// record and ranks, and the event that marks them complete.
bool enqueue_factor_end(hm_server* sv, int k) {
  Slot& s = sv->slots[k];
  const DevData& D = s.req->ds->D;
  const size_t nb = s.req->ds->tree.bk.size();
  bool ok = hipMemcpyAsync(s.h_abort, D.abort_flag, sizeof(int32_t), hipMemcpyDeviceToHost, sv->st) == hipSuccess &&
            hipMemcpyAsync(s.h_key, D.fail_key, sizeof(unsigned long long), hipMemcpyDeviceToHost, sv->st) ==
                hipSuccess &&
            hipMemcpyAsync(s.h_rank, D.rank, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, sv->st) == hipSuccess &&
            hipEventRecord(s.ev_fac, sv->st) == hipSuccess;
  s.factor_pending = true;
  return ok;
}

// Admits q into slot k: assembly, breakdown-flag reset and the slot's
// dataset descriptor, all enqueued on the server's stream.
bool admit(hm_server* sv, Request* q, int k) {
  hm_dataset* ds = q->ds;
  Slot& s = sv->slots[k];
  q->slot = k;
  s.req = q;
  q->state = RState::ACTIVE;
  q->level = 0;
  q->stats.t_queue = seconds_since(q->t_submit);
  sv->last_use[ds] = ++sv->use_clock;
  const hm_status a = assemble_launch(ds, &q->th, &q->ap, sv->st);
  if (a == HM_ERR_OOM || a == HM_ERR_ARG) {
    complete(sv, q, a);
    return true;
  }
  if (a != HM_OK) return false;
  sv->hD[k] = ds->D;
  if (hipMemcpyAsync(sv->dD + k, sv->hD + k, sizeof(DevData), hipMemcpyHostToDevice, sv->st) != hipSuccess ||
      launch_factor_init(ds->D, sv->st) != hipSuccess)
    return false;
  if ((int32_t)ds->level_begin.size() - 1 <= 0) return enqueue_factor_end(sv, k);
  return true;
}

// Enqueues the forward solve and log-determinant of slot k's request on the
// solve stream, after its factorisation's end event.
bool enqueue_solve(hm_server* sv, int k) {
  Slot& s = sv->slots[k];
  hm_dataset* ds = s.req->ds;
  DevData Ds = ds->D;
  Ds.ws = sv->solve_ws;
  return hipStreamWaitEvent(sv->st_solve, s.ev_fac, 0) == hipSuccess &&
         hipEventRecord(s.ev_sol0, sv->st_solve) == hipSuccess &&
         launch_solve(Ds, ds->d_Z, ds->d_perm, ds->r, ds->d_W, ds->d_diag_ids,
                      (int32_t)ds->plan.diag_leaf_ids.size(), ds->d_out, sv->st_solve) == hipSuccess &&
         hipMemcpyAsync(s.h_out, ds->d_out, sizeof(double) * (1 + ds->r), hipMemcpyDeviceToHost, sv->st_solve) ==
             hipSuccess &&
         hipEventRecord(s.ev_sol1, sv->st_solve) == hipSuccess;
}

float elapsed_s(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return NAN;
  }
  return ms * 1e-3f;
}

// Host phase part 1: requests whose factorisation or solve has finished, and
// cancellations.  Returns false on a device failure.
bool retire(hm_server* sv) {
  for (int k = 0; k < sv->max_active; ++k) {
    Slot& s = sv->slots[k];
    Request* q = s.req;
    if (!q) continue;
    hm_dataset* ds = q->ds;
    if (q->state == RState::ACTIVE && s.factor_pending) {
      const hipError_t e = hipEventQuery(s.ev_fac);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return false;
      s.factor_pending = false;
      ds->t_assemble = elapsed_s(ds->ev[0], ds->ev[1]);
      ds->t_factor = elapsed_s(ds->ev[1], s.ev_fac);
      ds->t_solve = 0;
      const hm_status fs = decode_factor_status(ds, *s.h_abort, *s.h_key);
      q->max_rank = max_lr_rank(ds, s.h_rank);
      if (q->cancel) {
        complete(sv, q, HM_ERR_CANCELLED);
      } else if (fs == HM_OK) {
        if (!enqueue_solve(sv, k)) return false;
        q->state = RState::SOLVING;
      } else {
        q->res.resize(q->r);
        fill_results(ds, nullptr, q->max_rank, q->res.data());
        complete(sv, q, fs);
      }
    } else if (q->state == RState::SOLVING) {
      const hipError_t e = hipEventQuery(s.ev_sol1);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return false;
      ds->t_solve = elapsed_s(s.ev_sol0, s.ev_sol1);
      q->res.resize(q->r);
      fill_results(ds, s.h_out, q->max_rank, q->res.data());
      complete(sv, q, HM_OK);
    } else if (q->state == RState::ACTIVE && q->cancel) {
      // stops between levels; the dataset's factor storage is left partly
      // factorised and is overwritten by its next assembly
      complete(sv, q, HM_ERR_CANCELLED);
    }
  }
  return true;
}

// Host phase part 2: admission in arrival order (see include/hmlik.h).
bool admit_queued(hm_server* sv) {
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    int k = -1;
    for (int j = 0; j < sv->max_active && k < 0; ++j)
      if (!sv->slots[j].req) k = j;
    if (k < 0) break;
    Request* q = *it;
    if (dataset_in_use(sv, q->ds)) {
      ++it;
      continue;
    }
    if (!q->ds->store && !make_room(sv, q->ds, (int64_t)q->ds->store_bytes)) break;
    it = sv->queue.erase(it);
    if (!admit(sv, q, k)) return false;
  }
  return true;
}

void fail_all(hm_server* sv, hm_status s) {
  sv->failed = s;
  for (Request* q : sv->queue) complete(sv, q, s);
  sv->queue.clear();
  for (Slot& sl : sv->slots)
    if (sl.req) complete(sv, sl.req, s);
}

void worker_main(hm_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  if (hipSetDevice(sv->ctx->device) != hipSuccess) {
    fail_all(sv, HM_ERR_DEVICE);
    return;
  }
  std::vector<int> finishing;
  for (;;) {
    if (!retire(sv) || !admit_queued(sv)) {
      (void)hipGetLastError();
      fail_all(sv, HM_ERR_DEVICE);
      return;
    }
    bool occupied = false, solving = false;
    int32_t total = 0, members = 0;
    finishing.clear();
    for (int k = 0; k < sv->max_active; ++k) {
      Slot& s = sv->slots[k];
      sv->hseg[2 * k] = sv->hseg[2 * k + 1] = 0;
      if (!s.req) continue;
      occupied = true;
      Request* q = s.req;
      if (q->state == RState::SOLVING) solving = true;
      if (q->state != RState::ACTIVE || s.factor_pending) continue;
      const std::vector<int32_t>& lb = q->ds->level_begin;
      const int32_t nlev = (int32_t)lb.size() - 1;
      if (q->level >= nlev) continue;
      sv->hseg[2 * k] = lb[q->level];
      sv->hseg[2 * k + 1] = lb[q->level + 1];
      total += lb[q->level + 1] - lb[q->level];
      ++members;
      if (++q->level == nlev) finishing.push_back(k);
    }
    if (!occupied && sv->queue.empty() && sv->stop) return;
    if (members == 0) {
      // nothing to launch: poll a running solve or factorisation record, or
      // wait for a submission
      if (solving || occupied)
        sv->cv_work.wait_for(lk, std::chrono::microseconds(200));
      else
        sv->cv_work.wait(lk);
      continue;
    }
    for (int k = 0; k < sv->max_active; ++k) {
      Request* q = sv->slots[k].req;
      if (q && sv->hseg[2 * k + 1] > sv->hseg[2 * k]) {
        ++q->stats.steps;
        q->stats.peak_batch = std::max(q->stats.peak_batch, members);
      }
    }
    // device phase: the lock is released so that submit, poll and cancel proceed
    lk.unlock();
    bool ok = hipMemcpyAsync(sv->dseg, sv->hseg, sizeof(int32_t) * 2 * sv->max_active, hipMemcpyHostToDevice,
                             sv->st) == hipSuccess &&
              launch_level_batch(sv->dD, sv->dseg, sv->max_active, total, NSLOTS, sv->st) == hipSuccess;
    for (int k : finishing) ok = ok && enqueue_factor_end(sv, k);
    ok = ok && hipStreamSynchronize(sv->st) == hipSuccess;
    lk.lock();
    if (!ok) {
      (void)hipGetLastError();
      fail_all(sv, HM_ERR_DEVICE);
      return;
    }
  }
}

void free_server(hm_server* sv) {
  (void)hipSetDevice(sv->ctx->device);
  if (sv->st) (void)hipStreamSynchronize(sv->st);
  if (sv->st_solve) (void)hipStreamSynchronize(sv->st_solve);
  for (Slot& s : sv->slots)
    for (hipEvent_t e : {s.ev_fac, s.ev_sol0, s.ev_sol1})
      if (e) (void)hipEventDestroy(e);
  if (sv->dD) (void)hipFree(sv->dD);
  if (sv->dseg) (void)hipFree(sv->dseg);
  if (sv->solve_ws) (void)hipFree(sv->solve_ws);
  if (sv->hD) (void)hipHostFree(sv->hD);
  if (sv->hseg) (void)hipHostFree(sv->hseg);
  if (sv->pinned) (void)hipHostFree(sv->pinned);
  if (sv->st) (void)hipStreamDestroy(sv->st);
  if (sv->st_solve) (void)hipStreamDestroy(sv->st_solve);
  (void)hipGetLastError();
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

}  // namespace

namespace hm_int {

void server_forget_dataset(hm_server* sv, hm_dataset* ds) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    if ((*it)->ds == ds) {
      complete(sv, *it, HM_ERR_CANCELLED);
      it = sv->queue.erase(it);
    } else {
      ++it;
    }
  }
  for (Slot& s : sv->slots)
    if (s.req && s.req->ds == ds) s.req->cancel = true;
  sv->cv_work.notify_all();
  sv->cv_done.wait(lk, [&] { return !dataset_in_use(sv, ds) || sv->failed != HM_OK; });
  sv->last_use.erase(ds);
  sv->ctx->datasets.erase(ds);   // the worker no longer counts its storage
}

}  // namespace hm_int

extern "C" {

hm_status hm_server_create(hm_ctx* ctx, const hm_server_opts* opts, hm_server** out) {
  if (!ctx || !opts || !out) return HM_ERR_ARG;
  *out = nullptr;
  if (opts->max_active < 1 || opts->max_active > 64 || opts->hbm_budget < 0) return HM_ERR_ARG;
  if (ctx->datasets.empty() || !ctx->ws) return HM_ERR_ARG;
  if (ctx->server.load()) return HM_ERR_BUSY;
  if (hipSetDevice(ctx->device) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_DEVICE;
  }
  hm_server* sv = new (std::nothrow) hm_server;
  if (!sv) return HM_ERR_OOM;
  sv->ctx = ctx;
  sv->max_active = opts->max_active;
  sv->budget = opts->hbm_budget;
  for (const hm_dataset* d : ctx->datasets) {
    sv->max_nblocks = std::max<int64_t>(sv->max_nblocks, (int64_t)d->tree.bk.size());
    sv->max_r = std::max(sv->max_r, d->r);
  }
  const int A = sv->max_active;
  sv->slots.resize(A);
  // per slot: abort flag, breakdown key, ranks, solve output (8-byte aligned pieces)
  const size_t per = 16 + 8 * (size_t)((sv->max_nblocks + 1) / 2) + 8 * (size_t)(1 + std::max(sv->max_r, 1));
  bool ok = hipStreamCreateWithFlags(&sv->st, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->st_solve, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc((void**)&sv->dD, sizeof(DevData) * A) == hipSuccess &&
            hipMalloc((void**)&sv->dseg, sizeof(int32_t) * 2 * A) == hipSuccess &&
            hipMalloc((void**)&sv->solve_ws, sizeof(double) * ctx->ws_stride) == hipSuccess &&
            hipHostMalloc((void**)&sv->hD, sizeof(DevData) * A, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&sv->hseg, sizeof(int32_t) * 2 * A, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&sv->pinned, per * A, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ok && k < A; ++k) {
    Slot& s = sv->slots[k];
    char* base = sv->pinned + per * k;
    s.h_abort = (int32_t*)base;
    s.h_key = (unsigned long long*)(base + 8);
    s.h_rank = (int32_t*)(base + 16);
    s.h_out = (double*)(base + 16 + 8 * ((sv->max_nblocks + 1) / 2));
    ok = hipEventCreate(&s.ev_fac) == hipSuccess && hipEventCreate(&s.ev_sol0) == hipSuccess &&
         hipEventCreate(&s.ev_sol1) == hipSuccess;
  }
  if (ok) {
    std::memset(sv->hD, 0, sizeof(DevData) * A);
    std::memset(sv->hseg, 0, sizeof(int32_t) * 2 * A);
    ok = hipMemcpy(sv->dD, sv->hD, sizeof(DevData) * A, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_server(sv);
    return HM_ERR_OOM;
  }
  hm_server* expected = nullptr;
  if (!ctx->server.compare_exchange_strong(expected, sv)) {
    free_server(sv);
    return HM_ERR_BUSY;
  }
  try {
    sv->worker = std::thread(worker_main, sv);
  } catch (...) {
    ctx->server.store(nullptr);
    free_server(sv);
    return HM_ERR_INTERNAL;
  }
  *out = sv;
  return HM_OK;
}

hm_status hm_server_submit(hm_server* sv, hm_dataset* ds, const hm_theta* theta, const hm_approx* approx,
                           uint64_t* ticket) {
  if (!sv || !ds || !ticket || ds->ctx != sv->ctx || ds->r < 1) return HM_ERR_ARG;
  const hm_status c = check_theta_approx(theta, approx);
  if (c != HM_OK) return c;
  if (sv->budget > 0 && (int64_t)ds->store_bytes > sv->budget) return HM_ERR_OOM;
  Request* q = new (std::nothrow) Request;
  if (!q) return HM_ERR_OOM;
  q->ds = ds;
  q->th = *theta;
  q->ap = *approx;
  q->r = ds->r;
  q->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->failed != HM_OK || sv->stop) {
    delete q;
    return sv->failed != HM_OK ? sv->failed : HM_ERR_ARG;
  }
  q->ticket = sv->next_ticket++;
  sv->reqs[q->ticket] = q;
  sv->queue.push_back(q);
  *ticket = q->ticket;
  sv->cv_work.notify_all();
  return HM_OK;
}

hm_status hm_server_poll(hm_server* sv, uint64_t ticket, int32_t wait, hm_result* out, hm_request_stats* stats,
                         int32_t* done) {
  if (!sv || !out || !done) return HM_ERR_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HM_ERR_ARG;
  Request* q = it->second;
  if (wait) sv->cv_done.wait(lk, [&] { return q->state == RState::DONE; });
  if (q->state != RState::DONE) {
    *done = 0;
    return HM_OK;
  }
  std::copy(q->res.begin(), q->res.end(), out);
  if (stats) *stats = q->stats;
  const hm_status s = q->status;
  sv->reqs.erase(it);
  delete q;
  *done = 1;
  return s;
}

hm_status hm_server_cancel(hm_server* sv, uint64_t ticket) {
  if (!sv) return HM_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HM_ERR_ARG;
  Request* q = it->second;
  if (q->state == RState::QUEUED) {
    sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), q));
    complete(sv, q, HM_ERR_CANCELLED);
  } else if (q->state == RState::ACTIVE) {
    q->cancel = true;
    sv->cv_work.notify_all();
  }
  return HM_OK;
}

void hm_server_destroy(hm_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Request* q : sv->queue) complete(sv, q, HM_ERR_CANCELLED);
    sv->queue.clear();
    sv->cv_work.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  hm_ctx* ctx = sv->ctx;
  free_server(sv);
  ctx->server.store(nullptr);
}

}  // extern "C"
