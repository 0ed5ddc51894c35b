// Request server of libhmlik (hm_server_* in include/hmlik.h): evaluations of
// eq. (4) of Section 3.1, the calls a likelihood maximiser issues, for a
// stream of (dataset, theta, accuracy) requests on resident datasets.
//
// Continuous batching over HIP streams: every batch slot has a stream of its
// own and its own share of the context's work-group workspace.  An admitted
// request's assembly (Section 2.1, Remark 2.4), its H-Cholesky levels
// (Section 3.2) and its forward solve are enqueued on its slot's stream, so
// the requests advance independently and their kernels overlap on the device
// (one level of one factorisation fills only a few dozen of the 256 CUs).
// A worker thread owns the context's device work: it feeds each slot's stream
// in chunks of levels (two chunks in flight, so that cancellation takes effect
// at a chunk boundary and the host never holds thousands of launches), retires
// finished requests, and admits queued ones as slots and memory free up.
// The tasks, their inputs and their order within each dataset are those of a
// single evaluation, so every result is bitwise that of hm_loglik.
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

constexpr int32_t CHUNK_LEVELS = 128;   // levels enqueued per chunk

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
  int32_t max_rank = 0;
  hm_status status = HM_OK;
  std::vector<hm_result> res;
  hm_request_stats stats{};
  Clock::time_point t_submit;
};

// One batch slot: its stream, its workspace share, the progress of its
// request's enqueued work, and host records written by asynchronous copies
// (pinned memory) with the events that say when they are complete.
struct Slot {
  Request* req = nullptr;
  hipStream_t st = nullptr;
  double* ws = nullptr;
  int32_t next_level = 0;        // first level not yet enqueued
  int32_t chunks = 0;            // chunks enqueued so far
  bool fac_enqueued = false;     // all levels and the breakdown record enqueued
  hipEvent_t ev_chunk[2] = {nullptr, nullptr};
  hipEvent_t ev_fac = nullptr, ev_sol0 = nullptr, ev_sol1 = nullptr;
  int32_t* h_capped = nullptr;   // rank-cap count of the evaluation
  unsigned long long* h_key = nullptr;
  int32_t* h_rank = nullptr;     // rank of every block after the factorisation (max_nblocks entries)
  int32_t* h_rank_C = nullptr;   // the same after the assembly
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
  int grid = 0;              // work-groups (= workspace slots) per batch slot
  char* pinned = nullptr;    // the slots' host records, one pinned allocation
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

// The dataset's descriptor with the slot's workspace share.
DevData slot_view(const Slot& s) {
  DevData D = s.req->ds->D;
  D.ws = s.ws;
  return D;
}

// 1: the chunk enqueued two chunks ago (and so everything before it) has
// finished; 0: not yet; -1: device error.
int chunk_window_free(const Slot& s) {
  if (s.chunks < 2) return 1;
  const hipError_t e = hipEventQuery(s.ev_chunk[s.chunks % 2]);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return -1;
}

// 1: everything enqueued on the slot's stream has finished; 0: not yet; -1: error.
int slot_idle(const Slot& s) {
  if (s.chunks == 0) return 1;
  const hipError_t e = hipEventQuery(s.fac_enqueued ? s.ev_fac : s.ev_chunk[(s.chunks - 1) % 2]);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return -1;
}

// Enqueues the next chunk of levels of slot k's factorisation; after the last
// level, the copies of its breakdown record and ranks and the end event.
bool enqueue_chunk(hm_server* sv, int k) {
  Slot& s = sv->slots[k];
  hm_dataset* ds = s.req->ds;
  const std::vector<int32_t>& lb = ds->level_begin;
  const int32_t nlev = (int32_t)lb.size() - 1;
  const DevData D = slot_view(s);
  const int32_t l0 = s.next_level, l1 = std::min(nlev, l0 + CHUNK_LEVELS);
  if (launch_factor_levels(D, lb.data(), l0, l1, sv->grid, s.st) != hipSuccess) return false;
  s.next_level = l1;
  if (hipEventRecord(s.ev_chunk[s.chunks % 2], s.st) != hipSuccess) return false;
  ++s.chunks;
  ++s.req->stats.steps;
  if (l1 < nlev) return true;
  const size_t nb = ds->tree.bk.size();
  s.fac_enqueued = true;
  return hipMemcpyAsync(s.h_capped, D.capped, sizeof(int32_t), hipMemcpyDeviceToHost, s.st) == hipSuccess &&
         hipMemcpyAsync(s.h_key, D.fail_key, sizeof(unsigned long long), hipMemcpyDeviceToHost, s.st) ==
             hipSuccess &&
         hipMemcpyAsync(s.h_rank, D.rank, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s.st) == hipSuccess &&
         hipEventRecord(s.ev_fac, s.st) == hipSuccess;
}

// Admits q into slot k: assembly and the first chunk of levels on the slot's
// stream.
bool admit(hm_server* sv, Request* q, int k) {
  hm_dataset* ds = q->ds;
  Slot& s = sv->slots[k];
  q->slot = k;
  s.req = q;
  s.next_level = 0;
  s.chunks = 0;
  s.fac_enqueued = false;
  q->state = RState::ACTIVE;
  q->stats.t_queue = seconds_since(q->t_submit);
  sv->last_use[ds] = ++sv->use_clock;
  const hm_status a = assemble_launch(ds, &q->th, &q->ap, s.st, s.ws, sv->grid);
  if (a == HM_ERR_OOM || a == HM_ERR_ARG) {
    complete(sv, q, a);
    return true;
  }
  return a == HM_OK &&
         hipMemcpyAsync(s.h_rank_C, ds->D.rank, sizeof(int32_t) * ds->tree.bk.size(), hipMemcpyDeviceToHost,
                        s.st) == hipSuccess &&
         enqueue_chunk(sv, k);
}

// Enqueues the forward solve and log-determinant of slot k's request after
// its factorisation, on the slot's stream.
bool enqueue_solve(hm_server* sv, int k) {
  Slot& s = sv->slots[k];
  hm_dataset* ds = s.req->ds;
  DevData D = slot_view(s);
  D.W = ds->d_W;
  D.r = ds->r;
  return hipEventRecord(s.ev_sol0, s.st) == hipSuccess &&
         launch_solve(D, ds->d_Z, ds->d_perm, ds->plan.slevel_begin.data(),
                      (int32_t)ds->plan.slevel_begin.size() - 1, sv->grid, ds->d_diag_ids,
                      (int32_t)ds->plan.diag_leaf_ids.size(), ds->d_out, s.st) == hipSuccess &&
         hipMemcpyAsync(s.h_out, ds->d_out, sizeof(double) * (1 + ds->r), hipMemcpyDeviceToHost, s.st) ==
             hipSuccess &&
         hipEventRecord(s.ev_sol1, s.st) == hipSuccess;
}

float elapsed_s(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return NAN;
  }
  return ms * 1e-3f;
}

// Advances every occupied slot: feeds chunks, handles a finished
// factorisation or solve, and cancellations.  Returns false on a device error.
bool progress(hm_server* sv) {
  for (int k = 0; k < sv->max_active; ++k) {
    Slot& s = sv->slots[k];
    Request* q = s.req;
    if (!q) continue;
    hm_dataset* ds = q->ds;
    if (q->state == RState::ACTIVE && q->cancel) {
      // nothing more is enqueued; the request ends once its stream is idle
      const int idle = slot_idle(s);
      if (idle < 0) return false;
      if (idle) complete(sv, q, HM_ERR_CANCELLED);
      continue;
    }
    if (q->state == RState::ACTIVE && !s.fac_enqueued) {
      const int w = chunk_window_free(s);
      if (w < 0) return false;
      if (w && !enqueue_chunk(sv, k)) return false;
      continue;
    }
    if (q->state == RState::ACTIVE) {
      const hipError_t e = hipEventQuery(s.ev_fac);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return false;
      ds->t_assemble = elapsed_s(ds->ev[0], ds->ev[1]);
      ds->t_factor = elapsed_s(ds->ev[1], s.ev_fac);
      ds->t_solve = 0;
      const hm_status fs = decode_factor_status(ds, *s.h_key);
      q->max_rank = max_lr_rank(ds, s.h_rank);
      ds->rank_capped = *s.h_capped;
      ds->bytes_C = storage_bytes(ds, s.h_rank_C);
      ds->bytes_L = storage_bytes(ds, s.h_rank);
      if (fs == HM_OK) {
        if (!enqueue_solve(sv, k)) return false;
        q->state = RState::SOLVING;
      } else {
        q->res.resize(q->r);
        fill_results(ds, nullptr, q->max_rank, q->res.data());
        complete(sv, q, fs);
      }
      continue;
    }
    if (q->state == RState::SOLVING) {
      const hipError_t e = hipEventQuery(s.ev_sol1);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return false;
      ds->t_solve = elapsed_s(s.ev_sol0, s.ev_sol1);
      q->res.resize(q->r);
      fill_results(ds, s.h_out, q->max_rank, q->res.data());
      complete(sv, q, HM_OK);
    }
  }
  return true;
}

// Admission in arrival order (see include/hmlik.h).
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
  for (;;) {
    if (!progress(sv) || !admit_queued(sv)) {
      (void)hipGetLastError();
      fail_all(sv, HM_ERR_DEVICE);
      return;
    }
    int32_t admitted = 0;
    for (const Slot& s : sv->slots) admitted += s.req != nullptr;
    for (Slot& s : sv->slots)
      if (s.req) s.req->stats.peak_batch = std::max(s.req->stats.peak_batch, admitted);
    const bool occupied = admitted > 0;
    if (!occupied && sv->queue.empty() && sv->stop) return;
    // poll the streams while requests run; otherwise sleep until a submission
    if (occupied)
      sv->cv_work.wait_for(lk, std::chrono::microseconds(200));
    else
      sv->cv_work.wait(lk);
  }
}

void free_server(hm_server* sv) {
  (void)hipSetDevice(sv->ctx->device);
  for (Slot& s : sv->slots) {
    if (s.st) (void)hipStreamSynchronize(s.st);
    for (hipEvent_t e : {s.ev_chunk[0], s.ev_chunk[1], s.ev_fac, s.ev_sol0, s.ev_sol1})
      if (e) (void)hipEventDestroy(e);
    if (s.st) (void)hipStreamDestroy(s.st);
  }
  if (sv->pinned) (void)hipHostFree(sv->pinned);
  (void)hipGetLastError();
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

}  // namespace

namespace hm_int {

bool server_store_attached(hm_server* sv, const hm_dataset* ds) {
  std::lock_guard<std::mutex> lk(sv->mu);
  return ds->store != nullptr;
}

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
    if (s.req && s.req->ds == ds && s.req->state == RState::ACTIVE) s.req->cancel = true;
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
  if (opts->max_active < 1 || opts->max_active > 16 || opts->hbm_budget < 0) return HM_ERR_ARG;
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
  sv->grid = NSLOTS / opts->max_active;
  for (const hm_dataset* d : ctx->datasets) {
    sv->max_nblocks = std::max<int64_t>(sv->max_nblocks, (int64_t)d->tree.bk.size());
    sv->max_r = std::max(sv->max_r, d->r);
  }
  const int A = sv->max_active;
  sv->slots.resize(A);
  // per slot: rank-cap count, breakdown key, ranks after the factorisation and
  // after the assembly, solve output (8-byte aligned pieces)
  const size_t rank_bytes = 8 * (size_t)((sv->max_nblocks + 1) / 2);
  const size_t per = 16 + 2 * rank_bytes + 8 * (size_t)(1 + std::max(sv->max_r, 1));
  bool ok = hipHostMalloc((void**)&sv->pinned, per * A, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ok && k < A; ++k) {
    Slot& s = sv->slots[k];
    char* base = sv->pinned + per * k;
    s.h_capped = (int32_t*)base;
    s.h_key = (unsigned long long*)(base + 8);
    s.h_rank = (int32_t*)(base + 16);
    s.h_rank_C = (int32_t*)(base + 16 + rank_bytes);
    s.h_out = (double*)(base + 16 + 2 * rank_bytes);
    s.ws = ctx->ws + (int64_t)k * sv->grid * ctx->ws_stride;
    ok = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&s.ev_chunk[0]) == hipSuccess && hipEventCreate(&s.ev_chunk[1]) == hipSuccess &&
         hipEventCreate(&s.ev_fac) == hipSuccess && hipEventCreate(&s.ev_sol0) == hipSuccess &&
         hipEventCreate(&s.ev_sol1) == hipSuccess;
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
  if (approx && approx->prec != HM_FP64) return HM_ERR_ARG;   // served and batched forms: FP64
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
  ds->fused_solved = false;   // the served solve overwrites the solve buffer
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
  // every request has finished; the context's direct calls may run again
  sv->ctx->server.store(nullptr);
  free_server(sv);
}

}  // extern "C"
