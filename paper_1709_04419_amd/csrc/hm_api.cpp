// C ABI of libhmlik (declared in include/hmlik.h): context, dataset (trees,
// schedule and device storage, built once per set of locations), and the
// per-theta evaluation of eq. (4) of Section 3.1.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <set>
#include <vector>

#include "../../include/hmlik.h"
#include "hm_device.h"
#include "hm_internal.h"
#include "hm_plan.h"

using namespace hm;
using namespace hm_int;

namespace {

hm_status dev_alloc(hm_dataset* ds, size_t bytes, void** out) {
  void* p = nullptr;
  if (bytes == 0) bytes = 64;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_OOM;
  }
  ds->bufs.push_back(DevBuf{p, bytes});
  *out = p;
  return HM_OK;
}

template <class T>
hm_status upload(hm_dataset* ds, const std::vector<T>& v, T** out) {
  void* p = nullptr;
  hm_status s = dev_alloc(ds, v.size() * sizeof(T), &p);
  if (s != HM_OK) return s;
  if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return HM_ERR_DEVICE;
  *out = static_cast<T*>(p);
  return HM_OK;
}

#define TRY(x)                        \
  do {                                \
    hm_status _s = (x);               \
    if (_s != HM_OK) return _s;       \
  } while (0)
#define HIPTRY(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) {                        \
      (void)hipGetLastError();                      \
      return HM_ERR_DEVICE;                         \
    }                                               \
  } while (0)

// Taylor coefficients a_k of 1/Gamma(1+z) = sum a_k z^k (a_0 = 1), i.e. the
// coefficients of 1/Gamma(z) = sum_k a_{k-1} z^k (Abramowitz & Stegun 6.1.34).
constexpr long double RG[8] = {1.0L,
                               0.5772156649015328606L,
                               -0.6558780715202538811L,
                               -0.0420026350340952355L,
                               0.1665386113822914895L,
                               -0.0421977345555443367L,
                               -0.0096219715278769736L,
                               0.0072189432466630995L};

// Per-theta constants of the K_nu evaluation (Temme's method needs
// Gamma_1(mu) = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu) and
// Gamma_2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2 for |mu| <= 1/2).
MaternConst make_matern(const hm_theta& th) {
  MaternConst c{};
  c.sigma2 = th.sigma2;
  c.inv_ell = 1.0 / th.ell;
  c.nu = th.nu;
  c.nugget = th.nugget;
  const long double nu = th.nu;
  c.norm = (double)(1.0L / (powl(2.0L, nu - 1.0L) * tgammal(nu)));
  const long double N = floorl(nu + 0.5L);
  const long double mu = nu - N;
  c.mu = (double)mu;
  c.nrec = (int32_t)N;
  c.half = (th.nu == 0.5) ? 1 : (th.nu == 1.5) ? 3 : (th.nu == 2.5) ? 5 : 0;
  const long double gp = tgammal(1.0L + mu), gm = tgammal(1.0L - mu);
  c.gp = (double)gp;
  c.gm = (double)gm;
  long double g1;
  if (fabsl(mu) < 1e-3L) {
    // odd part of 1/Gamma(1+z): Gamma_1(mu) = -(a1 + a3 mu^2 + a5 mu^4 + a7 mu^6)
    const long double m2 = mu * mu;
    g1 = -(RG[1] + m2 * (RG[3] + m2 * (RG[5] + m2 * RG[7])));
  } else {
    g1 = (1.0L / gm - 1.0L / gp) / (2.0L * mu);
  }
  c.g1 = (double)g1;
  c.g2 = (double)((1.0L / gm + 1.0L / gp) / 2.0L);
  c.fact = (mu == 0.0L) ? 1.0 : (double)(mu * 3.14159265358979323846264338327950288L /
                                         sinl(mu * 3.14159265358979323846264338327950288L));
  return c;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// While a request server runs on a context it alone issues the context's
// device work; the direct entry points then return HM_ERR_BUSY.
bool busy(const hm_ctx* c) { return c->server.load() != nullptr; }

// The dataset's kernels use the context's current workspace.
void use_ctx_ws(hm_dataset* ds) {
  ds->D.ws = ds->ctx->ws;
  ds->D.ws_stride = ds->ctx->ws_stride;
}

// Carves the factor storage at `base` into the dense-leaf pool, the low-rank
// factor pool and the update-term pool (each 256-byte aligned); returns its
// size in bytes.  With base == nullptr only the size is computed.
size_t store_layout(const Plan& P, void* base, DevData& D) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t a = up(sizeof(double) * (size_t)P.dense_pool);
  const size_t b = up(sizeof(double) * (size_t)P.lr_pool);
  const size_t c = up(sizeof(double) * (size_t)P.term_pool);
  const size_t d = up(sizeof(double) * (size_t)P.stage_pool);
  if (base) {
    char* q = static_cast<char*>(base);
    D.dense = (double*)q;
    D.lr = (double*)(q + a);
    D.termbuf = (double*)(q + a + b);
    D.stage = (double*)(q + a + b + c);
  } else {
    D.dense = D.lr = D.termbuf = D.stage = nullptr;
  }
  return a + b + c + d + 256;
}

}  // namespace

namespace hm_int {

hm_status attach_store(hm_dataset* ds) {
  if (ds->store) return HM_OK;
  void* p = nullptr;
  if (hipMalloc(&p, ds->store_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_OOM;
  }
  ds->store = p;
  store_layout(ds->plan, p, ds->D);
  return HM_OK;
}

void release_store(hm_dataset* ds) {
  if (!ds->store) return;
  (void)hipSetDevice(ds->ctx->device);
  (void)hipStreamSynchronize(ds->ctx->stream);
  (void)hipFree(ds->store);
  ds->store = nullptr;
  store_layout(ds->plan, nullptr, ds->D);
  ds->assembled = ds->factored = false;
}

}  // namespace hm_int

namespace {

hm_status build_device(hm_dataset* ds) {
  const Tree& T = ds->tree;
  const Plan& P = ds->plan;
  DevData& D = ds->D;
  D = DevData{};
  D.n = T.n;
  TRY(upload(ds, T.bk, const_cast<Block**>(&D.bk)));
  TRY(upload(ds, T.cl, const_cast<Cluster**>(&D.cl)));
  TRY(upload(ds, T.diag_of, const_cast<int32_t**>(&D.diag_of)));
  D.nblocks = (int32_t)T.bk.size();
  void* p;
  TRY(upload(ds, P.dense_off, const_cast<int64_t**>(&D.dense_off)));
  TRY(upload(ds, P.lr_off, const_cast<int64_t**>(&D.lr_off)));
  TRY(upload(ds, P.lr_voff, const_cast<int64_t**>(&D.lr_voff)));
  TRY(upload(ds, P.lr_cap, const_cast<int32_t**>(&D.lr_cap)));
  TRY(upload(ds, P.stage_off, const_cast<int64_t**>(&D.stage_off)));
  {
    std::vector<int32_t> z(2 * T.bk.size(), 0);
    TRY(upload(ds, z, &D.ts_app));
  }
  {
    std::vector<int32_t> rk(T.bk.size(), 0);
    TRY(upload(ds, rk, &D.rank));
  }
  ds->store_bytes = store_layout(P, nullptr, D);
  TRY(attach_store(ds));
  TRY(upload(ds, P.terms, const_cast<TermDef**>(&D.terms)));
  TRY(upload(ds, P.insts, const_cast<TermInst**>(&D.insts)));
  {
    // the factor tasks, then the data solve's tasks that the stream program
    // runs beside them (ids from ntasks on, no program index)
    std::vector<Task> all(P.tasks);
    all.insert(all.end(), P.ftasks.begin(), P.ftasks.end());
    TRY(upload(ds, all, const_cast<Task**>(&D.tasks)));
    std::vector<int32_t> prog(P.task_prog);
    prog.resize(all.size(), -1);
    TRY(upload(ds, prog, const_cast<int32_t**>(&D.task_prog)));
  }
  TRY(upload(ds, ds->order, &ds->d_order));
  D.order = ds->d_order;
  TRY(upload(ds, P.deps, const_cast<int32_t**>(&D.deps)));
  D.ntasks = (int32_t)P.tasks.size();
  TRY(dev_alloc(ds, 256, &p));
  D.fail_key = (unsigned long long*)p;
  D.capped = (int32_t*)((char*)p + 64);
  TRY(upload(ds, P.sub_begin, const_cast<int32_t**>(&D.sub_begin)));
  TRY(upload(ds, P.sub_end, const_cast<int32_t**>(&D.sub_end)));
  TRY(upload(ds, P.sub_leaves, const_cast<int32_t**>(&D.sub_leaves)));
  TRY(upload(ds, P.stasks, const_cast<Task**>(&D.stasks)));
  TRY(upload(ds, P.btasks, &ds->d_btasks));
  TRY(upload(ds, P.apply_chunks, &ds->d_chunks));
  TRY(upload(ds, P.sop_begin, const_cast<int32_t**>(&D.sop_begin)));
  TRY(upload(ds, P.sops, const_cast<SolveOp**>(&D.sops)));
  TRY(dev_alloc(ds, sizeof(double) * T.bk.size(), &p));
  D.logdet_part = (double*)p;
  TRY(upload(ds, P.dense_ids, const_cast<int32_t**>(&D.dense_ids)));
  D.ndense = (int32_t)P.dense_ids.size();
  TRY(upload(ds, P.lr_ids, const_cast<int32_t**>(&D.lr_ids)));
  D.nlr = (int32_t)P.lr_ids.size();
  TRY(upload(ds, P.diag_leaf_ids, &ds->d_diag_ids));
  TRY(upload(ds, T.perm, &ds->d_perm));
  // workspace slots (one per resident work-group): the largest of
  //   - the single-task flush of a block of at most max_lr_rows rows and
  //     columns: (m + n) x 2 K_MAX accumulated factors plus truncation scratch
  //     (also covers ACA's m x K_MAX and n x K_MAX factors of such blocks);
  //   - an explicit block of at most dflush x dflush with the transposed
  //     triangular factor of its pivoted QR;
  //   - the big blocks' steps: stacked R factors (TS_GMAX p x p per factor,
  //     p <= 2 K_MAX) plus the core truncation's scratch, or a row block of
  //     the truncated factor (ts_rows x K_MAX), or ACA's used flags.
  const int64_t mr = P.max_lr_rows > 64 ? P.max_lr_rows : 64;
  D.dflush = DENSE_FLUSH * T.leaf_size;
  const int64_t df = D.dflush;
  int64_t stride = 2 * mr * (2 * K_MAX) + mr + 2 * (2 * K_MAX + 1) * (2 * K_MAX) + 4096;
  if (stride < df * df + (df + 1) * df + 64) stride = df * df + (df + 1) * df + 64;
  int64_t big_rows = 0;
  for (int32_t b : P.lr_ids)
    if (P.lr_cap[b] == 2 * K_MAX) big_rows = std::max(big_rows, std::max(T.bk[b].m, T.bk[b].n));
  if (big_rows > 0) {
    const int64_t p = 2 * K_MAX;
    const int64_t ts = 2 * TS_GMAX * p * p + (p + 1) * p + 4096;
    stride = std::max(stride, ts);
    stride = std::max(stride, ts_rows(big_rows) * K_MAX + 64);
    stride = std::max(stride, big_rows + 2 * (K_MAX + 1) * K_MAX + 64);
  }
  stride = (stride + 63) & ~(int64_t)63;
  hm_ctx* c = ds->ctx;
  if (c->ws_stride < stride) {
    HIPTRY(hipStreamSynchronize(c->stream));
    if (c->ws) (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_stride = 0;
    void* w = nullptr;
    if (hipMalloc(&w, sizeof(double) * stride * NSLOTS) != hipSuccess) {
      (void)hipGetLastError();
      return HM_ERR_OOM;
    }
    c->ws = (double*)w;
    c->ws_stride = stride;
  }
  use_ctx_ws(ds);
  TRY(dev_alloc(ds, sizeof(double) * (P.tasks.size() + 1), &p));
  D.task_flops = (double*)p;
  if (getenv("HMLIK_TASK_TIMES")) {
    TRY(dev_alloc(ds, sizeof(int64_t) * 7 * (P.tasks.size() + 1), &p));
    D.task_times = (int64_t*)p;
    ds->tt_buf = D.task_times;
  }
  return HM_OK;
}

}  // namespace

extern "C" {

const char* hm_status_string(hm_status s) {
  switch (s) {
    case HM_OK: return "ok";
    case HM_ERR_ARG: return "invalid argument";
    case HM_ERR_NOT_SPD: return "H-Cholesky breakdown: non-positive pivot";
    case HM_ERR_OOM: return "device out of memory";
    case HM_ERR_DEVICE: return "HIP runtime error";
    case HM_ERR_INTERNAL: return "internal invariant failed (planner or schedule)";
    case HM_ERR_CANCELLED: return "request cancelled";
    case HM_ERR_BUSY: return "a request server owns this context";
  }
  return "unknown status";
}

hm_status hm_ctx_create(int device, void* stream, hm_ctx** out) {
  if (!out) return HM_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return HM_ERR_DEVICE;
  }
  HIPTRY(hipSetDevice(device));
  // this GPU's copy of the allocation-free entry point's workspace
  if (noalloc_scratch_init(device) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_DEVICE;
  }
  hm_ctx* c = new (std::nothrow) hm_ctx;
  if (!c) return HM_ERR_OOM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  *out = c;
  return HM_OK;
}

void hm_ctx_destroy(hm_ctx* ctx) {
  if (!ctx) return;
  if (hm_server* sv = ctx->server.load()) hm_server_destroy(sv);
  if (ctx->ws) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->ws);
  }
  delete ctx;
}

hm_status hm_dataset_create(hm_ctx* ctx, const double* coords_in, int64_t n, int32_t d, const hm_tree_opts* opts,
                            int32_t coords_on_device, hm_dataset** out) {
  if (!ctx || !coords_in || !opts || !out || n < 1 || d != 2) return HM_ERR_ARG;
  *out = nullptr;
  if (busy(ctx)) return HM_ERR_BUSY;
  if (opts->leaf_size < 1 || opts->leaf_size > LEAF_MAX) return HM_ERR_ARG;
  if (!std::isfinite(opts->eta) || opts->eta < 0.0) return HM_ERR_ARG;
  HIPTRY(hipSetDevice(ctx->device));
  // the planner runs on the host: device coordinates are copied over first
  std::vector<double> host_coords;
  const double* coords = coords_in;
  if (coords_on_device) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, coords_in) != hipSuccess || at.type != hipMemoryTypeDevice ||
        at.device != ctx->device) {
      (void)hipGetLastError();
      return HM_ERR_ARG;
    }
    try {
      host_coords.resize(2 * (size_t)n);
    } catch (const std::bad_alloc&) {
      return HM_ERR_OOM;
    }
    HIPTRY(hipMemcpyAsync(host_coords.data(), coords_in, sizeof(double) * 2 * n, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    coords = host_coords.data();
  }
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(coords[i])) return HM_ERR_ARG;
  hm_dataset* ds = new (std::nothrow) hm_dataset;
  if (!ds) return HM_ERR_OOM;
  ds->ctx = ctx;
  try {
    build_tree(coords, n, opts->leaf_size, opts->eta, ds->tree);
    build_plan(ds->tree, ds->plan);
  } catch (const std::bad_alloc&) {
    delete ds;
    return HM_ERR_OOM;
  } catch (const std::length_error&) {
    delete ds;              // the task graph outgrows the schedule's 32-bit offsets
    return HM_ERR_OOM;
  } catch (const std::exception&) {
    delete ds;
    return HM_ERR_INTERNAL;
  }
  {
    const auto& tasks = ds->plan.tasks;
    ds->order.resize(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i) ds->order[i] = (int32_t)i;
    ds->level_begin.clear();
    int32_t cur = -1;
    for (int32_t i = 0; i < (int32_t)tasks.size(); ++i)
      if (tasks[i].level != cur) {
        ds->level_begin.push_back(i);
        cur = tasks[i].level;
      }
    ds->level_begin.push_back((int32_t)tasks.size());
  }
  hm_status s = build_device(ds);
  if (s == HM_OK) {
    // permuted coordinates
    std::vector<double> x(n), y(n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] = coords[2 * ds->tree.perm[i]];
      y[i] = coords[2 * ds->tree.perm[i] + 1];
    }
    double *dx = nullptr, *dy = nullptr;
    s = upload(ds, x, &dx);
    if (s == HM_OK) s = upload(ds, y, &dy);
    ds->D.px = dx;
    ds->D.py = dy;
  }
  if (s == HM_OK) {
    for (int i = 0; i < 4 && s == HM_OK; ++i)
      if (hipEventCreate(&ds->ev[i]) != hipSuccess) s = HM_ERR_DEVICE;
  }
  if (s != HM_OK) {
    hm_dataset_destroy(ds);
    return s;
  }
  ctx->datasets.insert(ds);
  *out = ds;
  return HM_OK;
}

void hm_dataset_destroy(hm_dataset* ds) {
  if (!ds) return;
  if (hm_server* sv = ds->ctx->server.load()) server_forget_dataset(sv, ds);
  (void)hipSetDevice(ds->ctx->device);
  (void)hipStreamSynchronize(ds->ctx->stream);
  for (auto& b : ds->bufs) (void)hipFree(b.p);
  for (void* q : {(void*)ds->d_Z, (void*)ds->d_W, (void*)ds->d_out, (void*)ds->d_op, (void*)ds->d_part, ds->c_store,
                  (void*)ds->d_iperm})
    if (q) (void)hipFree(q);
  if (ds->store) (void)hipFree(ds->store);
  for (int i = 0; i < 4; ++i)
    if (ds->ev[i]) (void)hipEventDestroy(ds->ev[i]);
  for (hipEvent_t e : ds->mev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t x : ds->xs)
    if (x) (void)hipStreamDestroy(x);
  ds->ctx->datasets.erase(ds);
  delete ds;
}

hm_status hm_dataset_release(hm_dataset* ds) {
  if (!ds) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  release_store(ds);
  return HM_OK;
}

hm_status hm_dataset_footprint(const hm_dataset* ds, int64_t* resident_bytes, int64_t* factor_bytes,
                               int32_t* attached) {
  if (!ds) return HM_ERR_ARG;
  if (resident_bytes) {
    int64_t s = 0;
    for (const auto& b : ds->bufs) s += (int64_t)b.bytes;
    *resident_bytes = s;
  }
  if (factor_bytes) *factor_bytes = (int64_t)ds->store_bytes;
  if (attached) {
    hm_server* sv = ds->ctx->server.load();
    *attached = sv ? server_store_attached(sv, ds) : ds->store != nullptr;
  }
  return HM_OK;
}

hm_status hm_dataset_set_z(hm_dataset* ds, const double* Z, int32_t r, int32_t on_device) {
  if (!ds || !Z || r < 1 || r > 64) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  const int64_t n = ds->tree.n;
  // validate before anything changes: on an error the old Z stays in place
  if (!on_device) {
    for (int64_t i = 0; i < n * (int64_t)r; ++i)
      if (!std::isfinite(Z[i])) return HM_ERR_ARG;
  } else {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, Z) != hipSuccess || at.type != hipMemoryTypeDevice ||
        at.device != ds->ctx->device) {
      (void)hipGetLastError();
      return HM_ERR_ARG;
    }
  }
  HIPTRY(hipSetDevice(ds->ctx->device));
  double *z = ds->d_Z, *w = ds->d_W, *o = ds->d_out;
  const bool grow = r > ds->zcap;
  if (grow) {
    z = w = o = nullptr;
    const size_t bz = sizeof(double) * n * r;
    if (hipMalloc((void**)&z, bz) != hipSuccess || hipMalloc((void**)&w, bz) != hipSuccess ||
        hipMalloc((void**)&o, sizeof(double) * (1 + r)) != hipSuccess) {
      (void)hipGetLastError();
      for (void* q : {(void*)z, (void*)w, (void*)o})
        if (q) (void)hipFree(q);
      return HM_ERR_OOM;
    }
  }
  const bool ok = hipMemcpyAsync(z, Z, sizeof(double) * n * r,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 ds->ctx->stream) == hipSuccess &&
                  hipStreamSynchronize(ds->ctx->stream) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (grow)
      for (void* q : {(void*)z, (void*)w, (void*)o}) (void)hipFree(q);
    return HM_ERR_DEVICE;
  }
  if (grow) {
    for (void* q : {(void*)ds->d_Z, (void*)ds->d_W, (void*)ds->d_out})
      if (q) (void)hipFree(q);
    ds->d_Z = z;
    ds->d_W = w;
    ds->d_out = o;
    ds->zcap = r;
  }
  ds->r = r;
  ds->fused_solved = false;
  return HM_OK;
}

}  // extern "C"

namespace hm_int {

hm_status alloc_matrix_copy(hm_dataset* ds) {
  const Plan& P = ds->plan;
  const size_t b = sizeof(double) * ((size_t)P.dense_pool + (size_t)P.lr_pool) +
                   sizeof(int32_t) * ds->tree.bk.size() + 256;
  if (hipMalloc(&ds->c_store, b) != hipSuccess) {
    (void)hipGetLastError();
    ds->c_store = nullptr;
    return HM_ERR_OOM;
  }
  ds->c_bytes = b;
  return HM_OK;
}

hm_status check_theta_approx(const hm_theta* th, const hm_approx* ap) {
  if (!th || !ap) return HM_ERR_ARG;
  if (!finite_pos(th->sigma2) || !finite_pos(th->ell) || !finite_pos(th->nu)) return HM_ERR_ARG;
  if (!std::isfinite(th->nugget) || th->nugget < 0.0) return HM_ERR_ARG;
  if (ap->fixed_rank < 0 || ap->fixed_rank > K_MAX) return HM_ERR_ARG;
  if (ap->fixed_rank == 0 && !finite_pos(ap->eps)) return HM_ERR_ARG;
  if (ap->fixed_rank > 0 && !(std::isfinite(ap->eps) && ap->eps >= 0.0)) return HM_ERR_ARG;
  if (th->nu > 50.0) return HM_ERR_ARG;
  if (ap->refine_max_iter < 0 || ap->refine_max_iter > 100 || !std::isfinite(ap->refine_tol) ||
      ap->refine_tol < 0.0)
    return HM_ERR_ARG;
  if (ap->prec == HM_FP64) {
    if (ap->refine_max_iter != 0 || ap->refine_tol != 0.0) return HM_ERR_ARG;
  } else if (ap->prec != HM_MIXED) {
    return HM_ERR_ARG;
  }
  return HM_OK;
}

int64_t storage_bytes(const hm_dataset* ds, const int32_t* rank) {
  int64_t e = ds->plan.n_dense_entries;
  for (int32_t b : ds->plan.lr_ids) {
    const Block& bk = ds->tree.bk[b];
    e += (bk.m + bk.n) * (int64_t)rank[b];
  }
  return 8 * e;
}

hm_status assemble_launch(hm_dataset* ds, const hm_theta* th, const hm_approx* ap, hipStream_t st, double* ws,
                          int grid) {
  TRY(check_theta_approx(th, ap));
  HIPTRY(hipSetDevice(ds->ctx->device));
  TRY(attach_store(ds));
  use_ctx_ws(ds);
  DevData& D = ds->D;
  D.mc = make_matern(*th);
  D.kfix = ap->fixed_rank;
  D.eps = (ap->fixed_rank > 0) ? 0.0 : ap->eps;
  D.kmax = (ap->fixed_rank > 0) ? ap->fixed_rank : K_MAX;
  D.mixed = ap->prec == HM_MIXED ? 1 : 0;
  ds->prec = ap->prec;
  ds->refine_max_iter = ap->refine_max_iter;
  ds->refine_tol = ap->refine_tol;
  // the mixed form refines C~^{-1} Z with the assembled matrix: keep a copy
  if (D.mixed && !ds->c_store) TRY(alloc_matrix_copy(ds));
  DevData Dl = D;
  if (ws) Dl.ws = ws;
  HIPTRY(hipEventRecord(ds->ev[0], st));
  HIPTRY(launch_eval_init(Dl, st));
  HIPTRY(launch_assemble(Dl, st));
  HIPTRY(launch_aca(Dl, ws ? grid : NSLOTS, st));
  ds->theta_set = true;
  ds->c_valid = false;
  if ((ds->keep_c || D.mixed) && ds->c_store) {
    const Plan& P = ds->plan;
    char* q = static_cast<char*>(ds->c_store);
    const size_t bd = sizeof(double) * (size_t)P.dense_pool, bl = sizeof(double) * (size_t)P.lr_pool;
    HIPTRY(hipMemcpyAsync(q, D.dense, bd, hipMemcpyDeviceToDevice, st));
    HIPTRY(hipMemcpyAsync(q + bd, D.lr, bl, hipMemcpyDeviceToDevice, st));
    HIPTRY(hipMemcpyAsync(q + bd + bl, D.rank, sizeof(int32_t) * ds->tree.bk.size(), hipMemcpyDeviceToDevice, st));
    ds->c_valid = true;
  }
  HIPTRY(hipEventRecord(ds->ev[1], st));
  return HM_OK;
}

hm_status decode_factor_status(hm_dataset* ds, unsigned long long key) {
  ds->assembled = false;
  ds->factored = true;
  ds->fail_block = -1;
  ds->fail_pivot = -1;
  if (key != ~0ull) {
    const int64_t prog = (int64_t)(key >> 8);
    ds->fail_pivot = (int32_t)(key & 0xff);
    ds->fail_block = (prog >= 0 && prog < (int64_t)ds->plan.prog_obj.size()) ? ds->plan.prog_obj[prog] : -1;
    ds->factor_status = HM_ERR_NOT_SPD;
    return HM_ERR_NOT_SPD;
  }
  ds->factor_status = HM_OK;
  return HM_OK;
}

int32_t max_lr_rank(const hm_dataset* ds, const int32_t* rank) {
  int32_t mr = 0;
  for (int32_t b : ds->plan.lr_ids) mr = rank[b] > mr ? rank[b] : mr;
  return mr;
}

void fill_results(const hm_dataset* ds, const double* res, int32_t max_rank, hm_result* out) {
  const double c0 = -0.5 * (double)ds->tree.n * std::log(2.0 * 3.14159265358979323846);
  for (int c = 0; c < ds->r; ++c) {
    hm_result& o = out[c];
    std::memset(&o, 0, sizeof(o));
    o.status = ds->factor_status;
    o.n = ds->tree.n;
    o.max_rank = max_rank;
    o.rank_capped = ds->rank_capped;
    o.bytes_C = ds->bytes_C;
    o.bytes_L = ds->factor_status == HM_OK ? ds->bytes_L : 0;
    o.fail_block = ds->fail_block;
    o.fail_pivot = ds->fail_pivot;
    o.t_assemble = ds->t_assemble;
    o.t_factor = ds->t_factor;
    o.t_solve = ds->t_solve;
    if (ds->factor_status == HM_OK) {
      o.logdet = res[0];
      o.quadform = res[1 + c];
      if (ds->prec == HM_MIXED && (size_t)c < ds->ref_quad.size()) {
        // eq. (4) with the refined quadratic form Z^T C~^{-1} Z
        o.refine_quad = ds->ref_quad[c];
        o.refine_resid = ds->ref_resid[c];
        o.refine_iters = ds->ref_iters;
        o.loglik = c0 - 0.5 * o.logdet - 0.5 * o.refine_quad;
      } else {
        o.refine_quad = o.quadform;
        o.loglik = c0 - 0.5 * o.logdet - 0.5 * o.quadform;
      }
    } else {
      o.logdet = o.quadform = o.loglik = o.refine_quad = NAN;
    }
  }
}

}  // namespace hm_int

extern "C" {

hm_status hm_assemble(hm_dataset* ds, const hm_theta* th, const hm_approx* ap) {
  if (!ds) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  TRY(assemble_launch(ds, th, ap, ds->ctx->stream, nullptr, NSLOTS));
  HIPTRY(hipEventSynchronize(ds->ev[1]));
  float ms = 0;
  HIPTRY(hipEventElapsedTime(&ms, ds->ev[0], ds->ev[1]));
  ds->t_assemble = ms * 1e-3;
  {
    std::vector<int32_t> rk(ds->tree.bk.size());
    HIPTRY(hipMemcpy(rk.data(), ds->D.rank, sizeof(int32_t) * rk.size(), hipMemcpyDeviceToHost));
    ds->bytes_C = storage_bytes(ds, rk.data());
  }
  ds->assembled = true;
  ds->fused_solved = false;
  ds->factored = false;
  return HM_OK;
}

static hm_status finish_factor(hm_dataset* ds) {
  DevData& D = ds->D;
  unsigned long long key = 0;
  HIPTRY(hipMemcpy(&key, D.fail_key, sizeof(key), hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(&ds->rank_capped, D.capped, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (D.task_times && getenv("HMLIK_TASK_TIMES")) {
    const char* path = getenv("HMLIK_TASK_TIMES");
    std::vector<int64_t> tt(7 * ds->plan.tasks.size());
    if (hipMemcpy(tt.data(), D.task_times, sizeof(int64_t) * tt.size(), hipMemcpyDeviceToHost) == hipSuccess) {
      if (FILE* f = fopen(path, "w")) {
        fprintf(f, "task kind obj level ninst start end qr svd apply solve form\n");
        for (size_t i = 0; i < ds->plan.tasks.size(); ++i) {
          const Task& t = ds->plan.tasks[i];
          fprintf(f, "%zu %d %d %d %d", i, (int)t.kind, t.obj, t.level, t.ninst);
          for (int q = 0; q < 7; ++q) fprintf(f, " %lld", (long long)tt[7 * i + q]);
          fprintf(f, "\n");
        }
        fclose(f);
      }
    }
  }
  return decode_factor_status(ds, key);
}

// Work-groups and workspace slots of each stream of the stream program
// (disjoint slot ranges within the context's NSLOTS).  Four streams: the
// general levels 256, the big-block flush steps 128, the two wave streams 64
// each.  Six: streams 0 and 4 (general levels) 128 each, 1 and 5 (flush
// steps) and 2, 3 (waves) 64 each.  Eight: streams 0, 4, 6 (general levels)
// 80 each, 1, 5, 7 (flush steps) 48 each, 2, 3 (waves) 64 each.
static constexpr int32_t MS_GRID4[4] = {256, 128, 64, 64};
static constexpr int32_t MS_SLOT_BASE4[4] = {0, 256, 384, 448};
static constexpr int32_t MS_GRID6[6] = {128, 64, 64, 64, 128, 64};
static constexpr int32_t MS_SLOT_BASE6[6] = {0, 128, 192, 256, 320, 448};
static constexpr int32_t MS_GRID8[8] = {80, 48, 64, 64, 80, 48, 80, 48};
static constexpr int32_t MS_SLOT_BASE8[8] = {0, 80, 128, 192, 256, 336, 384, 464};
// every stream's slot range [base, base + grid) inside the NSLOTS slots and
// disjoint from every other stream's
static constexpr bool slot_ranges_ok(const int32_t* grid, const int32_t* base, int ns) {
  for (int a = 0; a < ns; ++a) {
    if (grid[a] < 1 || base[a] < 0 || base[a] + grid[a] > NSLOTS) return false;
    for (int b = 0; b < ns; ++b)
      if (a != b && base[a] < base[b] + grid[b] && base[b] < base[a] + grid[a]) return false;
  }
  return true;
}
static_assert(MS_STREAMS == 8, "stream tables for 4, 6 and 8 streams");
static_assert(slot_ranges_ok(MS_GRID4, MS_SLOT_BASE4, 4) && slot_ranges_ok(MS_GRID6, MS_SLOT_BASE6, 6) &&
                  slot_ranges_ok(MS_GRID8, MS_SLOT_BASE8, 8),
              "stream slot ranges");

// Streams of the program hm_tune_schedule builds: HMLIK_STREAMS (1, 4, 6 or
// 8) if set; otherwise as many as the HIP runtime has hardware queues for
// (GPU_MAX_HW_QUEUES: one per stream and one for the default stream; streams
// that share a hardware queue run their work in issue order, which costs more
// than the extra streams gain): 8 from 9 queues, 6 from 7, else 4.  1: the
// level-synchronous schedule on the caller's stream.
static int program_streams() {
  if (const char* v = getenv("HMLIK_SINGLE_STREAM")) {
    if (*v) return 1;
  }
  if (const char* v = getenv("HMLIK_STREAMS")) {
    const int k = atoi(v);
    if (k == 1 || k == 4 || k == 6 || k == 8) return k;
  }
  const char* q = getenv("GPU_MAX_HW_QUEUES");
  const int hwq = q ? atoi(q) : 4;
  return hwq >= 9 ? 8 : hwq >= 7 ? 6 : 4;
}

// Issues the factorisation's stream program: the extra streams first wait for
// the work already on st (the assembly), each launch waits for its events and
// records its own, and st finally waits for the extra streams' last launches.
static hipError_t launch_stream_program(hm_dataset* ds, const DevData& D, hipStream_t st) {
  const StreamProgram& g = ds->ms;
  hipEvent_t* fork = &ds->mev[g.nevents];
  DevData Dm = D;
  Dm.order = ds->d_morder;
  const int ns = g.nstreams;
  const int32_t* grid = ns == 8 ? MS_GRID8 : ns == 6 ? MS_GRID6 : MS_GRID4;
  const int32_t* slot = ns == 8 ? MS_SLOT_BASE8 : ns == 6 ? MS_SLOT_BASE6 : MS_SLOT_BASE4;
  hipStream_t sx[MS_STREAMS];
  sx[0] = st;
  for (int s = 1; s < ns; ++s) sx[s] = ds->xs[s - 1];
  hipError_t e = hipEventRecord(fork[0], st);
  for (int s = 1; s < ns && e == hipSuccess; ++s) e = hipStreamWaitEvent(sx[s], fork[0], 0);
  // HMLIK_PROGRESS=<launches>: synchronise every <launches> launches and
  // report progress on stderr (long factorisations; costs a sync per chunk)
  size_t chunk = 0;
  if (const char* v = getenv("HMLIK_PROGRESS")) chunk = (size_t)std::max(1, atoi(v));
  for (size_t k = 0; k < g.launches.size() && e == hipSuccess; ++k) {
    if (chunk && k > 0 && k % chunk == 0) {
      for (int s = 0; s < ns && e == hipSuccess; ++s) e = hipStreamSynchronize(sx[s]);
      fprintf(stderr, "hmlik factor: launch %zu of %zu (streams)\n", k, g.launches.size());
    }
    const MSLaunch& M = g.launches[k];
    for (int32_t w = 0; w < M.nwait && e == hipSuccess; ++w)
      e = hipStreamWaitEvent(sx[M.stream], ds->mev[g.waits[M.wait_begin + w]], 0);
    if (e == hipSuccess)
      e = launch_factor_range(Dm, M.t0, M.t1, grid[M.stream], slot[M.stream], sx[M.stream]);
    if (e == hipSuccess && M.rec >= 0) e = hipEventRecord(ds->mev[M.rec], sx[M.stream]);
  }
  for (int s = 1; s < ns && e == hipSuccess; ++s) {
    e = hipEventRecord(fork[s], sx[s]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, fork[s], 0);
  }
  return e;
}

hm_status hm_factor(hm_dataset* ds) {
  if (!ds || !ds->assembled) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  HIPTRY(hipSetDevice(ds->ctx->device));
  use_ctx_ws(ds);
  DevData& D = ds->D;
  hipStream_t st = ds->ctx->stream;
  HIPTRY(hipEventRecord(ds->ev[1], st));
  ds->fused_solved = false;
  if (ds->ms_valid) {
    // the program also runs the data's forward solve L~ v = Z (tree order, in
    // place in the solve buffer) beside the factorisation's tail
    DevData Dm = D;
    Dm.W = ds->d_W;
    Dm.r = ds->r;
    HIPTRY(launch_permute(ds->d_Z, ds->d_perm, ds->tree.n, ds->r, ds->d_W, st));
    HIPTRY(launch_stream_program(ds, Dm, st));
    ds->fused_solved = true;
  } else {
    const int32_t nlev = (int32_t)ds->level_begin.size() - 1;
    // HMLIK_PROGRESS=<levels>: synchronise every <levels> levels and report
    // progress on stderr (for long factorisations; costs a sync per chunk)
    int32_t chunk = nlev;
    if (const char* e = getenv("HMLIK_PROGRESS")) chunk = std::max(1, atoi(e));
    for (int32_t l0 = 0; l0 < nlev; l0 += chunk) {
      const int32_t l1 = std::min(nlev, l0 + chunk);
      HIPTRY(launch_factor_levels(D, ds->level_begin.data(), l0, l1, NSLOTS, st));
      if (l1 < nlev) {
        HIPTRY(hipStreamSynchronize(st));
        HIPTRY(hipEventRecord(ds->ev[2], st));
        HIPTRY(hipEventSynchronize(ds->ev[2]));
        float ms = 0;
        HIPTRY(hipEventElapsedTime(&ms, ds->ev[1], ds->ev[2]));
        fprintf(stderr, "hmlik factor: level %d of %d, task %d of %d, %.1f s\n", l1, nlev, ds->level_begin[l1],
                ds->level_begin[nlev], ms * 1e-3);
      }
    }
  }
  HIPTRY(hipEventRecord(ds->ev[2], st));
  HIPTRY(hipEventSynchronize(ds->ev[2]));
  float ms = 0;
  HIPTRY(hipEventElapsedTime(&ms, ds->ev[1], ds->ev[2]));
  ds->t_factor = ms * 1e-3;
  return finish_factor(ds);
}

// Iterative refinement of x = C~^{-1} Z (mixed form): x_0 = (L~ L~^T)^{-1} Z,
// then x += (L~ L~^T)^{-1} (Z - C~ x) with C~ the assembled matrix (FP64
// products), until the relative residual ||Z - C~ x|| / ||Z|| of every column
// is at most refine_tol or refine_max_iter corrections were applied.  Fills
// ds->ref_quad (Z^T x), ds->ref_resid and ds->ref_iters.  Tree order
// throughout; buffers: the operator buffers and the data's solve buffer.
static hm_status refine(hm_dataset* ds) {
  const int64_t n = ds->tree.n;
  const int r = ds->r;
  hipStream_t st = ds->ctx->stream;
  constexpr int G = 256;   // work-groups of the vector steps (partial sums)
  if (!ds->d_op && hipMalloc((void**)&ds->d_op, sizeof(double) * 3 * n * 64) != hipSuccess) {
    (void)hipGetLastError();
    ds->d_op = nullptr;
    return HM_ERR_OOM;
  }
  if (!ds->d_part && hipMalloc((void**)&ds->d_part, sizeof(double) * G * 2 * 64) != hipSuccess) {
    (void)hipGetLastError();
    ds->d_part = nullptr;
    return HM_ERR_OOM;
  }
  if (!ds->c_valid) return HM_ERR_ARG;
  double* Zt = ds->d_op;
  double* X = Zt + n * 64;
  double* Y = X + n * 64;
  double* R = ds->d_W;
  use_ctx_ws(ds);
  DevData D = ds->D;
  D.r = r;
  DevData Dc = D;   // the kept assembled matrix
  {
    const Plan& P = ds->plan;
    char* q = static_cast<char*>(ds->c_store);
    Dc.dense = (double*)q;
    Dc.lr = (double*)(q + sizeof(double) * (size_t)P.dense_pool);
    Dc.rank = (int32_t*)(q + sizeof(double) * ((size_t)P.dense_pool + (size_t)P.lr_pool));
  }
  const Plan& P = ds->plan;
  auto solve_in_place = [&](double* W) -> hm_status {
    DevData Ds = D;
    Ds.W = W;
    HIPTRY(launch_task_levels(Ds, Ds.stasks, P.slevel_begin.data(), (int32_t)P.slevel_begin.size() - 1, NSLOTS, st));
    HIPTRY(launch_task_levels(Ds, ds->d_btasks, P.blevel_begin.data(), (int32_t)P.blevel_begin.size() - 1, NSLOTS,
                              st));
    return HM_OK;
  };
  std::vector<double> part(G * 2 * 64);
  HIPTRY(launch_permute(ds->d_Z, ds->d_perm, n, r, Zt, st));
  HIPTRY(hipMemcpyAsync(X, Zt, sizeof(double) * n * r, hipMemcpyDeviceToDevice, st));
  TRY(solve_in_place(X));
  ds->ref_resid.assign(r, 0.0);
  int it = 0;
  for (;; ++it) {
    DevData Da = Dc;
    Da.W = X;
    Da.Y = Y;
    HIPTRY(launch_apply(Da, 2, ds->d_chunks, (int32_t)P.apply_chunks.size(), NSLOTS, st));
    HIPTRY(launch_refine_resid(Zt, Y, R, n, r, ds->d_part, G, st));
    HIPTRY(hipMemcpyAsync(part.data(), ds->d_part, sizeof(double) * G * 2 * r, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    double worst = 0.0;
    for (int c = 0; c < r; ++c) {
      double sr = 0.0, sz = 0.0;
      for (int g = 0; g < G; ++g) {
        sr += part[g * 2 * r + c];
        sz += part[g * 2 * r + r + c];
      }
      ds->ref_resid[c] = sz > 0.0 ? std::sqrt(sr / sz) : 0.0;
      worst = std::max(worst, ds->ref_resid[c]);
    }
    if (worst <= ds->refine_tol || it >= ds->refine_max_iter) break;
    TRY(solve_in_place(R));
    HIPTRY(launch_refine_update(X, R, Zt, n, r, ds->d_part, G, st));
  }
  ds->ref_iters = it;
  // Z^T x of the final x
  HIPTRY(launch_refine_update(X, nullptr, Zt, n, r, ds->d_part, G, st));
  HIPTRY(hipMemcpyAsync(part.data(), ds->d_part, sizeof(double) * G * 2 * r, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  ds->ref_quad.assign(r, 0.0);
  for (int c = 0; c < r; ++c)
    for (int g = 0; g < G; ++g) ds->ref_quad[c] += part[g * 2 * r + c];
  return HM_OK;
}

hm_status hm_solve(hm_dataset* ds, hm_result* out) {
  if (!ds || !out || !ds->factored || ds->r < 1) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  HIPTRY(hipSetDevice(ds->ctx->device));
  const int r = ds->r;
  DevData& D = ds->D;
  hipStream_t st = ds->ctx->stream;
  int32_t max_rank = 0;
  {
    std::vector<int32_t> rk(ds->tree.bk.size());
    HIPTRY(hipMemcpy(rk.data(), D.rank, sizeof(int32_t) * rk.size(), hipMemcpyDeviceToHost));
    max_rank = max_lr_rank(ds, rk.data());
    ds->bytes_L = storage_bytes(ds, rk.data());
  }
  std::vector<double> res(1 + r, NAN);
  if (ds->factor_status == HM_OK) {
    HIPTRY(hipEventRecord(ds->ev[2], st));
    DevData Ds = D;
    Ds.W = ds->d_W;
    Ds.r = r;
    if (ds->fused_solved) {
      // v = L~^-1 Z is already in the solve buffer (the factorisation's
      // program ran the solve): only the sums remain
      HIPTRY(launch_solve_reduce(Ds, ds->d_diag_ids, (int32_t)ds->plan.diag_leaf_ids.size(), ds->d_out, st));
    } else {
      HIPTRY(launch_solve(Ds, ds->d_Z, ds->d_perm, ds->plan.slevel_begin.data(),
                          (int32_t)ds->plan.slevel_begin.size() - 1, NSLOTS, ds->d_diag_ids,
                          (int32_t)ds->plan.diag_leaf_ids.size(), ds->d_out, st));
    }
    // the buffer is reused below (refinement) and by a later call
    ds->fused_solved = false;
    HIPTRY(hipEventRecord(ds->ev[3], st));
    HIPTRY(hipEventSynchronize(ds->ev[3]));
    float ms = 0;
    HIPTRY(hipEventElapsedTime(&ms, ds->ev[2], ds->ev[3]));
    ds->t_solve = ms * 1e-3;
    HIPTRY(hipMemcpy(res.data(), ds->d_out, sizeof(double) * (1 + r), hipMemcpyDeviceToHost));
    ds->ref_quad.clear();
    if (ds->prec == HM_MIXED) {
      HIPTRY(hipEventRecord(ds->ev[2], st));
      TRY(refine(ds));
      HIPTRY(hipEventRecord(ds->ev[3], st));
      HIPTRY(hipEventSynchronize(ds->ev[3]));
      float ms2 = 0;
      HIPTRY(hipEventElapsedTime(&ms2, ds->ev[2], ds->ev[3]));
      ds->t_solve += ms2 * 1e-3;
    }
  }
  fill_results(ds, res.data(), max_rank, out);
  return ds->factor_status;
}

hm_status hm_loglik(hm_dataset* ds, const hm_theta* th, const hm_approx* ap, hm_result* out) {
  if (!ds || !out) return HM_ERR_ARG;
  if (ds->r < 1) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  TRY(hm_assemble(ds, th, ap));
  hm_status s = hm_factor(ds);
  if (s != HM_OK && s != HM_ERR_NOT_SPD) return s;
  return hm_solve(ds, out);
}

hm_status hm_loglik_batch(hm_ctx* ctx, int32_t m, hm_dataset* const* ds, const hm_theta* theta,
                          const hm_approx* approx, hm_result* out) {
  if (!ctx || m < 1 || !ds || !theta || !approx || !out) return HM_ERR_ARG;
  if (busy(ctx)) return HM_ERR_BUSY;
  for (int32_t i = 0; i < m; ++i) {
    if (!ds[i] || ds[i]->ctx != ctx || ds[i]->r < 1) return HM_ERR_ARG;
    for (int32_t j = 0; j < i; ++j)
      if (ds[j] == ds[i]) return HM_ERR_ARG;
    TRY(check_theta_approx(&theta[i], &approx[i]));
  }
  // a request server with one slot per dataset (at most 16 on the device at
  // once), all requests submitted together
  const hm_server_opts opts{std::min<int32_t>(m, 16), 0};
  hm_server* sv = nullptr;
  TRY(hm_server_create(ctx, &opts, &sv));
  std::vector<uint64_t> tickets(m, 0);
  hm_status s = HM_OK;
  for (int32_t i = 0; i < m && s == HM_OK; ++i) s = hm_server_submit(sv, ds[i], &theta[i], &approx[i], &tickets[i]);
  hm_status any = HM_OK;
  size_t off = 0;
  for (int32_t i = 0; i < m; ++i) {
    if (!tickets[i]) continue;
    int32_t done = 0;
    const hm_status q = hm_server_poll(sv, tickets[i], 1, out + off, nullptr, &done);
    off += (size_t)ds[i]->r;
    if (q == HM_ERR_NOT_SPD) {
      any = HM_ERR_NOT_SPD;
    } else if (q != HM_OK && s == HM_OK) {
      s = q;
    }
  }
  hm_server_destroy(sv);
  return s != HM_OK ? s : any;
}

hm_status hm_tune_schedule(hm_dataset* ds, const hm_theta* theta, const hm_approx* approx) {
  if (!ds || ds->r < 1) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  TRY(check_theta_approx(theta, approx));
  HIPTRY(hipSetDevice(ds->ctx->device));
  const int32_t nt = (int32_t)ds->plan.tasks.size();
  if (!ds->tt_buf) {
    void* p = nullptr;
    TRY(dev_alloc(ds, sizeof(int64_t) * 7 * ((size_t)nt + 1), &p));
    ds->tt_buf = (int64_t*)p;
  }
  int64_t* saved = ds->D.task_times;
  ds->D.task_times = ds->tt_buf;
  hm_status s = hm_assemble(ds, theta, approx);
  if (s == HM_OK) s = hm_factor(ds);
  ds->D.task_times = saved;
  if (s != HM_OK) return s;
  std::vector<int64_t> tt(7 * (size_t)nt);
  HIPTRY(hipMemcpy(tt.data(), ds->tt_buf, sizeof(int64_t) * tt.size(), hipMemcpyDeviceToHost));
  // factor tasks: measured; the data solve's tasks (not timed in the run):
  // the mean of the factor's tasks of the same kind, an over-estimate (those
  // solve for many columns) that only orders the program
  const int32_t nf = (int32_t)ds->plan.ftasks.size();
  std::vector<double> dur(nt + (size_t)nf);
  double ksum[2] = {0.0, 0.0};
  int64_t kcnt[2] = {0, 0};
  for (int32_t t = 0; t < nt; ++t) {
    dur[t] = (double)(tt[7 * (size_t)t + 1] - tt[7 * (size_t)t]);
    const int8_t k = ds->plan.tasks[t].kind;
    if (k == TASK_SOLVE_SEQ || k == TASK_SOLVE_MV) {
      ksum[k == TASK_SOLVE_MV] += dur[t];
      ++kcnt[k == TASK_SOLVE_MV];
    }
  }
  for (int32_t k = 0; k < nf; ++k) {
    const int j = ds->plan.ftasks[k].kind == TASK_SOLVE_MV;
    dur[nt + (size_t)k] = kcnt[j] ? ksum[j] / (double)kcnt[j] : 1000.0;
  }
  std::vector<int32_t> order, level_begin;
  StreamProgram prog;
  const int nstreams = program_streams();
  const bool multi = nstreams > 1;
  try {
    schedule_by_durations(ds->plan, std::vector<double>(dur.begin(), dur.begin() + nt), order, level_begin);
    if (multi) {
      // timing records are in s_memrealtime ticks (100 MHz): 6 us per launch
      build_stream_program(ds->tree, ds->plan, dur, 600.0, true, nstreams, prog);
    }
  } catch (const std::exception&) {
    return HM_ERR_INTERNAL;
  }
  ds->level_begin = level_begin;
  ds->order = order;
  ds->ms_valid = false;
  if (multi) {
    const size_t no = prog.order.size();   // factor and data-solve tasks
    if (no != (size_t)nt + (size_t)nf) return HM_ERR_INTERNAL;
    if (!ds->d_morder) {
      void* q = nullptr;
      TRY(dev_alloc(ds, sizeof(int32_t) * no, &q));
      ds->d_morder = (int32_t*)q;
    }
    HIPTRY(hipMemcpy(ds->d_morder, prog.order.data(), sizeof(int32_t) * no, hipMemcpyHostToDevice));
    for (int s = 0; s < nstreams - 1; ++s)
      if (!ds->xs[s]) HIPTRY(hipStreamCreateWithFlags(&ds->xs[s], hipStreamNonBlocking));
    const size_t nev = (size_t)prog.nevents + MS_STREAMS;
    while (ds->mev.size() < nev) {
      hipEvent_t e = nullptr;
      HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ds->mev.push_back(e);
    }
    ds->ms = std::move(prog);
    ds->ms_valid = true;
  }
  HIPTRY(hipMemcpy(ds->d_order, ds->order.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice));
  return HM_OK;
}

hm_status hm_dataset_info(const hm_dataset* ds, int64_t* n, int64_t* nclusters, int64_t* nblocks,
                          int64_t* ntasks, int64_t* nlevels) {
  if (!ds) return HM_ERR_ARG;
  if (n) *n = ds->tree.n;
  if (nclusters) *nclusters = (int64_t)ds->tree.cl.size();
  if (nblocks) *nblocks = (int64_t)ds->tree.bk.size();
  if (ntasks) *ntasks = (int64_t)ds->plan.tasks.size();
  if (nlevels) *nlevels = ds->ms_valid ? (int64_t)ds->ms.launches.size() : (int64_t)ds->level_begin.size() - 1;
  return HM_OK;
}

hm_status hm_dataset_export_tree(const hm_dataset* ds, int64_t* perm, int64_t* ranges, double* boxes) {
  if (!ds) return HM_ERR_ARG;
  const Tree& T = ds->tree;
  if (perm) std::memcpy(perm, T.perm.data(), sizeof(int64_t) * T.n);
  for (size_t c = 0; c < T.cl.size(); ++c) {
    if (ranges) {
      ranges[2 * c] = T.cl[c].begin;
      ranges[2 * c + 1] = T.cl[c].end;
    }
    if (boxes) {
      boxes[4 * c] = T.cl[c].lo[0];
      boxes[4 * c + 1] = T.cl[c].lo[1];
      boxes[4 * c + 2] = T.cl[c].hi[0];
      boxes[4 * c + 3] = T.cl[c].hi[1];
    }
  }
  return HM_OK;
}

hm_status hm_dataset_export_blocks(const hm_dataset* ds, int64_t* rc, int8_t* kind) {
  if (!ds) return HM_ERR_ARG;
  const Tree& T = ds->tree;
  for (size_t b = 0; b < T.bk.size(); ++b) {
    if (rc) {
      rc[4 * b] = T.bk[b].r0;
      rc[4 * b + 1] = T.bk[b].c0;
      rc[4 * b + 2] = T.bk[b].m;
      rc[4 * b + 3] = T.bk[b].n;
    }
    if (kind) kind[b] = T.bk[b].kind;
  }
  return HM_OK;
}

hm_status hm_get_block(hm_dataset* ds, int64_t block, double* data, int32_t* rank) {
  if (!ds || !data || !rank || block < 0 || block >= (int64_t)ds->tree.bk.size()) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  if (!ds->store) return HM_ERR_ARG;
  const Block& b = ds->tree.bk[block];
  HIPTRY(hipSetDevice(ds->ctx->device));
  HIPTRY(hipStreamSynchronize(ds->ctx->stream));
  if (b.kind == BK_DENSE) {
    HIPTRY(hipMemcpy(data, ds->D.dense + ds->plan.dense_off[block], sizeof(double) * b.m * b.n,
                     hipMemcpyDeviceToHost));
    *rank = -1;
    return HM_OK;
  }
  if (b.kind == BK_LR) {
    int32_t k = 0;
    HIPTRY(hipMemcpy(&k, ds->D.rank + block, sizeof(int32_t), hipMemcpyDeviceToHost));
    const double* U = ds->D.lr + ds->plan.lr_off[block];
    const double* V = ds->D.lr + ds->plan.lr_voff[block];
    HIPTRY(hipMemcpy(data, U, sizeof(double) * b.m * k, hipMemcpyDeviceToHost));
    HIPTRY(hipMemcpy(data + b.m * k, V, sizeof(double) * b.n * k, hipMemcpyDeviceToHost));
    *rank = k;
    return HM_OK;
  }
  return HM_ERR_ARG;
}

hm_status hm_factor_flops(hm_dataset* ds, double* flops) {
  if (!ds || !flops || !ds->factored) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  HIPTRY(hipSetDevice(ds->ctx->device));
  HIPTRY(hipStreamSynchronize(ds->ctx->stream));
  std::vector<double> f(ds->plan.tasks.size());
  if (!f.empty())
    HIPTRY(hipMemcpy(f.data(), ds->D.task_flops, sizeof(double) * f.size(), hipMemcpyDeviceToHost));
  double s = 0.0;
  for (double v : f) s += v;
  *flops = s;
  return HM_OK;
}

hm_status hm_get_term(hm_dataset* ds, int64_t term, double* data, int32_t* kind, int64_t* A, int64_t* B,
                      int64_t* rows, int32_t* k) {
  if (!ds || term < 0 || term >= (int64_t)ds->plan.terms.size() || !kind || !A || !B || !rows || !k)
    return HM_ERR_ARG;
  const TermDef& t = ds->plan.terms[term];
  *kind = t.kind;
  *A = t.A;
  *B = t.B;
  *rows = t.rows;
  *k = 0;
  if (t.kind == TK_DD) return HM_OK;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  if (!ds->store) return HM_ERR_ARG;
  const int32_t R = (t.kind == TK_LRA) ? t.A : t.B;
  HIPTRY(hipSetDevice(ds->ctx->device));
  HIPTRY(hipStreamSynchronize(ds->ctx->stream));
  HIPTRY(hipMemcpy(k, ds->D.rank + R, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (data && *k > 0)
    HIPTRY(hipMemcpy(data, ds->D.termbuf + t.buf, sizeof(double) * t.rows * (*k), hipMemcpyDeviceToHost));
  return HM_OK;
}

hm_status hm_test_truncate(hm_dataset* ds, const double* X, int64_t m, const double* Y, int64_t n, int32_t r,
                           double eps, int32_t fixed_rank, double* U, double* V, int32_t* k, double* seconds) {
  const bool expl = (Y == nullptr);
  if (!ds || !X || !U || !V || !k || m < 1 || n < 1) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  if (expl ? (r != 0 || n > 4 * LEAF_MAX) : (r < 1 || r > 2 * K_MAX)) return HM_ERR_ARG;
  if (fixed_rank < 0 || fixed_rank > K_MAX || (fixed_rank == 0 && !finite_pos(eps))) return HM_ERR_ARG;
  const int64_t need = expl ? m * n + (n | 1) * (m < n ? m : n) + 64
                            : (m + n) * (int64_t)r + 2 * (int64_t)(r + 1) * r + 64;
  use_ctx_ws(ds);
  if (need > ds->D.ws_stride) return HM_ERR_ARG;
  const int64_t xs = expl ? m * n : m * (int64_t)r;
  HIPTRY(hipSetDevice(ds->ctx->device));
  hipStream_t st = ds->ctx->stream;
  DevData D = ds->D;
  D.kfix = fixed_rank;
  D.eps = fixed_rank > 0 ? 0.0 : eps;
  D.kmax = fixed_rank > 0 ? fixed_rank : K_MAX;
  void *dX = nullptr, *dY = nullptr, *dU = nullptr, *dV = nullptr, *dk = nullptr, *dph = nullptr;
  hm_status s = HM_OK;
  if (hipMalloc(&dX, sizeof(double) * xs) != hipSuccess ||
      (!expl && hipMalloc(&dY, sizeof(double) * n * r) != hipSuccess) ||
      hipMalloc(&dU, sizeof(double) * m * K_MAX) != hipSuccess ||
      hipMalloc(&dV, sizeof(double) * n * K_MAX) != hipSuccess || hipMalloc(&dk, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&dph, sizeof(int64_t) * 4) != hipSuccess)
    s = HM_ERR_OOM;
  if (s == HM_OK) {
    float ms = 0;
    if (hipMemcpy(dX, X, sizeof(double) * xs, hipMemcpyHostToDevice) != hipSuccess ||
        (!expl && hipMemcpy(dY, Y, sizeof(double) * n * r, hipMemcpyHostToDevice) != hipSuccess) ||
        hipEventRecord(ds->ev[0], st) != hipSuccess ||
        launch_truncate_test(D, (double*)dX, m, (double*)dY, n, r, (double*)dU, (double*)dV, (int32_t*)dk,
                             (int64_t*)dph, st) !=
            hipSuccess ||
        hipEventRecord(ds->ev[1], st) != hipSuccess || hipEventSynchronize(ds->ev[1]) != hipSuccess ||
        hipEventElapsedTime(&ms, ds->ev[0], ds->ev[1]) != hipSuccess ||
        hipMemcpy(k, dk, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
      s = HM_ERR_DEVICE;
    if (s == HM_OK && (hipMemcpy(U, dU, sizeof(double) * m * (*k), hipMemcpyDeviceToHost) != hipSuccess ||
                       hipMemcpy(V, dV, sizeof(double) * n * (*k), hipMemcpyDeviceToHost) != hipSuccess))
      s = HM_ERR_DEVICE;
    if (seconds) {
      int64_t ph[3] = {0, 0, 0};
      (void)hipMemcpy(ph, dph, sizeof(ph), hipMemcpyDeviceToHost);
      seconds[0] = ms * 1e-3;
      for (int q = 0; q < 3; ++q) seconds[1 + q] = ph[q] * 1e-8;   // 100 MHz clock
    }
  }
  (void)hipGetLastError();
  for (void* q : {dX, dY, dU, dV, dk, dph})
    if (q) (void)hipFree(q);
  return s;
}

hm_status hm_truncate_noalloc(hm_ctx* ctx, const double* X, int64_t m, const double* Y, int64_t n, int32_t r,
                              double eps, int32_t fixed_rank, double* U, double* V, int32_t* k) {
  const bool expl = (Y == nullptr);
  if (!ctx || !X || !U || !V || !k || m < 1 || n < 1) return HM_ERR_ARG;
  if (busy(ctx)) return HM_ERR_BUSY;
  if (expl ? (r != 0 || n > 4 * LEAF_MAX) : (r < 1 || r > 2 * K_MAX)) return HM_ERR_ARG;
  if (fixed_rank < 0 || fixed_rank > K_MAX || (fixed_rank == 0 && !finite_pos(eps))) return HM_ERR_ARG;
  // workspace of the kernel (as in hm_test_truncate) within the fixed array
  const int64_t need = expl ? m * n + (n | 1) * (m < n ? m : n) + 64
                            : (m + n) * (int64_t)r + 2 * (int64_t)(r + 1) * r + 64;
  if (need > NOALLOC_DOUBLES - 64) return HM_ERR_ARG;
  double* base = noalloc_scratch(ctx->device);
  if (!base) return HM_ERR_DEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_DEVICE;
  }
  DevData D{};
  D.kfix = fixed_rank;
  D.eps = fixed_rank > 0 ? 0.0 : eps;
  D.kmax = fixed_rank > 0 ? fixed_rank : K_MAX;
  if (launch_truncate_noalloc(D, base, X, m, Y, n, r, U, V, k, ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_DEVICE;
  }
  return HM_OK;
}

hm_status hm_dataset_keep_matrix(hm_dataset* ds, int32_t keep) {
  // (the mixed form allocates the copy itself, see assemble_launch)
  if (!ds) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  HIPTRY(hipSetDevice(ds->ctx->device));
  if (!keep) {
    if (ds->c_store) {
      HIPTRY(hipStreamSynchronize(ds->ctx->stream));
      (void)hipFree(ds->c_store);
    }
    ds->c_store = nullptr;
    ds->c_bytes = 0;
    ds->keep_c = ds->c_valid = false;
    return HM_OK;
  }
  if (!ds->c_store) TRY(alloc_matrix_copy(ds));
  ds->keep_c = true;
  return HM_OK;
}

hm_status hm_apply(hm_dataset* ds, int32_t op, const double* W, double* Y, int32_t r, int32_t on_device) {
  if (!ds || !W || !Y || r < 1 || r > 64 || op < HM_OP_L || op > HM_OP_C_EXACT) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  const bool need_factor = op == HM_OP_L || op == HM_OP_LT || op == HM_OP_SOLVE;
  if (need_factor && !(ds->factored && ds->factor_status == HM_OK && ds->store)) return HM_ERR_ARG;
  if (op == HM_OP_C && !ds->c_valid) return HM_ERR_ARG;
  if (op == HM_OP_C_EXACT && !ds->theta_set) return HM_ERR_ARG;
  const int64_t n = ds->tree.n;
  if (on_device) {
    hipPointerAttribute_t a{}, b{};
    if (hipPointerGetAttributes(&a, W) != hipSuccess || hipPointerGetAttributes(&b, Y) != hipSuccess ||
        a.type != hipMemoryTypeDevice || b.type != hipMemoryTypeDevice || a.device != ds->ctx->device ||
        b.device != ds->ctx->device) {
      (void)hipGetLastError();
      return HM_ERR_ARG;
    }
  } else {
    for (int64_t i = 0; i < n * (int64_t)r; ++i)
      if (!std::isfinite(W[i])) return HM_ERR_ARG;
  }
  HIPTRY(hipSetDevice(ds->ctx->device));
  hipStream_t st = ds->ctx->stream;
  if (!ds->d_op) {
    if (hipMalloc((void**)&ds->d_op, sizeof(double) * 3 * n * 64) != hipSuccess) {
      (void)hipGetLastError();
      ds->d_op = nullptr;
      return HM_ERR_OOM;
    }
  }
  double* A = ds->d_op;              // input, tree order
  double* B = A + n * 64;            // output, tree order
  double* T = B + n * 64;            // input-order staging of host data
  const double* src = W;
  if (!on_device) {
    HIPTRY(hipMemcpyAsync(T, W, sizeof(double) * n * r, hipMemcpyHostToDevice, st));
    src = T;
  }
  HIPTRY(launch_permute(src, ds->d_perm, n, r, A, st));
  use_ctx_ws(ds);
  DevData D = ds->D;
  D.W = A;
  D.Y = B;
  D.r = r;
  const double* res = B;
  if (op == HM_OP_L || op == HM_OP_LT) {
    HIPTRY(launch_apply(D, op == HM_OP_L ? 0 : 1, ds->d_chunks, (int32_t)ds->plan.apply_chunks.size(), NSLOTS, st));
  } else if (op == HM_OP_C) {
    const Plan& P = ds->plan;
    char* q = static_cast<char*>(ds->c_store);
    D.dense = (double*)q;
    D.lr = (double*)(q + sizeof(double) * (size_t)P.dense_pool);
    D.rank = (int32_t*)(q + sizeof(double) * ((size_t)P.dense_pool + (size_t)P.lr_pool));
    HIPTRY(launch_apply(D, 2, ds->d_chunks, (int32_t)ds->plan.apply_chunks.size(), NSLOTS, st));
  } else if (op == HM_OP_SOLVE) {
    HIPTRY(launch_task_levels(D, D.stasks, ds->plan.slevel_begin.data(), (int32_t)ds->plan.slevel_begin.size() - 1,
                              NSLOTS, st));
    HIPTRY(launch_task_levels(D, ds->d_btasks, ds->plan.blevel_begin.data(),
                              (int32_t)ds->plan.blevel_begin.size() - 1, NSLOTS, st));
    res = A;
  } else {
    for (int32_t c0 = 0; c0 < r; c0 += 4) {
      DevData Dc = D;
      Dc.W = A + c0 * n;
      Dc.Y = B + c0 * n;
      Dc.r = std::min(4, r - c0);
      HIPTRY(launch_dense_matvec(Dc, st));
    }
  }
  if (on_device) {
    HIPTRY(launch_unpermute(res, ds->d_perm, n, r, Y, st));
    HIPTRY(hipStreamSynchronize(st));
  } else {
    HIPTRY(launch_unpermute(res, ds->d_perm, n, r, T, st));
    HIPTRY(hipMemcpyAsync(Y, T, sizeof(double) * n * r, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
  }
  return HM_OK;
}

hm_status hm_exact_block(hm_dataset* ds, int64_t i0, int64_t ni, int64_t j0, int64_t nj, double* out, int64_t ldo,
                         int32_t on_device) {
  if (!ds || !out) return HM_ERR_ARG;
  const int64_t n = ds->tree.n;
  if (i0 < 0 || ni < 0 || j0 < 0 || nj < 0 || i0 > n - ni || j0 > n - nj || ldo < (ni > 1 ? ni : 1))
    return HM_ERR_ARG;
  if (!ds->theta_set) return HM_ERR_ARG;
  if (busy(ds->ctx)) return HM_ERR_BUSY;
  if (ni == 0 || nj == 0) return HM_OK;
  if (nj > 1 && ldo > (INT64_MAX - ni) / (nj - 1)) return HM_ERR_ARG;
  HIPTRY(hipSetDevice(ds->ctx->device));
  hipStream_t st = ds->ctx->stream;
  if (on_device) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, out) != hipSuccess || a.type != hipMemoryTypeDevice ||
        a.device != ds->ctx->device) {
      (void)hipGetLastError();
      return HM_ERR_ARG;
    }
  }
  if (!ds->d_iperm) {
    std::vector<int64_t> ip(n);
    for (int64_t q = 0; q < n; ++q) ip[ds->tree.perm[q]] = q;
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(int64_t) * n) != hipSuccess) {
      (void)hipGetLastError();
      return HM_ERR_OOM;
    }
    ds->d_iperm = (int64_t*)p;
    HIPTRY(hipMemcpy(ds->d_iperm, ip.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice));
  }
  if (on_device) {
    HIPTRY(launch_exact_block(ds->D, ds->d_iperm, i0, ni, j0, nj, out, ldo, st));
    HIPTRY(hipStreamSynchronize(st));
    return HM_OK;
  }
  double* tmp = nullptr;
  if (hipMalloc((void**)&tmp, sizeof(double) * ni * nj) != hipSuccess) {
    (void)hipGetLastError();
    return HM_ERR_OOM;
  }
  hipError_t e = launch_exact_block(ds->D, ds->d_iperm, i0, ni, j0, nj, tmp, ni, st);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(out, sizeof(double) * ldo, tmp, sizeof(double) * ni, sizeof(double) * ni, nj,
                         hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  return e == hipSuccess ? HM_OK : HM_ERR_DEVICE;
}

hm_status hm_simulate(hm_dataset* ds, const hm_theta* theta, const hm_approx* approx, const double* W, double* Z,
                      int32_t r, int32_t on_device) {
  if (!ds || !W || !Z || r < 1 || r > 64) return HM_ERR_ARG;
  TRY(hm_assemble(ds, theta, approx));
  const hm_status s = hm_factor(ds);
  if (s != HM_OK) return s;
  return hm_apply(ds, HM_OP_L, W, Z, r, on_device);
}

hm_status hm_inverse_accuracy(hm_dataset* ds, const double* x0, int32_t iters, double* norm) {
  if (!ds || !x0 || !norm || iters < 1) return HM_ERR_ARG;
  if (!(ds->factored && ds->factor_status == HM_OK && ds->theta_set)) return HM_ERR_ARG;
  const int64_t n = ds->tree.n;
  std::vector<double> x(x0, x0 + n), y(n), t(n);
  auto nrm = [](const std::vector<double>& v) {
    double s = 0.0;
    for (double a : v) s += a * a;
    return std::sqrt(s);
  };
  double s = nrm(x);
  if (!(s > 0.0) || !std::isfinite(s)) return HM_ERR_ARG;
  for (double& a : x) a /= s;
  // power iteration on A^T A, A = I - (L L^T)^{-1} C, A^T = I - C (L L^T)^{-1}
  double lam = 0.0;
  for (int32_t it = 0; it < iters; ++it) {
    TRY(hm_apply(ds, HM_OP_C_EXACT, x.data(), t.data(), 1, 0));
    TRY(hm_apply(ds, HM_OP_SOLVE, t.data(), y.data(), 1, 0));
    for (int64_t i = 0; i < n; ++i) y[i] = x[i] - y[i];            // y = A x
    TRY(hm_apply(ds, HM_OP_SOLVE, y.data(), t.data(), 1, 0));
    TRY(hm_apply(ds, HM_OP_C_EXACT, t.data(), x.data(), 1, 0));
    for (int64_t i = 0; i < n; ++i) x[i] = y[i] - x[i];            // x = A^T y
    lam = nrm(x);                                                   // ||A^T A x|| with ||x|| = 1
    if (!(lam > 0.0)) break;
    for (double& a : x) a /= lam;
  }
  *norm = std::sqrt(lam);
  return HM_OK;
}

}  // extern "C"
