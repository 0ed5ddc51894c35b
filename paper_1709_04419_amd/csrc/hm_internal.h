// Library-internal definitions of the handles declared opaque in
// include/hmlik.h, shared by the evaluation entry points (hm_api.cpp) and the
// request server (hm_server.cpp).
#pragma once
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdint>
#include <set>
#include <vector>

#include "../../include/hmlik.h"
#include "hm_device.h"
#include "hm_plan.h"

struct hm_ctx {
  int device;
  hipStream_t stream;
  // workspace slots shared by the context's datasets (evaluations on one
  // context are ordered on its stream); grown when a dataset needs more
  double* ws = nullptr;
  int64_t ws_stride = 0;
  // the context's live datasets (the server's view of resident factor storage)
  std::set<hm_dataset*> datasets;
  // non-null while a request server owns the context's device work
  std::atomic<hm_server*> server{nullptr};
};

namespace hm_int {

constexpr int NSLOTS = 512;   // workspace slots (ACA and level-kernel work-groups)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace hm_int

struct hm_dataset {
  hm_ctx* ctx = nullptr;
  hm::Tree tree;
  hm::Plan plan;
  std::vector<hm_int::DevBuf> bufs;   // resident: trees, plan, schedule, Z, small per-evaluation arrays
  // factor storage (dense leaves, low-rank factors, update-term buffers): the
  // theta-dependent bulk of the dataset, one allocation that can be released
  // between evaluations and is re-attached by the next one
  void* store = nullptr;
  size_t store_bytes = 0;
  hm::DevData D{};
  int64_t* d_perm = nullptr;
  int32_t* d_diag_ids = nullptr;
  double* d_Z = nullptr;
  double* d_W = nullptr;
  double* d_out = nullptr;
  int32_t r = 0;                      // columns of Z
  int32_t zcap = 0;                   // columns d_Z, d_W and d_out hold
  bool assembled = false, factored = false;
  hm_status factor_status = HM_OK;
  int64_t fail_block = -1;
  int32_t fail_pivot = -1;
  int32_t rank_capped = 0;            // rank-cap count of the last evaluation
  int64_t bytes_C = 0, bytes_L = 0;   // storage of C~ and L~ at the actual ranks
  double t_assemble = 0, t_factor = 0, t_solve = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // operators (hm_apply): the backward solve's tasks, the row chunks, three
  // n x 64 buffers (allocated on first use)
  hm::Task* d_btasks = nullptr;
  int32_t* d_chunks = nullptr;
  double* d_op = nullptr;
  int64_t* d_iperm = nullptr;         // input index -> tree position (hm_exact_block, first use)
  // copy of the assembled matrix C~ (dense pool, low-rank pool, ranks), made by
  // every assembly while keep_c is set
  bool keep_c = false;
  bool c_valid = false;
  void* c_store = nullptr;
  size_t c_bytes = 0;
  bool theta_set = false;             // an assembly has set theta (the exact covariance product)
  // arithmetic of the last assembly (hm_precision) and its refinement controls
  int32_t prec = HM_FP64;
  int32_t refine_max_iter = 0;
  double refine_tol = 0.0;
  double* d_part = nullptr;           // partial sums of the refinement (NSLOTS_RED x 128 doubles)
  // per column: refined Z^T x, its relative residual, and the corrections applied
  std::vector<double> ref_quad, ref_resid;
  int32_t ref_iters = 0;
  std::vector<int32_t> level_begin;   // position in `order` where each level starts (+ end)
  std::vector<int32_t> order;         // execution order (task ids), level by level
  int32_t* d_order = nullptr;
  int64_t* tt_buf = nullptr;          // per-task timing records (allocated on first use)
  // factorisation on several streams (built by hm_tune_schedule): the program,
  // its task order on the device, the extra streams and the events
  bool ms_valid = false;
  hm::StreamProgram ms;
  int32_t* d_morder = nullptr;
  hipStream_t xs[hm::MS_STREAMS - 1] = {};
  std::vector<hipEvent_t> mev;        // ms.nevents, then MS_STREAMS (fork / join)
  // the program also runs the data's forward solve (tasks plan.ftasks after the
  // factor tasks; combined task and program-index arrays on the device), and
  // whether the last factorisation did so for the current data
  bool ms_fused = false;
  hm::Task* d_ctasks = nullptr;
  int32_t* d_cprog = nullptr;
  bool fused_solved = false;
};

namespace hm_int {

// allocates the copy of the assembled matrix (dense pool, low-rank pool, ranks)
hm_status alloc_matrix_copy(hm_dataset* ds);
// theta and accuracy checks shared by every evaluation entry point
hm_status check_theta_approx(const hm_theta* th, const hm_approx* ap);
// allocates the factor storage if it is not attached
hm_status attach_store(hm_dataset* ds);
// frees the factor storage (after the context's stream has drained)
void release_store(hm_dataset* ds);
// sets theta and the accuracy, attaches the factor storage and enqueues the
// assembly on `st`, bracketed by ds->ev[0], ds->ev[1]; with ws != nullptr the
// ACA kernel runs `grid` work-groups on the workspace slots starting at ws
// (else NSLOTS on the context's workspace)
hm_status assemble_launch(hm_dataset* ds, const hm_theta* th, const hm_approx* ap, hipStream_t st, double* ws,
                          int grid);
// decodes a finished factorisation's breakdown record into ds->factor_status,
// fail_block and fail_pivot (key: min over failed pivots of program index << 8 | pivot)
hm_status decode_factor_status(hm_dataset* ds, unsigned long long key);
// bytes of the dense leaves plus the low-rank factors at the ranks `rank`
int64_t storage_bytes(const hm_dataset* ds, const int32_t* rank);
// largest rank among the low-rank leaves, from a host copy of the rank array
int32_t max_lr_rank(const hm_dataset* ds, const int32_t* rank);
// fills r results from the solve output (log-det, then v^T v per column)
void fill_results(const hm_dataset* ds, const double* res, int32_t max_rank, hm_result* out);
// cancels the server's queued requests on `ds` and waits until none of its
// requests is on the device (before the dataset is destroyed)
void server_forget_dataset(hm_server* sv, hm_dataset* ds);
// whether ds has factor storage attached, read under the server's lock (the
// worker attaches and releases storage while the server runs)
bool server_store_attached(hm_server* sv, const hm_dataset* ds);

}  // namespace hm_int
