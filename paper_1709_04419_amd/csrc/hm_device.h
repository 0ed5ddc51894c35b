// Device-side view of a dataset's plan and storage, passed by value to the
// kernels.  Plain pointers into device memory owned by the library.
#pragma once
#include <cstdint>

#include "hm_plan.h"

namespace hm {

// Per-theta constants of the Matern entry generator (eq. (2) of Section 2.2,
// plus the nugget of the remark in Section 2.4).  Filled on the host.
struct MaternConst {
  double sigma2, inv_ell, nu, nugget;
  double norm;        // 1 / (2^(nu-1) Gamma(nu))
  double mu;          // nu - N, |mu| <= 1/2
  int32_t nrec;       // N = round-half-up(nu): K_nu from (K_mu, K_mu+1) by N-1 recurrences
  int32_t half;       // 1, 3, 5 for nu = 1/2, 3/2, 5/2 (closed forms), 0 otherwise
  double g1, g2;      // Temme's Gamma_1(mu), Gamma_2(mu)
  double gp, gm;      // Gamma(1 + mu), Gamma(1 - mu)
  double fact;        // mu pi / sin(mu pi)
};

struct DevData {
  int64_t n;
  const double* px;           // permuted coordinates (SoA)
  const double* py;
  const Block* bk;
  const Cluster* cl;
  const int32_t* diag_of;
  int32_t nblocks;
  // storage
  double* dense;
  const int64_t* dense_off;
  double* lr;
  const int64_t* lr_off;      // U of a low-rank block (m x cap, ld m)
  const int64_t* lr_voff;     // V (n x cap, ld n)
  const int32_t* lr_cap;      // cap: K_MAX, or 2 K_MAX for big blocks (flush in place, TASK_TS_*)
  double* stage;              // staging of the big blocks' flush steps
  const int64_t* stage_off;
  int32_t* ts_app;            // big block: column where the current step appends its term
  int32_t* rank;              // per block (low-rank leaves)
  double* termbuf;
  const TermDef* terms;
  const TermInst* insts;
  // the final forward solve: its tasks (level order) and the permuted data
  const Task* stasks;
  double* W;                  // n x r, leading dimension n
  double* Y;                  // n x r output of the operator products (TASK_APPLY)
  int32_t r;
  // schedule
  const Task* tasks;
  const int32_t* order;       // execution order of the tasks, level by level
  const int32_t* deps;
  int32_t ntasks;
  unsigned long long* fail_key;   // min over (program index << 8 | pivot) of failed pivots
  int32_t* capped;                // ACA runs / truncations where the rank cap bound in the accuracy mode
  const int32_t* task_prog;       // program-order index of each task
  int64_t* task_times;            // optional: start/end real-time stamps per task (nullptr: off)
  double* task_flops;             // algorithmic flops of each factorization task
  // structure helpers
  const int32_t* sub_begin;
  const int32_t* sub_end;
  const int32_t* sub_leaves;
  const int32_t* sop_begin;
  const SolveOp* sops;
  // outputs
  double* logdet_part;        // per block id (diagonal dense leaves)
  // workspace: one slot per resident workgroup
  double* ws;
  int64_t ws_stride;
  // lists for the bulk kernels
  const int32_t* dense_ids;
  int32_t ndense;
  const int32_t* lr_ids;
  int32_t nlr;
  // approximation
  MaternConst mc;
  double eps;
  int32_t kfix;
  int32_t kmax;               // rank cap (K_MAX, or kfix)
  int32_t mixed;              // 1: low-rank factors FP32-valued, their products in FP32 (HM_MIXED)
  int32_t dflush;             // low-rank blocks of at most dflush x dflush take their updates explicitly
};

}  // namespace hm

#include <hip/hip_runtime_api.h>

namespace hm {
hipError_t launch_assemble(const DevData& D, hipStream_t st);
hipError_t launch_aca(const DevData& D, int grid, hipStream_t st);
hipError_t launch_truncate_test(const DevData& D, const double* X, int64_t m, const double* Y, int64_t n,
                                int r, double* U, double* V, int32_t* kout, int64_t* phases, hipStream_t st);
// Allocation-free truncation: a fixed per-GPU device array of NOALLOC_DOUBLES
// doubles (counters, then workspace).  noalloc_scratch_init resolves this
// GPU's copy once (hipGetSymbolAddress with the device current);
// noalloc_scratch returns it (nullptr before init).
constexpr int64_t NOALLOC_DOUBLES = 4 << 20;   // 32 MiB
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch_init(int device);
double* noalloc_scratch(int device);
hipError_t launch_truncate_noalloc(DevData D, double* base, const double* X, int64_t m, const double* Y, int64_t n,
                                   int r, double* U, double* V, int32_t* kout, hipStream_t st);
// Clears the breakdown record and the rank-cap counter of an evaluation (before
// its assembly).
hipError_t launch_eval_init(const DevData& D, hipStream_t st);
// Launches levels [l0, l1) of the task DAG, one kernel per level.
hipError_t launch_factor_levels(const DevData& D, const int32_t* level_begin, int32_t l0, int32_t l1, int max_grid,
                                hipStream_t st);
// Tasks order[t0 .. t1) of D.order on at most max_grid work-groups that use
// workspace slots slot_base .. slot_base + max_grid - 1.
hipError_t launch_factor_range(const DevData& D, int32_t t0, int32_t t1, int max_grid, int32_t slot_base,
                               hipStream_t st);
// One level of several datasets' factorisations in one launch: Ds (device
// array of nseg DevData), seg (device, 2 nseg ints: the level's task range per
// dataset), total = the number of tasks over all of them.
hipError_t launch_level_batch(const DevData* Ds, const int32_t* seg, int32_t nseg, int32_t total, int max_grid,
                              hipStream_t st);
// Operators on D.W / D.Y (n x D.r, tree order, leading dimension n):
// `nlev` levels [level_begin[l], level_begin[l + 1]) of a solve task graph
// (tasks on the device, in level order); the row-chunk product of mode 0 (L),
// 1 (L^T) or 2 (symmetric matrix of the stored lower blocks); the exact
// covariance product Y = C W (entries of eq. 2 plus nugget formed on the fly,
// D.r <= 4); and the permutations between input and tree order.
hipError_t launch_task_levels(const DevData& D, const Task* tasks, const int32_t* level_begin, int32_t nlev,
                              int max_grid, hipStream_t st);
hipError_t launch_apply(const DevData& D, int mode, const int32_t* chunks, int32_t nchunks, int max_grid,
                        hipStream_t st);
hipError_t launch_dense_matvec(const DevData& D, hipStream_t st);
hipError_t launch_exact_block(const DevData& D, const int64_t* iperm, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                              double* out, int64_t ldo, hipStream_t st);
// Refinement vector steps on n x r arrays (leading dimension n), with
// per-work-group partial sums (fixed order) in part (grid x (2 r) doubles):
//   resid:  R = Z - Y; part[g][c] = sum R^2, part[g][r + c] = sum Z^2 (column c)
//   update: X += Dx; part[g][c] = sum Z X (column c, after the update)
hipError_t launch_refine_resid(const double* Z, const double* Y, double* R, int64_t n, int r, double* part, int grid,
                               hipStream_t st);
hipError_t launch_refine_update(double* X, const double* Dx, const double* Z, int64_t n, int r, double* part,
                                int grid, hipStream_t st);
hipError_t launch_permute(const double* Z, const int64_t* perm, int64_t n, int r, double* W, hipStream_t st);
hipError_t launch_unpermute(const double* W, const int64_t* perm, int64_t n, int r, double* Z, hipStream_t st);
// Forward solve L v = Z (Z permuted into W, then the solve task levels
// slevel_begin[0 .. nslev]), log-determinant and v^T v into out.
// log-det and v^T v sums of an already solved W (the data solve ran inside
// the factorisation's stream program).
hipError_t launch_solve_reduce(const DevData& D, const int32_t* diag_ids, int32_t ndiag, double* out, hipStream_t st);
hipError_t launch_solve(const DevData& D, const double* Z, const int64_t* perm, const int32_t* slevel_begin,
                        int32_t nslev, int max_grid, const int32_t* diag_ids, int32_t ndiag, double* out,
                        hipStream_t st);
}  // namespace hm
