// Host-side structures: cluster tree, block cluster tree and the symbolic
// H-Cholesky schedule.  Everything here depends on the locations only (never
// on theta), so it is built once per dataset and reused for every likelihood
// evaluation.  Shared between the host planner (hm_plan.cpp) and the device
// runtime (hm_device.hip); plain-old-data only.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hm {

// Largest rank a low-rank block may carry (assembly, truncation, update
// accumulation).  Also the largest rank of an accumulated update list before
// it is truncated.  Both are named constants of the method.
constexpr int K_MAX = 64;
constexpr int R_ACC = 64;
// Low-rank blocks whose clusters both hold at most DENSE_FLUSH * n_min points
// take their pending updates on the explicit matrix and are truncated once.
constexpr int DENSE_FLUSH = 4;
// Largest leaf size n_min the device kernels accept (dense tiles <= 64 x 64).
constexpr int LEAF_MAX = 64;

enum BlockKind : int8_t { BK_NODE = 0, BK_DENSE = 1, BK_LR = 2 };

struct Cluster {
  int64_t begin, end;      // contiguous range of permuted positions
  double lo[2], hi[2];     // tight axis-parallel bounding box
  int32_t son[2];          // -1 for a leaf
  int32_t level;
};

struct Block {
  int32_t row, col;        // cluster ids (tau, sigma)
  int8_t kind;
  int32_t son_begin, nsons;  // into Tree::sons
  int64_t r0, c0, m, n;    // global permuted ranges
};

// Term kinds: how the factor X Y^T of an update is obtained.
enum TermKind : int8_t {
  TK_LRA = 0,  // A low-rank:  X = U_A,        Y = L_B V_A  (computed)
  TK_LRB = 1,  // B low-rank:  X = L_A V_B (computed),  Y = U_B
  TK_DD = 2,   // both dense:  X = D_A,        Y = D_B
};

struct TermDef {
  int8_t kind;
  int32_t A, B;            // factor blocks
  int64_t rows;            // rows of the computed factor (0 for TK_DD)
  int64_t buf;             // offset (doubles) of the computed factor, ld = rows, K_MAX cols
};

// One term restricted to one leaf: leaf(lr0.., lc0..) -= X[xr0.., :] Y[yr0.., :]^T
struct TermInst {
  int32_t term;
  int32_t lr0, lc0;        // offset of the region inside the leaf
  int32_t mx, ny;          // region size
  int64_t xr0, yr0;        // first row used in X and in Y
};

enum TaskKind : int8_t {
  TASK_DIAG = 0,       // dense diagonal leaf: flush + Cholesky
  TASK_OFFD = 1,       // dense off-diagonal leaf: flush + triangular solve
  TASK_LR = 2,         // low-rank leaf: flush (truncation), then V <- L^-1 V if a0 == 1
  TASK_TERM = 3,       // compute the product factor of a term
  TASK_SOLVE_SEQ = 4,  // W(rows of cluster a0) <- L^-1 W(same rows), the cluster's solve program
  TASK_SOLVE_MV = 5,   // W(rows of cluster a1) -= L_blk(those rows, :) W(cols of blk), blk = a0
  TASK_TERM_ROWS = 6,  // rows of cluster a1 of the product factor of term obj
  // Factored flush of a big low-rank block obj (see ts_rows) as steps: before
  // term a0 (1-based; a0 = T + 1 is the final truncation after the last of its
  // T terms) the accumulated [U, -X_1, ..][V, Y_1, ..] is truncated if its rank
  // would exceed R_ACC, then term a0 is appended:
  TASK_TS_A = 7,       //   row block a1: Householder QR of its rows (if truncating)
  TASK_TS_B = 8,       //   stacked R factors: QR, core SVD, small factors; new rank
  TASK_TS_C = 9,       //   row block a1: its rows of the truncated factor, then the term's columns
  // operators of the factor / matrix on the data (obj = -1 only):
  TASK_SOLVE_SEQ_T = 10,  // W(rows of cluster a0) <- L^-T W(same rows), its solve program backwards
  TASK_SOLVE_MV_T = 11,   // W(rows of cluster a1) -= L_blk(:, those rows)^T W(rows of blk), blk = a0
  TASK_APPLY = 12,        // Y(rows of cluster a1) = M W(.) for M = L (a0 = 0), L^T (1), C~ (2)
};
// W of the solve tasks: obj >= 0 is the V factor of that low-rank block (its
// rows relative to the block's column cluster), obj = -1 the permuted data of
// the final forward solve.

struct Task {
  int8_t kind;
  int32_t obj;             // block id (DIAG/OFFD/LR/SOLVE_*, -1: the data) or term id (TERM*)
  int32_t dep_begin, ndeps;  // into Plan::deps (task indices, already in ticket order)
  int32_t inst_begin, ninst; // into Plan::insts (leaf tasks)
  int32_t diag;            // DIAG/OFFD: diagonal leaf block of the column cluster; LR: column cluster
  int32_t level;           // longest-path depth
  int32_t a0, a1;          // kind-specific (see TaskKind)
};

// Solves over clusters of at most SOLVE_SEQ points run as one task; larger
// ones are split at their sons, with the coupling product W2 -= L21 W1 done in
// row chunks of at most SOLVE_CHUNK points.  Term products with more than
// TERM_SPLIT rows are computed in row chunks of at most SOLVE_CHUNK points.
constexpr int64_t SOLVE_SEQ = 512;
constexpr int64_t SOLVE_CHUNK = 512;
constexpr int64_t TERM_SPLIT = 1024;

// Low-rank blocks with more than TS_BIG rows or columns take their factored
// flush as TASK_TS_* steps: their factors are stored with 2 K_MAX columns, the
// accumulation lives there in place, and every truncation runs on row blocks
// of the two factors in parallel (QR of each row block, then one QR of the
// stacked R factors: tall-skinny QR).
#ifndef HM_TS_BIG
#define HM_TS_BIG 256
#endif
#ifndef HM_TS_MINROWS
#define HM_TS_MINROWS 256
#endif
constexpr int64_t TS_BIG = HM_TS_BIG;
constexpr int TS_GMAX = 16;                     // row blocks per factor at most
constexpr int64_t TS_MINROWS = HM_TS_MINROWS;   // rows per row block at least (>= 2 K_MAX)
// Row blocks of a factor with `rows` rows: g blocks of ceil(rows / g) rows.
inline int ts_blocks(int64_t rows) {
  int64_t g = (rows + TS_MINROWS - 1) / TS_MINROWS;
  if (g > TS_GMAX) g = TS_GMAX;
  return g < 1 ? 1 : (int)g;
}
inline int64_t ts_rows(int64_t rows) {
  const int g = ts_blocks(rows);
  return (rows + g - 1) / g;
}
// Whether an m x n low-rank block is big: more than TS_BIG rows or columns,
// and every row block of both factors at least 2 K_MAX rows high (it holds a
// triangular factor of up to 2 K_MAX columns).
inline bool ts_big(int64_t m, int64_t n) {
  const int64_t lo = m < n ? m : n, hi = m < n ? n : m;
  return hi > TS_BIG && lo >= 2 * K_MAX;
}

// One step of the H forward substitution W <- L_cc^{-1} W over a cluster c:
//   SOP_TRSV  : W[off .. off+m) <- L_blk^{-1} W[off ..)   (blk dense diagonal leaf)
//   SOP_MATVEC: W[off .. off+m(blk)) -= L_blk W[off2 .. off2+n(blk))
enum SolveOpKind : int8_t { SOP_TRSV = 0, SOP_MATVEC = 1 };
struct SolveOp {
  int8_t kind;
  int32_t blk;
  int64_t off, off2;       // relative to the cluster's first position
};

struct Tree {
  int64_t n = 0;
  int32_t leaf_size = 0;
  double eta = 0;
  std::vector<int64_t> perm;     // perm[i] = input index at permuted position i
  std::vector<Cluster> cl;       // pre-order
  std::vector<Block> bk;         // pre-order
  std::vector<int32_t> sons;     // block sons storage
  std::vector<int32_t> diag_of;  // cluster id -> diagonal block id
};

struct Plan {
  // the forward solve of the data as tasks that depend on the factor tasks they
  // read (ids: factor tasks 0 .. tasks.size()-1, then these from tasks.size()),
  // in program order; run inside the stream program, beside the factorisation
  std::vector<Task> ftasks;
  std::vector<int32_t> fdeps;
  // storage
  std::vector<int64_t> dense_off;   // block id -> offset (doubles) in dense pool, -1 otherwise
  std::vector<int64_t> lr_off;      // block id -> offset of U (m x cap), then V (n x cap), cap = lr_cap
  std::vector<int64_t> lr_voff;     // block id -> offset of V
  std::vector<int32_t> lr_cap;      // block id -> columns of its U and V storage (K_MAX, or 2 K_MAX if big)
  // big low-rank blocks (TASK_TS_*): offset of their staging area (row-block
  // Householder coefficients and the small factors of the last truncation),
  // -1 otherwise; stage_pool doubles in all
  std::vector<int64_t> stage_off;
  int64_t stage_pool = 0;
  int64_t dense_pool = 0, lr_pool = 0, term_pool = 0;
  std::vector<int32_t> dense_ids, lr_ids, diag_leaf_ids;  // leaves by kind (pre-order)
  // leaves (pre-order) of every block's subtree: sub_leaves[sub_begin[b] .. sub_end[b])
  std::vector<int32_t> sub_begin, sub_end, sub_leaves;
  // terms and their per-leaf instances, CSR by leaf
  std::vector<TermDef> terms;
  std::vector<TermInst> insts;
  // tasks in ticket order and their dependencies
  std::vector<Task> tasks;
  std::vector<int32_t> task_prog;   // ticket index -> program-order index
  std::vector<int32_t> prog_obj;    // program-order index -> block/term id
  std::vector<int32_t> deps;
  // solve programs per cluster, CSR
  std::vector<int32_t> sop_begin;
  std::vector<SolveOp> sops;
  // the final forward solve L v = Z as its own task graph (solve tasks with
  // obj = -1), in level order: stasks[slevel_begin[l] .. slevel_begin[l + 1])
  std::vector<Task> stasks;
  std::vector<int32_t> sdeps;
  std::vector<int32_t> slevel_begin;
  // the backward solve L^T x = y as a task graph, in level order
  std::vector<Task> btasks;
  std::vector<int32_t> bdeps;
  std::vector<int32_t> blevel_begin;
  // row chunks (clusters of at most SOLVE_CHUNK points) of the whole index
  // set, left to right: the independent tasks of an operator product
  std::vector<int32_t> apply_chunks;
  // work counters (algorithmic)
  int64_t n_dense_entries = 0;
  int64_t max_lr_rows = 0;      // max(m, n) over low-rank leaves
  int32_t max_level = 0;
};

// Builds the cluster tree (geometric bisection) and the lower-triangular
// block tree with standard admissibility.  coords: n x 2 row-major.
void build_tree(const double* coords, int64_t n, int32_t leaf_size, double eta, Tree& t);
// Symbolic H-Cholesky: terms, instances, tasks, dependencies, solve programs.
void build_plan(const Tree& t, Plan& p);
// Level schedule of the factorisation tasks from measured durations (seconds
// or any unit): order = task ids level by level, level_begin[l] .. [l + 1] the
// tasks of level l, every dependency in an earlier level, and within a level
// the longer tasks first.
void schedule_by_durations(const Plan& p, const std::vector<double>& dur, std::vector<int32_t>& order,
                           std::vector<int32_t>& level_begin);

// Factorisation on several streams.  Task classes: (0) every task not named
// below, (1) the big blocks' flush steps (TASK_TS_*), (2) low-rank flushes of
// blocks above MS_LONG_ROWS rows or columns.  MS_STREAM_CLASS gives each
// stream its class: classes 0 and 1 run levels built as in
// schedule_by_durations (a free stream of the class takes the most critical
// ready tasks and every ready task no longer than the longest of them, so a
// further stream of the class picks up what the first left while it is busy);
// class 2 runs waves (a free stream takes every ready task) on two streams.
// A program uses the first nstreams of these streams: 4 (one stream each for
// classes 0 and 1), 6 (two each) or MS_STREAMS = 8 (three each).  Stream 0 is
// the caller's.  A launch runs
// tasks order[t0 .. t1) on its stream;
// before it, its stream waits for the events waits[wait_begin .. + nwait)
// (each recorded after an earlier launch of another stream); after it, event
// rec (>= 0) is recorded.  The launches are listed in the order the host issues
// them; every dependency of a task is met by an earlier launch of its own
// stream or by such a wait.
constexpr int MS_STREAMS = 8;
constexpr int8_t MS_STREAM_CLASS[MS_STREAMS] = {0, 1, 2, 2, 0, 1, 0, 1};
constexpr int MS_LONG_ROWS = 128;
struct MSLaunch {
  int8_t stream;
  int32_t t0, t1;
  int32_t wait_begin, nwait;
  int32_t rec;
};
struct StreamProgram {
  int32_t nstreams = 0;
  std::vector<int32_t> order;
  std::vector<MSLaunch> launches;
  std::vector<int32_t> waits;
  int32_t nevents = 0;
  double modelled_seconds = 0;   // makespan of the simulation that built it
};
// Tasks of the program: the factorisation's (p.tasks) and, when fused, the
// data solve's (p.ftasks, ids from p.tasks.size(); class 0, the general tasks); dur
// holds one duration per task of the program.
void build_stream_program(const Tree& t, const Plan& p, const std::vector<double>& dur, double launch_overhead,
                          bool fused, int nstreams, StreamProgram& out);
// Throws std::logic_error if a dependency is not met as stated above.
void validate_stream_program(const Plan& p, const StreamProgram& g, bool fused);

}  // namespace hm
