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
  TASK_DIAG = 0,    // dense diagonal leaf: flush + Cholesky
  TASK_OFFD = 1,    // dense off-diagonal leaf: flush + triangular solve
  TASK_LR = 2,      // low-rank leaf: flush (truncation) + V <- L^-1 V
  TASK_TERM = 3,    // compute the product factor of a term
};

struct Task {
  int8_t kind;
  int32_t obj;             // block id (DIAG/OFFD/LR) or term id (TERM)
  int32_t dep_begin, ndeps;  // into Plan::deps (task indices, already in ticket order)
  int32_t inst_begin, ninst; // into Plan::insts (leaf tasks)
  int32_t diag;            // DIAG/OFFD: diagonal leaf block of the column cluster; LR: column cluster
  int32_t level;           // longest-path depth
};

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
  // storage
  std::vector<int64_t> dense_off;   // block id -> offset (doubles) in dense pool, -1 otherwise
  std::vector<int64_t> lr_off;      // block id -> offset of U (m*K_MAX) then V (n*K_MAX)
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

}  // namespace hm
