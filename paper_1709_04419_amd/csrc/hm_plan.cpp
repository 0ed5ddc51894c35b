// Host planner: cluster tree, block cluster tree and symbolic H-Cholesky.
//
// Cluster tree (Appendix B, Definition B.1): geometric bisection.  A cluster
// with more than n_min points is split along the longest side of its tight
// bounding box (lowest axis on ties) at the median of the total order
// (coordinate, original index); the first son gets floor(|t|/2) points.  The
// permutation is the left-to-right order of the leaves.
//
// Block cluster tree (Definitions B.2, B.3): lower triangle only, standard
// admissibility min(diam^2) <= eta^2 dist^2 with dist^2 > 0, evaluated with a
// fixed operation order.  This file is compiled without floating-point
// contraction so that the partition is reproducible bit for bit.
//
// Symbolic H-Cholesky (Section 3.2: the factor keeps the block structure of
// the matrix; log|C| = 2 sum log L_ii): the recursive formatted Cholesky with
// deferred, per-leaf ordered updates is run once without numbers.  It records
//   * every update term (what its factors X, Y are made of),
//   * for every leaf the ordered list of restricted terms it must subtract,
//   * the tasks (dense diagonal, dense off-diagonal, low-rank leaf, term
//     product) with their data dependencies,
//   * the forward-substitution programs over clusters.
// The device executes the tasks in any order compatible with the
// dependencies; each leaf still applies its terms in program order, so the
// arithmetic per leaf is fixed.
#include "hm_plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <deque>
#include <map>
#include <queue>
#include <set>
#include <stdexcept>

namespace hm {

namespace {

struct TreeBuilder {
  const double* P;
  int64_t n;
  int32_t nmin;
  Tree& t;
  std::vector<int64_t> work;

  int32_t build(int64_t b, int64_t e, int32_t level) {
    Cluster c{};
    c.begin = b;
    c.end = e;
    c.level = level;
    c.son[0] = c.son[1] = -1;
    for (int ax = 0; ax < 2; ++ax) {
      double lo = P[2 * work[b] + ax], hi = lo;
      for (int64_t i = b + 1; i < e; ++i) {
        double v = P[2 * work[i] + ax];
        if (v < lo) lo = v;
        if (v > hi) hi = v;
      }
      c.lo[ax] = lo;
      c.hi[ax] = hi;
    }
    int32_t id = (int32_t)t.cl.size();
    t.cl.push_back(c);
    if (e - b <= nmin) return id;
    double ext0 = c.hi[0] - c.lo[0], ext1 = c.hi[1] - c.lo[1];
    int ax = (ext1 > ext0) ? 1 : 0;  // lowest axis on ties
    const double* Pp = P;
    std::sort(work.begin() + b, work.begin() + e, [Pp, ax](int64_t i, int64_t j) {
      double a = Pp[2 * i + ax], bb = Pp[2 * j + ax];
      return a < bb || (a == bb && i < j);
    });
    int64_t half = (e - b) / 2;
    int32_t s0 = build(b, b + half, level + 1);
    int32_t s1 = build(b + half, e, level + 1);
    t.cl[id].son[0] = s0;
    t.cl[id].son[1] = s1;
    return id;
  }
};

inline bool is_leaf(const Cluster& c) { return c.son[0] < 0; }

double diam2(const Cluster& c) {
  double dx = c.hi[0] - c.lo[0];
  double dy = c.hi[1] - c.lo[1];
  double a = dx * dx;
  double b = dy * dy;
  return a + b;
}

double dist2(const Cluster& a, const Cluster& b) {
  double s = 0.0;
  for (int ax = 0; ax < 2; ++ax) {
    double g = 0.0;
    double g1 = b.lo[ax] - a.hi[ax];
    double g2 = a.lo[ax] - b.hi[ax];
    if (g1 > g) g = g1;
    if (g2 > g) g = g2;
    double gg = g * g;
    s = s + gg;
  }
  return s;
}

bool admissible(const Cluster& a, const Cluster& b, double eta) {
  double d2 = dist2(a, b);
  if (!(d2 > 0.0)) return false;
  double da = diam2(a), db = diam2(b);
  double dm = da < db ? da : db;
  double e2 = eta * eta;
  double rhs = e2 * d2;
  return dm <= rhs;
}

struct BlockBuilder {
  Tree& t;
  double eta;
  int32_t build(int32_t r, int32_t s) {
    const Cluster& R = t.cl[r];
    const Cluster& S = t.cl[s];
    Block b{};
    b.row = r;
    b.col = s;
    b.kind = BK_NODE;
    b.r0 = R.begin;
    b.c0 = S.begin;
    b.m = R.end - R.begin;
    b.n = S.end - S.begin;
    b.son_begin = -1;
    b.nsons = 0;
    int32_t id = (int32_t)t.bk.size();
    t.bk.push_back(b);
    if (r == s) t.diag_of[r] = id;
    if (r != s && admissible(R, S, eta)) {
      t.bk[id].kind = BK_LR;
      return id;
    }
    if (is_leaf(R) && is_leaf(S)) {
      t.bk[id].kind = BK_DENSE;
      return id;
    }
    int32_t rows[2], cols[2];
    int nr = 0, nc = 0;
    if (is_leaf(R)) rows[nr++] = r; else { rows[nr++] = R.son[0]; rows[nr++] = R.son[1]; }
    if (is_leaf(S)) cols[nc++] = s; else { cols[nc++] = S.son[0]; cols[nc++] = S.son[1]; }
    int32_t local[4];
    int ns = 0;
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nc; ++j) {
        if (r == s && t.cl[rows[i]].begin < t.cl[cols[j]].begin) continue;
        local[ns++] = build(rows[i], cols[j]);
      }
    t.bk[id].son_begin = (int32_t)t.sons.size();
    t.bk[id].nsons = ns;
    for (int i = 0; i < ns; ++i) t.sons.push_back(local[i]);
    return id;
  }
};

}  // namespace

void build_tree(const double* coords, int64_t n, int32_t leaf_size, double eta, Tree& t) {
  if (n < 1 || leaf_size < 1) throw std::invalid_argument("n and leaf_size must be >= 1");
  t = Tree{};
  t.n = n;
  t.leaf_size = leaf_size;
  t.eta = eta;
  TreeBuilder tb{coords, n, leaf_size, t, {}};
  tb.work.resize(n);
  for (int64_t i = 0; i < n; ++i) tb.work[i] = i;
  tb.build(0, n, 0);
  t.perm = tb.work;
  t.diag_of.assign(t.cl.size(), -1);
  BlockBuilder bb{t, eta};
  bb.build(0, 0);
}

// ---------------------------------------------------------------- planner

namespace {

struct Planner {
  const Tree& T;
  Plan& P;
  std::vector<int32_t> final_task;                  // block -> task that finalises it
  std::vector<std::vector<TermInst>> leaf_insts;    // block -> ordered instances
  std::vector<Task> tasks;                          // program order
  std::vector<std::vector<int32_t>> tdeps;
  std::vector<std::vector<int32_t>> term_tasks;     // term -> tasks computing its factor (none for TK_DD)
  std::vector<int32_t> sub_end;                     // block -> one past its pre-order subtree
  std::vector<int32_t> leaf_rank;                   // block -> #leaves with smaller id

  Planner(const Tree& t, Plan& p) : T(t), P(p) {}

  const Block& B(int32_t b) const { return T.bk[b]; }
  const Cluster& C(int32_t c) const { return T.cl[c]; }

  int32_t son(int32_t b, int32_t r, int32_t c) const {
    const Block& bb = B(b);
    for (int i = 0; i < bb.nsons; ++i) {
      int32_t s = T.sons[bb.son_begin + i];
      if (B(s).row == r && B(s).col == c) return s;
    }
    throw std::logic_error("missing block son");
  }

  void leaves_of(int32_t b, std::vector<int32_t>& out) const {
    for (int32_t i = leaf_rank[b]; i < leaf_rank[sub_end[b]]; ++i) out.push_back(P.sub_leaves[i]);
  }

  // set while the fused data solve is emitted: negative dependencies then
  // name factor tasks (-1 - id) rather than unfinished blocks
  bool factor_deps_coded = false;

  int32_t new_task(int8_t kind, int32_t obj, std::vector<int32_t> deps, int32_t a0 = 0, int32_t a1 = 0) {
    std::sort(deps.begin(), deps.end());
    deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
    if (!deps.empty() && deps.front() < 0 && !factor_deps_coded)
      throw std::logic_error("dependency on an unfinished block");
    Task t{};
    t.kind = kind;
    t.obj = obj;
    t.diag = -1;
    t.a0 = a0;
    t.a1 = a1;
    if (tasks.size() >= (size_t)INT32_MAX) throw std::length_error("task graph: more tasks than 32-bit ids");
    tasks.push_back(t);
    tdeps.push_back(std::move(deps));
    return (int32_t)tasks.size() - 1;
  }

  // Clusters below x (x itself if small enough) of at most `limit` points
  // (or leaves), left to right.
  void chunks_of(int32_t x, int64_t limit, std::vector<int32_t>& out) const {
    if (C(x).end - C(x).begin <= limit || is_leaf(C(x))) {
      out.push_back(x);
      return;
    }
    chunks_of(C(x).son[0], limit, out);
    chunks_of(C(x).son[1], limit, out);
  }

  // Leaves of block b whose rows meet the rows of cluster q, in pre-order.
  void leaves_in_rows(int32_t b, int32_t q, std::vector<int32_t>& out) const {
    for (int32_t i = leaf_rank[b]; i < leaf_rank[sub_end[b]]; ++i) {
      const int32_t l = P.sub_leaves[i];
      if (B(l).r0 < C(q).end && B(l).r0 + B(l).m > C(q).begin) out.push_back(l);
    }
  }

  // The forward substitution W(c) <- L_cc^{-1} W(c) of target `tgt` (a
  // low-rank block's V, or -1 for the data) as tasks: clusters of at most
  // SOLVE_SEQ points in one task by their solve program; larger ones as
  // W(c1) solve, W(c2) -= L21 W(c1) in row chunks, W(c2) solve.  Every row
  // receives the same operations in the same order as the cluster's solve
  // program.  `deps` must precede every task; with factor_deps the tasks also
  // wait for the factor leaves they read.  Returns the task after which all of
  // W(c) is final.
  int32_t emit_solve(int32_t tgt, int32_t c, const std::vector<int32_t>& deps, bool factor_deps) {
    const int32_t d = T.diag_of[c];
    if (C(c).end - C(c).begin <= SOLVE_SEQ || is_leaf(C(c))) {
      std::vector<int32_t> dp = deps;
      if (factor_deps) {
        std::vector<int32_t> lv;
        leaves_of(d, lv);
        for (int32_t l : lv) dp.push_back(final_task[l]);
      }
      return new_task(TASK_SOLVE_SEQ, tgt, dp, c, 0);
    }
    const int32_t c1 = C(c).son[0], c2 = C(c).son[1];
    const int32_t t1 = emit_solve(tgt, c1, deps, factor_deps);
    const int32_t b21 = son(d, c2, c1);
    std::vector<int32_t> qs;
    chunks_of(c2, SOLVE_CHUNK, qs);
    std::vector<int32_t> mv = deps;
    for (int32_t q : qs) {
      std::vector<int32_t> dp = deps;
      dp.push_back(t1);
      if (factor_deps) {
        std::vector<int32_t> lv;
        leaves_in_rows(b21, q, lv);
        for (int32_t l : lv) dp.push_back(final_task[l]);
      }
      mv.push_back(new_task(TASK_SOLVE_MV, tgt, dp, b21, q));
    }
    return emit_solve(tgt, c2, mv, factor_deps);
  }

  // The backward substitution W(c) <- L_cc^{-T} W(c) of the data: clusters of
  // at most SOLVE_SEQ points in one task (their solve program backwards);
  // larger ones as W(c2) solve, W(c1) -= L21^T W(c2) in row chunks of c1,
  // W(c1) solve.  Returns the task after which all of W(c) is final.
  int32_t emit_solve_t(int32_t c, const std::vector<int32_t>& deps) {
    const int32_t d = T.diag_of[c];
    if (C(c).end - C(c).begin <= SOLVE_SEQ || is_leaf(C(c))) return new_task(TASK_SOLVE_SEQ_T, -1, deps, c, 0);
    const int32_t c1 = C(c).son[0], c2 = C(c).son[1];
    const int32_t t2 = emit_solve_t(c2, deps);
    const int32_t b21 = son(d, c2, c1);
    std::vector<int32_t> qs;
    chunks_of(c1, SOLVE_CHUNK, qs);
    std::vector<int32_t> mv = deps;
    for (int32_t q : qs) {
      std::vector<int32_t> dp = deps;
      dp.push_back(t2);
      mv.push_back(new_task(TASK_SOLVE_MV_T, -1, dp, b21, q));
    }
    return emit_solve_t(c1, mv);
  }

  // Sorts the tasks recorded since `tasks` was cleared into levels (longest
  // path) and stores them with their dependencies renumbered.
  void leveled(std::vector<Task>& out, std::vector<int32_t>& odeps, std::vector<int32_t>& obegin) {
    const int32_t ns = (int32_t)tasks.size();
    std::vector<int32_t> lev(ns, 0);
    for (int32_t i = 0; i < ns; ++i)
      for (int32_t d : tdeps[i]) {
        if (d >= i) throw std::logic_error("operator dependency not earlier in program order");
        lev[i] = std::max(lev[i], lev[d] + 1);
      }
    std::vector<int32_t> ord(ns);
    for (int32_t i = 0; i < ns; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return lev[a] < lev[b]; });
    std::vector<int32_t> rk(ns);
    for (int32_t i = 0; i < ns; ++i) rk[ord[i]] = i;
    out.clear();
    odeps.clear();
    obegin.clear();
    for (int32_t k = 0; k < ns; ++k) {
      const int32_t i = ord[k];
      Task t = tasks[i];
      t.level = lev[i];
      if (obegin.size() <= (size_t)t.level) obegin.push_back(k);
      t.dep_begin = (int32_t)odeps.size();
      for (int32_t d : tdeps[i]) odeps.push_back(rk[d]);
      t.ndeps = (int32_t)tdeps[i].size();
      t.inst_begin = t.ninst = 0;
      out.push_back(t);
    }
    obegin.push_back(ns);
  }

  void push(int32_t bid, int64_t R0, int64_t C0, int32_t term, int64_t xoff, int64_t yoff,
            int64_t mx, int64_t ny) {
    const Block& b = B(bid);
    if (b.kind != BK_NODE) {
      TermInst in{};
      in.term = term;
      in.lr0 = (int32_t)(R0 - b.r0);
      in.lc0 = (int32_t)(C0 - b.c0);
      in.mx = (int32_t)mx;
      in.ny = (int32_t)ny;
      in.xr0 = xoff;
      in.yr0 = yoff;
      leaf_insts[bid].push_back(in);
      return;
    }
    if (R0 != b.r0 || C0 != b.c0 || mx != b.m || ny != b.n)
      throw std::logic_error("partial target on a non-leaf block");
    for (int i = 0; i < b.nsons; ++i) {
      int32_t s = T.sons[b.son_begin + i];
      const Block& sb = B(s);
      push(s, sb.r0, sb.c0, term, xoff + (sb.r0 - R0), yoff + (sb.c0 - C0), sb.m, sb.n);
    }
  }

  struct Target {
    int32_t bid;
    int64_t R0, C0;
  };

  Target sub_target(const Target& tg, int32_t t, int32_t s) const {
    Target o{tg.bid, C(t).begin, C(s).begin};
    if (B(tg.bid).kind == BK_NODE) o.bid = son(tg.bid, t, s);
    return o;
  }

  void update(const Target& tg, int32_t A, int32_t Bb) {
    int8_t ka = B(A).kind, kb = B(Bb).kind;
    int64_t mx = B(A).m, ny = B(Bb).m;
    if (ka == BK_LR || kb == BK_LR || (ka == BK_DENSE && kb == BK_DENSE)) {
      TermDef d{};
      d.A = A;
      d.B = Bb;
      std::vector<int32_t> deps;
      if (P.terms.size() >= (size_t)INT32_MAX) throw std::length_error("task graph: more terms than 32-bit ids");
      int32_t tid = (int32_t)P.terms.size();
      if (ka == BK_LR) {
        d.kind = TK_LRA;
        d.rows = ny;
        deps.push_back(final_task[A]);
        std::vector<int32_t> lv;
        leaves_of(Bb, lv);
        for (int32_t l : lv) deps.push_back(final_task[l]);
      } else if (kb == BK_LR) {
        d.kind = TK_LRB;
        d.rows = mx;
        deps.push_back(final_task[Bb]);
        std::vector<int32_t> lv;
        leaves_of(A, lv);
        for (int32_t l : lv) deps.push_back(final_task[l]);
      } else {
        d.kind = TK_DD;
        d.rows = 0;
      }
      d.buf = -1;
      term_tasks.emplace_back();
      if (d.rows > 0) {
        // rows of the computed factor = rows of the H-block applied
        const int32_t hrow = (d.kind == TK_LRA) ? B(Bb).row : B(A).row;
        if (d.rows > TERM_SPLIT) {
          std::vector<int32_t> qs;
          chunks_of(hrow, SOLVE_CHUNK, qs);
          for (int32_t q : qs) term_tasks[tid].push_back(new_task(TASK_TERM_ROWS, tid, deps, 0, q));
        } else {
          term_tasks[tid].push_back(new_task(TASK_TERM, tid, deps));
        }
      }
      P.terms.push_back(d);
      push(tg.bid, tg.R0, tg.C0, tid, 0, 0, mx, ny);
      return;
    }
    int32_t tau = B(A).row, rho = B(A).col, sig = B(Bb).row;
    int32_t ts[2], ss[2], rs[2];
    int nt = 0, nss = 0, nr = 0;
    if (ka == BK_NODE && !is_leaf(C(tau))) { ts[nt++] = C(tau).son[0]; ts[nt++] = C(tau).son[1]; }
    else ts[nt++] = tau;
    if (kb == BK_NODE && !is_leaf(C(sig))) { ss[nss++] = C(sig).son[0]; ss[nss++] = C(sig).son[1]; }
    else ss[nss++] = sig;
    if (!is_leaf(C(rho))) { rs[nr++] = C(rho).son[0]; rs[nr++] = C(rho).son[1]; }
    else rs[nr++] = rho;
    bool diag = tau == sig;
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nss; ++j) {
        if (diag && C(ts[i]).begin < C(ss[j]).begin) continue;
        Target sub = sub_target(tg, ts[i], ss[j]);
        for (int k = 0; k < nr; ++k) {
          int32_t a = (ka != BK_NODE) ? A : son(A, ts[i], rs[k]);
          int32_t b = (kb != BK_NODE) ? Bb : son(Bb, ss[j], rs[k]);
          update(sub, a, b);
        }
      }
  }

  void inst_deps_one(const TermInst& in, std::vector<int32_t>& deps) const {
    const TermDef& d = P.terms[in.term];
    if (d.kind == TK_DD) {
      deps.push_back(final_task[d.A]);
      deps.push_back(final_task[d.B]);
    } else {
      for (int32_t q : term_tasks[in.term]) deps.push_back(q);
    }
  }

  std::vector<int32_t> inst_deps(int32_t bid) const {
    std::vector<int32_t> deps;
    for (const TermInst& in : leaf_insts[bid]) inst_deps_one(in, deps);
    return deps;
  }

  // Factored flush of a big low-rank block (T >= 1 pending terms) as steps
  // 1 .. T + 1 of TASK_TS_A (per row block), TASK_TS_B, TASK_TS_C (per row
  // block); `extra` must precede the final truncation.  Returns the final
  // step's row-block tasks.
  std::vector<int32_t> emit_ts(int32_t bid, const std::vector<int32_t>& extra) {
    const Block& b = B(bid);
    const int gx = ts_blocks(b.m), gy = ts_blocks(b.n), g = gx + gy;
    const int32_t T1 = (int32_t)leaf_insts[bid].size() + 1;
    std::vector<int32_t> prevC;   // C tasks of the previous step, by row block
    for (int32_t i = 1; i <= T1; ++i) {
      // every task of step i reads the rank of term i (whether to truncate),
      // so all of them wait for the term's producers
      std::vector<int32_t> term_dp;
      if (i < T1) inst_deps_one(leaf_insts[bid][i - 1], term_dp);
      std::vector<int32_t> as;
      for (int q = 0; q < g; ++q) {
        std::vector<int32_t> dp = term_dp;
        if (!prevC.empty()) dp.push_back(prevC[q]);
        as.push_back(new_task(TASK_TS_A, bid, dp, i, q));
      }
      std::vector<int32_t> bd = as;
      if (i == T1) bd.insert(bd.end(), extra.begin(), extra.end());
      const int32_t tb = new_task(TASK_TS_B, bid, bd, i, 0);
      std::vector<int32_t> cd{tb};
      prevC.clear();
      for (int q = 0; q < g; ++q) prevC.push_back(new_task(TASK_TS_C, bid, cd, i, q));
    }
    return prevC;
  }

  // Term buffers by liveness.  A computed term factor is written by its
  // producer tasks and read while the leaves that hold its instances are
  // flushed; every such read happens before final_task of that leaf (the
  // flush task, or a task that depends on it).  Sweeping the program order, a
  // term's buffer is released after the last of those final tasks and given
  // to a later term of the same row count whose producers are at least
  // TERM_REUSE_SLACK longest-path levels later than every one of them; the
  // new producers then depend on those final tasks, so no schedule can
  // overwrite a factor that is still to be read.
  void share_term_buffers() {
    constexpr int32_t TERM_REUSE_SLACK = 8;
    const int32_t nt = (int32_t)tasks.size(), nterm = (int32_t)P.terms.size();
    std::vector<int32_t> lev(nt, 0);
    for (int32_t i = 0; i < nt; ++i)
      for (int32_t d : tdeps[i]) lev[i] = std::max(lev[i], lev[d] + 1);
    std::vector<std::vector<int32_t>> cons(nterm);
    for (size_t b = 0; b < leaf_insts.size(); ++b)
      for (const TermInst& in : leaf_insts[b])
        if (P.terms[in.term].rows > 0) cons[in.term].push_back(final_task[b]);
    std::vector<int32_t> first(nterm, -1), last(nterm, -1), conslev(nterm, 0);
    std::vector<std::vector<int32_t>> at_first(nt + 1), at_free(nt + 1);
    for (int32_t k = 0; k < nterm; ++k) {
      if (P.terms[k].rows <= 0 || term_tasks[k].empty()) continue;
      auto& c = cons[k];
      std::sort(c.begin(), c.end());
      c.erase(std::unique(c.begin(), c.end()), c.end());
      first[k] = *std::min_element(term_tasks[k].begin(), term_tasks[k].end());
      last[k] = *std::max_element(term_tasks[k].begin(), term_tasks[k].end());
      for (int32_t q : c) {
        if (q < 0) throw std::logic_error("term consumer without a final task");
        last[k] = std::max(last[k], q);
        conslev[k] = std::max(conslev[k], lev[q]);
      }
      at_first[first[k]].push_back(k);
      at_free[last[k] + 1].push_back(k);
    }
    struct Slot {
      int64_t off;
      int32_t prev;   // term that held it last
    };
    std::map<int64_t, std::deque<Slot>> free_by_rows;
    P.term_pool = 0;
    for (int32_t i = 0; i <= nt; ++i) {
      for (int32_t k : at_free[i]) free_by_rows[P.terms[k].rows].push_back(Slot{P.terms[k].buf, k});
      if (i == nt) break;
      for (int32_t k : at_first[i]) {
        TermDef& d = P.terms[k];
        int32_t plev = nt;
        for (int32_t q : term_tasks[k]) plev = std::min(plev, lev[q]);
        auto& fl = free_by_rows[d.rows];
        bool got = false;
        for (int probe = 0; probe < 8 && probe < (int)fl.size(); ++probe) {
          const Slot sl = fl[probe];
          if (conslev[sl.prev] + TERM_REUSE_SLACK >= plev) continue;
          fl.erase(fl.begin() + probe);
          d.buf = sl.off;
          for (int32_t q : term_tasks[k])
            for (int32_t c : cons[sl.prev]) tdeps[q].push_back(c);
          got = true;
          break;
        }
        if (!got) {
          d.buf = P.term_pool;
          P.term_pool += d.rows * K_MAX;
        }
      }
    }
  }

  void htrsm(int32_t bid) {
    const Block& b = B(bid);
    int32_t sig = b.col;
    if (b.kind == BK_DENSE) {
      std::vector<int32_t> deps = inst_deps(bid);
      int32_t d = T.diag_of[sig];
      deps.push_back(final_task[d]);
      int32_t t = new_task(TASK_OFFD, bid, deps);
      tasks[t].diag = d;
      final_task[bid] = t;
      return;
    }
    if (b.kind == BK_LR) {
      std::vector<int32_t> lv;
      leaves_of(T.diag_of[sig], lv);
      std::vector<int32_t> lfin;
      for (int32_t l : lv) lfin.push_back(final_task[l]);
      if (ts_big(b.m, b.n) && !leaf_insts[bid].empty()) {
        // the flush as parallel steps, then V <- L^{-1} V as solve tasks
        const std::vector<int32_t> fin = emit_ts(bid, lfin);
        final_task[bid] = emit_solve(bid, sig, fin, false);
        return;
      }
      std::vector<int32_t> deps = inst_deps(bid);
      deps.insert(deps.end(), lfin.begin(), lfin.end());
      int32_t t = new_task(TASK_LR, bid, deps);
      tasks[t].diag = sig;
      if (b.n > SOLVE_SEQ && !is_leaf(C(sig))) {
        // V <- L_{sigma sigma}^{-1} V as a chain of solve tasks (the flush task
        // already waits for every leaf of L_{sigma sigma})
        tasks[t].a0 = 0;
        final_task[bid] = emit_solve(bid, sig, {t}, false);
      } else {
        tasks[t].a0 = 1;
        final_task[bid] = t;
      }
      return;
    }
    int32_t rho = b.row;
    int32_t rows[2];
    int nr = 0;
    if (is_leaf(C(rho))) rows[nr++] = rho; else { rows[nr++] = C(rho).son[0]; rows[nr++] = C(rho).son[1]; }
    if (is_leaf(C(sig))) {
      for (int i = 0; i < nr; ++i) htrsm(son(bid, rows[i], sig));
      return;
    }
    int32_t s1 = C(sig).son[0], s2 = C(sig).son[1];
    int32_t L21 = son(T.diag_of[sig], s2, s1);
    for (int i = 0; i < nr; ++i) {
      int32_t b1 = son(bid, rows[i], s1);
      int32_t b2 = son(bid, rows[i], s2);
      htrsm(b1);
      update(Target{b2, C(rows[i]).begin, C(s2).begin}, b1, L21);
      htrsm(b2);
    }
  }

  void hchol(int32_t c) {
    int32_t d = T.diag_of[c];
    if (is_leaf(C(c))) {
      int32_t t = new_task(TASK_DIAG, d, inst_deps(d));
      tasks[t].diag = d;
      final_task[d] = t;
      return;
    }
    int32_t c1 = C(c).son[0], c2 = C(c).son[1];
    hchol(c1);
    int32_t b21 = son(d, c2, c1);
    htrsm(b21);
    update(Target{T.diag_of[c2], C(c2).begin, C(c2).begin}, b21, b21);
    hchol(c2);
  }

  void solve_prog(int32_t c, int64_t base, std::vector<SolveOp>& out) const {
    int32_t d = T.diag_of[c];
    if (is_leaf(C(c))) {
      SolveOp op{};
      op.kind = SOP_TRSV;
      op.blk = d;
      op.off = C(c).begin - base;
      op.off2 = 0;
      out.push_back(op);
      return;
    }
    int32_t c1 = C(c).son[0], c2 = C(c).son[1];
    solve_prog(c1, base, out);
    int32_t b21 = son(d, c2, c1);
    std::vector<int32_t> lv;
    leaves_of(b21, lv);
    for (int32_t l : lv) {
      SolveOp op{};
      op.kind = SOP_MATVEC;
      op.blk = l;
      op.off = B(l).r0 - base;
      op.off2 = B(l).c0 - base;
      out.push_back(op);
    }
    solve_prog(c2, base, out);
  }

  void run() {
    const int32_t nb = (int32_t)T.bk.size();
    // leaves in pre-order and subtree extents
    sub_end.assign(nb, 0);
    for (int32_t b = nb - 1; b >= 0; --b) {
      const Block& bb = B(b);
      sub_end[b] = b + 1;
      for (int i = 0; i < bb.nsons; ++i) sub_end[b] = std::max(sub_end[b], sub_end[T.sons[bb.son_begin + i]]);
    }
    leaf_rank.assign(nb + 1, 0);
    P.sub_leaves.clear();
    for (int32_t b = 0; b < nb; ++b) {
      leaf_rank[b] = (int32_t)P.sub_leaves.size();
      if (B(b).kind != BK_NODE) P.sub_leaves.push_back(b);
    }
    leaf_rank[nb] = (int32_t)P.sub_leaves.size();
    P.sub_begin.assign(nb, 0);
    P.sub_end.assign(nb, 0);
    for (int32_t b = 0; b < nb; ++b) {
      P.sub_begin[b] = leaf_rank[b];
      P.sub_end[b] = leaf_rank[sub_end[b]];
    }
    // storage
    P.dense_off.assign(nb, -1);
    P.lr_off.assign(nb, -1);
    P.lr_voff.assign(nb, -1);
    P.lr_cap.assign(nb, 0);
    P.stage_off.assign(nb, -1);
    P.stage_pool = 0;
    P.dense_pool = P.lr_pool = P.term_pool = 0;
    P.n_dense_entries = 0;
    P.max_lr_rows = 0;
    for (int32_t b = 0; b < nb; ++b) {
      const Block& bb = B(b);
      if (bb.kind == BK_DENSE) {
        P.dense_off[b] = P.dense_pool;
        P.dense_pool += bb.m * bb.n;
        P.n_dense_entries += bb.m * bb.n;
        P.dense_ids.push_back(b);
        if (bb.row == bb.col) P.diag_leaf_ids.push_back(b);
      } else if (bb.kind == BK_LR) {
        const bool big = ts_big(bb.m, bb.n);
        const int32_t cap = big ? 2 * K_MAX : K_MAX;
        P.lr_cap[b] = cap;
        P.lr_off[b] = P.lr_pool;
        P.lr_voff[b] = P.lr_pool + bb.m * cap;
        P.lr_pool += (bb.m + bb.n) * (int64_t)cap;
        P.lr_ids.push_back(b);
        if (big) {
          P.stage_off[b] = P.stage_pool;
          const int64_t g = ts_blocks(bb.m) + ts_blocks(bb.n);
          P.stage_pool += g * 2 * K_MAX * (1 + K_MAX);
        } else {
          P.max_lr_rows = std::max(P.max_lr_rows, std::max(bb.m, bb.n));
        }
      }
    }
    // symbolic factorisation in program order
    final_task.assign(nb, -1);
    leaf_insts.assign(nb, {});
    hchol(0);
    share_term_buffers();
    // levels (longest path) and ticket order
    const int32_t nt = (int32_t)tasks.size();
    std::vector<int32_t> level(nt, 0);
    for (int32_t i = 0; i < nt; ++i) {
      int32_t lv = 0;
      for (int32_t d : tdeps[i]) {
        if (d >= i) throw std::logic_error("dependency not earlier in program order");
        lv = std::max(lv, level[d] + 1);
      }
      level[i] = lv;
    }
    std::vector<int32_t> order(nt);
    for (int32_t i = 0; i < nt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return level[a] < level[b]; });
    std::vector<int32_t> rank(nt);
    for (int32_t i = 0; i < nt; ++i) rank[order[i]] = i;
    P.tasks.clear();
    P.deps.clear();
    P.insts.clear();
    P.max_level = 0;
    std::vector<int32_t> ts_inst(nb, -1);   // big block -> first of its instances in P.insts
    for (int32_t k = 0; k < nt; ++k) {
      int32_t i = order[k];
      Task t = tasks[i];
      t.level = level[i];
      P.max_level = std::max(P.max_level, level[i]);
      // dependency and instance lists are indexed with 32 bits on both sides
      if (P.deps.size() + tdeps[i].size() > (size_t)INT32_MAX || P.insts.size() + leaf_insts.size() > (size_t)INT32_MAX)
        throw std::length_error("task graph: more dependencies or instances than 32-bit offsets");
      t.dep_begin = (int32_t)P.deps.size();
      for (int32_t d : tdeps[i]) P.deps.push_back(rank[d]);
      t.ndeps = (int32_t)tdeps[i].size();
      t.inst_begin = (int32_t)P.insts.size();
      t.ninst = 0;
      if (t.kind == TASK_DIAG || t.kind == TASK_OFFD || t.kind == TASK_LR) {
        for (const TermInst& in : leaf_insts[t.obj]) P.insts.push_back(in);
        t.ninst = (int32_t)leaf_insts[t.obj].size();
      } else if (t.kind == TASK_TS_A || t.kind == TASK_TS_B || t.kind == TASK_TS_C) {
        if (ts_inst[t.obj] < 0) {
          ts_inst[t.obj] = (int32_t)P.insts.size();
          for (const TermInst& in : leaf_insts[t.obj]) P.insts.push_back(in);
        }
        t.inst_begin = ts_inst[t.obj];
        t.ninst = (int32_t)leaf_insts[t.obj].size();
      }
      P.tasks.push_back(t);
      P.task_prog.push_back(i);
    }
    P.prog_obj.resize(nt);
    for (int32_t i = 0; i < nt; ++i) P.prog_obj[i] = tasks[i].obj;
    // the data's forward solve again, now depending on the factor tasks whose
    // blocks it reads: final_task is re-coded as -1 - (task id) while it is
    // emitted, so those dependencies are told apart from the solve's own
    {
      const std::vector<int32_t> saved = final_task;
      // (a block without a final task decodes out of range, which the
      // validation rejects)
      for (int32_t& f : final_task) f = f >= 0 ? -1 - rank[f] : INT32_MIN;
      tasks.clear();
      tdeps.clear();
      factor_deps_coded = true;
      emit_solve(-1, 0, {}, true);
      factor_deps_coded = false;
      final_task = saved;
      const int32_t nf = (int32_t)tasks.size();
      P.ftasks.clear();
      P.fdeps.clear();
      for (int32_t i = 0; i < nf; ++i) {
        Task t = tasks[i];
        t.level = 0;
        if (P.fdeps.size() + tdeps[i].size() > (size_t)INT32_MAX)
          throw std::length_error("task graph: more dependencies than 32-bit offsets");
        t.dep_begin = (int32_t)P.fdeps.size();
        t.ndeps = (int32_t)tdeps[i].size();
        for (int32_t d : tdeps[i]) {
          if (d < 0) {
            P.fdeps.push_back(-1 - d);
          } else {
            if (d >= i) throw std::logic_error("data solve dependency not earlier in program order");
            P.fdeps.push_back(nt + d);
          }
        }
        P.ftasks.push_back(t);
      }
    }
    // solve programs for every cluster
    const int32_t nc = (int32_t)T.cl.size();
    P.sop_begin.assign(nc + 1, 0);
    P.sops.clear();
    for (int32_t c = 0; c < nc; ++c) {
      P.sop_begin[c] = (int32_t)P.sops.size();
      solve_prog(c, C(c).begin, P.sops);
    }
    P.sop_begin[nc] = (int32_t)P.sops.size();
    // the final forward solve as a task graph of its own (it runs after the
    // whole factorisation, so it needs no dependencies on factor tasks)
    tasks.clear();
    tdeps.clear();
    emit_solve(-1, 0, {}, false);
    leveled(P.stasks, P.sdeps, P.slevel_begin);
    // the backward solve with L^T, and the row chunks of operator products
    tasks.clear();
    tdeps.clear();
    emit_solve_t(0, {});
    leveled(P.btasks, P.bdeps, P.blevel_begin);
    tasks.clear();
    tdeps.clear();
    P.apply_chunks.clear();
    chunks_of(0, SOLVE_CHUNK, P.apply_chunks);
  }
};

}  // namespace

// A solve task's target rows: the low-rank block's column cluster (obj >= 0)
// or the whole index set (obj = -1); every cluster and block it reads lies
// inside them.
template <class F>
static void check_solve_task(const Tree& T, const Task& t, F fail) {
  const int32_t nb = (int32_t)T.bk.size(), nc = (int32_t)T.cl.size();
  int64_t lo = 0, hi = T.n;
  if (t.obj >= 0) {
    if (t.obj >= nb || T.bk[t.obj].kind != BK_LR) fail("solve target");
    lo = T.bk[t.obj].c0;
    hi = lo + T.bk[t.obj].n;
  }
  if (t.kind == TASK_SOLVE_SEQ) {
    if (t.a0 < 0 || t.a0 >= nc) fail("solve cluster");
    if (T.cl[t.a0].begin < lo || T.cl[t.a0].end > hi) fail("solve cluster rows");
    return;
  }
  if (t.a0 < 0 || t.a0 >= nb || t.a1 < 0 || t.a1 >= nc) fail("solve product ids");
  const Block& b = T.bk[t.a0];
  const Cluster& q = T.cl[t.a1];
  if (b.r0 < lo || b.r0 + b.m > hi || b.c0 < lo || b.c0 + b.n > hi) fail("solve product block");
  if (q.begin < b.r0 || q.end > b.r0 + b.m) fail("solve product chunk");
}

// Bounds and ordering checks of everything the device will index with.
static void validate(const Tree& T, const Plan& P) {
  auto fail = [](const char* what) { throw std::logic_error(what); };
  const int64_t nb = (int64_t)T.bk.size(), nt = (int64_t)P.tasks.size();
  for (int64_t k = 0; k < nt; ++k) {
    const Task& t = P.tasks[k];
    for (int32_t q = 0; q < t.ndeps; ++q) {
      const int32_t d = P.deps[t.dep_begin + q];
      if (d < 0 || d >= k) fail("dependency not earlier in ticket order");
    }
    if (t.kind == TASK_TERM || t.kind == TASK_TERM_ROWS) {
      if (t.obj < 0 || t.obj >= (int32_t)P.terms.size()) fail("term id");
      if (t.kind == TASK_TERM_ROWS) {
        const TermDef& d = P.terms[t.obj];
        const int32_t hrow = (d.kind == TK_LRA) ? T.bk[d.B].row : T.bk[d.A].row;
        const Cluster& H = T.cl[hrow];
        if (t.a1 < 0 || t.a1 >= (int32_t)T.cl.size()) fail("term chunk cluster");
        const Cluster& q = T.cl[t.a1];
        if (d.kind == TK_DD || q.begin < H.begin || q.end > H.end) fail("term chunk rows");
      }
      continue;
    }
    if (t.kind == TASK_SOLVE_SEQ || t.kind == TASK_SOLVE_MV) {
      check_solve_task(T, t, fail);
      continue;
    }
    if (t.obj < 0 || t.obj >= nb) fail("task block id");
    const Block& b = T.bk[t.obj];
    if (t.kind == TASK_TS_A || t.kind == TASK_TS_B || t.kind == TASK_TS_C) {
      if (b.kind != BK_LR || !ts_big(b.m, b.n) || P.lr_cap[t.obj] != 2 * K_MAX ||
          P.stage_off[t.obj] < 0)
        fail("big low-rank step block");
      if (t.a0 < 1 || t.a0 > t.ninst + 1) fail("big low-rank step index");
      if (t.kind != TASK_TS_B && (t.a1 < 0 || t.a1 >= ts_blocks(b.m) + ts_blocks(b.n))) fail("row block");
      if (ts_rows(b.m) < 2 * K_MAX || ts_rows(b.n) < 2 * K_MAX) fail("row block height");
    } else if (t.kind == TASK_LR) {
      if (b.kind != BK_LR || t.diag != b.col) fail("low-rank task");
    } else {
      if (b.kind != BK_DENSE || b.m > LEAF_MAX || b.n > LEAF_MAX) fail("dense task");
      if (t.diag < 0 || t.diag >= nb || T.bk[t.diag].kind != BK_DENSE || T.bk[t.diag].m != b.n) fail("diag leaf");
    }
    for (int32_t q = 0; q < t.ninst; ++q) {
      const TermInst& in = P.insts[t.inst_begin + q];
      const TermDef& d = P.terms[in.term];
      if (in.lr0 < 0 || in.lc0 < 0 || in.lr0 + in.mx > b.m || in.lc0 + in.ny > b.n) fail("instance region");
      const Block& A = T.bk[d.A];
      const Block& B = T.bk[d.B];
      const int64_t xrows = (d.kind == TK_LRB) ? d.rows : A.m;
      const int64_t yrows = (d.kind == TK_LRA) ? d.rows : B.m;
      if (in.xr0 < 0 || in.xr0 + in.mx > xrows || in.yr0 < 0 || in.yr0 + in.ny > yrows) fail("instance rows");
      if (d.kind == TK_DD && (A.kind != BK_DENSE || B.kind != BK_DENSE || A.n != B.n)) fail("dd term");
      if (d.kind == TK_LRA && A.kind != BK_LR) fail("lrA term");
      if (d.kind == TK_LRB && B.kind != BK_LR) fail("lrB term");
    }
  }
  for (int64_t b = 0; b < nb; ++b) {
    if (P.sub_begin[b] < 0 || P.sub_end[b] < P.sub_begin[b] || P.sub_end[b] > (int32_t)P.sub_leaves.size())
      fail("subtree leaf range");
    for (int32_t q = P.sub_begin[b]; q < P.sub_end[b]; ++q) {
      const Block& l = T.bk[P.sub_leaves[q]];
      const Block& bb = T.bk[b];
      if (l.r0 < bb.r0 || l.r0 + l.m > bb.r0 + bb.m || l.c0 < bb.c0 || l.c0 + l.n > bb.c0 + bb.n)
        fail("subtree leaf outside its block");
    }
  }
  for (const TermDef& d : P.terms)
    if (d.kind != TK_DD && (d.buf < 0 || d.buf + d.rows * K_MAX > P.term_pool)) fail("term buffer");
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<Task>& ts = pass ? P.btasks : P.stasks;
    const std::vector<int32_t>& tdp = pass ? P.bdeps : P.sdeps;
    const std::vector<int32_t>& lb = pass ? P.blevel_begin : P.slevel_begin;
    const int64_t ns = (int64_t)ts.size();
    if (lb.empty() || lb.back() != ns) fail("solve levels");
    for (int64_t k = 0; k < ns; ++k) {
      const Task& t = ts[k];
      const int8_t seq = pass ? TASK_SOLVE_SEQ_T : TASK_SOLVE_SEQ, mv = pass ? TASK_SOLVE_MV_T : TASK_SOLVE_MV;
      if (t.obj != -1 || (t.kind != seq && t.kind != mv)) fail("solve task kind");
      Task u = t;
      u.kind = (t.kind == seq) ? TASK_SOLVE_SEQ : TASK_SOLVE_MV;
      if (pass && u.kind == TASK_SOLVE_MV) {
        // the transposed product writes rows of the block's columns
        const Block& b = T.bk[t.a0];
        const Cluster& q = T.cl[t.a1];
        if (q.begin < b.c0 || q.end > b.c0 + b.n || b.r0 + b.m > T.n) fail("backward product chunk");
      } else {
        check_solve_task(T, u, fail);
      }
      for (int32_t q = 0; q < t.ndeps; ++q) {
        const int32_t d = tdp[t.dep_begin + q];
        if (d < 0 || d >= k || ts[d].level >= t.level) fail("solve dependency");
      }
    }
  }
  // the data solve beside the factorisation: solve tasks on the data, each
  // dependency a factor task or an earlier task of this list
  for (size_t k = 0; k < P.ftasks.size(); ++k) {
    const Task& t = P.ftasks[k];
    if (t.obj != -1 || (t.kind != TASK_SOLVE_SEQ && t.kind != TASK_SOLVE_MV)) fail("fused solve task kind");
    check_solve_task(T, t, fail);
    if (t.dep_begin < 0 || t.ndeps < 0 || (size_t)t.dep_begin + t.ndeps > P.fdeps.size()) fail("fused solve deps");
    for (int32_t q = 0; q < t.ndeps; ++q) {
      const int32_t d = P.fdeps[t.dep_begin + q];
      if (d < 0 || d >= nt + (int64_t)k) fail("fused solve dependency");
    }
  }
  int64_t covered = 0;
  for (int32_t q : P.apply_chunks) {
    if (q < 0 || q >= (int32_t)T.cl.size() || T.cl[q].begin != covered) fail("operator chunks");
    covered = T.cl[q].end;
  }
  if (covered != T.n) fail("operator chunks cover");
  for (size_t c = 0; c + 1 < P.sop_begin.size(); ++c) {
    const int64_t len = T.cl[c].end - T.cl[c].begin;
    for (int32_t o = P.sop_begin[c]; o < P.sop_begin[c + 1]; ++o) {
      const SolveOp& op = P.sops[o];
      const Block& b = T.bk[op.blk];
      if (op.off < 0 || op.off + b.m > len) fail("solve op rows");
      if (op.kind == SOP_MATVEC && (op.off2 < 0 || op.off2 + b.n > len)) fail("solve op cols");
      if (op.kind == SOP_TRSV && (b.kind != BK_DENSE || b.m != b.n)) fail("solve op diag");
    }
  }
}

void build_plan(const Tree& t, Plan& p) {
  p = Plan{};
  Planner pl(t, p);
  pl.run();
  validate(t, p);
}

}  // namespace hm

namespace hm {

// Greedy level building.  tail(t) is the longest chain of measured durations
// from t to the end of the factorisation (t included).  Each level starts from
// the ready task of longest tail, t*, and takes delta = its duration; every
// ready task whose tail exceeds tail(t*) - delta must run now (deferring it by
// one level would lengthen the schedule), and delta grows to the longest of
// those; every other ready task of duration at most delta runs now as well,
// for free.  Longer, non-critical tasks wait for a level of their own length.
void schedule_by_durations(const Plan& p, const std::vector<double>& dur, std::vector<int32_t>& order,
                           std::vector<int32_t>& level_begin) {
  const int32_t nt = (int32_t)p.tasks.size();
  if ((int32_t)dur.size() != nt) throw std::logic_error("one duration per task");
  std::vector<int32_t> sbeg(nt + 1, 0), succ(p.deps.size());
  for (int32_t t = 0; t < nt; ++t)
    for (int32_t q = 0; q < p.tasks[t].ndeps; ++q) ++sbeg[p.deps[p.tasks[t].dep_begin + q] + 1];
  for (int32_t t = 0; t < nt; ++t) sbeg[t + 1] += sbeg[t];
  {
    std::vector<int32_t> fill(sbeg.begin(), sbeg.end() - 1);
    for (int32_t t = 0; t < nt; ++t)
      for (int32_t q = 0; q < p.tasks[t].ndeps; ++q) succ[fill[p.deps[p.tasks[t].dep_begin + q]]++] = t;
  }
  // dependencies precede their tasks in plan order, so one backward sweep
  std::vector<double> tail(nt, 0.0);
  for (int32_t t = nt - 1; t >= 0; --t) {
    double m = 0.0;
    for (int32_t q = sbeg[t]; q < sbeg[t + 1]; ++q) m = std::max(m, tail[succ[q]]);
    tail[t] = m + std::max(0.0, dur[t]);
  }
  std::vector<int32_t> need(nt);
  std::set<std::pair<double, int32_t>> by_dur, by_tail;
  for (int32_t t = 0; t < nt; ++t) {
    need[t] = p.tasks[t].ndeps;
    if (!need[t]) {
      by_dur.insert({dur[t], t});
      by_tail.insert({tail[t], t});
    }
  }
  order.clear();
  order.reserve(nt);
  level_begin.assign(1, 0);
  std::vector<int32_t> cur;
  while ((int32_t)order.size() < nt) {
    if (by_tail.empty()) throw std::logic_error("schedule: no ready task (dependency cycle)");
    cur.clear();
    const double tmax = by_tail.rbegin()->first;
    double delta = dur[by_tail.rbegin()->second];
    for (bool grew = true; grew;) {
      grew = false;
      for (auto it = by_tail.rbegin(); it != by_tail.rend() && it->first > tmax - delta; ++it)
        if (dur[it->second] > delta) {
          delta = dur[it->second];
          grew = true;
        }
    }
    for (auto it = by_tail.rbegin(); it != by_tail.rend() && it->first > tmax - delta; ++it) cur.push_back(it->second);
    for (auto it = by_dur.begin(); it != by_dur.end() && it->first <= delta; ++it) cur.push_back(it->second);
    std::sort(cur.begin(), cur.end());
    cur.erase(std::unique(cur.begin(), cur.end()), cur.end());
    for (int32_t t : cur) {
      by_dur.erase({dur[t], t});
      by_tail.erase({tail[t], t});
    }
    // longer tasks first: the level's work-groups take them round-robin
    std::stable_sort(cur.begin(), cur.end(), [&](int32_t a, int32_t b) { return dur[a] > dur[b]; });
    for (int32_t t : cur) order.push_back(t);
    level_begin.push_back((int32_t)order.size());
    for (int32_t t : cur)
      for (int32_t q = sbeg[t]; q < sbeg[t + 1]; ++q) {
        const int32_t s2 = succ[q];
        if (--need[s2] == 0) {
          by_dur.insert({dur[s2], s2});
          by_tail.insert({tail[s2], s2});
        }
      }
  }
}

}  // namespace hm

namespace hm {

// The stream program is built by simulating the execution with the measured
// durations: a stream of levels (0 and 1) forms its next level, whenever it is
// free, from the ready tasks of its class by the rule of schedule_by_durations
// (a level lasts as long as its longest task, or its total work over 256 CUs if
// that is more); a wave stream takes, whenever it is free, every ready task of
// its class.  A task counts as finished when its launch ends (the event
// granularity).  Launches are then issued in order of simulated start.
void build_stream_program(const Tree& t, const Plan& p, const std::vector<double>& dur, double ovh,
                          bool fused, int nstreams, StreamProgram& out) {
  if (nstreams != 4 && nstreams != 6 && nstreams != 8) throw std::logic_error("stream program: 4, 6 or 8 streams");
  const int32_t nfac = (int32_t)p.tasks.size();
  const int32_t nt = nfac + (fused ? (int32_t)p.ftasks.size() : 0);
  if ((int32_t)dur.size() != nt) throw std::logic_error("one duration per task");
  auto task = [&](int32_t i) -> const Task& { return i < nfac ? p.tasks[i] : p.ftasks[i - nfac]; };
  auto dep = [&](int32_t i, int32_t q) { return i < nfac ? p.deps[p.tasks[i].dep_begin + q]
                                                       : p.fdeps[p.ftasks[i - nfac].dep_begin + q]; };
  std::vector<int8_t> cls(nt, 0);
  for (int32_t i = 0; i < nfac; ++i) {
    const Task& tk = p.tasks[i];
    if (tk.kind == TASK_TS_A || tk.kind == TASK_TS_B || tk.kind == TASK_TS_C) {
      cls[i] = 1;
    } else if (tk.kind == TASK_LR) {
      const Block& b = t.bk[tk.obj];
      if (std::max(b.m, b.n) > MS_LONG_ROWS) cls[i] = 2;
    }
  }
  std::vector<int32_t> sbeg(nt + 1, 0);
  for (int32_t i = 0; i < nt; ++i)
    for (int32_t q = 0; q < task(i).ndeps; ++q) ++sbeg[dep(i, q) + 1];
  for (int32_t i = 0; i < nt; ++i) sbeg[i + 1] += sbeg[i];
  std::vector<int32_t> succ(sbeg[nt]);
  {
    std::vector<int32_t> fill(sbeg.begin(), sbeg.end() - 1);
    for (int32_t i = 0; i < nt; ++i)
      for (int32_t q = 0; q < task(i).ndeps; ++q) succ[fill[dep(i, q)]++] = i;
  }
  std::vector<double> d(nt), tail(nt, 0.0);
  for (int32_t i = 0; i < nt; ++i) d[i] = std::max(0.0, dur[i]);
  for (int32_t i = nt - 1; i >= 0; --i) {
    double m = 0.0;
    for (int32_t q = sbeg[i]; q < sbeg[i + 1]; ++q) m = std::max(m, tail[succ[q]]);
    tail[i] = m + d[i];
  }
  struct Sim {
    int8_t stream;
    double start, end;
    std::vector<int32_t> tasks;
  };
  std::vector<Sim> sims;
  std::vector<int32_t> need(nt), launch_of(nt, -1);
  std::set<std::pair<double, int32_t>> by_dur[2], by_tail[2];
  std::vector<int32_t> waveq;
  auto ready = [&](int32_t i) {
    if (cls[i] == 2) {
      waveq.push_back(i);
    } else {
      by_dur[cls[i]].insert({d[i], i});
      by_tail[cls[i]].insert({tail[i], i});
    }
  };
  for (int32_t i = 0; i < nt; ++i) {
    need[i] = task(i).ndeps;
    if (!need[i]) ready(i);
  }
  using Ev = std::pair<double, int32_t>;   // (end time, launch id)
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> ends;
  double free_at[MS_STREAMS] = {};
  double now = 0.0;
  int32_t done = 0;
  while (done < nt) {
    while (!ends.empty() && ends.top().first <= now) {
      const int32_t L = ends.top().second;
      ends.pop();
      for (int32_t i : sims[L].tasks) {
        ++done;
        for (int32_t q = sbeg[i]; q < sbeg[i + 1]; ++q)
          if (--need[succ[q]] == 0) ready(succ[q]);
      }
    }
    if (done == nt) break;
    for (int sa = 0; sa < nstreams; ++sa) {
      const int a = MS_STREAM_CLASS[sa];
      if (a > 1 || free_at[sa] > now || by_tail[a].empty()) continue;
      const double tmax = by_tail[a].rbegin()->first;
      double delta = d[by_tail[a].rbegin()->second];
      for (bool grew = true; grew;) {
        grew = false;
        for (auto it = by_tail[a].rbegin(); it != by_tail[a].rend() && it->first > tmax - delta; ++it)
          if (d[it->second] > delta) {
            delta = d[it->second];
            grew = true;
          }
      }
      Sim L{(int8_t)sa, now, 0.0, {}};
      for (auto it = by_tail[a].rbegin(); it != by_tail[a].rend() && it->first > tmax - delta; ++it)
        L.tasks.push_back(it->second);
      for (auto it = by_dur[a].begin(); it != by_dur[a].end() && it->first <= delta; ++it) L.tasks.push_back(it->second);
      std::sort(L.tasks.begin(), L.tasks.end());
      L.tasks.erase(std::unique(L.tasks.begin(), L.tasks.end()), L.tasks.end());
      double work = 0.0;
      for (int32_t i : L.tasks) {
        by_dur[a].erase({d[i], i});
        by_tail[a].erase({tail[i], i});
        work += d[i];
      }
      L.end = now + std::max(delta, work / 256.0) + ovh;
      free_at[sa] = L.end;
      ends.push({L.end, (int32_t)sims.size()});
      sims.push_back(std::move(L));
    }
    for (int s = 0; s < nstreams && !waveq.empty(); ++s) {
      if (MS_STREAM_CLASS[s] != 2 || free_at[s] > now) continue;
      Sim L{(int8_t)s, now, 0.0, {}};
      double mx = 0.0, work = 0.0;
      for (int32_t i : waveq) {
        mx = std::max(mx, d[i]);
        work += d[i];
      }
      L.tasks.swap(waveq);
      waveq.clear();
      L.end = now + std::max(mx, work / 64.0) + ovh;
      free_at[s] = L.end;
      ends.push({L.end, (int32_t)sims.size()});
      sims.push_back(std::move(L));
    }
    if (ends.empty()) throw std::logic_error("stream program: no task can start (dependency cycle)");
    now = std::max(now, ends.top().first);
  }
  // issue order: by simulated start (ties: creation order)
  std::vector<int32_t> ord(sims.size());
  for (size_t i = 0; i < sims.size(); ++i) ord[i] = (int32_t)i;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return sims[a].start < sims[b].start; });
  std::vector<int32_t> pos_of(sims.size());
  for (size_t k = 0; k < ord.size(); ++k) pos_of[ord[k]] = (int32_t)k;
  for (size_t L = 0; L < sims.size(); ++L)
    for (int32_t i : sims[L].tasks) launch_of[i] = pos_of[L];
  out = StreamProgram{};
  out.nstreams = nstreams;
  out.order.reserve(nt);
  out.launches.resize(ord.size());
  std::vector<int32_t> rec_of(ord.size(), -1);
  // last launch (issue position) of stream s2 that stream s already waits for
  int32_t waited[MS_STREAMS][MS_STREAMS];
  for (auto& row : waited)
    for (int32_t& v : row) v = -1;
  for (size_t k = 0; k < ord.size(); ++k) {
    Sim& L = sims[ord[k]];
    MSLaunch& M = out.launches[k];
    M.stream = L.stream;
    M.rec = -1;
    // longer tasks first (round-robin over the launch's work-groups)
    std::stable_sort(L.tasks.begin(), L.tasks.end(), [&](int32_t a, int32_t b) { return d[a] > d[b]; });
    M.t0 = (int32_t)out.order.size();
    for (int32_t i : L.tasks) out.order.push_back(i);
    M.t1 = (int32_t)out.order.size();
    // per other stream, the latest launch this one depends on
    int32_t need_from[MS_STREAMS];
    for (int32_t& v : need_from) v = -1;
    for (int32_t i : L.tasks)
      for (int32_t q = 0; q < task(i).ndeps; ++q) {
        const int32_t u = dep(i, q);
        const int32_t lu = launch_of[u];
        const int su = out.launches[lu].stream;
        if (lu >= (int32_t)k) throw std::logic_error("stream program: dependency issued later");
        if (su != M.stream) need_from[su] = std::max(need_from[su], lu);
      }
    M.wait_begin = (int32_t)out.waits.size();
    M.nwait = 0;
    for (int s2 = 0; s2 < MS_STREAMS; ++s2) {
      const int32_t lu = need_from[s2];
      if (lu < 0 || lu <= waited[M.stream][s2]) continue;
      if (rec_of[lu] < 0) {
        rec_of[lu] = out.nevents++;
        out.launches[lu].rec = rec_of[lu];
      }
      out.waits.push_back(rec_of[lu]);
      ++M.nwait;
      waited[M.stream][s2] = lu;
    }
  }
  double end = 0.0;
  for (const Sim& L : sims) end = std::max(end, L.end);
  out.modelled_seconds = end;
  validate_stream_program(p, out, fused);
}

void validate_stream_program(const Plan& p, const StreamProgram& g, bool fused) {
  auto fail = [](const char* what) { throw std::logic_error(what); };
  const int32_t nfac = (int32_t)p.tasks.size();
  const int32_t nt = nfac + (fused ? (int32_t)p.ftasks.size() : 0);
  auto task = [&](int32_t i) -> const Task& { return i < nfac ? p.tasks[i] : p.ftasks[i - nfac]; };
  auto dep = [&](int32_t i, int32_t q) { return i < nfac ? p.deps[p.tasks[i].dep_begin + q]
                                                       : p.fdeps[p.ftasks[i - nfac].dep_begin + q]; };
  if ((int32_t)g.order.size() != nt) fail("stream program: order is not a permutation");
  if (g.nstreams < 1 || g.nstreams > MS_STREAMS) fail("stream program: stream count");
  std::vector<int32_t> launch_of(nt, -1);
  for (size_t k = 0; k < g.launches.size(); ++k) {
    const MSLaunch& M = g.launches[k];
    if (M.stream < 0 || M.stream >= g.nstreams || M.t0 < 0 || M.t1 < M.t0 || M.t1 > nt) fail("stream program: launch");
    if (M.wait_begin < 0 || M.nwait < 0 || M.wait_begin + M.nwait > (int32_t)g.waits.size())
      fail("stream program: wait range");
    if (M.rec < -1 || M.rec >= g.nevents) fail("stream program: event");
    for (int32_t q = M.t0; q < M.t1; ++q) {
      const int32_t i = g.order[q];
      if (i < 0 || i >= nt || launch_of[i] >= 0) fail("stream program: order is not a permutation");
      launch_of[i] = (int32_t)k;
    }
  }
  // event e -> launch that records it (each event recorded once)
  std::vector<int32_t> rec_launch(g.nevents, -1);
  for (size_t k = 0; k < g.launches.size(); ++k)
    if (g.launches[k].rec >= 0) {
      if (rec_launch[g.launches[k].rec] >= 0) fail("stream program: event recorded twice");
      rec_launch[g.launches[k].rec] = (int32_t)k;
    }
  // covered[s][s2]: latest launch of stream s2 whose completion stream s has
  // waited for, so far in issue order (waits carry over to later launches of s)
  std::vector<int32_t> covered(MS_STREAMS * MS_STREAMS, -1);
  for (size_t k = 0; k < g.launches.size(); ++k) {
    const MSLaunch& M = g.launches[k];
    for (int32_t w = 0; w < M.nwait; ++w) {
      const int32_t e = g.waits[M.wait_begin + w];
      const int32_t lr = rec_launch[e];
      if (lr < 0 || lr >= (int32_t)k) fail("stream program: wait on an event not yet recorded");
      const int s2 = g.launches[lr].stream;
      int32_t& c = covered[M.stream * MS_STREAMS + s2];
      c = std::max(c, lr);
    }
    for (int32_t q = M.t0; q < M.t1; ++q) {
      const int32_t i = g.order[q];
      for (int32_t r = 0; r < task(i).ndeps; ++r) {
        const int32_t u = dep(i, r);
        const int32_t lu = launch_of[u];
        if (lu >= (int32_t)k) fail("stream program: dependency not in an earlier launch");
        const int su = g.launches[lu].stream;
        // same stream: in order; other stream: an awaited launch of that stream
        // at or after the dependency's launch (launches of one stream complete in order)
        if (su != M.stream && covered[M.stream * MS_STREAMS + su] < lu)
          fail("stream program: cross-stream dependency without a wait");
      }
    }
  }
}

}  // namespace hm
