"""CPU check of the factorisation task graph's data hazards on the term
buffers (hm_plan.cpp): a term's product factor is written by its TERM /
TERM_ROWS tasks and read by the leaf tasks that take its restricted
instances (DIAG / OFFD / LR, and the step tasks TS_* of a big block's step
for that term); buffers are shared by later terms of the same height.  For
the task graph of real point sets:

  * read after write: every reader has every writer of the term among its
    ancestors;
  * write after read: when a buffer passes from one term to the next, every
    reader of the first is an ancestor of every writer of the second;
  * distinct buffers do not overlap, and sharing happens (the check is not
    vacuous);
  * a control: with the sharing dependencies ignored the same check finds
    write-after-read hazards;
  * read after write on the factor's blocks: every block a task reads (the
    factors of its update terms, the diagonal leaf of a triangular solve, the
    L blocks of a solve program, the blocks of a term product) is finished by
    its last writer among the task's ancestors; a control without the term
    products' dependencies finds reads that would race;
  * the data's forward solve: any two of its tasks whose rows of W conflict
    (one writes rows the other reads or writes) are ordered by dependencies.
Compiled into a small host harness (g++)."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1709_04419_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_04419_amd", "csrc")

HARNESS = r"""
#include "hm_plan.h"
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <vector>
using namespace hm;

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  const long n = atol(argv[2]);
  const int leaf = atoi(argv[3]);
  std::vector<double> P(2 * n);
  if (fread(P.data(), 8, 2 * n, f) != (size_t)(2 * n)) return 1;
  fclose(f);
  Tree t; build_tree(P.data(), n, leaf, 2.0, t);
  Plan p; build_plan(t, p);
  const int32_t nt = (int32_t)p.tasks.size(), nterm = (int32_t)p.terms.size();
  // writers and readers of every term
  std::vector<std::vector<int32_t>> wr(nterm), rd(nterm);
  for (int32_t i = 0; i < nt; ++i) {
    const Task& k = p.tasks[i];
    if (k.kind == TASK_TERM || k.kind == TASK_TERM_ROWS) {
      wr[k.obj].push_back(i);
    } else if (k.kind == TASK_DIAG || k.kind == TASK_OFFD || k.kind == TASK_LR) {
      for (int32_t q = 0; q < k.ninst; ++q) rd[p.insts[k.inst_begin + q].term].push_back(i);
    } else if (k.kind == TASK_TS_A || k.kind == TASK_TS_B || k.kind == TASK_TS_C) {
      if (k.a0 >= 1 && k.a0 <= k.ninst) rd[p.insts[k.inst_begin + k.a0 - 1].term].push_back(i);
    }
  }
  // ancestors as bitsets, in ticket order (every dependency has a lower id);
  // with `sharing` false the dependencies that buffer reuse added are left out:
  // a reader of a buffer's previous term is then no longer an ancestor of the
  // next term's writers
  auto hazards = [&](bool sharing, long& raw, long& war, long& pairs) {
    std::vector<int32_t> prev_of(nterm, -1);
    std::map<int64_t, std::vector<int32_t>> by_off;
    for (int32_t k = 0; k < nterm; ++k)
      if (p.terms[k].rows > 0 && !wr[k].empty()) by_off[p.terms[k].buf].push_back(k);
    for (auto& e : by_off) {
      auto& v = e.second;
      std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
        return *std::min_element(wr[a].begin(), wr[a].end()) < *std::min_element(wr[b].begin(), wr[b].end());
      });
      for (size_t q = 1; q < v.size(); ++q) prev_of[v[q]] = v[q - 1];
    }
    // the sharing edges: writer of a term <- readers of the buffer's previous term
    std::vector<std::vector<int32_t>> skip(nt);
    if (!sharing)
      for (int32_t k = 0; k < nterm; ++k)
        if (prev_of[k] >= 0)
          for (int32_t w : wr[k]) skip[w] = rd[prev_of[k]];
    const size_t words = ((size_t)nt + 63) / 64;
    std::vector<uint64_t> anc((size_t)nt * words, 0);
    for (int32_t i = 0; i < nt; ++i) {
      uint64_t* ai = &anc[(size_t)i * words];
      const Task& k = p.tasks[i];
      for (int32_t q = 0; q < k.ndeps; ++q) {
        const int32_t d = p.deps[k.dep_begin + q];
        if (!sharing && std::find(skip[i].begin(), skip[i].end(), d) != skip[i].end()) continue;
        const uint64_t* ad = &anc[(size_t)d * words];
        for (size_t w = 0; w < words; ++w) ai[w] |= ad[w];
        ai[d / 64] |= 1ull << (d % 64);
      }
    }
    auto is_anc = [&](int32_t a, int32_t of) { return (anc[(size_t)of * words + a / 64] >> (a % 64)) & 1; };
    raw = war = pairs = 0;
    for (int32_t k = 0; k < nterm; ++k) {
      if (p.terms[k].rows <= 0) continue;
      for (int32_t c : rd[k])
        for (int32_t w : wr[k]) raw += !is_anc(w, c);
      if (prev_of[k] < 0) continue;
      ++pairs;
      for (int32_t c : rd[prev_of[k]])
        for (int32_t w : wr[k]) war += !is_anc(c, w);
    }
  };
  long raw, war, pairs, raw0, war0, pairs0;
  hazards(true, raw, war, pairs);
  hazards(false, raw0, war0, pairs0);
  // distinct buffers: disjoint ranges [buf, buf + rows * K_MAX)
  std::map<int64_t, int64_t> ext;
  for (const TermDef& d : p.terms)
    if (d.rows > 0) ext[d.buf] = std::max(ext[d.buf], d.rows * (int64_t)K_MAX);
  long overlaps = 0;
  int64_t end = -1;
  for (auto& e : ext) {
    overlaps += e.first < end;
    end = std::max(end, e.first + e.second);
  }
  long terms_with_buf = 0;
  for (const TermDef& d : p.terms) terms_with_buf += d.rows > 0;
  // read after write on the factor's blocks: every block a task reads is
  // finished (its last writer ran) before the task starts
  const int32_t nb = (int32_t)t.bk.size();
  std::vector<int32_t> last(nb, -1);
  auto writes_block = [](int8_t kind) {
    return kind == TASK_DIAG || kind == TASK_OFFD || kind == TASK_LR || kind == TASK_TS_A || kind == TASK_TS_B ||
           kind == TASK_TS_C || kind == TASK_SOLVE_SEQ || kind == TASK_SOLVE_MV;
  };
  for (int32_t i = 0; i < nt; ++i)
    if (writes_block(p.tasks[i].kind) && p.tasks[i].obj >= 0) last[p.tasks[i].obj] = i;
  auto leaves_rows = [&](int32_t b, int64_t lo, int64_t hi, std::vector<int32_t>& out) {
    for (int32_t q = p.sub_begin[b]; q < p.sub_end[b]; ++q) {
      const Block& l = t.bk[p.sub_leaves[q]];
      if (l.r0 < hi && l.r0 + l.m > lo) out.push_back(p.sub_leaves[q]);
    }
  };
  auto inst_reads = [&](const TermInst& in, std::vector<int32_t>& out) {
    const TermDef& d = p.terms[in.term];
    if (d.kind == TK_LRA) out.push_back(d.A);
    else if (d.kind == TK_LRB) out.push_back(d.B);
    else { out.push_back(d.A); out.push_back(d.B); }
  };
  auto reads_of = [&](int32_t i, std::vector<int32_t>& out) {
    out.clear();
    const Task& k = p.tasks[i];
    switch (k.kind) {
      case TASK_TERM: case TASK_TERM_ROWS: {
        const TermDef& d = p.terms[k.obj];
        const int32_t lrb = d.kind == TK_LRA ? d.A : d.B, hb = d.kind == TK_LRA ? d.B : d.A;
        int64_t lo = 0, hi = t.n;
        if (k.kind == TASK_TERM_ROWS) { lo = t.cl[k.a1].begin; hi = t.cl[k.a1].end; }
        out.push_back(lrb);
        leaves_rows(hb, lo, hi, out);
        break;
      }
      case TASK_DIAG: case TASK_OFFD: case TASK_LR:
        for (int32_t q = 0; q < k.ninst; ++q) inst_reads(p.insts[k.inst_begin + q], out);
        if (k.kind == TASK_OFFD) out.push_back(k.diag);
        if (k.kind == TASK_LR && k.a0 == 1) leaves_rows(t.diag_of[k.diag], 0, t.n, out);
        break;
      case TASK_TS_A: case TASK_TS_B: case TASK_TS_C:
        if (k.a0 >= 1 && k.a0 <= k.ninst) inst_reads(p.insts[k.inst_begin + k.a0 - 1], out);
        break;
      case TASK_SOLVE_SEQ:
        for (int32_t q = p.sop_begin[k.a0]; q < p.sop_begin[k.a0 + 1]; ++q) leaves_rows(p.sops[q].blk, 0, t.n, out);
        break;
      case TASK_SOLVE_MV:
        leaves_rows(k.a0, t.cl[k.a1].begin, t.cl[k.a1].end, out);
        break;
      default: break;
    }
  };
  // ancestors again, optionally without the dependencies of the term products
  // (the control: their reads of the factor blocks are then unordered)
  auto block_raw = [&](bool term_deps, long& viol, long& checked) {
    const size_t words = ((size_t)nt + 63) / 64;
    std::vector<uint64_t> anc((size_t)nt * words, 0);
    for (int32_t i = 0; i < nt; ++i) {
      const Task& k = p.tasks[i];
      if (!term_deps && (k.kind == TASK_TERM || k.kind == TASK_TERM_ROWS)) continue;
      uint64_t* ai = &anc[(size_t)i * words];
      for (int32_t q = 0; q < k.ndeps; ++q) {
        const int32_t d = p.deps[k.dep_begin + q];
        const uint64_t* ad = &anc[(size_t)d * words];
        for (size_t w = 0; w < words; ++w) ai[w] |= ad[w];
        ai[d / 64] |= 1ull << (d % 64);
      }
    }
    viol = checked = 0;
    std::vector<int32_t> rb;
    for (int32_t i = 0; i < nt; ++i) {
      reads_of(i, rb);
      for (int32_t b : rb) {
        if (b == p.tasks[i].obj || last[b] < 0) continue;
        ++checked;
        viol += !((anc[(size_t)i * words + last[b] / 64] >> (last[b] % 64)) & 1);
      }
    }
  };
  // the data solve (tasks on the rows of W): two tasks whose row ranges
  // conflict (one writes what the other reads or writes) are ordered
  const int32_t nf = (int32_t)p.ftasks.size();
  std::vector<std::vector<uint64_t>> fanc(nf, std::vector<uint64_t>(((size_t)nf + 63) / 64, 0));
  for (int32_t i = 0; i < nf; ++i) {
    const Task& k = p.ftasks[i];
    for (int32_t q = 0; q < k.ndeps; ++q) {
      const int32_t d = p.fdeps[k.dep_begin + q] - nt;   // factor tasks: negative, skipped
      if (d < 0) continue;
      for (size_t w = 0; w < fanc[i].size(); ++w) fanc[i][w] |= fanc[d][w];
      fanc[i][d / 64] |= 1ull << (d % 64);
    }
  }
  auto wrange = [&](const Task& k, int64_t& w0, int64_t& w1, int64_t& r0, int64_t& r1) {
    if (k.kind == TASK_SOLVE_SEQ) {
      w0 = r0 = t.cl[k.a0].begin;
      w1 = r1 = t.cl[k.a0].end;
    } else {
      w0 = t.cl[k.a1].begin;
      w1 = t.cl[k.a1].end;
      r0 = t.bk[k.a0].c0;
      r1 = r0 + t.bk[k.a0].n;
    }
  };
  long w_conflicts = 0, w_unordered = 0;
  for (int32_t i = 0; i < nf; ++i)
    for (int32_t j = i + 1; j < nf; ++j) {
      int64_t wi0, wi1, ri0, ri1, wj0, wj1, rj0, rj1;
      wrange(p.ftasks[i], wi0, wi1, ri0, ri1);
      wrange(p.ftasks[j], wj0, wj1, rj0, rj1);
      auto meet = [](int64_t a0, int64_t a1, int64_t b0, int64_t b1) { return a0 < b1 && b0 < a1; };
      if (!(meet(wi0, wi1, wj0, wj1) || meet(wi0, wi1, rj0, rj1) || meet(wj0, wj1, ri0, ri1))) continue;
      ++w_conflicts;
      const bool ordered = ((fanc[j][i / 64] >> (i % 64)) & 1) || ((fanc[i][j / 64] >> (j % 64)) & 1);
      w_unordered += !ordered;
    }
  printf("{\"solve_conflicts\": %ld, \"solve_unordered\": %ld}\n", w_conflicts, w_unordered);
  long braw, bchecked, braw0, bchecked0;
  block_raw(true, braw, bchecked);
  block_raw(false, braw0, bchecked0);
  printf("{\"block_reads_checked\": %ld, \"block_raw\": %ld, \"block_raw_without_term_deps\": %ld}\n", bchecked,
         braw, braw0);
  printf("{\"tasks\": %d, \"terms_with_buffer\": %ld, \"buffers\": %zu, \"shared_pairs\": %ld, \"raw\": %ld, "
         "\"war\": %ld, \"overlaps\": %ld, \"war_without_sharing_deps\": %ld, \"pool_end\": %lld, "
         "\"term_pool\": %lld}\n", nt, terms_with_buf, ext.size(), pairs, raw, war, overlaps, war0,
         (long long)end, (long long)p.term_pool);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("hazards")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), os.path.join(CSRC, "hm_plan.cpp"),
                    "-o", str(exe)], check=True, timeout=600)
    return d, exe


@pytest.mark.parametrize("n,leaf", [(3000, 32), (12000, 64)])
def test_term_buffer_hazards(harness, n, leaf):
    d, exe = harness
    pts = d / f"p{n}.bin"
    wl.basin_clusters(n, 41).astype(np.float64).tofile(pts)
    out = subprocess.run([str(exe), str(pts), str(n), str(leaf)], capture_output=True, text=True, timeout=600,
                         check=True)
    lines = out.stdout.strip().splitlines()
    solve = json.loads(lines[-3])
    # the data solve's tasks that touch the same rows of W are ordered
    assert solve["solve_conflicts"] > 0 and solve["solve_unordered"] == 0
    blocks = json.loads(lines[-2])
    r = json.loads(lines[-1])
    # every block read follows the block's last writer; the control (term
    # products without their dependencies) finds reads that would not
    assert blocks["block_reads_checked"] > 0 and blocks["block_raw"] == 0
    assert blocks["block_raw_without_term_deps"] > 0
    assert r["raw"] == 0 and r["war"] == 0 and r["overlaps"] == 0
    assert r["shared_pairs"] > 0 and r["buffers"] < r["terms_with_buffer"]
    assert r["war_without_sharing_deps"] > 0
    assert r["pool_end"] <= r["term_pool"]
