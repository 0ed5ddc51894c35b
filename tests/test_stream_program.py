"""CPU checks of the multi-stream factorisation schedule (hm_plan.cpp:
build_stream_program / validate_stream_program), compiled into a small host
harness: for the task graph of a real point set and seeded random durations,
the program covers every task once, every dependency is met by an earlier
launch of the same stream or by a wait on an event recorded after it, and the
validator rejects programs with a wait removed or two launches swapped."""
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
#include <cstdio>
#include <random>
#include <stdexcept>
#include <vector>
using namespace hm;
static bool rejects(const Plan& p, const StreamProgram& g) {
  try { validate_stream_program(p, g); } catch (const std::logic_error&) { return true; }
  return false;
}
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  long n = atol(argv[2]);
  int leaf = atoi(argv[3]);
  std::vector<double> P(2 * n);
  if (fread(P.data(), 8, 2 * n, f) != (size_t)(2 * n)) return 1;
  fclose(f);
  Tree t; build_tree(P.data(), n, leaf, 2.0, t);
  Plan p; build_plan(t, p);
  const int nt = (int)p.tasks.size();
  std::mt19937_64 rng(atoi(argv[4]));
  std::exponential_distribution<double> ex(1.0);
  std::vector<double> dur(nt);
  for (int i = 0; i < nt; ++i) dur[i] = 100.0 * ex(rng);
  StreamProgram g;
  build_stream_program(t, p, dur, 1.0, g);
  int per[MS_STREAMS] = {0}, waits_total = 0, dropped_ok = 0, dropped_tried = 0;
  for (auto& L : g.launches) { per[L.stream]++; waits_total += L.nwait; }
  for (size_t k = 0; k < g.launches.size() && dropped_tried < 20; ++k)
    if (g.launches[k].nwait > 0) {
      StreamProgram b = g; b.launches[k].nwait -= 1; ++dropped_tried;
      dropped_ok += rejects(p, b);
    }
  // swap two adjacent launches of one stream that depend on each other
  int swapped_rejected = -1;
  for (size_t k = 0; k + 1 < g.launches.size() && swapped_rejected < 0; ++k) {
    StreamProgram b = g;
    std::swap(b.launches[k], b.launches[k + 1]);
    if (rejects(p, b)) swapped_rejected = 1;
  }
  printf("{\"tasks\": %d, \"launches\": %zu, \"per_stream\": [%d, %d, %d, %d], \"waits\": %d, \"events\": %d, "
         "\"dropped_tried\": %d, \"dropped_rejected\": %d, \"swap_rejected\": %d}\n", nt, g.launches.size(),
         per[0], per[1], per[2], per[3], waits_total, g.nevents, dropped_tried, dropped_ok, swapped_rejected);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("msprog")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), os.path.join(CSRC, "hm_plan.cpp"),
                    "-o", str(exe)], check=True, timeout=600)
    return d, exe


@pytest.mark.parametrize("n,leaf,seed", [(3000, 32, 1), (12000, 64, 2)])
def test_stream_program_valid_and_validator_strict(harness, n, leaf, seed):
    d, exe = harness
    pts = d / f"p{n}.bin"
    wl.basin_clusters(n, 41).astype(np.float64).tofile(pts)
    out = subprocess.run([str(exe), str(pts), str(n), str(leaf), str(seed)], capture_output=True, text=True,
                         timeout=600, check=True)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    assert sum(r["per_stream"]) == r["launches"]
    assert r["per_stream"][0] > 0 and r["per_stream"][2] + r["per_stream"][3] > 0
    assert r["waits"] > 0 and r["events"] > 0
    # every wait the builder emits is needed: removing any one breaks a dependency
    assert r["dropped_tried"] > 0 and r["dropped_rejected"] == r["dropped_tried"]
    assert r["swap_rejected"] == 1
