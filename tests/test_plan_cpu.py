"""The host plan of resumed iteration batches (csrc/plan.h), on the CPU.

A time step that its queued launches leave undecided is resumed from the
host in batches of 1, 1, 2, 4, ... launches, each judged by an end of step
over its iterates.  The batch sizes, the iteration limit and the ring of
iterate buffers (record slot l % nbuf) must keep every launched range valid
over thousands of batches: an unbounded shift once made a resumed range
negative after about 30 batches.  The header is pure integer arithmetic;
this test compiles it with a small driver and walks long steps.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_13555_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "plan.h"
using namespace ocip;
// Walk a step resumed after `launched0` queued iterates until max_iters, the
// way the host driver does, and check every batch and end-of-step range.
static int walk(int launched0, int max_iters, int nbuf, long *batches) {
  int launched = launched0, extra = 0;
  while (launched < max_iters) {
    ++extra;
    const int count = resumed_batch(extra, launched, max_iters, nbuf);
    if (!batch_range_ok(launched, count)) return 1;
    const int first = launched + 1, last = launched + count;
    if (!end_range_ok(first, last, nbuf)) return 2;
    if (count < 1 || count > nbuf - 1 || count > kMaxBatch) return 3;
    if (last > max_iters && count != 1) return 4;
    launched = last;
    ++*batches;
  }
  if (launched != (launched0 > max_iters ? launched0 : max_iters)) return 5;
  return 0;
}
int main() {
  // the batch sizes: 1, 1, 2, 4, ..., 64, and 64 from then on (no overflow)
  const int expect[10] = {1, 1, 2, 4, 8, 16, 32, 64, 64, 64};
  for (int e = 1; e <= 10; ++e)
    if (resume_count(e) != expect[e - 1]) { printf("count %d\n", e); return 1; }
  for (int e = 11; e < 100000; ++e)
    if (resume_count(e) != kMaxBatch) { printf("count %d\n", e); return 1; }
  if (batch_range_ok(-1, 1) || batch_range_ok(0, 0) || batch_range_ok(0, kMaxBatch + 1)) return 1;
  if (end_range_ok(0, 1, 9) || end_range_ok(3, 2, 9) || end_range_ok(1, 9, 9)) return 1;
  if (!end_range_ok(1, 8, 9)) return 1;
  long batches = 0;
  const int nbufs[] = {9, 10, 17, 33, 65};
  const int limits[] = {1, 2, 7, 64, 65, 1000, 2700, 100000, 1000000};
  const int starts[] = {1, 2, 4, 8, 64};
  for (int nb : nbufs)
    for (int mi : limits)
      for (int l0 : starts) {
        const int rc = walk(l0, mi, nb, &batches);
        if (rc) { printf("walk rc=%d nbuf=%d max_iters=%d launched=%d\n", rc, nb, mi, l0); return 1; }
      }
  printf("ok %ld\n", batches);
  return 0;
}
"""


def test_resumed_batches_stay_in_range(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "plan_driver.cpp"
    exe = tmp_path / "plan_driver"
    src.write_text(DRIVER)
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
    assert int(out.stdout.split()[1]) > 10000   # thousands of resumed batches walked


ENSEMBLE_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "plan.h"
using namespace ocip;
// One batch of an ensemble class: problems planning first_i .. last_i, the
// class's launches at its nodes up to its longest range, each problem's
// work-groups computing ens_levels iterates and its reduction work-group
// reducing ens_reduced_before iterates before the launch's first; then the
// final reduction of ens_trailing iterates.  Every iterate of every range must
// be computed once, in order, by consecutive launches, and reduced once,
// after it is computed (its records written by an earlier launch).
static int batch(const std::vector<int> &first, const std::vector<int> &last, int ki) {
  const int n = (int)first.size();
  int L = 0;
  for (int i = 0; i < n; ++i) L = last[i] - first[i] + 1 > L ? last[i] - first[i] + 1 : L;
  for (int i = 0; i < n; ++i) {
    const int len = last[i] - first[i] + 1;
    std::vector<int> computed(len, 0), reduced(len, 0), when(len, -1);
    int next = first[i], launches = 0;
    for (int node = 1; node <= L; ++node) {
      if (!ens_launch_node(node, ki)) continue;
      ++launches;
      const int l = first[i] - 1 + node;   // the launch's first iterate
      const int kk = ens_levels(first[i], last[i], node, ki);
      if (kk < 0 || kk > ki) return 1;
      if (kk > 0 && l != next) return 2;   // consecutive, in order
      for (int j = 0; j < kk; ++j) { computed[l + j - first[i]]++; when[l + j - first[i]] = launches; }
      if (kk > 0) next = l + kk;
      // the reduction work-group: iterates l - r .. l - 1, from the launch before
      const int r = ens_reduced_before(node, ki);
      if (kk > 0)   // (an idle problem's reduction work-group returns too)
        for (int j = 1; j <= r; ++j) {
          const int it = l - j;
          if (it < first[i]) return 3;   // (the batch before reduced those)
          if (when[it - first[i]] != launches - 1) return 4;
          reduced[it - first[i]]++;
        }
    }
    if (next != last[i] + 1) return 5;
    const int t = ens_trailing(first[i], last[i], ki);
    if (t < 1 || t > ki) return 6;
    for (int j = 0; j < t; ++j) {
      const int it = last[i] - j;
      if (when[it - first[i]] != when[len - 1]) return 7;   // the last launch's iterates
      reduced[it - first[i]]++;
    }
    for (int j = 0; j < len; ++j)
      if (computed[j] != 1 || reduced[j] != 1) return 8;
  }
  return 0;
}
int main() {
  unsigned s = 12345u;
  auto rnd = [&](int m) { s = s * 1664525u + 1013904223u; return (int)((s >> 8) % (unsigned)m); };
  long checked = 0;
  for (int trial = 0; trial < 20000; ++trial) {
    const int ki = trial % 3 == 0 ? 1 : (trial % 3 == 1 ? 3 : 4);
    const int n = 1 + rnd(6);
    std::vector<int> first(n), last(n);
    for (int i = 0; i < n; ++i) {
      first[i] = 1 + rnd(200);
      last[i] = first[i] + rnd(70);
    }
    const int rc = batch(first, last, ki);
    if (rc) { printf("rc=%d trial=%d ki=%d\n", rc, trial, ki); return 1; }
    checked += n;
  }
  printf("ok %ld\n", checked);
  return 0;
}
"""


def test_ensemble_launch_plan_covers_every_iterate_once(tmp_path):
    """The ensemble's multi-iterate launches (plan.h, evaluated by the queue
    kernels themselves): over random batches of problems with different
    ranges and 1, 3 or 4 iterates per launch, every iterate is computed once
    by consecutive launches and its e reduced once, by the next launch's
    reduction work-group or the batch's final reduction."""
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "ens_driver.cpp"
    exe = tmp_path / "ens_driver"
    src.write_text(ENSEMBLE_DRIVER)
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
