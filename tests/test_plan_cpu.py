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
