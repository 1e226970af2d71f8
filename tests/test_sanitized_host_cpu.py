"""The library's pure host C++ under AddressSanitizer and UndefinedBehaviorSanitizer.

The Gauss-Legendre rule (csrc/quadrature.cpp, behind oci_gauss_legendre) and
the resumed-batch plan (csrc/plan.h) build without the HIP runtime, so they
are compiled here with the host compiler's sanitizers and driven over their
whole input range: every rule size 1 .. 4096 (and the refused sizes), and
long resumed steps.  Any out-of-bounds access, overflow or other undefined
behaviour aborts the driver.  (The HIP host driver itself links the HIP
runtime and is exercised by the GPU tests.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_13555_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <vector>
#include "oci.h"
#include "plan.h"
int main() {
  std::vector<double> mu, w;
  for (int n = 1; n <= 4096; n = n < 64 ? n + 1 : n * 2) {
    mu.assign(n, 0.0);
    w.assign(n, 0.0);
    if (oci_gauss_legendre(n, mu.data(), w.data()) != OCI_OK) { printf("rc %d\n", n); return 1; }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += w[i];
    if (std::fabs(s - 2.0) > 1e-11) { printf("sum %d %.17g\n", n, s); return 1; }
    for (int i = 1; i < n; ++i) if (!(mu[i] > mu[i - 1])) { printf("order %d\n", n); return 1; }
  }
  double d[4];
  if (oci_gauss_legendre(0, d, d) != OCI_EINVAL || oci_gauss_legendre(4097, d, d) != OCI_EINVAL ||
      oci_gauss_legendre(4, nullptr, d) != OCI_EINVAL) { printf("refusals\n"); return 1; }
  long total = 0;
  for (int nbuf : {7, 9, 65})
    for (int mi : {1, 1000, 1000000}) {
      int launched = 8, extra = 0;
      while (launched < mi) {
        const int c = ocip::resumed_batch(++extra, launched, mi, nbuf);
        if (!ocip::end_range_ok(launched + 1, launched + c, nbuf)) { printf("range\n"); return 1; }
        launched += c;
        ++total;
      }
    }
  printf("ok %ld\n", total);
  return 0;
}
"""


def test_host_code_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    src = tmp_path / "sanitize_driver.cpp"
    exe = tmp_path / "sanitize_driver"
    src.write_text(DRIVER)
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", INCLUDE, "-I", CSRC]
    build = subprocess.run([cxx] + flags + [str(src), os.path.join(CSRC, "quadrature.cpp"), "-o",
                                            str(exe)], capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.startswith("ok ")
