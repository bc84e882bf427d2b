"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host eigensolvers of the library (the Davidson subspace problem and the batched
symmetric eigensolves of large PNO blocks) are plain C++: they are compiled here with
g++ and both sanitizers, together with a small driver, and run on random matrices of
several sizes, including 1 x 1.  Any invalid access or undefined operation aborts the
driver.  Skipped where g++ or the sanitizer runtimes are missing.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <cstdio>
#include <random>
#include <vector>
namespace pnoeom {
int host_eig(int, const double*, double*, double*, double*, int);
int host_syev(int, const double*, double*, double*);
int host_syev_batched(int, const int*, int, double*, double*, double*, int);
}
int main() {
  std::mt19937_64 g(7);
  std::normal_distribution<double> nd;
  for (int n : {1, 2, 5, 17, 40, 64}) {
    std::vector<double> a((size_t)n * n), wr(n), wi(n), vr((size_t)n * n), w(n), v((size_t)n * n);
    for (auto& x : a) x = nd(g);
    for (int nvec : {-1, 1, n / 2}) {
      if (pnoeom::host_eig(n, a.data(), wr.data(), wi.data(), vr.data(), nvec) != 0) return 1;
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) a[(size_t)i * n + j] = a[(size_t)j * n + i];
    if (pnoeom::host_syev(n, a.data(), w.data(), v.data()) != 0) return 2;
  }
  // batched: three blocks of different sizes in a padded stack
  const int ld = 24, nmat = 3;
  const int nsz[nmat] = {24, 7, 1};
  std::vector<double> A((size_t)nmat * ld * ld, 0.0), ev((size_t)nmat * ld), Vt((size_t)nmat * ld * ld);
  for (int m = 0; m < nmat; ++m)
    for (int i = 0; i < nsz[m]; ++i)
      for (int j = 0; j <= i; ++j) {
        const double x = nd(g);
        A[(size_t)m * ld * ld + (size_t)i * ld + j] = x;
        A[(size_t)m * ld * ld + (size_t)j * ld + i] = x;
      }
  if (pnoeom::host_syev_batched(nmat, nsz, ld, A.data(), ev.data(), Vt.data(), 2) != 0) return 3;
  std::printf("ok\n");
  return 0;
}
'''


def test_host_eigensolvers_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    drv = tmp_path / "drv.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_1802_06738_amd", "csrc", "eig.cpp"), str(drv), "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()):
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stderr[-3000:]
