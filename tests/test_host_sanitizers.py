"""Host code under sanitizers (CPU only): the constants (binary128 root finding,
eq. yoyo2 residues, the per-degree cache) and the degree choice, built with g++
under AddressSanitizer + UndefinedBehaviorSanitizer, and under ThreadSanitizer
with several threads filling and reading the cache at once.  A small C++ driver
calls every degree, the argument checks and the degree choice; any sanitizer
report fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2306_16778_amd", "csrc", "constants.cpp")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
#include "expm_pfd.h"

static int check_all(int first) {
  for (int k = 0; k < 32; ++k) {
    const int d = 2 + 2 * ((first + k) % 32);
    std::vector<double> th(d), a(d);
    if (expm_pfd_constants(d, th.data(), a.data()) != 0) return 1;
    for (double x : th) if (!std::isfinite(x)) return 2;
    for (double x : a) if (!std::isfinite(x)) return 3;
  }
  return 0;
}

int main(int argc, char** argv) {
  const int threads = argc > 1 ? std::atoi(argv[1]) : 1;
  std::vector<int> rc(threads, 0);
  std::vector<std::thread> ts;
  for (int i = 0; i < threads; ++i) ts.emplace_back([&rc, i] { rc[i] = check_all(7 * i); });
  for (auto& t : ts) t.join();
  for (int r : rc) if (r) { std::printf("constants failed %d\n", r); return 1; }
  double th[2], a[2];
  if (expm_pfd_constants(3, th, a) != EXPM_PFD_ERR_DEGREE) return 4;
  if (expm_pfd_constants(66, th, a) != EXPM_PFD_ERR_DEGREE) return 5;
  if (expm_pfd_constants(4, nullptr, a) != EXPM_PFD_ERR_NULL) return 6;
  int d = 0;
  double b = 0;
  if (expm_pfd_choose_degree(1e-7, 16, &d, &b) != 0 || d > 30) return 7;
  if (expm_pfd_choose_degree(1e-12, 16, &d, &b) != 1) return 8;
  if (expm_pfd_choose_degree(1e-8, 3, &d, &b) != EXPM_PFD_ERR_ARG) return 9;
  std::printf("ok\n");
  return 0;
}
"""


def _build_and_run(tmp_path, flags, threads):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I",
           os.path.join(ROOT, "include"), SRC, str(drv), "-o", str(exe), "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # (the library link order check is off: the environment may preload a library of its own)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([str(exe), str(threads)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and "ok" in out.stdout, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "Sanitizer" not in out.stderr, out.stderr


def test_constants_under_address_and_undefined_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], 1)


def test_constants_cache_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], 4)
