"""Host checks of the kernels' own float64 arctangent (mu3e_atan.hpp), built
with the host C++ compiler: it must agree with the C library's atan2 to a
few units in the last place on the first quadrant, where the triplet fit
takes its arc angles (Section IV-B)."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2206_11535_amd", "csrc")

PROGRAM = r"""
#include "mu3e_atan.hpp"
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
static int64_t ord(double v) { int64_t i; memcpy(&i, &v, 8); return i; }
int main() {
  srand48(7);
  int64_t worst = 0;
  for (int k = 0; k < 2000000; ++k) {
    double y = drand48(), x = drand48();
    if (k % 4 == 1) y *= 1e-6;            // nearly flat
    if (k % 4 == 2) x *= 1e-6;            // nearly vertical
    if (k % 4 == 3) {                     // wide exponent range
      y = ldexp(y, (int)(drand48() * 80) - 40);
      x = ldexp(x, (int)(drand48() * 80) - 40);
    }
    const int64_t d = llabs(ord(mu3e::atan2_q1(y, x)) - ord(atan2(y, x)));
    if (d > worst) worst = d;
  }
  // octant edges and special points
  const double tp8 = 0.41421356237309503;
  const double pts[][2] = {{0.0, 0.0}, {0.0, 1.0}, {1.0, 0.0}, {1.0, 1.0}, {tp8, 1.0},
                           {nextafter(tp8, 1.0), 1.0}, {1.0, tp8}, {1.0, 3e-30}};
  int64_t edge = 0;
  for (const auto& p : pts) {
    const int64_t d = llabs(ord(mu3e::atan2_q1(p[0], p[1])) - ord(atan2(p[0], p[1])));
    if (d > edge) edge = d;
  }
  printf("%lld %lld\n", (long long)worst, (long long)edge);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_atan2_q1_against_libm(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "t"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src), "-lm"])
    worst, edge = map(int, subprocess.check_output([str(exe)], text=True).split())
    assert worst <= 2, worst
    assert edge <= 1, edge
