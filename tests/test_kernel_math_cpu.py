"""Host checks of the kernels' own float64 arctangent (mu3e_atan.hpp), built
with the host C++ compiler: it must agree with the C library's atan2 to a
few units in the last place, on the first quadrant (the arc angles of the
triplet fit, Section IV-B) and on all four (turning angles of the vertex
stage, Section IV-C), signed zeros included."""
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
static int64_t ulps(double a, double b) {
  if (a == b) return 0;                       // also +0 == -0
  if (signbit(a) != signbit(b)) return 1LL << 62;
  return llabs(ord(a) - ord(b));
}
int main() {
  srand48(7);
  int64_t worst_q1 = 0, worst_full = 0;
  for (int k = 0; k < 2000000; ++k) {
    double y = drand48(), x = drand48();
    if (k % 4 == 1) y *= 1e-6;            // nearly flat
    if (k % 4 == 2) x *= 1e-6;            // nearly vertical
    if (k % 4 == 3) {                     // wide exponent range
      const int e = (int)(drand48() * 560) - 280;
      y = ldexp(y, e + (int)(drand48() * 20) - 10);
      x = ldexp(x, e);
    }
    const int64_t d = ulps(mu3e::atan2_q1(y, x), atan2(y, x));
    if (d > worst_q1) worst_q1 = d;
    const double sy = (k & 1) ? -y : y, sx = (k & 2) ? -x : x;   // all quadrants
    const int64_t e = ulps(mu3e::atan2_full(sy, sx), atan2(sy, sx));
    if (e > worst_full) worst_full = e;
  }
  // octant edges, axes and signed zeros
  const double tp8 = 0.41421356237309503;
  const double pts[][2] = {{0.0, 0.0}, {0.0, 1.0}, {1.0, 0.0}, {1.0, 1.0}, {tp8, 1.0},
                           {nextafter(tp8, 1.0), 1.0}, {1.0, tp8}, {1.0, 3e-30}, {0.0, -1.0},
                           {-0.0, -1.0}, {-0.0, 1.0}, {-1.0, 0.0}, {-1.0, -1.0}, {1e-80, -1.0}};
  int64_t edge = 0;
  for (const auto& p : pts) {
    const int64_t d = ulps(mu3e::atan2_full(p[0], p[1]), atan2(p[0], p[1]));
    if (d > edge) edge = d;
  }
  // the float32 version against the C library's atan2f
  int64_t worst_f = 0;
  for (int k = 0; k < 2000000; ++k) {
    float y = (float)drand48(), x = (float)drand48();
    if (k % 4 == 1) y *= 1e-6f;
    if (k % 4 == 2) x *= 1e-6f;
    if (k % 4 == 3) {
      const int e = (int)(drand48() * 100) - 50;
      y = ldexpf(y, e + (int)(drand48() * 20) - 10);
      x = ldexpf(x, e);
    }
    if (k & 1) y = -y;
    if (k & 2) x = -x;
    const float a = mu3e::atan2f_full(y, x), b = atan2f(y, x);
    int32_t ia, ib;
    memcpy(&ia, &a, 4);
    memcpy(&ib, &b, 4);
    const int64_t d = a == b ? 0 : (signbit(a) != signbit(b) ? (1LL << 40) : llabs((int64_t)ia - (int64_t)ib));
    if (d > worst_f) worst_f = d;
  }
  printf("%lld %lld %lld %lld\n", (long long)worst_q1, (long long)worst_full, (long long)edge, (long long)worst_f);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_atan2_against_libm(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "t"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src), "-lm"])
    worst_q1, worst_full, edge, worst_f = map(int, subprocess.check_output([str(exe)], text=True).split())
    assert worst_f <= 4, worst_f
    assert worst_q1 <= 2, worst_q1
    assert worst_full <= 2, worst_full
    assert edge <= 1, edge


def test_pair_index_split_with_approximate_reciprocal():
    """The cuts split a flat pair index p < n * m into (p // n, p % n) as the
    float32 truncation of (p + 0.5) * r with r the hardware reciprocal of n
    (about 1 ulp): the split stays exact for every n <= 128 and p < 128 n
    with r off by up to 2 ulp either way (float32 arithmetic emulated)."""
    import numpy as np
    for n in range(1, 129):
        p = np.arange(n * 128, dtype=np.int64)
        pf = p.astype(np.float32) + np.float32(0.5)
        r = np.float32(1.0) / np.float32(n)
        for step in (-2, -1, 0, 1, 2):
            rr = r
            for _ in range(abs(step)):
                rr = np.nextafter(rr, np.float32(np.inf if step > 0 else -np.inf), dtype=np.float32)
            q = (pf * rr).astype(np.float32).astype(np.int32)
            assert np.array_equal(q, p // n), (n, step)
