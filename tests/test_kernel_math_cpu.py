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


WINDOW_PROGRAM = r"""
#include "mu3e_window.hpp"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
// Delta lambda as the float64 selection computes it (Section IV-A)
static bool pass64(float z0, float z1, float z2, const float* R, float lo, float hi) {
  const double d = ((double)z2 - (double)z1) / ((double)R[2] - (double)R[1]) -
                   ((double)z1 - (double)z0) / ((double)R[1] - (double)R[0]);
  return d >= (double)lo && d <= (double)hi;
}
int main() {
  srand48(11);
  long wrong = 0, wrong_tight = 0, amb = 0, n = 0;
  double widest = 0;
  for (int trial = 0; trial < 400; ++trial) {
    float R[3] = {(float)(5 + 95 * drand48()), (float)(5 + 95 * drand48()), (float)(5 + 95 * drand48())};
    if (R[0] > R[1]) { float t = R[0]; R[0] = R[1]; R[1] = t; }
    if (R[1] > R[2]) { float t = R[1]; R[1] = R[2]; R[2] = t; }
    if (R[0] > R[1]) { float t = R[0]; R[0] = R[1]; R[1] = t; }
    if (!(R[0] < R[1] && R[1] < R[2])) continue;
    const float lo = (float)(-0.5 * drand48()), hi = (float)(lo + 0.5 * drand48());
    const float inv12 = 1.0f / (R[2] - R[1]), d01 = R[1] - R[0], dl_abs = fabsf(lo) + fabsf(hi);
    const double scale = trial % 4 == 3 ? 1e3 : 200;   // hit z up to +-200 mm, some far larger
    for (int k = 0; k < 5000; ++k) {
      const float z1 = (float)(scale * (2 * drand48() - 1));
      const float z2 = (float)(z1 + 1.5 * scale * (2 * drand48() - 1));
      const mu3e::ZWindow w = mu3e::dl_window_f(z1, z2, inv12, d01, lo, hi, dl_abs);
      const double za = 0.5 * ((double)w.in_lo + w.out_lo), e = 0.5 * ((double)w.in_lo - w.out_lo);
      const double zb = 0.5 * ((double)w.in_hi + w.out_hi);
      // the ambiguous band relative to the scale of the edge
      const double t12 = ((double)z2 - z1) / ((double)R[2] - R[1]);
      const double ref = fabs(za) + fabs(zb) + d01 * (fabs(t12) + dl_abs);
      if (e / ref > widest) widest = e / ref;
      for (int j = 0; j < 8; ++j) {
        // z0 a fraction of a band to several bands from either edge
        const double mult[4] = {0.05, 0.5, 2, 8};
        const double edge = (j & 1) ? zb : za;
        const float z0 = (float)(edge + (2 * drand48() - 1) * mult[(j >> 1) & 3] * e);
        const bool p = pass64(z0, z1, z2, R, lo, hi);
        const bool sure = z0 > w.in_lo && z0 < w.in_hi;
        const bool cand = z0 >= w.out_lo && z0 <= w.out_hi;
        wrong += (sure && !p) || (!cand && p);
        amb += cand && !sure;
        // the same window with a band 64 times narrower must get some wrong
        const double et = e / 64;
        const bool sure_t = z0 > za + et && z0 < zb - et, cand_t = z0 >= za - et && z0 <= zb + et;
        wrong_tight += (sure_t && !p) || (!cand_t && p);
        ++n;
      }
    }
  }
  printf("%ld %ld %ld %ld %.6e\n", n, wrong, wrong_tight, amb, widest);
  return 0;
}
"""


def test_dlambda_z0_window(tmp_path):
    """The join tests Delta lambda as a window on z0 whose float32 edges
    carry a bound on their rounding error (mu3e_window.hpp): on random
    radii, windows and hit pairs, with z0 drawn at a fraction of the
    ambiguous band to several bands from either edge, no z0 the window calls
    a sure pass fails the float64 test and none outside its outer edges
    passes it.  The same check with a band 64 times narrower does find wrong
    decisions (so the bound is not vacuous: it is needed), and the band stays
    below 64 u of its scale (so few candidates go to float64)."""
    src = tmp_path / "w.cpp"
    src.write_text(WINDOW_PROGRAM)
    exe = tmp_path / "w"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, "-o", str(exe), str(src),
                           "-lm"])
    n, wrong, wrong_tight, amb, widest = subprocess.check_output([str(exe)], text=True).split()
    n, wrong, wrong_tight, amb = int(n), int(wrong), int(wrong_tight), int(amb)
    assert n > 10_000_000 // 2, n
    assert wrong == 0, wrong
    assert wrong_tight > 0
    assert 0.2 * n < amb < 0.8 * n          # the draws straddle the band
    assert float(widest) < 64 * 2.0 ** -24, widest
