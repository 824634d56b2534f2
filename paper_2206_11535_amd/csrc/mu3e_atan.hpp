// Float64 arctangent of a first-quadrant point, for the arc angles of the
// triplet fit (Section IV-B), where the angles enter a float64 difference of
// products.  Plain arithmetic only (no HIP includes), so that the host test
// compiles it with a C++ compiler alone.
#pragma once

#include <math.h>

#if defined(__HIP__)
#define MU3E_HD __host__ __device__
#else
#define MU3E_HD
#endif

namespace mu3e {

// atan2(y, x) for finite x >= 0, y >= 0 (magnitudes 1e-90 .. 1e90), in
// [0, pi/2]; 0 when both are 0.  One division reduces the argument to
// |u| <= tan(pi/8): u = min/max, or
// (min - max)/(min + max) with atan(min/max) = pi/4 + atan(u) above tan(pi/8);
// then atan(u) = u + u^3 P(u^2) with the degree-9 polynomial P of
// atan_coeffs.py (relative error below 4e-17 before rounding); the result
// is pi/2 - atan(x/y) when y > x.  About 25 float64 operations and no
// float64 division or reciprocal; the general atan2 also handles signs,
// infinities and the other quadrants.
MU3E_HD inline double atan2_q1(double y, double x) {
  const bool swap = y > x;
  const double hi = swap ? y : x, lo = swap ? x : y;   // 0 <= lo <= hi
  const bool mid = lo > 0.41421356237309503 * hi;      // lo / hi > tan(pi/8)
  double num = mid ? lo - hi : lo;
  double den = mid ? lo + hi : (hi > 0.0 ? hi : 1.0);
  // the quotient is scale-free: bring den into the float32 range of the seed
  const double sc = den < 1e-30 ? 0x1p+200 : (den > 1e30 ? 0x1p-200 : 1.0);
  num *= sc;
  den *= sc;
  // num / den with a float32 reciprocal refined by two Newton steps and a
  // final residual correction (within an ulp, no float64 division)
  const double r0 = (double)(1.0f / (float)den);
  const double r1 = fma(r0, fma(-den, r0, 1.0), r0);
  const double r = fma(r1, fma(-den, r1, 1.0), r1);
  const double q = num * r;
  const double u = fma(fma(-den, q, num), r, q);
  const double s = u * u;
  double p = 0.021218539805649099546;
  p = fma(p, s, -0.043555219035647212182);
  p = fma(p, s, 0.056912234889686052638);
  p = fma(p, s, -0.066408526597346613603);
  p = fma(p, s, 0.076900351150696277612);
  p = fma(p, s, -0.090907798689403329392);
  p = fma(p, s, 0.11111106534664103835);
  p = fma(p, s, -0.14285714192066069085);
  p = fma(p, s, 0.19999999999045716163);
  p = fma(p, s, -0.33333333333329938344);
  double a = fma(u * s, p, u);
  if (mid) a += 0.78539816339744830962;                  // pi/4
  return swap ? 1.5707963267948966192 - a : a;           // pi/2 - atan(x/y)
}

// atan2(y, x) over all four quadrants from the first-quadrant one: the
// angle of (|x|, |y|), reflected to x < 0 and signed by y (the sign of a
// zero y decides, as for the C library: +-0 or +-pi).  Finite inputs of
// magnitude 1e-90 .. 1e90 (or zero).
MU3E_HD inline double atan2_full(double y, double x) {
  const double a = atan2_q1(fabs(y), fabs(x));
  const double b = signbit(x) ? 3.14159265358979323846 - a : a;
  return signbit(y) ? -b : b;
}

// float32 arctangent over all four quadrants, the float32 counterpart of
// atan2_full for the float32 fit: the same reduction (quotient by the
// reciprocal of the larger magnitude), and the degree-4 polynomial in u^2
// that atan_coeffs.py fits with five terms (relative error below 1e-9 before
// rounding, far under float32's 6e-8).  Finite inputs of magnitude
// 1e-20 .. 1e20 (or zero); a zero y's sign decides as in the C library.
MU3E_HD inline float atan2f_full(float y, float x) {
  const float ay = fabsf(y), ax = fabsf(x);
  const bool swap = ay > ax;
  const float hi = swap ? ay : ax, lo = swap ? ax : ay;
  const bool mid = lo > 0.41421356f * hi;
  float num = mid ? lo - hi : lo;
  float den = mid ? lo + hi : (hi > 0.0f ? hi : 1.0f);
  const float sc = den < 1e-20f ? 0x1p+64f : (den > 1e20f ? 0x1p-64f : 1.0f);
  num *= sc;
  den *= sc;
#if defined(__HIP_DEVICE_COMPILE__)
  const float u = num * __builtin_amdgcn_rcpf(den);
#else
  const float u = num / den;
#endif
  const float s = u * u;
  float p = -0.0606607136221f;
  p = fmaf(p, s, 0.105885721751f);
  p = fmaf(p, s, -0.142427443032f);
  p = fmaf(p, s, 0.199984236986f);
  p = fmaf(p, s, -0.333333142486f);
  float a = fmaf(u * s, p, u);
  if (mid) a += 0.785398163397f;                    // pi/4
  a = swap ? 1.57079632679f - a : a;                // pi/2 - atan(x/y)
  a = signbit(x) ? 3.14159265359f - a : a;
  return signbit(y) ? -a : a;
}

}  // namespace mu3e
