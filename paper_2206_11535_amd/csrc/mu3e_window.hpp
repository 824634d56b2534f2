// The Delta lambda window of the cuts as a window on z0 (Section IV-A,
// Delta lambda cut).  Plain arithmetic only (no HIP includes), so that the
// host test compiles it with a C++ compiler alone.
#pragma once

#include <math.h>

#if defined(__HIP__)
#define MU3E_HD __host__ __device__
#else
#define MU3E_HD
#endif

namespace mu3e {

// With t12 = (z2 - z1) / (R2 - R1) fixed by an (h1, h2) pair,
// Delta lambda = t12 - (z1 - z0) / (R1 - R0) increases with z0 (R1 > R0), so
// it lies in [lo, hi] exactly when z0 lies in
// [z1 - (t12 - lo)(R1 - R0), z1 - (t12 - hi)(R1 - R0)].  The edges are
// computed in float32 from inv12 = 1 / (R2 - R1) and d01 = R1 - R0 (both
// rounded to float32); each is within 7 u (|edge| + d01 (|t12| + |lo|))
// of the exact one, u = 2^-24 (the roundings of z2 - z1, of inv12 and its
// product, of t12 - lo, of d01 and of the fused multiply-add), and e, 16 u
// times a sum that covers both edges, bounds it with room for the rounding
// of the edge +- e themselves.  Inside [in_lo, in_hi] the combination
// passes with a margin far above the float64 rounding of Delta lambda,
// outside [out_lo, out_hi] it fails, in between float64 decides.
// dl_abs = |lo| + |hi|.
struct ZWindow {
  float in_lo, in_hi, out_lo, out_hi;
};

MU3E_HD inline ZWindow dl_window_f(float z1, float z2, float inv12, float d01, float lo, float hi, float dl_abs) {
  const float t12 = (z2 - z1) * inv12;
  const float za = fmaf(-(t12 - lo), d01, z1);
  const float zb = fmaf(-(t12 - hi), d01, z1);
  const float e = 16.0f * 5.9604645e-8f * (fabsf(za) + fabsf(zb) + d01 * (fabsf(t12) + dl_abs));
  return {za + e, zb - e, za - e, zb + e};
}

}  // namespace mu3e
