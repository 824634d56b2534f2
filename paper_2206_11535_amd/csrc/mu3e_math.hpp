// Device arithmetic of the online event selection (gfx950).
//
// Everything here is templated on the scalar type: the kernels evaluate in
// float32, and re-evaluate a candidate in float64 only when a float32 value
// falls inside a bound on its own rounding error around a decision edge (a
// cut window, the chi2 < 32 cut, the nearest-hit choice, a circle tangency).
// Cancellation-prone geometric primitives (coordinate differences, the
// transverse cross product, squared chords) are always formed in float64
// from the float32 hits: on gfx950 float64 FMA runs at the non-packed float32
// rate, and these few operations remove the error amplification of nearly
// straight tracks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mu3e_atan.hpp"

namespace mu3e {

constexpr double kCLight = 0.299792458;   // p[MeV] = kCLight * B[T] * R[mm]
constexpr double kMassE = 0.51099895;     // MeV
constexpr double kMassMu = 105.6583755;   // MeV
constexpr double kPiD = 3.14159265358979323846;
constexpr float kU32 = 5.9604645e-8f;     // unit roundoff of float32, 2^-24
constexpr int kMaxTiledLayerHits = 1023;   // hits per layer the cuts handle (tiled through LDS)

// Per-launch constants (by value in kernel arguments).
struct Consts {
  float R[4], zh[4], b, xx0, sig_pix;
  float dl_lo, dl_hi, c01_lo, c01_hi, c12_lo, c12_hi, rtc_lo, rtc_hi;
  float chi2_trk;
  int max_trip, max_trk, max_combo, max_lh;
  float de_max, r_target, target_tol, chi2_v, d_target, p_sum;
  // derived in float32
  float inv01, inv12;        // 1 / (R1 - R0), 1 / (R2 - R1)
  float d01, dl_abs;         // R1 - R0, |dl_lo| + |dl_hi|
  float invRR01, invRR12;    // 1 / (R0 R1), 1 / (R1 R2)
  float rtc_lo2, rtc_hi2;    // squared |r_tc| edges
};

// float32 quotient and square root on the device straight from the hardware
// reciprocal and root (about 1 ulp each, no rescaling of denormal or
// near-overflow operands: the fit's magnitudes stay far from both ends); the
// float64 overloads are exact operations.
__host__ __device__ inline float m_div(float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return a * __builtin_amdgcn_rcpf(b);
#else
  return a / b;
#endif
}
__host__ __device__ inline double m_div(double a, double b) { return a / b; }
__host__ __device__ inline float m_sqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
__host__ __device__ inline double m_sqrt(double x) { return sqrt(x); }
__host__ __device__ inline float m_atan2(float y, float x) { return atan2f_full(y, x); }
__host__ __device__ inline double m_atan2(double y, double x) { return atan2_full(y, x); }
__host__ __device__ inline float m_sin(float x) { return sinf(x); }
__host__ __device__ inline double m_sin(double x) { return sin(x); }
__host__ __device__ inline float m_cos(float x) { return cosf(x); }
__host__ __device__ inline double m_cos(double x) { return cos(x); }
__host__ __device__ inline float m_log(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_logf(x) * 0.693147180559945f;   // hardware log2 (about 1 ulp)
#else
  return logf(x);
#endif
}
__host__ __device__ inline double m_log(double x) { return log(x); }
__host__ __device__ inline float m_abs(float x) { return fabsf(x); }
__host__ __device__ inline double m_abs(double x) { return fabs(x); }

// ------------------------------------------------------------------ circle
// Transverse circle through three hits (Section IV-A, eq. rt-cut): signed
// circumradius r_tc = d01 d12 d20 / (2 [(h0-h1) x (h2-h1)]_z), positive for
// clockwise travel h0 -> h1 -> h2 (positive charge in B along +z); centre;
// chords.  Differences, cross product and squared chords in float64 (exact
// for float32 inputs up to the products' rounding).
template <class T>
struct Circle {
  T rho;          // |r_tc|
  T cx, cy;       // centre
  T d1, d2;       // chords h0-h1, h1-h2
  T cot1, cot2;   // cot(Phi_k / 2) of the arcs h0-h1 and h1-h2
  T z1, z2;       // longitudinal steps h1-h0, h2-h1
  double phi1, phi2;   // arc angles over h0-h1 and h1-h2 (float64)
  double kink;         // z1 Phi2 - z2 Phi1 (float64)
  double cross;   // [(h0-h1) x (h2-h1)]_z in float64
  int sgn;        // sign of r_tc
};

template <class T>
__host__ __device__ inline Circle<T> circle3(double x0, double y0, double z0, double x1, double y1, double z1,
                                             double x2, double y2, double z2) {
  Circle<T> c;
  const double ax = x0 - x1, ay = y0 - y1;
  const double bx = x2 - x1, by = y2 - y1;
  const double ex = x2 - x0, ey = y2 - y0;
  c.cross = ax * by - ay * bx;
  const double aa = ax * ax + ay * ay, bb = bx * bx + by * by, ee = ex * ex + ey * ey;
  c.sgn = c.cross > 0.0 ? 1 : -1;
  // |r_tc| = sqrt(aa bb ee) / (2 |cross|); centre relative to h1
  const T taa = (T)aa, tbb = (T)bb, tee = (T)ee, tcr = (T)c.cross;
  c.rho = m_div(m_sqrt(taa) * m_sqrt(tbb) * m_sqrt(tee), (T)2 * m_abs(tcr));
  const T inv = m_div((T)0.5, tcr);
  c.cx = (T)x1 + ((T)by * taa - (T)ay * tbb) * inv;
  c.cy = (T)y1 + ((T)ax * tbb - (T)bx * taa) * inv;
  c.d1 = m_sqrt(taa);
  c.d2 = m_sqrt(tbb);
  // Half the arc angle over a chord equals the triangle angle opposite to it
  // (inscribed angle), so cot(Phi_k/2) = |b^2 + c^2 - a^2| / (4 area) with
  // a the chord; the numerators are exact in float64 and stay accurate for
  // arcs close to a half circle, where asin(d / 2 rho) is ill-conditioned.
  // The absolute value selects the minor arc.
  const double acr = c.cross > 0.0 ? c.cross : -c.cross;
  const double n1 = fabs(bb + ee - aa), n2 = fabs(aa + ee - bb);
  if (sizeof(T) == 4) {   // float32 quotients of the exact float64 terms
    const float a2 = (float)(2.0 * acr);
    c.cot1 = (T)m_div((float)n1, a2);
    c.cot2 = (T)m_div((float)n2, a2);
  } else {
    c.cot1 = (T)(n1 / (2.0 * acr));
    c.cot2 = (T)(n2 / (2.0 * acr));
  }
  // Phi_k = 2 atan2(2 area, |b^2 + c^2 - a^2|) (minor arc, in [0, pi]);
  // both arguments are non-negative
  c.phi1 = 2.0 * atan2_q1(2.0 * acr, n1);
  c.phi2 = 2.0 * atan2_q1(2.0 * acr, n2);
  const double dz1 = z1 - z0, dz2 = z2 - z1;
  c.z1 = (T)dz1;
  c.z2 = (T)dz2;
  // The polar kink theta_2 - theta_1 and R_C2 - R_C1 are small differences of
  // O(1) quantities; both follow from this one product difference, formed
  // in float64 so that float32 arc angles do not dominate the fit's chi2.
  c.kink = dz1 * c.phi2 - dz2 * c.phi1;
  return c;
}

// Phi * cot(Phi/2) - 2 without cancellation for small arcs: the Taylor series
// of 2 x cot x - 2 (x = Phi/2) in float32 up to Phi = 1, direct beyond and in
// float64 (where the cancellation costs at most a few digits of 16).
template <class T>
__host__ __device__ inline T phicot_minus_2(T phi, T cot_half) {
  if (sizeof(T) == 4 && phi <= (T)1) {
    const T x2 = (T)0.25 * phi * phi;
    // -(2/3)x^2 - (2/45)x^4 - (4/945)x^6 - (2/4725)x^8 - (4/93555)x^10 - (2764/638512875)x^12
    T s = (T)(-2764.0 / 638512875.0);
    s = s * x2 + (T)(-4.0 / 93555.0);
    s = s * x2 + (T)(-2.0 / 4725.0);
    s = s * x2 + (T)(-4.0 / 945.0);
    s = s * x2 + (T)(-2.0 / 45.0);
    s = s * x2 + (T)(-2.0 / 3.0);
    return s * x2;
  }
  return phi * cot_half - (T)2;
}

// ------------------------------------------------------------- triplet fit
// Section IV-B, "Single Triplet Fit": minimise
//   chi2(R) = Phi_MS(R)^2 / sigma_Phi^2 + Theta_MS(R)^2 / sigma_Theta^2,
//   sigma_Theta = sigma_MS, sigma_Phi = sigma_MS / sin(theta),
// linearised around the transverse-circle solution (Phi_MS = 0).  The fit
// parameter is the 3D radius R (kappa = 1/R).  Each arc k has transverse
// chord d_k and longitudinal step z_k with R^2 = d_k^2/(4 sin^2(Phi_k/2)) +
// z_k^2/Phi_k^2; on the circle of radius rho the arc angles are
// Phi_k = 2 asin(d_k / 2 rho), the polar angles theta_k = atan2(rho Phi_k, z_k)
// and the 3D radii R_k = rho / sin(theta_k).  To first order in R - R_k
//   dPhi_k/dR = -2 R_k / D_k,  D_k = rho^2 cot(Phi_k/2) + 2 z_k^2 / Phi_k^3,
//   dtheta_k/dR = z_k rho^2 (Phi_k cot(Phi_k/2) - 2) / (D_k R_k^2 Phi_k^2 sin theta_k),
// the latter in a form free of the cancellation Phi_k + R_k dPhi_k/dR.
// Phi_MS = -(1/2) sum_k dPhi_k/dR (R - R_k), Theta_MS = theta_2(R) - theta_1(R),
// expanded at Rbar = (R_1 + R_2)/2.  sigma_MS is the Highland width for
// p = c B Rbar through x/X0 / sin(theta_mean), fixed in the minimisation.
// The arc angles are taken from the triangle (see circle3), which equals
// 2 asin(d_k / 2 rho) for the minor arc.
template <class T>
struct Fit {
  T kappa, s2kappa, chi2, rstar, s2r, th1, th2, phi2;
  T sth1, cth1;   // sin and cos of th1, from the arc length and step (no arctangent)
  Circle<T> c;
  bool ok;
};

template <class T>
__host__ __device__ inline Fit<T> fit_triplet(double x0, double y0, double z0, double x1, double y1, double z1,
                                              double x2, double y2, double z2, const Consts& C) {
  Fit<T> f;
  f.c = circle3<T>(x0, y0, z0, x1, y1, z1, x2, y2, z2);
  f.ok = false;
  if (f.c.cross == 0.0) return f;
  const T rho = f.c.rho;
  T phi[2], th[2], sth[2], cth[2], Rk[2], al[2], be[2];
  const T ck[2] = {f.c.cot1, f.c.cot2};
  const T zk[2] = {f.c.z1, f.c.z2};
  phi[0] = (T)f.c.phi1;
  phi[1] = (T)f.c.phi2;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T cot = ck[k];                                     // cot(Phi/2)
    const T arc = rho * phi[k];                              // transverse arc length
    const T len = m_sqrt(arc * arc + zk[k] * zk[k]);
    th[k] = m_atan2(arc, zk[k]);                             // output only
    const T ilen = m_div((T)1, len);
    sth[k] = arc * ilen;                                     // sin(theta_k)
    cth[k] = zk[k] * ilen;                                   // cos(theta_k)
    Rk[k] = m_div(rho, sth[k]);
    const T D = rho * rho * cot + m_div((T)2 * zk[k] * zk[k], phi[k] * phi[k] * phi[k]);
    al[k] = m_div(-(T)2 * Rk[k], D);
    be[k] = m_div(zk[k] * rho * rho * phicot_minus_2(phi[k], cot), D * Rk[k] * Rk[k] * phi[k] * phi[k] * sth[k]);
  }
  const T Rbar = (T)0.5 * (Rk[0] + Rk[1]);
  // theta_2 - theta_1 = atan2(rho K, rho^2 Phi1 Phi2 + z1 z2) and
  // R_2 - R_1 = (R_2^2 - R_1^2) / (R_1 + R_2) with
  // R_2^2 - R_1^2 = (z2/Phi2)^2 - (z1/Phi1)^2 = -K (z2 Phi1 + z1 Phi2) / (Phi1 Phi2)^2
  const T K = (T)f.c.kink;
  const T dth = m_atan2(rho * K, rho * rho * phi[0] * phi[1] + zk[0] * zk[1]);
  const T pp = phi[0] * phi[1];
  const T dR = -(T)0.5 * K * (zk[1] * phi[0] + zk[0] * phi[1]) / (pp * pp * (Rk[0] + Rk[1]));   // Rbar - R_1
  const T phi0 = -(T)0.5 * dR * (al[0] - al[1]);
  const T bphi = -(T)0.5 * (al[0] + al[1]);
  const T th0 = dth - dR * (be[1] + be[0]);
  const T bth = be[1] - be[0];
  // sin of the mean polar angle from the sines and cosines of the two:
  // sin th1 + sin th2 = 2 sin(mean) cos(half difference), and the half
  // difference's cosine is sqrt((1 + cos(th1 - th2)) / 2), both well
  // conditioned as th1 ~ th2 (no arctangent or sine evaluated)
  const T sn = m_div(sth[0] + sth[1], m_sqrt((T)2 * ((T)1 + cth[0] * cth[1] + sth[0] * sth[1])));
  const T s2 = sn * sn;
  const T p = (T)kCLight * (T)C.b * Rbar;
  const T X = m_div((T)C.xx0, sn);
  const T sms = m_div((T)13.6, p) * m_sqrt(X) * ((T)1 + (T)0.038 * m_log(X));
  const T den = s2 * bphi * bphi + bth * bth;
  if (!(den > (T)0) || !(sms > (T)0)) return f;
  const T num = phi0 * bth - th0 * bphi;
  const T sms2 = sms * sms;
  const T iden = m_div((T)1, den);
  f.rstar = Rbar - (s2 * phi0 * bphi + th0 * bth) * iden;
  f.s2r = sms2 * iden;
  f.chi2 = m_div(s2 * num * num * iden, sms2);
  f.kappa = m_div((T)f.c.sgn, f.rstar);
  const T r2 = f.rstar * f.rstar;
  f.s2kappa = m_div(f.s2r, r2 * r2);
  f.th1 = th[0];
  f.th2 = th[1];
  f.sth1 = sth[0];
  f.cth1 = cth[0];
  f.phi2 = phi[1];
  f.ok = f.rstar > (T)0 && f.chi2 == f.chi2;
  return f;
}

// Two-triplet track (Section IV-B, "Triplets Fit"): each triplet minimised on
// its own, kbar = weighted mean of the curvatures, chi2_global = sum of the
// triplets' quadratic chi2 evaluated at R = 1/|kbar|.
template <class T>
__host__ __device__ inline void combine(const Fit<T>& a, const Fit<T>& b, T& kbar, T& chi2) {
  const T wa = m_div((T)1, a.s2kappa), wb = m_div((T)1, b.s2kappa);
  kbar = m_div(a.kappa * wa + b.kappa * wb, wa + wb);
  const T R = m_div((T)1, m_abs(kbar));
  const T da = R - a.rstar, db = R - b.rstar;
  chi2 = a.chi2 + m_div(da * da, a.s2r) + b.chi2 + m_div(db * db, b.s2r);
}

// ---------------------------------------------------------- layer-3 point
// Section IV-B: the preliminary helix (circumcircle + the z advance of arc
// h1->h2 per radian of turning) crosses r = R3; the crossing reached first
// going forward from h2 is the prediction.  Returns 0 if the circle never
// reaches r = R3, 1 on success; *near = true when the reach decision lies
// within `tol` (relative) of a tangency.
template <class T>
__host__ __device__ inline int predict_l3(const Fit<T>& f, float x2, float y2, float z2, T R3, T tol,
                                          T& px, T& py, T& pz, bool* near) {
  const T cx = f.c.cx, cy = f.c.cy, rho = f.c.rho;
  const T cn = m_sqrt(cx * cx + cy * cy);
  const T outer = rho + R3, inner = m_abs(rho - R3);
  if (near) *near = m_abs(cn - outer) <= tol * outer || m_abs(cn - inner) <= tol * outer;
  if (!(cn > (T)0) || cn > outer || cn < inner) return 0;
  const T icn = m_div((T)1, cn);
  const T a = (R3 * R3 - rho * rho + cn * cn) * (T)0.5 * icn;
  T h2 = R3 * R3 - a * a;
  const T h = m_sqrt(h2 > (T)0 ? h2 : (T)0);
  const T ux = cx * icn, uy = cy * icn;
  const T vx = (T)x2 - cx, vy = (T)y2 - cy;                  // centre -> h2
  // Turning angle from h2 to each crossing q in the bending sense (clockwise
  // for sgn > 0), in (0, 2 pi]: as the pair (cos, sin) * |v||w| = (dot, cross),
  // cross taken in the bending sense.  The first crossing is chosen by
  // comparing the pairs (half-turn, then the sign of their cross product),
  // and only its angle is evaluated.
  T qx[2], qy[2], dt[2], cr[2];
  bool upper[2];   // angle in (pi, 2 pi]
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T s = k == 0 ? (T)-1 : (T)1;
    qx[k] = a * ux - s * h * uy;
    qy[k] = a * uy + s * h * ux;
    const T wx = qx[k] - cx, wy = qy[k] - cy;                // centre -> crossing
    const T c = vx * wy - vy * wx;                           // counter-clockwise sense
    cr[k] = f.c.sgn > 0 ? -c : c;
    dt[k] = vx * wx + vy * wy;
    upper[k] = cr[k] < (T)0 || (cr[k] == (T)0 && !(dt[k] < (T)0));
  }
  // crossing 1 comes strictly first: an earlier half-turn, or the same one
  // and a counter-clockwise turn from crossing 1 to crossing 0 (ties keep 0)
  const bool second = (!upper[1] && upper[0]) ||
                      (upper[1] == upper[0] && dt[0] * cr[1] - cr[0] * dt[1] < (T)0);
  const int k = second ? 1 : 0;
  T ang = m_atan2(second ? cr[1] : cr[0], second ? dt[1] : dt[0]);
  if (!(ang > (T)0)) ang += (T)(2.0 * kPiD);
  px = qx[k];
  py = qy[k];
  pz = (T)z2 + m_div(ang * f.c.z2, f.phi2);
  return 1;
}

// Highland width of the projected scattering angle (beta = 1).
template <class T>
__host__ __device__ inline T highland(T p, T x) {
  return m_div((T)13.6, p) * m_sqrt(x) * ((T)1 + (T)0.038 * m_log(x));
}

}  // namespace mu3e
