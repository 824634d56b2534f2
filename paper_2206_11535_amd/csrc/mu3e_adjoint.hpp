// Hand-written adjoint (reverse mode) of the triplet-fit chi2 with respect to
// the nine hit coordinates (Section IV-B, eq. objective-function, as
// evaluated by fit_triplet in mu3e_math.hpp).  The forward part repeats the
// arithmetic of fit_triplet and keeps its intermediates; the reverse sweep
// walks the same steps backwards.  The discrete choices (minor arc, series
// or direct branch, signs) are those of the forward evaluation.
#pragma once

#include "mu3e_math.hpp"

namespace mu3e {

// d/dPhi of the series branch of phicot_minus_2 (float32, Phi <= 1).
template <class T>
__host__ __device__ inline T phicot_series_dphi(T phi) {
  const T x2 = (T)0.25 * phi * phi;
  T s = (T)(6.0 * -2764.0 / 638512875.0);
  s = s * x2 + (T)(5.0 * -4.0 / 93555.0);
  s = s * x2 + (T)(4.0 * -2.0 / 4725.0);
  s = s * x2 + (T)(3.0 * -4.0 / 945.0);
  s = s * x2 + (T)(2.0 * -2.0 / 45.0);
  s = s * x2 + (T)(-2.0 / 3.0);
  return (T)0.5 * phi * s;
}

// chi2 of the triplet (h[0..2] = hit 0 xyz, ...) and w * d chi2 / d h added
// to g[9].  Returns false (g untouched) when the fit is degenerate.
template <class T>
__host__ __device__ inline bool fit_chi2_adjoint(const double* h, const Consts& C, T w, T& chi2_out, double* g) {
  // ------------------------------------------------------------ forward
  const double ax = h[0] - h[3], ay = h[1] - h[4];
  const double bx = h[6] - h[3], by = h[7] - h[4];
  const double ex = h[6] - h[0], ey = h[7] - h[1];
  const double cross = ax * by - ay * bx;
  if (cross == 0.0) return false;
  const double aa = ax * ax + ay * ay, bb = bx * bx + by * by, ee = ex * ex + ey * ey;
  const double sc = cross > 0.0 ? 1.0 : -1.0;
  const double acr = sc * cross;
  const double m1 = bb + ee - aa, m2 = aa + ee - bb;
  const double s1 = m1 >= 0.0 ? 1.0 : -1.0, s2n = m2 >= 0.0 ? 1.0 : -1.0;
  const double n1 = s1 * m1, n2 = s2n * m2;
  const T rho = m_sqrt((T)aa) * m_sqrt((T)bb) * m_sqrt((T)ee) / ((T)2 * (T)acr);
  const T ck[2] = {(T)(n1 / (2.0 * acr)), (T)(n2 / (2.0 * acr))};
  const double phid[2] = {2.0 * atan2(2.0 * acr, n1), 2.0 * atan2(2.0 * acr, n2)};
  const double dz[2] = {h[5] - h[2], h[8] - h[5]};
  const double Kd = dz[0] * phid[1] - dz[1] * phid[0];
  const T phi[2] = {(T)phid[0], (T)phid[1]};
  const T zk[2] = {(T)dz[0], (T)dz[1]};
  T arc[2], len[2], th[2], sth[2], Rk[2], D[2], al[2], gg[2], be[2];
  bool ser[2];
  for (int k = 0; k < 2; ++k) {
    arc[k] = rho * phi[k];
    len[k] = m_sqrt(arc[k] * arc[k] + zk[k] * zk[k]);
    th[k] = m_atan2(arc[k], zk[k]);
    sth[k] = arc[k] / len[k];
    Rk[k] = rho / sth[k];
    D[k] = rho * rho * ck[k] + (T)2 * zk[k] * zk[k] / (phi[k] * phi[k] * phi[k]);
    al[k] = -(T)2 * Rk[k] / D[k];
    ser[k] = sizeof(T) == 4 && phi[k] <= (T)1;
    gg[k] = phicot_minus_2(phi[k], ck[k]);
    be[k] = zk[k] * rho * rho * gg[k] / (D[k] * Rk[k] * Rk[k] * phi[k] * phi[k] * sth[k]);
  }
  const T K = (T)Kd;
  const T Rbar = (T)0.5 * (Rk[0] + Rk[1]);
  const T U = rho * K, V = rho * rho * phi[0] * phi[1] + zk[0] * zk[1];
  const T dth = m_atan2(U, V);
  const T pp = phi[0] * phi[1];
  const T Q = zk[1] * phi[0] + zk[0] * phi[1];
  const T Rs = Rk[0] + Rk[1];
  const T dR = -(T)0.5 * K * Q / (pp * pp * Rs);
  const T phi0 = -(T)0.5 * dR * (al[0] - al[1]);
  const T bphi = -(T)0.5 * (al[0] + al[1]);
  const T th0 = dth - dR * (be[1] + be[0]);
  const T bth = be[1] - be[0];
  const T tm = (T)0.5 * (th[0] + th[1]);
  const T sn = m_sin(tm);
  const T s2 = sn * sn;
  const T p = (T)kCLight * (T)C.b * Rbar;
  const T X = (T)C.xx0 / sn;
  const T lX = m_log(X), sX = m_sqrt(X);
  const T sms = (T)13.6 / p * sX * ((T)1 + (T)0.038 * lX);
  const T sms2 = sms * sms;
  const T den = s2 * bphi * bphi + bth * bth;
  if (!(den > (T)0) || !(sms > (T)0)) return false;
  const T num = phi0 * bth - th0 * bphi;
  const T chi2 = s2 * num * num / (den * sms2);
  chi2_out = chi2;
  // ------------------------------------------------------------ reverse
  const T inv = (T)1 / (den * sms2);
  T g_s2 = w * num * num * inv;
  const T g_num = w * (T)2 * s2 * num * inv;
  const T g_den = -w * chi2 / den;
  const T g_sms2 = -w * chi2 / sms2;
  g_s2 += g_den * bphi * bphi;
  T g_bphi = g_den * (T)2 * s2 * bphi - g_num * th0;
  T g_bth = g_den * (T)2 * bth + g_num * phi0;
  const T g_phi0 = g_num * bth;
  const T g_th0 = -g_num * bphi;
  // sigma_MS(p, X)
  const T g_sms = (T)2 * sms * g_sms2;
  const T g_p = -g_sms * sms / p;
  const T g_X = g_sms * (T)13.6 / (p * sX) * ((T)0.5 * ((T)1 + (T)0.038 * lX) + (T)0.038);
  T g_sn = -g_X * X / sn + g_s2 * (T)2 * sn;
  T g_Rbar = g_p * (T)kCLight * (T)C.b;
  const T g_tm = g_sn * m_cos(tm);
  T g_th[2] = {(T)0.5 * g_tm, (T)0.5 * g_tm};
  // th0 = dth - dR (be1 + be2), bth = be2 - be1
  const T g_dth = g_th0;
  T g_dR = -g_th0 * (be[0] + be[1]);
  T g_be[2] = {-g_th0 * dR - g_bth, -g_th0 * dR + g_bth};
  // phi0 = -dR (al1 - al2) / 2, bphi = -(al1 + al2) / 2
  g_dR += -(T)0.5 * (al[0] - al[1]) * g_phi0;
  T g_al[2] = {-(T)0.5 * dR * g_phi0 - (T)0.5 * g_bphi, (T)0.5 * dR * g_phi0 - (T)0.5 * g_bphi};
  // dR = -K Q / (2 pp^2 Rs)
  T g_K = -(T)0.5 * Q / (pp * pp * Rs) * g_dR;
  const T g_Q = -(T)0.5 * K / (pp * pp * Rs) * g_dR;
  const T g_pp = -(T)2 * dR / pp * g_dR;
  const T g_Rs = -dR / Rs * g_dR;
  T g_phi[2] = {g_Q * zk[1] + g_pp * phi[1], g_Q * zk[0] + g_pp * phi[0]};
  T g_z[2] = {g_Q * phi[1], g_Q * phi[0]};
  T g_R[2] = {g_Rs + (T)0.5 * g_Rbar, g_Rs + (T)0.5 * g_Rbar};
  // dth = atan2(U, V), U = rho K, V = rho^2 phi1 phi2 + z1 z2
  const T uv = U * U + V * V;
  const T g_U = g_dth * V / uv, g_V = -g_dth * U / uv;
  T g_rho = g_U * K + g_V * (T)2 * rho * phi[0] * phi[1];
  g_K += g_U * rho;
  g_phi[0] += g_V * rho * rho * phi[1];
  g_phi[1] += g_V * rho * rho * phi[0];
  g_z[0] += g_V * zk[1];
  g_z[1] += g_V * zk[0];
  T g_c[2] = {0, 0};
  for (int k = 0; k < 2; ++k) {
    // be = z rho^2 g / (D R^2 phi^2 sth)
    const T Db = D[k] * Rk[k] * Rk[k] * phi[k] * phi[k] * sth[k];
    const T g_Nb = g_be[k] / Db;
    const T g_Db = -g_be[k] * be[k] / Db;
    g_z[k] += g_Nb * rho * rho * gg[k];
    g_rho += g_Nb * (T)2 * rho * zk[k] * gg[k];
    const T g_g = g_Nb * zk[k] * rho * rho;
    T g_D = g_Db * Rk[k] * Rk[k] * phi[k] * phi[k] * sth[k];
    g_R[k] += g_Db * D[k] * (T)2 * Rk[k] * phi[k] * phi[k] * sth[k];
    g_phi[k] += g_Db * D[k] * Rk[k] * Rk[k] * (T)2 * phi[k] * sth[k];
    T g_sth = g_Db * D[k] * Rk[k] * Rk[k] * phi[k] * phi[k];
    if (ser[k]) {
      g_phi[k] += g_g * phicot_series_dphi(phi[k]);
    } else {
      g_phi[k] += g_g * ck[k];
      g_c[k] += g_g * phi[k];
    }
    // al = -2 R / D
    g_R[k] += g_al[k] * (-(T)2 / D[k]);
    g_D += -g_al[k] * al[k] / D[k];
    // D = rho^2 cot + 2 z^2 / phi^3
    const T p3 = phi[k] * phi[k] * phi[k];
    g_rho += g_D * (T)2 * rho * ck[k];
    g_c[k] += g_D * rho * rho;
    g_z[k] += g_D * (T)4 * zk[k] / p3;
    g_phi[k] += g_D * (-(T)6 * zk[k] * zk[k] / (p3 * phi[k]));
    // R = rho / sth
    g_rho += g_R[k] / sth[k];
    g_sth += -g_R[k] * Rk[k] / sth[k];
    // sth = arc / len, th = atan2(arc, z), len = sqrt(arc^2 + z^2)
    T g_arc = g_sth / len[k];
    T g_len = -g_sth * sth[k] / len[k];
    const T l2 = len[k] * len[k];
    g_arc += g_th[k] * zk[k] / l2;
    g_z[k] += -g_th[k] * arc[k] / l2;
    g_arc += g_len * arc[k] / len[k];
    g_z[k] += g_len * zk[k] / len[k];
    // arc = rho phi
    g_rho += g_arc * phi[k];
    g_phi[k] += g_arc * rho;
  }
  // ---- float64 primitives
  // K = dz1 phi2 - dz2 phi1
  double gdz[2] = {(double)g_z[0] + (double)g_K * phid[1], (double)g_z[1] - (double)g_K * phid[0]};
  double gphi[2] = {(double)g_phi[0] - (double)g_K * dz[1], (double)g_phi[1] + (double)g_K * dz[0]};
  // phi_k = 2 atan2(2 acr, n_k)
  double g_acr = 0, g_n[2] = {0, 0};
  const double nk[2] = {n1, n2};
  for (int k = 0; k < 2; ++k) {
    const double q = 4.0 * acr * acr + nk[k] * nk[k];
    g_acr += gphi[k] * 4.0 * nk[k] / q;
    g_n[k] += -gphi[k] * 4.0 * acr / q;
    // cot_k = n_k / (2 acr)
    g_n[k] += (double)g_c[k] / (2.0 * acr);
    g_acr += -(double)g_c[k] * nk[k] / (2.0 * acr * acr);
  }
  // rho = sqrt(aa bb ee) / (2 acr)
  const double rhod = (double)rho;
  double g_aa = (double)g_rho * rhod / (2.0 * aa);
  double g_bb = (double)g_rho * rhod / (2.0 * bb);
  double g_ee = (double)g_rho * rhod / (2.0 * ee);
  g_acr += -(double)g_rho * rhod / acr;
  // n1 = |bb + ee - aa|, n2 = |aa + ee - bb|, acr = |cross|
  g_bb += s1 * g_n[0] - s2n * g_n[1];
  g_ee += s1 * g_n[0] + s2n * g_n[1];
  g_aa += -s1 * g_n[0] + s2n * g_n[1];
  const double g_cross = sc * g_acr;
  // squared chords and the cross product
  const double g_ax = 2.0 * ax * g_aa + by * g_cross, g_ay = 2.0 * ay * g_aa - bx * g_cross;
  const double g_bx = 2.0 * bx * g_bb - ay * g_cross, g_by = 2.0 * by * g_bb + ax * g_cross;
  const double g_ex = 2.0 * ex * g_ee, g_ey = 2.0 * ey * g_ee;
  g[0] += g_ax - g_ex;
  g[1] += g_ay - g_ey;
  g[3] += -g_ax - g_bx;
  g[4] += -g_ay - g_by;
  g[6] += g_bx + g_ex;
  g[7] += g_by + g_ey;
  g[2] += -gdz[0];
  g[5] += gdz[0] - gdz[1];
  g[8] += gdz[1];
  return true;
}


// ------------------------------------------------------------- alignment
// theta[s] = (tx, ty, tz, alpha) of sensor s moves a hit to
// R_z(alpha) (x, y, z) + (tx, ty, tz).  Coordinates after alignment are
// formed in float64.  trig[2s], trig[2s + 1] = cos, sin of (double)alpha_s,
// computed once per sensor by the caller (align_trig).
__host__ __device__ inline void align_trig(const float* theta, int s, double* trig) {
  const double a = theta[4 * s + 3];
  trig[2 * s] = cos(a);
  trig[2 * s + 1] = sin(a);
}

__host__ __device__ inline void align_hit(const float* X, const float* Y, const float* Z, const uint16_t* S,
                                          const float* theta, const double* trig, int g, double* h, int& s,
                                          double& ca, double& sa) {
  s = S[g];
  const double tx = theta[4 * s], ty = theta[4 * s + 1], tz = theta[4 * s + 2];
  ca = trig[2 * s];
  sa = trig[2 * s + 1];
  const double x = X[g], y = Y[g];
  h[0] = ca * x - sa * y + tx;
  h[1] = sa * x + ca * y + ty;
  h[2] = (double)Z[g] + tz;
}

// The three aligned hits of triplet tr (global hit indices); false if an
// index or a sensor id is out of range.
__host__ __device__ inline bool align_triplet(const float* X, const float* Y, const float* Z, const uint16_t* S,
                                              int n_hits, int n_sensors, const float* theta, const double* trig,
                                              const int32_t* tr, double* h, int* s, double* ca, double* sa) {
  for (int k = 0; k < 3; ++k) {
    const int g = tr[k];
    if ((unsigned)g >= (unsigned)n_hits) return false;
    if (S[g] >= n_sensors) return false;
    align_hit(X, Y, Z, S, theta, trig, g, h + 3 * k, s[k], ca[k], sa[k]);
  }
  return true;
}

// chi2 of one triplet after alignment (float32 fit); NaN if degenerate.
__host__ __device__ inline float align_chi2_one(const float* X, const float* Y, const float* Z, const uint16_t* S,
                                                int n_hits, int n_sensors, const float* theta,
                                                const double* trig, const int32_t* tr, const Consts& C) {
  double h[9], ca[3], sa[3];
  int s[3];
  if (!align_triplet(X, Y, Z, S, n_hits, n_sensors, theta, trig, tr, h, s, ca, sa)) return __builtin_nanf("");
  const Fit<float> f = fit_triplet<float>(h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7], h[8], C);
  return f.ok ? f.chi2 : __builtin_nanf("");
}

// w * d chi2 / d theta of one triplet: gs[4k..4k+3] for the sensor s[k] of
// hit k.  False (nothing to add) if the triplet is degenerate.
__host__ __device__ inline bool align_grad_one(const float* X, const float* Y, const float* Z, const uint16_t* S,
                                               int n_hits, int n_sensors, const float* theta,
                                               const double* trig, const int32_t* tr, const Consts& C, float w,
                                               int* s, double* gs) {
  double h[9], ca[3], sa[3];
  if (!align_triplet(X, Y, Z, S, n_hits, n_sensors, theta, trig, tr, h, s, ca, sa)) return false;
  double g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float c;
  if (!fit_chi2_adjoint<float>(h, C, w, c, g)) return false;
  for (int k = 0; k < 3; ++k) {
    const double gx = g[3 * k], gy = g[3 * k + 1], gz = g[3 * k + 2];
    const double x0 = X[tr[k]], y0 = Y[tr[k]];
    // d(x', y') / d alpha of the rotated hit
    const double dxa = -sa[k] * x0 - ca[k] * y0, dya = ca[k] * x0 - sa[k] * y0;
    gs[4 * k] = gx;
    gs[4 * k + 1] = gy;
    gs[4 * k + 2] = gz;
    gs[4 * k + 3] = gx * dxa + gy * dya;
  }
  return true;
}

}  // namespace mu3e
