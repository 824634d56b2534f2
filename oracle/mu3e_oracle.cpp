// FP64 reference ("oracle") for the Mu3e online event selection.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
// link or call this file; only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark use it.  It shares no code with the GPU path.
//
// It follows the paper (arXiv 2206.11535, "Online Event Selection for Mu3e
// using GPUs") step by step, in double precision, by brute force:
//   Section IV-A  Selection Cuts       eq. sel-cut-delta-lambda, eq. sel-cut-phi,
//                                      eq. rt-cut; Alg. 2
//   Section IV-B  Track Reconstruction eq. objective-function,
//                                      eq. objective-function-global, the
//                                      weighted mean curvature; Alg. 3
//   Section IV-C  Vertex Fit           the weighted 2D vertex, eq. track-error,
//                                      the z back-projection, the vertex chi2;
//                                      Alg. 4
//   Section V-B   frame flow and the rule that an overflowing frame is kept; Alg. 1
// Readings of silent or garbled passages are listed in the design notes and
// repeated at the function that applies them.
//
// Every function that decides something also reports whether the decision is
// *ambiguous*: a tested quantity lies within a relative distance `amb` (1e-5)
// of a window edge, or an argmin has a near-tie.  The parity comparator drops
// ambiguous candidates and everything derived from them.
//
// The scalar type of the triplet fit is a template parameter so that the same
// code yields exact gradients with forward-mode dual numbers (Dual<N>).
//
// Parity pins (closed forms, invariants, noiseless helices, brute force) live
// in the test-suite; see the header of each section for what pins it.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#include <limits>
#include <omp.h>

namespace {

const double kC = 0.299792458;      // p[MeV] = kC * B[T] * R[mm]
const double kMe = 0.51099895;      // MeV
const double kMmu = 105.6583755;    // MeV
const double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ dual
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0; }
};
template <int N> Dual<N> mk(double v, const double* d) { Dual<N> r(v); for (int i = 0; i < N; ++i) r.d[i] = d[i]; return r; }
template <int N> Dual<N> chain(const Dual<N>& a, double v, double da) {
  Dual<N> r(v); for (int i = 0; i < N; ++i) r.d[i] = da * a.d[i]; return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v + b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v - b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r(-a.v); for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v * b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v / b.v); for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> bool operator<(const Dual<N>& a, double b) { return a.v < b; }
template <int N> bool operator>(const Dual<N>& a, double b) { return a.v > b; }
template <int N> bool operator==(const Dual<N>& a, double b) { return a.v == b; }
template <int N> Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> Dual<N> asin(const Dual<N>& a) { return chain(a, std::asin(a.v), 1.0 / std::sqrt(1.0 - a.v * a.v)); }
template <int N> Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }
template <int N> Dual<N> atan2(const Dual<N>& y, const Dual<N>& x) {
  double den = x.v * x.v + y.v * y.v;
  Dual<N> r(std::atan2(y.v, x.v));
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
  return r;
}
inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

// ------------------------------------------------------------------ params
struct Params {
  double r_layer[4], z_half[4], b, xx0, sigma_pix;
  double win[8];            // dlambda lo,hi; cosphi01 lo,hi; cosphi12 lo,hi; |rtc| lo,hi
  double chi2_track_max;
  int max_triplets, max_tracks, max_combos, max_layer_hits;
  double de_max, r_target, target_tol, chi2_vertex_max, d_target_max, p_sum_max;
  double amb;
};

enum { KEEP = 1u, TRIPLET_OVF = 2u, TRACK_OVF = 4u, COMBO_OVF = 8u, VERTEX = 16u, HITS_OVF = 32u };

// Decision with ambiguity: 1 sure pass, 0 sure fail, -1 ambiguous.
inline bool near_edge(double q, double e, double amb) { return std::fabs(q - e) <= amb * std::fabs(e); }
inline int window(double q, double lo, double hi, double amb) {
  if (near_edge(q, lo, amb) || near_edge(q, hi, amb)) return -1;
  return (q >= lo && q <= hi) ? 1 : 0;
}
// Conjunction of three-valued decisions: any sure fail -> fail; else any
// ambiguous -> ambiguous; else pass.
inline int conj(int a, int b) { if (a == 0 || b == 0) return 0; if (a < 0 || b < 0) return -1; return 1; }

inline double highland(double p, double x) {   // projected MS angle, beta = 1
  return 13.6 / p * std::sqrt(x) * (1.0 + 0.038 * std::log(x));
}

// ============================================================ Selection Cuts
// Section IV-A.  The detector is four concentric cylinders: in tan(lambda) and
// cos(Phi) the transverse radius of a hit is the nominal layer radius (the
// text's subscript r_{r,i} is read as r_{t,i}, a typo).  d_ij in eq. rt-cut are
// transverse distances because r_{t,c} is a transverse radius.  The sign of
// r_{t,c} follows the cross product (h0-h1) x (h2-h1): positive for clockwise
// (positive charge in B along +z).
// Pins: circumradius closed form, straight-line special case, rotation /
// z-translation invariance, mirror symmetry (tests/test_oracle_cuts.py).
struct CutQ { double dlambda, cosphi01, cosphi12, rtc; };

CutQ cut_quantities(const double* h0, const double* h1, const double* h2, const Params& P) {
  CutQ q;
  const double R0 = P.r_layer[0], R1 = P.r_layer[1], R2 = P.r_layer[2];
  double tl01 = (h1[2] - h0[2]) / (R1 - R0);           // tan(lambda_01)
  double tl12 = (h2[2] - h1[2]) / (R2 - R1);           // tan(lambda_12)
  q.dlambda = tl12 - tl01;                             // eq. sel-cut-delta-lambda
  q.cosphi01 = (h0[0] * h1[0] + h0[1] * h1[1]) / (R0 * R1);   // eq. sel-cut-phi
  q.cosphi12 = (h1[0] * h2[0] + h1[1] * h2[1]) / (R1 * R2);
  double cross = (h0[0] - h1[0]) * (h2[1] - h1[1]) - (h0[1] - h1[1]) * (h2[0] - h1[0]);
  double d01 = std::hypot(h0[0] - h1[0], h0[1] - h1[1]);
  double d12 = std::hypot(h1[0] - h2[0], h1[1] - h2[1]);
  double d20 = std::hypot(h2[0] - h0[0], h2[1] - h0[1]);
  q.rtc = (cross == 0.0) ? std::numeric_limits<double>::infinity()
                         : d01 * d12 * d20 / (2.0 * cross);   // eq. rt-cut
  return q;
}

int cut_decision(const CutQ& q, const Params& P) {
  int a = window(q.dlambda, P.win[0], P.win[1], P.amb);
  int b = window(q.cosphi01, P.win[2], P.win[3], P.amb);
  int c = window(q.cosphi12, P.win[4], P.win[5], P.amb);
  int d = std::isinf(q.rtc) ? 0 : window(std::fabs(q.rtc), P.win[6], P.win[7], P.amb);
  return conj(conj(a, b), conj(c, d));
}

// ========================================================== Triplet fit
// Section IV-B, "Single Triplet Fit".  The paper gives the objective
// chi2 = Phi_MS^2/sigma_Phi^2 + Theta_MS^2/sigma_Theta^2 with
// sigma_Theta^2 = sigma_MS^2 and sigma_Phi^2 = sigma_MS^2 / sin^2(.), and the
// method: linearise around the transverse circle through the three hits
// (Phi_MS = 0) with a first-order Taylor expansion.  Reading (the formulas
// themselves are not printed):
//   * fit parameter: the 3D radius R = p / (kC B); kappa = 1/R;
//   * per arc k (h0->h1, h1->h2) with transverse chord d_k and longitudinal
//     step z_k: R^2 = d_k^2 / (4 sin^2(Phi_k/2)) + z_k^2 / Phi_k^2; at the
//     circle solution (transverse radius rho = |r_tc|) Phi_Ck = 2 asin(d_k/2rho),
//     theta_Ck = atan2(rho Phi_Ck, z_k), R_Ck = rho / sin(theta_Ck);
//   * Phi_MS(R) = -(1/2) sum_k dPhi_k/dR (R - R_Ck),
//     Theta_MS(R) = theta_2(R) - theta_1(R), both to first order, centred at
//     Rbar_C = (R_C1 + R_C2)/2;
//   * the sin^2 in sigma_Phi is the polar angle (mean of the arcs' theta);
//   * sigma_MS is the Highland width for p = kC B Rbar_C and thickness
//     x/X0 / sin(theta), held fixed in the minimisation.
// Pins: noiseless helix -> R* = R_true exactly and chi2 = 0; the exact
// nonlinear minimum agrees to second order in the kink; pulls ~ N(0,1).
template <class T>
struct Fit {
  T kappa, sigma2_kappa, chi2, r_star, sigma2_r;
  T rtc, theta1, theta2, phi1, phi2, rbar_c, sigma_ms;
  T cx, cy;                 // circumcentre
  int sgn;
};

template <class T>
bool triplet_fit(const T* h0, const T* h1, const T* h2, const Params& P, Fit<T>& o) {
  using std::sqrt; using std::sin; using std::cos; using std::log; using std::asin;
  using std::atan2; using std::fabs;
  T ax = h0[0] - h1[0], ay = h0[1] - h1[1];
  T bx = h2[0] - h1[0], by = h2[1] - h1[1];
  T cross = ax * by - ay * bx;
  if (val(cross) == 0.0) return false;
  T d1 = sqrt((h1[0] - h0[0]) * (h1[0] - h0[0]) + (h1[1] - h0[1]) * (h1[1] - h0[1]));
  T d2 = sqrt((h2[0] - h1[0]) * (h2[0] - h1[0]) + (h2[1] - h1[1]) * (h2[1] - h1[1]));
  T d3 = sqrt((h0[0] - h2[0]) * (h0[0] - h2[0]) + (h0[1] - h2[1]) * (h0[1] - h2[1]));
  T rtc = d1 * d2 * d3 / (2.0 * cross);
  o.rtc = rtc;
  o.sgn = val(rtc) > 0 ? 1 : -1;
  T rho = fabs(rtc);
  // circumcentre relative to h1
  T aa = ax * ax + ay * ay, bb = bx * bx + by * by;
  T D = 2.0 * cross;
  o.cx = h1[0] + (by * aa - ay * bb) / D;
  o.cy = h1[1] + (ax * bb - bx * aa) / D;
  T dk[2] = {d1, d2};
  T zk[2] = {h1[2] - h0[2], h2[2] - h1[2]};
  T Phi[2], th[2], Rk[2], al[2], be[2];
  for (int k = 0; k < 2; ++k) {
    T s = dk[k] / (2.0 * rho);
    if (val(s) > 1.0) s = T(1.0);
    Phi[k] = 2.0 * asin(s);
    T sk = rho * Phi[k];
    th[k] = atan2(sk, zk[k]);
    Rk[k] = rho / sin(th[k]);
    T half = Phi[k] / 2.0;
    T cot = cos(half) / sin(half);
    al[k] = -2.0 * Rk[k] / (rho * rho * cot + 2.0 * zk[k] * zk[k] / (Phi[k] * Phi[k] * Phi[k]));
    be[k] = zk[k] * (Phi[k] + Rk[k] * al[k]) / (Rk[k] * Rk[k] * Phi[k] * Phi[k] * sin(th[k]));
  }
  T Rbar = (Rk[0] + Rk[1]) / 2.0;
  T Phi0 = -0.5 * (al[0] * (Rbar - Rk[0]) + al[1] * (Rbar - Rk[1]));
  T bPhi = -0.5 * (al[0] + al[1]);
  T Th0 = (th[1] - th[0]) + be[1] * (Rbar - Rk[1]) - be[0] * (Rbar - Rk[0]);
  T bTh = be[1] - be[0];
  T thbar = (th[0] + th[1]) / 2.0;
  T sn = sin(thbar);
  T s2 = sn * sn;
  T p = kC * P.b * Rbar;
  T X = P.xx0 / sn;
  T sms = 13.6 / p * sqrt(X) * (1.0 + 0.038 * log(X));
  T den = s2 * bPhi * bPhi + bTh * bTh;
  if (!(val(den) > 0.0)) return false;
  T delta = -(s2 * Phi0 * bPhi + Th0 * bTh) / den;
  T num = Phi0 * bTh - Th0 * bPhi;
  o.r_star = Rbar + delta;
  o.sigma2_r = sms * sms / den;
  o.chi2 = s2 * num * num / (den * sms * sms);
  o.kappa = (double)o.sgn / o.r_star;
  T r2 = o.r_star * o.r_star;
  o.sigma2_kappa = o.sigma2_r / (r2 * r2);
  o.theta1 = th[0]; o.theta2 = th[1]; o.phi1 = Phi[0]; o.phi2 = Phi[1];
  o.rbar_c = Rbar; o.sigma_ms = sms;
  return true;
}

// ============================================================ Extension
// Section IV-B, "Triplets Fit": the preliminary helix of the first triplet
// predicts the layer-3 position; the closest layer-3 hit forms the second
// triplet.  Reading: the helix is the transverse circumcircle with the z
// slope of arc 2 per radian of turning; the predicted point is the first
// crossing of r = R3 reached going forward from h2; the nearest hit is by 3D
// Euclidean distance with no search window; ties go to the lowest index.
// Returns false if the circle never reaches r = R3.
bool predict_l3(const double* h1, const double* h2, const Fit<double>& f, const Params& P, double* out,
                int* amb) {
  double R3 = P.r_layer[3];
  double cx = f.cx, cy = f.cy, rho = std::fabs(f.rtc);
  double cn = std::hypot(cx, cy);
  if (amb && (near_edge(cn, rho + R3, P.amb) || near_edge(cn, std::fabs(rho - R3), P.amb))) *amb = 1;
  if (cn == 0.0 || cn > rho + R3 || cn < std::fabs(rho - R3)) return false;
  double a = (R3 * R3 - rho * rho + cn * cn) / (2.0 * cn);
  double hh = std::sqrt(std::max(R3 * R3 - a * a, 0.0));
  double ex = cx / cn, ey = cy / cn;
  double best = 1e300, bx = 0, by = 0;
  for (int s = -1; s <= 1; s += 2) {
    double px = a * ex - s * hh * ey, py = a * ey + s * hh * ex;
    double psi_p = std::atan2(py - cy, px - cx);
    double psi_2 = std::atan2(h2[1] - cy, h2[0] - cx);
    double dphi = (f.sgn > 0) ? psi_2 - psi_p : psi_p - psi_2;   // clockwise for positive
    dphi = std::fmod(dphi, 2 * kPi);
    if (dphi <= 0) dphi += 2 * kPi;
    if (dphi < best) { best = dphi; bx = px; by = py; }
  }
  out[0] = bx; out[1] = by;
  out[2] = h2[2] + best * (h2[2] - h1[2]) / f.phi2;
  return true;
}

// Section IV-B, "Triplets Fit": the two triplet fits of a track combined.
// The curvature is the mean of the two kappas weighted by 1/sigma^2_kappa;
// chi2_global is the sum over both triplets of their quadratic chi2 (the
// minimum plus the curvature term) evaluated at Rbar = 1/|kbar| (eq.
// objective-function-global read as a function of the curvature).
void combine_fits(const Fit<double>& f1, const Fit<double>& f2, double& kbar, double& chi2) {
  double w1 = 1 / f1.sigma2_kappa, w2 = 1 / f2.sigma2_kappa;
  kbar = (f1.kappa * w1 + f2.kappa * w2) / (w1 + w2);
  double rbar = 1 / std::fabs(kbar);
  chi2 = f1.chi2 + (rbar - f1.r_star) * (rbar - f1.r_star) / f1.sigma2_r
       + f2.chi2 + (rbar - f2.r_star) * (rbar - f2.r_star) / f2.sigma2_r;
}

// ============================================================ Vertex
// Section IV-C.  Per-track circle: r_t = Rbar sin(theta_C1) (first arc),
// centre on the bending side of the h0-h1 chord.  sigma_MS at layer 0 from
// Highland with the track momentum.
struct Track {
  int hit[4];
  int charge;
  double kbar, chi2, rbar;
  double theta1, rt, cx, cy, sms0, E, p;
  const double* h0;   // layer-0 hit xyz
};

void track_circle(Track& t, const double* h0, const double* h1, const Params& P) {
  double dx = h1[0] - h0[0], dy = h1[1] - h0[1];
  double d = std::hypot(dx, dy);
  double rt = t.rbar * std::sin(t.theta1);
  if (rt < d / 2) rt = d / 2;
  double hh = std::sqrt(std::max(rt * rt - d * d / 4, 0.0));
  double ux = dx / d, uy = dy / d;
  double nx = uy, ny = -ux;          // right-hand normal of the motion
  double sg = t.charge > 0 ? 1.0 : -1.0;
  t.rt = rt;
  t.cx = (h0[0] + h1[0]) / 2 + sg * hh * nx;
  t.cy = (h0[1] + h1[1]) / 2 + sg * hh * ny;
  t.p = kC * P.b * t.rbar;
  t.E = std::sqrt(t.p * t.p + kMe * kMe);
  t.sms0 = highland(t.p, P.xx0 / std::sin(t.theta1));
  t.h0 = h0;
}

// A track given by its four hits (layers 0..3): both triplet fits, their
// combination and the transverse circle.  False if a fit fails.
bool track_from_hits(const double* q, const Params& P, Track& t) {
  Fit<double> f1, f2;
  if (!triplet_fit(q, q + 3, q + 6, P, f1) || !triplet_fit(q + 3, q + 6, q + 9, P, f2)) return false;
  double chi2;
  combine_fits(f1, f2, t.kbar, chi2);
  t.chi2 = chi2;
  t.charge = t.kbar > 0 ? 1 : -1;
  t.rbar = 1 / std::fabs(t.kbar);
  t.theta1 = f1.theta1;
  track_circle(t, q, q + 3, P);
  return true;
}

// turning angle travelled backwards from the layer-0 hit to point q
double back_angle(const Track& t, double qx, double qy) {
  double ps_q = std::atan2(qy - t.cy, qx - t.cx);
  double ps_0 = std::atan2(t.h0[1] - t.cy, t.h0[0] - t.cx);
  double d = (t.charge > 0) ? ps_q - ps_0 : ps_0 - ps_q;  // forward is clockwise for e+
  d = std::fmod(d, 2 * kPi);
  if (d < 0) d += 2 * kPi;
  return d;
}

double point_sigma2(const Track& t, double qx, double qy, const Params& P) {
  double s = t.rt * back_angle(t, qx, qy);                 // eq. track-error
  return t.sms0 * t.sms0 * s * s + P.sigma_pix * P.sigma_pix;
}

// distance in the (rho, z) half plane from (r, z) to the double-cone surface
double cone_distance(double r, double z, const Params& P) {
  double best = 1e300;
  for (int s = -1; s <= 1; s += 2) {
    double ax = P.r_target, az = 0.0, bx = 0.0, bz = s * 50.0;
    double vx = bx - ax, vz = bz - az;
    double t = ((r - ax) * vx + (z - az) * vz) / (vx * vx + vz * vz);
    t = std::min(1.0, std::max(0.0, t));
    double dx = r - (ax + t * vx), dz = z - (az + t * vz);
    best = std::min(best, std::hypot(dx, dz));
  }
  return best;
}

struct VertexOut { int pass; int amb; double x, y, z, chi2, dt, psum; int reached; };

// One e+ e+ e- track triple (Section IV-C, "Finding Possible Event Vertices"
// and "Signal Estimation").  Reports the minimum-chi2 passing combination.
VertexOut vertex_triple(const Track* T[3], const Params& P) {
  VertexOut r{0, 0, 0, 0, 0, std::numeric_limits<double>::infinity(), 0, 0, 0};
  const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  double px[3][2], py[3][2];
  int np[3];
  for (int k = 0; k < 3; ++k) {
    const Track& A = *T[pr[k][0]];
    const Track& B = *T[pr[k][1]];
    double dx = B.cx - A.cx, dy = B.cy - A.cy;
    double d = std::hypot(dx, dy);
    double sum = A.rt + B.rt, dif = std::fabs(A.rt - B.rt);
    if (near_edge(d, sum, P.amb) || (dif > 0 && near_edge(d, dif, P.amb))) r.amb = 1;
    if (d == 0.0 || d > sum || d < dif) return r;          // circles do not meet
    double a = (A.rt * A.rt - B.rt * B.rt + d * d) / (2 * d);
    double h = std::sqrt(std::max(A.rt * A.rt - a * a, 0.0));
    double ex = dx / d, ey = dy / d;
    np[k] = 0;
    for (int s = -1; s <= 1; s += 2) {
      double qx = A.cx + a * ex - s * h * ey, qy = A.cy + a * ey + s * h * ex;
      double lim = P.r_target + P.target_tol;
      double rq = std::hypot(qx, qy);
      if (near_edge(rq, lim, P.amb)) r.amb = 1;
      if (rq <= lim) { px[k][np[k]] = qx; py[k][np[k]] = qy; ++np[k]; }
    }
    if (np[k] == 0) return r;                                // none near target
  }
  r.reached = 1;
  for (int i0 = 0; i0 < np[0]; ++i0)
  for (int i1 = 0; i1 < np[1]; ++i1)
  for (int i2 = 0; i2 < np[2]; ++i2) {
    int sel[3] = {i0, i1, i2};
    double sw = 0, mx = 0, my = 0;
    for (int k = 0; k < 3; ++k) {
      double qx = px[k][sel[k]], qy = py[k][sel[k]];
      double s2 = 0.5 * (point_sigma2(*T[pr[k][0]], qx, qy, P) + point_sigma2(*T[pr[k][1]], qx, qy, P));
      sw += 1 / s2; mx += qx / s2; my += qy / s2;
    }
    mx /= sw; my /= sw;                                      // mu_t
    double cax[3], cay[3], zz[3], sg2[3];
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const Track& t = *T[k];
      double vx = mx - t.cx, vy = my - t.cy;
      double vn = std::hypot(vx, vy);
      if (vn == 0.0) { ok = false; break; }
      cax[k] = t.cx + t.rt * vx / vn;                        // point of closest approach
      cay[k] = t.cy + t.rt * vy / vn;
      double dphi = back_angle(t, cax[k], cay[k]);
      zz[k] = t.h0[2] - dphi * t.rbar * std::cos(t.theta1);  // z back-projection
      sg2[k] = point_sigma2(t, cax[k], cay[k], P);
    }
    if (!ok) continue;
    double wz = 0, mz = 0;
    for (int k = 0; k < 3; ++k) { wz += 1 / sg2[k]; mz += zz[k] / sg2[k]; }
    mz /= wz;
    double chi2 = 0;
    for (int k = 0; k < 3; ++k) {
      double dx = cax[k] - mx, dy = cay[k] - my, dz = zz[k] - mz;
      chi2 += (dx * dx + dy * dy + dz * dz) / sg2[k];
    }
    double dt = cone_distance(std::hypot(mx, my), mz, P);
    double sx = 0, sy = 0, sz = 0;
    for (int k = 0; k < 3; ++k) {
      const Track& t = *T[k];
      double ux = (cax[k] - t.cx) / t.rt, uy = (cay[k] - t.cy) / t.rt;
      double tx = t.charge > 0 ? uy : -uy, ty = t.charge > 0 ? -ux : ux;   // travel direction
      double pt = kC * P.b * t.rt;
      sx += pt * tx; sy += pt * ty; sz += t.p * std::cos(t.theta1);
    }
    double psum = std::sqrt(sx * sx + sy * sy + sz * sz);
    if (near_edge(chi2, P.chi2_vertex_max, P.amb) || near_edge(dt, P.d_target_max, P.amb) ||
        near_edge(psum, P.p_sum_max, P.amb)) r.amb = 1;
    bool pass = chi2 <= P.chi2_vertex_max && dt <= P.d_target_max && psum <= P.p_sum_max;
    if (pass) {
      if (r.pass && near_edge(chi2, r.chi2, P.amb)) r.amb = 1;   // reported-vertex near-tie
      if (!r.pass || chi2 < r.chi2) { r.x = mx; r.y = my; r.z = mz; r.chi2 = chi2; r.dt = dt; r.psum = psum; }
      r.pass = 1;
    }
  }
  return r;
}

// ============================================================ Refined vertex
// Section VII names a more precise vertex reconstruction than the rough
// estimate of Section IV-C as the next step; the paper gives no formula.
// Reading taken here: the refined vertex of an e+ e+ e- triple is the point v
// that minimises
//     J(v, phi) = sum_k |H_k(phi_k) - v|^2 / sigma_k^2
// jointly over v and one turning angle phi_k per track.  H_k(phi) is the point
// of track k's helix reached after turning phi backwards (in the transverse
// plane) from its layer-0 hit; sigma_k^2 is eq. track-error's variance at the
// track's point of closest approach to the rough estimate, held fixed during
// the minimisation.  Only triples whose rough estimate passes the three signal
// tests are refined, starting from that estimate and its closest-approach
// angles.  J has 9 - 6 = 3 degrees of freedom.
// The minimiser is found by Levenberg-Marquardt on the nine weighted
// residuals, with a central-difference Jacobian and a Gaussian-elimination
// solve: slow and plain.
// Pins: noiseless decays (exact vertex), a displaced third track against the
// closed-form vertex of three weighted straight lines, an independent solver
// from the same start, rotation and z-translation invariance
// (tests/test_oracle_refine.py).

// Point of track t after turning phi backwards from its layer-0 hit.
void helix_point(const Track& t, double phi, double* p) {
  double ps0 = std::atan2(t.h0[1] - t.cy, t.h0[0] - t.cx);
  double ps = ps0 + (t.charge > 0 ? phi : -phi);     // backwards of a clockwise (e+) track is ccw
  p[0] = t.cx + t.rt * std::cos(ps);
  p[1] = t.cy + t.rt * std::sin(ps);
  p[2] = t.h0[2] - phi * t.rbar * std::cos(t.theta1);
}

// Weighted residuals of J at x = (v, phi_0, phi_1, phi_2): r[3k + i].
void refine_residual(const Track* T[3], const double* s2, const double* x, double* r) {
  for (int k = 0; k < 3; ++k) {
    double p[3];
    helix_point(*T[k], x[3 + k], p);
    double sk = std::sqrt(s2[k]);
    for (int i = 0; i < 3; ++i) r[3 * k + i] = (p[i] - x[i]) / sk;
  }
}

double sumsq9(const double* r) { double s = 0; for (int i = 0; i < 9; ++i) s += r[i] * r[i]; return s; }

// Solve the n x n system A d = b in place by Gaussian elimination with
// partial pivoting; false if A is singular.
bool gauss_solve(double* A, double* b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r) if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = b[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
    b[c] = s / A[c * n + c];
  }
  return true;
}

struct RefineOut { int status, iters; double x[6], J, s2[3]; VertexOut rough; };

// status: 1 converged, 0 the rough estimate does not pass, -1 no convergence.
RefineOut refine_triple(const Track* T[3], const Params& P) {
  RefineOut o{};
  o.rough = vertex_triple(T, P);
  if (!o.rough.pass) return o;
  double x[6] = {o.rough.x, o.rough.y, o.rough.z, 0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    const Track& t = *T[k];
    double vx = o.rough.x - t.cx, vy = o.rough.y - t.cy, vn = std::hypot(vx, vy);
    double cax = t.cx + t.rt * vx / vn, cay = t.cy + t.rt * vy / vn;   // closest approach
    x[3 + k] = back_angle(t, cax, cay);
    o.s2[k] = point_sigma2(t, cax, cay, P);
  }
  double r[9], J, lam = 1e-3;
  refine_residual(T, o.s2, x, r);
  J = sumsq9(r);
  o.status = -1;
  for (int it = 1; it <= 500; ++it) {
    double Jac[9][6];
    for (int j = 0; j < 6; ++j) {                        // central differences
      double h = j < 3 ? 1e-6 : 1e-7, xp[6], xm[6], rp[9], rm[9];
      for (int i = 0; i < 6; ++i) xp[i] = xm[i] = x[i];
      xp[j] += h; xm[j] -= h;
      refine_residual(T, o.s2, xp, rp);
      refine_residual(T, o.s2, xm, rm);
      for (int i = 0; i < 9; ++i) Jac[i][j] = (rp[i] - rm[i]) / (2 * h);
    }
    double A[36], g[6];
    for (int a = 0; a < 6; ++a) {
      g[a] = 0;
      for (int i = 0; i < 9; ++i) g[a] += Jac[i][a] * r[i];
      for (int b = 0; b < 6; ++b) {
        double s = 0;
        for (int i = 0; i < 9; ++i) s += Jac[i][a] * Jac[i][b];
        A[a * 6 + b] = s;
      }
    }
    bool accepted = false, tiny = false;
    while (lam < 1e16) {
      double M[36], d[6];
      for (int i = 0; i < 36; ++i) M[i] = A[i];
      for (int a = 0; a < 6; ++a) { M[a * 6 + a] *= 1 + lam; d[a] = -g[a]; }
      if (!gauss_solve(M, d, 6)) { lam *= 10; continue; }
      double dv = std::max({std::fabs(d[0]), std::fabs(d[1]), std::fabs(d[2])});
      double dp = std::max({std::fabs(d[3]), std::fabs(d[4]), std::fabs(d[5])});
      if (dv < 1e-10 && dp < 1e-12) { tiny = true; break; }   // converged: the step vanishes
      double xn[6], rn[9];
      for (int a = 0; a < 6; ++a) xn[a] = x[a] + d[a];
      refine_residual(T, o.s2, xn, rn);
      double Jn = sumsq9(rn);
      if (Jn <= J) {
        for (int a = 0; a < 6; ++a) x[a] = xn[a];
        for (int i = 0; i < 9; ++i) r[i] = rn[i];
        J = Jn;
        lam = std::max(lam / 10, 1e-12);
        accepted = true;
        break;
      }
      lam *= 10;
    }
    o.iters = it;
    if (tiny) { o.status = 1; break; }
    if (!accepted) break;                                // no descent left but the step is not small
  }
  for (int a = 0; a < 6; ++a) o.x[a] = x[a];
  o.J = J;
  return o;
}

// ============================================================ per frame
struct TripRec { int f, h[3]; double rtc; int pass, amb; };
struct TrackRec { int f, h[4]; int charge; double kbar, chi2; int pass, amb; };
struct TripleRec { int f, t[3][3]; int pass, amb; };
struct Stats { long long combos, pairs01, pairs12, joins, fits, tracks_tested; };

struct FrameOut {
  uint32_t flags, amb;         // amb bits use the flag bit positions
  int32_t counts[3], namb[3];
  double vtx[4];
  std::vector<TripRec> trips;
  std::vector<TrackRec> tracks;
  std::vector<TripleRec> triples;
  Stats st;
};

void process_frame(int f, const float* X, const float* Y, const float* Z, const int32_t* lo,
                   const Params& P, FrameOut& out, bool want_lists) {
  out.flags = 0; out.amb = 0;
  out.counts[0] = out.counts[1] = out.counts[2] = 0;
  out.namb[0] = out.namb[1] = out.namb[2] = 0;
  for (int i = 0; i < 4; ++i) out.vtx[i] = std::numeric_limits<double>::quiet_NaN();
  std::memset(&out.st, 0, sizeof(out.st));
  int b[5];
  for (int l = 0; l <= 4; ++l) b[l] = lo[4 * f + l];
  for (int l = 0; l < 4; ++l)
    if (b[l + 1] - b[l] > P.max_layer_hits) { out.flags = HITS_OVF | KEEP; return; }
  auto H = [&](int i, double* h) { h[0] = X[i]; h[1] = Y[i]; h[2] = Z[i]; };
  // ---- Selection Cuts (Alg. 2): brute force over all n0*n1*n2 combinations
  struct Cand { int h[3]; double rtc; int amb; };
  std::vector<Cand> sel;
  int n_amb_trip = 0;
  for (int i0 = b[0]; i0 < b[1]; ++i0)
  for (int i1 = b[1]; i1 < b[2]; ++i1)
  for (int i2 = b[2]; i2 < b[3]; ++i2) {
    double h0[3], h1[3], h2[3];
    H(i0, h0); H(i1, h1); H(i2, h2);
    CutQ q = cut_quantities(h0, h1, h2, P);
    int d = cut_decision(q, P);
    out.st.combos++;
    if (d < 0) ++n_amb_trip;
    if (d != 0) sel.push_back({{i0, i1, i2}, q.rtc, d < 0});
    if (want_lists && d != 0) out.trips.push_back({f, {i0, i1, i2}, q.rtc, d > 0 ? 1 : 0, d < 0 ? 1 : 0});
  }
  int n_pass = 0;
  for (auto& c : sel) n_pass += c.amb ? 0 : 1;
  out.counts[0] = n_pass;                      // sure passes (ambiguous ones excluded)
  out.namb[0] = n_amb_trip;
  // count semantics: exact; overflow iff count > cap (Section VI-B compares the
  // count against the cap of 768 with a strict inequality)
  int lo_cnt = n_pass, hi_cnt = n_pass + n_amb_trip;
  if (lo_cnt > P.max_triplets) out.flags |= TRIPLET_OVF;
  if (n_amb_trip) out.amb |= TRIPLET_OVF | TRACK_OVF | COMBO_OVF | VERTEX;   // descendants excused
  if (hi_cnt > P.max_triplets && lo_cnt <= P.max_triplets) out.amb |= TRIPLET_OVF;
  if (out.flags & TRIPLET_OVF) { out.flags |= KEEP; return; }
  // ---- Track Reconstruction (Alg. 3)
  std::vector<Track> tracks;
  int n_amb_trk = 0;
  for (auto& c : sel) {
    double h0[3], h1[3], h2[3];
    H(c.h[0], h0); H(c.h[1], h1); H(c.h[2], h2);
    Fit<double> f1;
    out.st.fits++;
    if (!triplet_fit(h0, h1, h2, P, f1)) continue;
    double pr[3];
    int pamb = 0;
    bool reach = predict_l3(h1, h2, f1, P, pr, &pamb);
    if (!reach) {
      if (pamb || c.amb) {                                   // could have reached: excuse
        if (want_lists) out.tracks.push_back({f, {c.h[0], c.h[1], c.h[2], -1}, f1.sgn, 0.0, 0.0, 0, 1});
        ++n_amb_trk;
      }
      continue;
    }
    int best = -1; double bd = 1e300, second = 1e300;
    for (int i3 = b[3]; i3 < b[4]; ++i3) {
      double dx = X[i3] - pr[0], dy = Y[i3] - pr[1], dz = Z[i3] - pr[2];
      double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < bd) { second = bd; bd = d2; best = i3; }
      else if (d2 < second) second = d2;
    }
    if (best < 0) continue;                                  // empty layer 3
    bool amb = c.amb || pamb || (second - bd <= P.amb * second);
    double h3[3];
    H(best, h3);
    Fit<double> f2;
    out.st.fits++;
    out.st.tracks_tested++;
    if (!triplet_fit(h1, h2, h3, P, f2)) continue;
    if (f2.sgn != f1.sgn) continue;                          // opposite bending: reject
    double kbar, chi2;
    combine_fits(f1, f2, kbar, chi2);
    double rbar = 1 / std::fabs(kbar);
    if (near_edge(chi2, P.chi2_track_max, P.amb)) amb = true;
    bool pass = chi2 < P.chi2_track_max;                     // strict (Section IV-B)
    if (want_lists && (pass || amb))
      out.tracks.push_back({f, {c.h[0], c.h[1], c.h[2], best}, f1.sgn, kbar, chi2, pass ? 1 : 0, amb ? 1 : 0});
    if (amb) { ++n_amb_trk; continue; }
    if (!pass) continue;
    Track t;
    t.hit[0] = c.h[0]; t.hit[1] = c.h[1]; t.hit[2] = c.h[2]; t.hit[3] = best;
    t.charge = kbar > 0 ? 1 : -1;
    t.kbar = kbar; t.chi2 = chi2; t.rbar = rbar; t.theta1 = f1.theta1;
    tracks.push_back(t);
  }
  out.counts[1] = (int)tracks.size();
  out.namb[1] = n_amb_trk;
  if (n_amb_trk) out.amb |= TRACK_OVF | COMBO_OVF | VERTEX;
  if ((int)tracks.size() > P.max_tracks) out.flags |= TRACK_OVF;
  if (out.flags & TRACK_OVF) { out.flags |= KEEP; return; }
  // ---- Vertex Fit (Alg. 4)
  std::vector<double> hb(tracks.size() * 6);
  for (size_t k = 0; k < tracks.size(); ++k) {
    double* h0 = &hb[6 * k];
    double* h1 = h0 + 3;
    H(tracks[k].hit[0], h0); H(tracks[k].hit[1], h1);
    track_circle(tracks[k], h0, h1, P);
  }
  std::vector<int> pos, neg;
  for (size_t k = 0; k < tracks.size(); ++k) (tracks[k].charge > 0 ? pos : neg).push_back((int)k);
  struct Tri { int t[3]; };
  std::vector<Tri> combos;
  int n_amb_e = 0;
  for (size_t i = 0; i < pos.size(); ++i)
  for (size_t j = i + 1; j < pos.size(); ++j)
  for (size_t e = 0; e < neg.size(); ++e) {
    const Track &A = tracks[pos[i]], &B = tracks[pos[j]], &C = tracks[neg[e]];
    double sE = A.E + B.E + C.E;
    double lo_e = kMmu - P.de_max, hi_e = kMmu + P.de_max;
    int d = window(sE, lo_e, hi_e, P.amb);
    if (d < 0) ++n_amb_e;
    if (d == 1) combos.push_back({{pos[i], pos[j], neg[e]}});
    if (want_lists && d != 0) {
      TripleRec tr;
      tr.f = f; tr.pass = d > 0 ? 1 : 0; tr.amb = d < 0 ? 1 : 0;
      const Track* abc[3] = {&A, &B, &C};
      for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 3; ++r) tr.t[q][r] = abc[q]->hit[r];
      out.triples.push_back(tr);
    }
  }
  out.counts[2] = (int)combos.size();
  out.namb[2] = n_amb_e;
  if (n_amb_e) out.amb |= COMBO_OVF | VERTEX;
  if ((int)combos.size() > P.max_combos) { out.flags |= COMBO_OVF | KEEP; return; }
  bool found = false;
  double bestchi = std::numeric_limits<double>::infinity();
  for (auto& c : combos) {
    const Track* T3[3] = {&tracks[c.t[0]], &tracks[c.t[1]], &tracks[c.t[2]]};
    VertexOut v = vertex_triple(T3, P);
    if (v.amb) out.amb |= VERTEX;
    if (v.pass) {
      if (found && near_edge(v.chi2, bestchi, P.amb)) out.amb |= VERTEX;
      if (!found || v.chi2 < bestchi) {
        bestchi = v.chi2;
        out.vtx[0] = v.x; out.vtx[1] = v.y; out.vtx[2] = v.z; out.vtx[3] = v.chi2;
      }
      found = true;
    }
  }
  if (found) out.flags |= VERTEX | KEEP;
}

Params unpack(const double* p) {
  // layout documented in oracle.py (PARAM_FIELDS)
  Params P;
  int k = 0;
  for (int i = 0; i < 4; ++i) P.r_layer[i] = p[k++];
  for (int i = 0; i < 4; ++i) P.z_half[i] = p[k++];
  P.b = p[k++]; P.xx0 = p[k++]; P.sigma_pix = p[k++];
  for (int i = 0; i < 8; ++i) P.win[i] = p[k++];
  P.chi2_track_max = p[k++];
  P.max_triplets = (int)p[k++]; P.max_tracks = (int)p[k++];
  P.max_combos = (int)p[k++]; P.max_layer_hits = (int)p[k++];
  P.de_max = p[k++]; P.r_target = p[k++]; P.target_tol = p[k++];
  P.chi2_vertex_max = p[k++]; P.d_target_max = p[k++]; P.p_sum_max = p[k++];
  P.amb = p[k++];
  return P;
}

struct Result {
  std::vector<FrameOut> frames;
  double seconds;
};

}  // namespace

extern "C" {

int oc_param_count() { return 31; }

// Run the whole selection over n_frames frames.  Returns an opaque handle.
void* oc_run(const float* x, const float* y, const float* z, const int32_t* lo, int n_frames,
             const double* params, int want_lists, int n_threads) {
  Params P = unpack(params);
  Result* R = new Result;
  R->frames.resize(n_frames);
  if (n_threads > 0) omp_set_num_threads(n_threads);
  double t0 = omp_get_wtime();
#pragma omp parallel for schedule(dynamic, 64)
  for (int f = 0; f < n_frames; ++f) process_frame(f, x, y, z, lo, P, R->frames[f], want_lists != 0);
  R->seconds = omp_get_wtime() - t0;
  return R;
}

double oc_seconds(void* h) { return static_cast<Result*>(h)->seconds; }
int oc_threads_used(int n_threads) {
  int n = 0;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}

void oc_sizes(void* h, long long* n_trips, long long* n_tracks, long long* n_triples) {
  Result* R = static_cast<Result*>(h);
  long long a = 0, b = 0, c = 0;
  for (auto& f : R->frames) { a += f.trips.size(); b += f.tracks.size(); c += f.triples.size(); }
  *n_trips = a; *n_tracks = b; *n_triples = c;
}

// frame outputs: flags[F], amb[F], counts[3F] (sure), namb[3F] (ambiguous), vtx[4F]; stats[6]
void oc_frames(void* h, uint32_t* flags, uint32_t* amb, int32_t* counts, int32_t* namb, double* vtx,
               long long* stats) {
  Result* R = static_cast<Result*>(h);
  for (int k = 0; k < 6; ++k) stats[k] = 0;
  for (size_t f = 0; f < R->frames.size(); ++f) {
    const FrameOut& o = R->frames[f];
    flags[f] = o.flags; amb[f] = o.amb;
    for (int k = 0; k < 3; ++k) { counts[3 * f + k] = o.counts[k]; namb[3 * f + k] = o.namb[k]; }
    for (int k = 0; k < 4; ++k) vtx[4 * f + k] = o.vtx[k];
    stats[0] += o.st.combos; stats[4] += o.st.fits; stats[5] += o.st.tracks_tested;
  }
}

// trips: int32 [n][6] (frame, h0, h1, h2, pass, amb) + double rtc[n]
// tracks: int32 [n][8] (frame, h0..h3, charge, pass, amb) + double [n][2] (kbar, chi2)
// triples: int32 [n][12] (frame, triplet hits of track a (3), b (3), c (3), pass, amb)
void oc_lists(void* h, int32_t* trips, double* trip_rtc, int32_t* tracks, double* track_f, int32_t* triples) {
  Result* R = static_cast<Result*>(h);
  long long a = 0, b = 0, c = 0;
  for (auto& f : R->frames) {
    for (auto& t : f.trips) {
      int32_t* o = trips + 6 * a;
      o[0] = t.f; o[1] = t.h[0]; o[2] = t.h[1]; o[3] = t.h[2]; o[4] = t.pass; o[5] = t.amb;
      trip_rtc[a++] = t.rtc;
    }
    for (auto& t : f.tracks) {
      int32_t* o = tracks + 8 * b;
      o[0] = t.f; for (int k = 0; k < 4; ++k) o[1 + k] = t.h[k];
      o[5] = t.charge; o[6] = t.pass; o[7] = t.amb;
      track_f[2 * b] = t.kbar; track_f[2 * b + 1] = t.chi2;
      ++b;
    }
    for (auto& t : f.triples) {
      int32_t* o = triples + 12 * c;
      o[0] = t.f;
      for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 3; ++r) o[1 + 3 * q + r] = t.t[q][r];
      o[10] = t.pass; o[11] = t.amb;
      ++c;
    }
  }
}

void oc_free(void* h) { delete static_cast<Result*>(h); }

// Cut quantities for explicit triplets: out [n][4] = dlambda, cosphi01, cosphi12, rtc;
// dec[n] = 1 pass, 0 fail, -1 ambiguous.
void oc_cut_quantities(const double* h /*[n][9]*/, int n, const double* params, double* out, int32_t* dec) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    CutQ q = cut_quantities(h + 9 * i, h + 9 * i + 3, h + 9 * i + 6, P);
    out[4 * i] = q.dlambda; out[4 * i + 1] = q.cosphi01; out[4 * i + 2] = q.cosphi12; out[4 * i + 3] = q.rtc;
    dec[i] = cut_decision(q, P);
  }
}

// Triplet fit for explicit triplets: out [n][14] = kappa, sigma2_kappa, chi2, r_star,
// sigma2_r, rtc, theta1, theta2, phi1, phi2, rbar_c, sigma_ms, cx, cy; ok[n].
void oc_fit(const double* h /*[n][9]*/, int n, const double* params, double* out, int32_t* ok) {
  Params P = unpack(params);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    Fit<double> f;
    ok[i] = triplet_fit(h + 9 * i, h + 9 * i + 3, h + 9 * i + 6, P, f) ? 1 : 0;
    double* o = out + 14 * i;
    if (!ok[i]) { for (int k = 0; k < 14; ++k) o[k] = std::numeric_limits<double>::quiet_NaN(); continue; }
    double v[14] = {f.kappa, f.sigma2_kappa, f.chi2, f.r_star, f.sigma2_r, f.rtc, f.theta1,
                    f.theta2, f.phi1, f.phi2, f.rbar_c, f.sigma_ms, f.cx, f.cy};
    std::memcpy(o, v, sizeof v);
  }
}

// Predicted layer-3 point for explicit triplets: out [n][3]; ok[n].
void oc_predict_l3(const double* h /*[n][9]*/, int n, const double* params, double* out, int32_t* ok) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    Fit<double> f;
    ok[i] = 0;
    if (!triplet_fit(h + 9 * i, h + 9 * i + 3, h + 9 * i + 6, P, f)) continue;
    ok[i] = predict_l3(h + 9 * i + 3, h + 9 * i + 6, f, P, out + 3 * i, nullptr) ? 1 : 0;
  }
}

// Track from four explicit hits: out [n][4] = kbar, chi2, theta1, rbar; ok[n]
// (0 fit failed, 1 ok; the chi2 cut is not applied here).
void oc_track4(const double* h /*[n][12]*/, int n, const double* params, double* out, int32_t* ok) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    const double* q = h + 12 * i;
    Fit<double> f1, f2;
    ok[i] = 0;
    if (!triplet_fit(q, q + 3, q + 6, P, f1) || !triplet_fit(q + 3, q + 6, q + 9, P, f2)) continue;
    if (f1.sgn != f2.sgn) continue;
    double kbar, chi2;
    combine_fits(f1, f2, kbar, chi2);
    out[4 * i] = kbar;
    out[4 * i + 1] = chi2;
    out[4 * i + 2] = f1.theta1; out[4 * i + 3] = 1 / std::fabs(kbar);
    ok[i] = 1;
  }
}

// Vertex for explicit track triples given by four hits each (e+, e+, e-):
// h [n][3][12]; out [n][10] = pass, x, y, z, chi2, sumE, amb, dtarget, psum,
// reached (all three pairs have an intersection near the target).
void oc_vertex4(const double* h, int n, const double* params, double* out) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    double* o = out + 10 * i;
    for (int k = 0; k < 10; ++k) o[k] = std::numeric_limits<double>::quiet_NaN();
    Track T[3];
    bool ok = true;
    for (int k = 0; k < 3 && ok; ++k) ok = track_from_hits(h + 36 * i + 12 * k, P, T[k]);
    if (!ok) continue;
    const Track* T3[3] = {&T[0], &T[1], &T[2]};
    VertexOut v = vertex_triple(T3, P);
    o[0] = v.pass; o[1] = v.x; o[2] = v.y; o[3] = v.z; o[4] = v.chi2;
    o[5] = T[0].E + T[1].E + T[2].E; o[6] = v.amb;
    o[7] = v.dt; o[8] = v.psum; o[9] = v.reached;
  }
}

// Refined vertex of explicit track triples given by four hits each (e+, e+,
// e-): h [n][3][12]; out [n][16] = x, y, z, J, phi_0, phi_1, phi_2,
// sigma2_0, sigma2_1, sigma2_2, rough x, rough y, rough z, rough chi2,
// iterations, rough amb; status [n] = 1 converged, 0 the rough estimate does
// not pass, -1 no convergence, -2 a track fit fails.
void oc_refine4(const double* h, int n, const double* params, double* out, int32_t* status) {
  Params P = unpack(params);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    double* o = out + 16 * i;
    for (int k = 0; k < 16; ++k) o[k] = std::numeric_limits<double>::quiet_NaN();
    Track T[3];
    bool ok = true;
    for (int k = 0; k < 3 && ok; ++k) ok = track_from_hits(h + 36 * i + 12 * k, P, T[k]);
    if (!ok) { status[i] = -2; continue; }
    const Track* T3[3] = {&T[0], &T[1], &T[2]};
    RefineOut r = refine_triple(T3, P);
    status[i] = r.status;
    o[15] = r.rough.amb;
    if (!r.rough.pass) continue;
    for (int k = 0; k < 3; ++k) { o[k] = r.x[k]; o[4 + k] = r.x[3 + k]; o[7 + k] = r.s2[k]; }
    o[3] = r.J;
    o[10] = r.rough.x; o[11] = r.rough.y; o[12] = r.rough.z; o[13] = r.rough.chi2;
    o[14] = r.iters;
  }
}

// The weighted residuals of the refined-vertex objective for tracks given by
// four hits: h [n][3][12], x [n][6] = (v, phi), s2 [n][3]; r [n][9] (NaN when
// a track fit fails).
void oc_refine_residual(const double* h, const double* x, const double* s2, int n, const double* params,
                        double* r) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    Track T[3];
    bool ok = true;
    for (int k = 0; k < 3 && ok; ++k) ok = track_from_hits(h + 36 * i + 12 * k, P, T[k]);
    if (!ok) { for (int k = 0; k < 9; ++k) r[9 * i + k] = std::numeric_limits<double>::quiet_NaN(); continue; }
    const Track* T3[3] = {&T[0], &T[1], &T[2]};
    refine_residual(T3, s2 + 3 * i, x + 6 * i, r + 9 * i);
  }
}

// Per-track vertex-stage quantities of tracks given by four hits:
// out [n][9] = kbar, rbar, rt, cx, cy, sms0, E, p, theta1; ok[n].
void oc_track_geom(const double* h /*[n][12]*/, int n, const double* params, double* out, int32_t* ok) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    const double* q = h + 12 * i;
    double* o = out + 9 * i;
    ok[i] = 0;
    for (int k = 0; k < 9; ++k) o[k] = std::numeric_limits<double>::quiet_NaN();
    Track t;
    if (!track_from_hits(q, P, t)) continue;
    const double v[9] = {t.kbar, t.rbar, t.rt, t.cx, t.cy, t.sms0, t.E, t.p, t.theta1};
    std::memcpy(o, v, sizeof v);
    ok[i] = 1;
  }
}

// Backward turning angle from the layer-0 hit to a transverse point q, the
// path length s = rt * angle and the position variance of eq. track-error at
// q, for tracks given by four hits: q [n][2], out [n][3]; ok[n].
void oc_track_point(const double* h /*[n][12]*/, const double* qxy, int n, const double* params, double* out,
                    int32_t* ok) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) {
    const double* q = h + 12 * i;
    double* o = out + 3 * i;
    ok[i] = 0;
    o[0] = o[1] = o[2] = std::numeric_limits<double>::quiet_NaN();
    Track t;
    if (!track_from_hits(q, P, t)) continue;
    const double a = back_angle(t, qxy[2 * i], qxy[2 * i + 1]);
    o[0] = a;
    o[1] = t.rt * a;
    o[2] = point_sigma2(t, qxy[2 * i], qxy[2 * i + 1], P);
    ok[i] = 1;
  }
}

// Distance from (rho, z) points to the double-cone target surface: rz [n][2].
void oc_cone_distance(const double* rz, int n, const double* params, double* out) {
  Params P = unpack(params);
  for (int i = 0; i < n; ++i) out[i] = cone_distance(rz[2 * i], rz[2 * i + 1], P);
}

// ---------------------------------------------------------- alignment
// Summed triplet-fit chi2 L(theta) = sum_t chi2_t(A(h; theta)) over explicit
// triplets, with A_s(h) = R_z(alpha_s) h + (tx, ty, tz)_s per sensor s, and
// its exact gradient by forward-mode dual numbers (12 directions per
// triplet: the four parameters of each of its three hits' sensors).
// theta [S][4], grad [S][4] (accumulated); weight [n] optional (NULL = 1):
// L = sum_t weight_t chi2_t.  Returns L.
double oc_align_loss_grad(const float* x, const float* y, const float* z, const uint16_t* sensor,
                          const int32_t* trip /*[n][3]*/, int n, const double* theta, int n_sensors,
                          const double* params, double* grad, int with_grad, const double* weight) {
  Params P = unpack(params);
  double L = 0;
  std::vector<double> G(with_grad ? (size_t)n_sensors * 4 : 0, 0.0);
#pragma omp parallel
  {
    std::vector<double> g(with_grad ? (size_t)n_sensors * 4 : 0, 0.0);
    double l = 0;
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (with_grad) {
        Dual<12> h[3][3];
        for (int k = 0; k < 3; ++k) {
          int hi = trip[3 * i + k];
          int s = sensor[hi];
          const double* th = theta + 4 * s;
          double ca = std::cos(th[3]), sa = std::sin(th[3]);
          double X0 = x[hi], Y0 = y[hi], Z0 = z[hi];
          double dv[12];
          // x' = ca X - sa Y + tx ; y' = sa X + ca Y + ty ; z' = Z + tz
          std::memset(dv, 0, sizeof dv); dv[4 * k + 0] = 1; dv[4 * k + 3] = -sa * X0 - ca * Y0;
          h[k][0] = mk<12>(ca * X0 - sa * Y0 + th[0], dv);
          std::memset(dv, 0, sizeof dv); dv[4 * k + 1] = 1; dv[4 * k + 3] = ca * X0 - sa * Y0;
          h[k][1] = mk<12>(sa * X0 + ca * Y0 + th[1], dv);
          std::memset(dv, 0, sizeof dv); dv[4 * k + 2] = 1;
          h[k][2] = mk<12>(Z0 + th[2], dv);
        }
        Fit<Dual<12>> f;
        if (!triplet_fit(h[0], h[1], h[2], P, f)) continue;
        const double w = weight ? weight[i] : 1.0;
        l += w * f.chi2.v;
        for (int k = 0; k < 3; ++k) {
          int s = sensor[trip[3 * i + k]];
          for (int j = 0; j < 4; ++j) g[4 * s + j] += w * f.chi2.d[4 * k + j];
        }
      } else {
        double h[3][3];
        for (int k = 0; k < 3; ++k) {
          int hi = trip[3 * i + k];
          const double* th = theta + 4 * sensor[hi];
          double ca = std::cos(th[3]), sa = std::sin(th[3]);
          h[k][0] = ca * x[hi] - sa * y[hi] + th[0];
          h[k][1] = sa * x[hi] + ca * y[hi] + th[1];
          h[k][2] = z[hi] + th[2];
        }
        Fit<double> f;
        if (!triplet_fit(h[0], h[1], h[2], P, f)) continue;
        l += (weight ? weight[i] : 1.0) * f.chi2;
      }
    }
#pragma omp critical
    {
      L += l;
      for (size_t k = 0; k < g.size(); ++k) G[k] += g[k];
    }
  }
  for (size_t k = 0; k < G.size(); ++k) grad[k] += G[k];
  return L;
}

}  // extern "C"
