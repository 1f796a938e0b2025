// FP64 reference ("oracle") of the differentiable Gaussian rasterizer used by
// 4DGCPro: projection of anisotropic 3D Gaussians (Sec. 3.1, Eq. 1 and the
// factorisation of the covariance), front-to-back compositing of ordered
// Gaussians (Eq. 2), progressive rendering of nested layers (Eq. 4), frame
// composition from a keyframe and residuals (Sec. 3.2, pose update and Eq. 7),
// and its analytic backward.
//
// TEST INFRASTRUCTURE ONLY. This file is compiled into liboracle.so and is
// used by the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark. It shares no code with the GPU library and must never be on the
// product path.
//
// The oracle is the plain per-pixel definition: every pixel scans its
// candidate Gaussians (all of them in brute-force mode, or those whose
// conservative footprint covers the pixel's bucket), orders them by depth and
// composites them. There are no tiles, no sorted pair lists and no
// transmittance recovery. The projection Jacobian for the backward is obtained
// by forward-mode dual numbers through the same plain projection code.
//
// Conventions where the paper is silent (each one is also listed in the
// design notes of the repository):
//  * alpha = min(alpha_max, o * G); a Gaussian contributes iff alpha >= alpha_min;
//  * the traversal stops before Gaussian i if T * (1 - alpha_i) < t_stop
//    (Gaussian i is not included);
//  * order: increasing depth key, ties broken by lower index, where the key is
//    the float32 rounding (to nearest) of the camera-space depth t_z of the
//    exactly composed frame mean (computed here in FP64); a Gaussian is culled
//    iff t_z <= near_plane;
//  * pixel (u, v) is sampled at (u + 0.5, v + 0.5);
//  * EWA projection with the Jacobian's x/z, y/z clamped at 1.3 times the
//    half-field-of-view tangent, plus `dilation` on the 2D covariance diagonal;
//  * colour = max(0, sum_k f_k Y_k(d) + 0.5) with the real orthonormal SH
//    basis (Condon-Shortley phase) and d the unit vector camera -> mean;
//  * o = sigmoid(logit), s = exp(log_scale), R = R(q / |q|).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t width, height, sh_degree, n_levels;
  int32_t level_counts[8];
  int32_t res_channels;  // 0 (no residuals), 8, 11 or 11 + 3K
  int32_t pad_;
  double near_plane, dilation, alpha_min, alpha_max, t_stop;
  double bg[3];
  // Multiplier of the first-order FP32 error bounds that decide which
  // decisions a float32 evaluation may take the other way (see "Ambiguous
  // decisions" below); 0 switches the exploration of alternatives off.
  double band_safety;
} oc_settings;

}  // extern "C"

namespace {

constexpr int kMaxC = 59;  // 11 + 3 * 16

// ---------------------------------------------------------------- dual numbers
template <int D>
struct Dual {
  double v;
  double d[D];
  Dual() : v(0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT
};
template <int D> Dual<D> operator+(const Dual<D>& a, const Dual<D>& b) { Dual<D> r; r.v = a.v + b.v; for (int i = 0; i < D; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int D> Dual<D> operator-(const Dual<D>& a, const Dual<D>& b) { Dual<D> r; r.v = a.v - b.v; for (int i = 0; i < D; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int D> Dual<D> operator-(const Dual<D>& a) { Dual<D> r; r.v = -a.v; for (int i = 0; i < D; ++i) r.d[i] = -a.d[i]; return r; }
template <int D> Dual<D> operator*(const Dual<D>& a, const Dual<D>& b) { Dual<D> r; r.v = a.v * b.v; for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int D> Dual<D> operator/(const Dual<D>& a, const Dual<D>& b) { Dual<D> r; r.v = a.v / b.v; double ib = 1.0 / b.v; for (int i = 0; i < D; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib; return r; }
template <int D> Dual<D> operator+(const Dual<D>& a, double b) { Dual<D> r = a; r.v += b; return r; }
template <int D> Dual<D> operator+(double a, const Dual<D>& b) { return b + a; }
template <int D> Dual<D> operator-(const Dual<D>& a, double b) { Dual<D> r = a; r.v -= b; return r; }
template <int D> Dual<D> operator-(double a, const Dual<D>& b) { Dual<D> r = -b; r.v += a; return r; }
template <int D> Dual<D> operator*(const Dual<D>& a, double b) { Dual<D> r; r.v = a.v * b; for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * b; return r; }
template <int D> Dual<D> operator*(double a, const Dual<D>& b) { return b * a; }
template <int D> Dual<D> operator/(const Dual<D>& a, double b) { return a * (1.0 / b); }
template <int D> Dual<D> operator/(double a, const Dual<D>& b) { return Dual<D>(a) / b; }
template <int D> Dual<D> exp(const Dual<D>& a) { Dual<D> r; r.v = std::exp(a.v); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * r.v; return r; }
template <int D> Dual<D> sqrt(const Dual<D>& a) { Dual<D> r; r.v = std::sqrt(a.v); double g = 0.5 / r.v; for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * g; return r; }

inline double val(double x) { return x; }
template <int D> inline double val(const Dual<D>& x) { return x.v; }
inline double exp(double x) { return std::exp(x); }
inline double sqrt(double x) { return std::sqrt(x); }

// --------------------------------------------------------------- SH basis
// Real spherical harmonics, orthonormal on the unit sphere, Condon-Shortley
// phase, index k = l^2 + l + m, for degree <= 3 (written for a unit vector).
template <class T>
void sh_basis(int deg, const T& x, const T& y, const T& z, T* Y) {
  const double pi = 3.14159265358979323846;
  Y[0] = T(0.5 / std::sqrt(pi));
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (deg < 2) return;
  const double c2a = 0.5 * std::sqrt(15.0 / pi);
  const double c2b = 0.25 * std::sqrt(5.0 / pi);
  const double c2c = 0.25 * std::sqrt(15.0 / pi);
  Y[4] = c2a * (x * y);
  Y[5] = -c2a * (y * z);
  Y[6] = c2b * (3.0 * (z * z) - 1.0);
  Y[7] = -c2a * (x * z);
  Y[8] = c2c * (x * x - y * y);
  if (deg < 3) return;
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
  const double c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  Y[9] = -c3a * (y * (3.0 * (x * x) - y * y));
  Y[10] = c3b * (x * y * z);
  Y[11] = -c3c * (y * (5.0 * (z * z) - 1.0));
  Y[12] = c3d * (z * (5.0 * (z * z) - 3.0));
  Y[13] = -c3c * (x * (5.0 * (z * z) - 1.0));
  Y[14] = c3e * (z * (x * x - y * y));
  Y[15] = -c3a * (x * (x * x - 3.0 * (y * y)));
}

// ----------------------------------------------------------- quaternions
// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
template <class T>
void quat_rot(const T q[4], T R[9]) {
  const T &w = q[0], &x = q[1], &y = q[2], &z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Hamilton product a (x) b, components (w, x, y, z).
template <class T>
void quat_mul(const T a[4], const T b[4], T out[4]) {
  out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

struct Cam {
  double R[9], t[3], fx, fy, cx, cy;
};

Cam load_cam(const double* c) {
  Cam k;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) k.R[3 * i + j] = c[4 * i + j];
    k.t[i] = c[4 * i + 3];
  }
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  return k;
}

inline int n_coeffs(int deg) { return (deg + 1) * (deg + 1); }
inline int n_channels(int deg) { return 11 + 3 * n_coeffs(deg); }

// ------------------------------------------------- frame composition (O1)
// Keyframe params (FP64 values of the float32 inputs) composed with the
// residuals of frames 0..f: mean, logit, log-scale and SH add; the rotation
// quaternion is left-multiplied, q_f = dq_f (x) q_{f-1}.
void compose_frame(const oc_settings& s, int n, const double* P, const double* res, int f, int i, double* out) {
  const int C = n_channels(s.sh_degree);
  for (int c = 0; c < C; ++c) out[c] = P[(size_t)c * n + i];
  if (!res || s.res_channels <= 0) return;
  const int Rc = s.res_channels;
  for (int t = 0; t <= f; ++t) {
    const double* r = res + (size_t)t * Rc * n;
    for (int c = 0; c < 3; ++c) out[c] += r[(size_t)c * n + i];
    double dq[4], q[4], o[4];
    for (int c = 0; c < 4; ++c) { dq[c] = r[(size_t)(3 + c) * n + i]; q[c] = out[6 + c]; }
    quat_mul(dq, q, o);
    for (int c = 0; c < 4; ++c) out[6 + c] = o[c];
    out[10] += r[(size_t)7 * n + i];
    if (Rc >= 11) for (int c = 0; c < 3; ++c) out[3 + c] += r[(size_t)(8 + c) * n + i];
    if (Rc > 11) for (int c = 11; c < Rc && c < C; ++c) out[c] += r[(size_t)c * n + i];
  }
}

// Reading: a Gaussian with any non-finite composed parameter is culled.
bool all_finite(const oc_settings& s, const double* p) {
  const int C = n_channels(s.sh_degree);
  for (int c = 0; c < C; ++c)
    if (!std::isfinite(p[c])) return false;
  return true;
}

// ------------------------------------------ float32 accuracy (readings)
// The oracle decides every discrete step (near-plane cull, depth order, the
// alpha cut, the transmittance stop) in FP64. A float32 evaluation of the same
// function can take a decision the other way when the FP64 margin is below its
// rounding error, so the oracle states the accuracy it asks of a float32
// evaluation and explores both outcomes of every decision inside that band
// (scaled by band_safety). u = 2^-24 is the float32 unit roundoff. The asked
// accuracy is that of a careful evaluation from float32 inputs:
//  * depth: exact up to its float32 rounding (the order key), i.e. computed in
//    higher precision from the exactly composed frame mean;
//  * 2D mean: one float32 rounding, 2u |m|;
//  * conic: (kConicOps + 8 per composed frame) u times its magnitude scale,
//    grown by sqrt(a c / det) (a cancellation-free determinant);
//  * the quadratic form: 6 roundings of the magnitude of its terms;
//  * exp, sigmoid and the product o G: 8u, plus the float32 sums of the
//    frame's opacity-logit deltas.
constexpr double kU = 5.9604644775390625e-08;  // 2^-24
constexpr double kConicOps = 24.0;  // roundings on the path params -> conic, per unit of conditioning

// ------------------------------------------------------ projection (O2-O4)
template <class T>
struct Proj {
  T mx, my, A, B, C, o, rgb[3];
  // diagnostics (value only)
  double s2d[3], tz, radius;
  double t_cam[3];     // camera-space mean
  double conic_err[3];  // conditioning-scaled magnitudes of (A, B, C), see error_bounds
  int flags;  // bit0 x-clamp, bit1 y-clamp, bit2..4 colour clamp r,g,b
};

// Projects one Gaussian with composed params p (C channels) into camera k.
// Returns false if it is culled (non-positive quaternion norm, det <= 0).
// The near-plane test is decided by the caller on the FP64 depth t_z.
template <class T>
bool project(const T* p, const oc_settings& s, const Cam& k, Proj<T>& out) {
  const int deg = s.sh_degree;
  const int K = n_coeffs(deg);
  T q[4] = {p[6], p[7], p[8], p[9]};
  double qn2 = val(q[0]) * val(q[0]) + val(q[1]) * val(q[1]) + val(q[2]) * val(q[2]) + val(q[3]) * val(q[3]);
  if (!(qn2 > 0.0)) return false;
  T qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int c = 0; c < 4; ++c) q[c] = q[c] / qn;
  T Rg[9];
  quat_rot(q, Rg);
  T sc[3] = {exp(p[3]), exp(p[4]), exp(p[5])};
  // world covariance  Sigma = R diag(s^2) R^T  (Sec. 3.1)
  T Sig[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T acc(0.0);
      for (int j = 0; j < 3; ++j) acc = acc + Rg[3 * a + j] * (sc[j] * sc[j]) * Rg[3 * b + j];
      Sig[3 * a + b] = acc;
    }
  // camera-space mean
  T t[3];
  for (int a = 0; a < 3; ++a) t[a] = k.R[3 * a] * p[0] + k.R[3 * a + 1] * p[1] + k.R[3 * a + 2] * p[2] + k.t[a];
  const double limx = 1.3 * (0.5 * s.width / k.fx);
  const double limy = 1.3 * (0.5 * s.height / k.fy);
  T ux = t[0] / t[2], uy = t[1] / t[2];
  out.flags = 0;
  if (val(ux) > limx) { ux = T(limx); out.flags |= 1; }
  if (val(ux) < -limx) { ux = T(-limx); out.flags |= 1; }
  if (val(uy) > limy) { uy = T(limy); out.flags |= 2; }
  if (val(uy) < -limy) { uy = T(-limy); out.flags |= 2; }
  // EWA Jacobian of the perspective map
  T J[6] = {k.fx / t[2], T(0.0), -k.fx * ux / t[2], T(0.0), k.fy / t[2], -k.fy * uy / t[2]};
  T M[6];  // J * R_wc
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = J[3 * a] * k.R[b] + J[3 * a + 1] * k.R[3 + b] + J[3 * a + 2] * k.R[6 + b];
  T cov[3];  // (xx, xy, yy) of M Sigma M^T
  {
    T SM0[3], SM1[3];
    for (int a = 0; a < 3; ++a) {
      SM0[a] = Sig[3 * a] * M[0] + Sig[3 * a + 1] * M[1] + Sig[3 * a + 2] * M[2];
      SM1[a] = Sig[3 * a] * M[3] + Sig[3 * a + 1] * M[4] + Sig[3 * a + 2] * M[5];
    }
    cov[0] = M[0] * SM0[0] + M[1] * SM0[1] + M[2] * SM0[2];
    cov[1] = M[0] * SM1[0] + M[1] * SM1[1] + M[2] * SM1[2];
    cov[2] = M[3] * SM1[0] + M[4] * SM1[1] + M[5] * SM1[2];
  }
  cov[0] = cov[0] + s.dilation;
  cov[2] = cov[2] + s.dilation;
  T det = cov[0] * cov[2] - cov[1] * cov[1];
  if (!(val(det) > 0.0)) return false;
  out.A = cov[2] / det;
  out.B = -cov[1] / det;
  out.C = cov[0] / det;
  {
    // Accuracy asked of a float32 evaluation of the conic (see error_bounds):
    // each entry within eps_c of its magnitude scale, where eps_c grows with
    // sqrt(a c / det), the conditioning of the 2D covariance, because b and
    // the determinant lose relative accuracy as the footprint thins.
    const double ca = val(cov[0]), cc = val(cov[2]), dt = val(det);
    const double kappa = std::sqrt(std::max(1.0, ca * cc / dt));
    const double A = val(out.A), Cc = val(out.C);
    out.conic_err[0] = kappa * std::fabs(A);
    out.conic_err[1] = kappa * std::sqrt(std::fabs(A * Cc));
    out.conic_err[2] = kappa * std::fabs(Cc);
  }
  for (int a = 0; a < 3; ++a) out.t_cam[a] = val(t[a]);
  out.mx = k.fx * t[0] / t[2] + k.cx;
  out.my = k.fy * t[1] / t[2] + k.cy;
  out.o = 1.0 / (1.0 + exp(-p[10]));
  // colour in the viewing direction
  double cpos[3];
  for (int a = 0; a < 3; ++a) cpos[a] = -(k.R[a] * k.t[0] + k.R[3 + a] * k.t[1] + k.R[6 + a] * k.t[2]);
  T dv[3] = {p[0] - cpos[0], p[1] - cpos[1], p[2] - cpos[2]};
  T dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int a = 0; a < 3; ++a) dv[a] = dv[a] / dn;
  T Y[16];
  sh_basis(deg, dv[0], dv[1], dv[2], Y);
  for (int c = 0; c < 3; ++c) {
    T acc(0.5);
    for (int j = 0; j < K; ++j) acc = acc + p[11 + 3 * j + c] * Y[j];
    if (val(acc) < 0.0) { acc = T(0.0); out.flags |= 4 << c; }
    out.rgb[c] = acc;
  }
  out.s2d[0] = val(cov[0]); out.s2d[1] = val(cov[1]); out.s2d[2] = val(cov[2]);
  out.tz = val(t[2]);
  double mid = 0.5 * (out.s2d[0] + out.s2d[2]);
  double lmax = mid + std::sqrt(std::max(0.0, 0.25 * (out.s2d[0] - out.s2d[2]) * (out.s2d[0] - out.s2d[2]) + out.s2d[1] * out.s2d[1]));
  double o = val(out.o);
  out.radius = (o >= s.alpha_min) ? std::sqrt(2.0 * std::log(o / s.alpha_min)) * std::sqrt(lmax) : 0.0;
  return true;
}

// ------------------------------------------------------- scene projection
struct Rec {  // one visible (frame-view, Gaussian)
  int idx;
  float key;         // float32 rounding of t_z: the order key
  bool key_amb;      // t_z lies within FP64 rounding of a float32 rounding boundary
  double tz;         // FP64 camera-space depth
  double tz_err;     // bound on the FP64 error of t_z
  double pos_err;    // asked float32 accuracy of the 2D mean (pixels)
  double conic_err[3];  // asked float32 accuracy of (A, B, C)
  double o_err;      // asked relative accuracy of o and of the evaluation of exp
  bool culled;       // t_z <= near_plane
  bool near_amb;     // t_z within its FP64 error bound of near_plane
  double mx, my, A, B, C, o, rgb[3], radius;
  int flags;         // projection clamps (Jacobian x/y, colour r/g/b)
};

struct Scene {
  oc_settings s;
  int n, F, V, B;
  std::vector<double> P, res;          // FP64 copies of the float32 inputs
  std::vector<Cam> cams;
};

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

// Error bounds of one record (see "float32 accuracy" above). nf is the number
// of composed residual frames (0 for a keyframe). The depth t_z is evaluated
// here in FP64: a few roundings of 2^-53 of the magnitudes involved.
void error_bounds(const Cam& k, const double* p, int nf, const Proj<double>& pr, Rec& r) {
  double mag = std::fabs(k.t[2]);
  for (int j = 0; j < 3; ++j) mag += std::fabs(k.R[6 + j] * p[j]);
  const double tz = pr.t_cam[2];
  r.tz = tz;
  r.tz_err = 16.0 * kU64 * mag;
  r.key = (float)tz;
  // the rounding boundaries between the key and its float32 neighbours
  const double up = (double)std::nextafter(r.key, INFINITY), dn = (double)std::nextafter(r.key, -INFINITY);
  const double kd = (double)r.key;
  r.key_amb = std::fabs(tz - 0.5 * (kd + up)) <= r.tz_err || std::fabs(tz - 0.5 * (kd + dn)) <= r.tz_err;
  r.pos_err = 2.0 * kU * std::max(std::fabs(pr.mx), std::fabs(pr.my));
  const double ec = (kConicOps + 8.0 * nf) * kU;
  for (int j = 0; j < 3; ++j) r.conic_err[j] = ec * pr.conic_err[j];
  r.o_err = 8.0 * kU + nf * kU * (std::fabs(p[10]) + 1.0) * (1.0 - pr.o);
}

// The record of Gaussian i with composed params p in camera k; false if it is
// culled (and not within the error bound of the near plane).
bool make_record(const oc_settings& s, const Cam& k, const double* p, int i, int nf, Rec& r) {
  if (!all_finite(s, p)) return false;
  // FP64 depth first: Gaussians far behind the near plane are never projected
  double tz = k.R[6] * p[0] + k.R[7] * p[1] + k.R[8] * p[2] + k.t[2];
  if (!(tz > 0.5 * s.near_plane)) return false;
  Proj<double> pr;
  if (!project(p, s, k, pr)) return false;
  if (!(pr.o >= s.alpha_min)) return false;  // can never reach alpha_min
  error_bounds(k, p, nf, pr, r);
  r.culled = !(r.tz > s.near_plane);
  r.near_amb = s.band_safety > 0.0 && std::fabs(r.tz - s.near_plane) <= r.tz_err;
  if (r.culled && !r.near_amb) return false;
  r.idx = i;
  r.mx = pr.mx; r.my = pr.my; r.A = pr.A; r.B = pr.B; r.C = pr.C; r.o = pr.o;
  for (int c = 0; c < 3; ++c) r.rgb[c] = pr.rgb[c];
  r.radius = pr.radius;
  r.flags = pr.flags;
  return true;
}

// All records of frame-view b in front of the near plane (or within the error
// bound of its depth from it), sorted by (key, index).
std::vector<Rec> project_view(const Scene& sc, int b) {
  const oc_settings& s = sc.s;
  const int n = sc.n;
  const int f = b / sc.V;
  const Cam& k = sc.cams[b];
  std::vector<Rec> out;
  out.reserve(n);
  const double* res = sc.res.empty() ? nullptr : sc.res.data();
  std::vector<std::vector<Rec>> part;
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  part.resize(nt);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double p[kMaxC];
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      compose_frame(s, n, sc.P.data(), res, f, i, p);
      Rec r;
      if (make_record(s, k, p, i, res ? f + 1 : 0, r)) part[tid].push_back(r);
    }
  }
  for (auto& v : part) out.insert(out.end(), v.begin(), v.end());
  std::sort(out.begin(), out.end(), [](const Rec& a, const Rec& b) {
    if (a.key != b.key) return a.key < b.key;
    return a.idx < b.idx;
  });
  return out;
}

// Candidate lists per bucket of kBucket x kBucket pixels (bucketed mode):
// every record whose conservative disc (radius + 2 px) meets the bucket, in
// (key, index) order.
constexpr int kBucket = 8;
struct Buckets {
  int bw, bh;
  std::vector<std::vector<int>> lists;  // indices into the record vector
};

Buckets make_buckets(const oc_settings& s, const std::vector<Rec>& recs) {
  Buckets bk;
  bk.bw = (s.width + kBucket - 1) / kBucket;
  bk.bh = (s.height + kBucket - 1) / kBucket;
  bk.lists.assign((size_t)bk.bw * bk.bh, {});
  for (int r = 0; r < (int)recs.size(); ++r) {
    const Rec& e = recs[r];
    double rad = e.radius + 2.0;
    // pixel sample points are at u + 0.5
    int u0 = (int)std::floor(e.mx - rad - 0.5), u1 = (int)std::ceil(e.mx + rad - 0.5);
    int v0 = (int)std::floor(e.my - rad - 0.5), v1 = (int)std::ceil(e.my + rad - 0.5);
    u0 = std::max(u0, 0); v0 = std::max(v0, 0);
    u1 = std::min(u1, s.width - 1); v1 = std::min(v1, s.height - 1);
    if (u0 > u1 || v0 > v1) continue;
    for (int by = v0 / kBucket; by <= v1 / kBucket; ++by)
      for (int bx = u0 / kBucket; bx <= u1 / kBucket; ++bx) bk.lists[(size_t)by * bk.bw + bx].push_back(r);
  }
  return bk;
}

// One kept candidate of a pixel.
struct Kept {
  int rec;
  int idx;
  double araw;  // o * G (before the alpha_max clamp)
  double G;
  double eps;   // bound on the relative float32 error of araw
};

// Per-pixel scan (O5): candidates with o * G >= alpha_min, or within the band
// of alpha_min in which a float32 evaluation may decide the other way, in
// order. The relative error of o * exp(power) is the absolute error of power
// (from the 2D mean, the conic and the evaluation of the quadratic form) plus
// that of o and of exp.
void pixel_candidates(const std::vector<Rec>& recs, const int* cand, int ncand, double px, double py,
                      const oc_settings& s, std::vector<Kept>& out) {
  out.clear();
  for (int j = 0; j < ncand; ++j) {
    const Rec& e = recs[cand ? cand[j] : j];
    double dx = px - e.mx, dy = py - e.my;
    double q = e.A * dx * dx + 2.0 * e.B * dx * dy + e.C * dy * dy;
    double power = -0.5 * q;
    double G = std::exp(power);
    double araw = e.o * G;
    const double gx = e.A * dx + e.B * dy, gy = e.B * dx + e.C * dy;
    const double qabs = std::fabs(e.A) * dx * dx + 2.0 * std::fabs(e.B * dx * dy) + std::fabs(e.C) * dy * dy;
    const double dpow = 0.5 * (e.conic_err[0] * dx * dx + 2.0 * e.conic_err[1] * std::fabs(dx * dy) +
                               e.conic_err[2] * dy * dy) +
                        std::sqrt(gx * gx + gy * gy) * e.pos_err + 6.0 * kU * 0.5 * qabs;
    const double eps = dpow + e.o_err;
    if (araw >= s.alpha_min * (1.0 - s.band_safety * eps)) out.push_back({cand ? cand[j] : j, e.idx, araw, G, eps});
  }
}

struct PixOut {
  double rgb[3];
  double T;
  int ncontrib;
  int stop_k;  // position in the kept list where the traversal ended
  uint64_t sig;
};

inline uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  return h;
}

// Plain compositing of one level (Eq. 2 / Eq. 4): the FP64 decisions.
PixOut composite(const std::vector<Rec>& recs, const std::vector<Kept>& L, int nl, const oc_settings& s,
                 std::vector<int>* contrib) {
  PixOut o;
  double T = 1.0, C[3] = {0, 0, 0};
  int nc = 0;
  uint64_t h = 1469598103934665603ULL;
  if (contrib) contrib->clear();
  size_t k = 0;
  for (; k < L.size(); ++k) {
    const Kept& e = L[k];
    if (e.idx >= nl) continue;
    if (recs[e.rec].culled) continue;
    if (!(e.araw >= s.alpha_min)) continue;
    double a = std::min(s.alpha_max, e.araw);
    double Tn = T * (1.0 - a);
    if (Tn < s.t_stop) break;
    const Rec& r = recs[e.rec];
    for (int c = 0; c < 3; ++c) C[c] += r.rgb[c] * a * T;
    T = Tn;
    ++nc;
    h = mix(h, (uint64_t)e.idx * 2 + (e.araw > s.alpha_max ? 1 : 0));
    if (contrib) contrib->push_back((int)k);
  }
  h = mix(h, 0xabcdefULL + k);
  for (int c = 0; c < 3; ++c) o.rgb[c] = C[c] + T * s.bg[c];
  o.T = T;
  o.ncontrib = nc;
  o.stop_k = (int)k;
  o.sig = h;
  return o;
}

// Ambiguous decisions. A decision whose FP64 margin is inside the band that a
// float32 evaluation can cross is explored both ways: the alpha cut of a
// candidate with araw within its relative bound of alpha_min, and the T-stop
// test with T' within the bound accumulated along the path (two roundings per
// factor plus the relative error of each alpha, scaled by alpha / (1 - alpha)).
// Every such bound is multiplied by band_safety. The exactly defined
// decisions are explored both ways only where the FP64 evaluation itself
// cannot settle them: the near-plane cull of a Gaussian with t_z within its
// FP64 error of near, and the order of two neighbours one of whose depths lies
// within its FP64 error of a float32 rounding boundary next to the other's key. Up to
// kMaxBranch decisions are explored on one path; the colours of all explored
// paths are the accepted results of the pixel. If more ambiguous decisions lie
// on one path the pixel is marked as excluded (nvar = -1).
constexpr int kMaxBranch = 4;
constexpr int kMaxVar = 1 << kMaxBranch;

struct VarCtx {
  const std::vector<Rec>* recs;
  const std::vector<Kept>* L;
  const std::vector<int>* order;  // positions in L (the level's candidates, possibly permuted)
  const oc_settings* s;
  double* out;  // [kMaxVar][3]
  int nout;
  bool overflow;
  int nflags;
};

void var_emit(VarCtx& c, double T, double r, double g, double b) {
  if (c.nout >= kMaxVar) { c.overflow = true; return; }
  const oc_settings& s = *c.s;
  double* o = c.out + 3 * c.nout++;
  o[0] = r + T * s.bg[0]; o[1] = g + T * s.bg[1]; o[2] = b + T * s.bg[2];
}

void var_dfs(VarCtx& c, size_t k, double T, double epsT, double r, double g, double b, int br);

void var_take(VarCtx& c, size_t k, bool include, double T, double epsT, double r, double g, double b, int br) {
  const oc_settings& s = *c.s;
  if (!include) { var_dfs(c, k + 1, T, epsT, r, g, b, br); return; }
  const Kept& e = (*c.L)[(*c.order)[k]];
  const bool clamped = e.araw > s.alpha_max;
  double a = std::min(s.alpha_max, e.araw);
  double Tn = T * (1.0 - a);
  double epsN = epsT + 2.0 * kU + (clamped ? 0.0 : e.eps * a / (1.0 - a));
  bool stop = Tn < s.t_stop;
  const Rec& q = (*c.recs)[e.rec];
  if (std::fabs(Tn - s.t_stop) <= s.band_safety * epsN * Tn) {
    c.nflags++;
    if (br >= kMaxBranch) { c.overflow = true; return; }
    // explore the other outcome
    if (stop)
      var_dfs(c, k + 1, Tn, epsN, r + q.rgb[0] * a * T, g + q.rgb[1] * a * T, b + q.rgb[2] * a * T, br + 1);
    else
      var_emit(c, T, r, g, b);
    if (c.overflow) return;
  }
  if (stop) { var_emit(c, T, r, g, b); return; }
  var_dfs(c, k + 1, Tn, epsN, r + q.rgb[0] * a * T, g + q.rgb[1] * a * T, b + q.rgb[2] * a * T, br);
}

void var_dfs(VarCtx& c, size_t k, double T, double epsT, double r, double g, double b, int br) {
  const oc_settings& s = *c.s;
  const std::vector<int>& ord = *c.order;
  for (; k < ord.size(); ++k) {
    const Kept& e = (*c.L)[ord[k]];
    const Rec& rec = (*c.recs)[e.rec];
    bool inc = !rec.culled && e.araw >= s.alpha_min;
    bool amb = rec.near_amb || std::fabs(e.araw - s.alpha_min) <= s.band_safety * e.eps * s.alpha_min;
    if (!inc && !amb) continue;
    if (amb) {
      c.nflags++;
      if (br >= kMaxBranch) { c.overflow = true; return; }
      var_take(c, k, !inc, T, epsT, r, g, b, br + 1);
      if (c.overflow) return;
    }
    var_take(c, k, inc, T, epsT, r, g, b, br);
    return;
  }
  var_emit(c, T, r, g, b);
}

// All accepted colours of one pixel-level: the depth-order alternatives (each
// unsettled pair of neighbours up to the end of the FP64 traversal swapped or not)
// times the alternatives of the other decisions. Returns nvar.
int pixel_variants(const std::vector<Rec>& recs, const std::vector<Kept>& L, int nl, const oc_settings& s,
                   int stop_k, double* vbuf) {
  if (!(s.band_safety > 0.0)) return 0;
  std::vector<int> ord;
  for (int k = 0; k < (int)L.size(); ++k)
    if (L[k].idx < nl) ord.push_back(k);
  std::vector<int> ties;
  for (size_t j = 0; j + 1 < ord.size(); ++j) {
    if (ord[j] > stop_k) break;
    const Rec& a = recs[L[ord[j]].rec];
    const Rec& b = recs[L[ord[j + 1]].rec];
    if ((a.key_amb || b.key_amb) && std::nextafter(a.key, INFINITY) >= b.key) {
      if (!ties.empty() && ties.back() == (int)j - 1) return -1;  // three mutual near-ties
      ties.push_back((int)j);
    }
  }
  const int nt = (int)ties.size();
  if (nt > kMaxBranch) return -1;
  VarCtx c{&recs, &L, nullptr, &s, vbuf, 0, false, nt};
  for (int m = 0; m < (1 << nt); ++m) {
    std::vector<int> perm = ord;
    for (int t = 0; t < nt; ++t)
      if (m >> t & 1) std::swap(perm[ties[t]], perm[ties[t] + 1]);
    c.order = &perm;
    var_dfs(c, 0, 1.0, 0.0, 0.0, 0.0, 0.0, nt);
    if (c.overflow) return -1;
  }
  return c.nflags == 0 ? 0 : c.nout;
}

// ------------------------------------------------ finite differences (O8)
double kept_araw(const Rec& e, double px, double py) {
  const double dx = px - e.mx, dy = py - e.my;
  return e.o * std::exp(-0.5 * (e.A * dx * dx + 2.0 * e.B * dx * dy + e.C * dy * dy));
}

// The kept candidates of one pixel (alpha >= alpha_min) among a bucket's
// records in (key, index) order, leaving out one Gaussian, built only as far
// as the traversals ask for them.
struct LazyKept {
  const std::vector<int>* lst;
  const std::vector<Rec>* R;
  int skip_idx;
  double px, py, amin;
  size_t pos;
  std::vector<Kept> kept;
  bool extend() {
    while (pos < lst->size()) {
      const int ci = (*lst)[pos++];
      const Rec& e = (*R)[ci];
      if (e.idx == skip_idx) continue;
      const double a = kept_araw(e, px, py);
      if (a >= amin) { kept.push_back({ci, e.idx, a, 0.0, 0.0}); return true; }
    }
    return false;
  }
};

inline bool rec_before(const Rec& a, const Rec& b) { return a.key < b.key || (a.key == b.key && a.idx < b.idx); }

bool load_scene(Scene& sc, const oc_settings* s, int n, const float* params, int F, const float* res, int V,
                const float* cams) {
  if (!s || n < 0 || F < 1 || V < 1 || !params || !cams) return false;
  if (s->sh_degree < 0 || s->sh_degree > 3 || s->n_levels < 1 || s->n_levels > 8) return false;
  sc.s = *s;
  sc.n = n; sc.F = F; sc.V = V; sc.B = F * V;
  const int C = n_channels(s->sh_degree);
  sc.P.assign(params, params + (size_t)C * n);
  if (res && s->res_channels > 0) {
    sc.res.assign(res, res + (size_t)F * s->res_channels * n);
  } else {
    sc.s.res_channels = 0;
  }
  sc.cams.resize(sc.B);
  for (int b = 0; b < sc.B; ++b) {
    double c[16];
    for (int j = 0; j < 16; ++j) c[j] = cams[16 * b + j];
    sc.cams[b] = load_cam(c);
  }
  return true;
}

}  // namespace

extern "C" {

int oc_n_channels(int deg) { return n_channels(deg); }

// OpenMP threads of the following calls (n >= 1); returns the previous maximum.
int oc_set_threads(int n) {
#ifdef _OPENMP
  const int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
#else
  (void)n;
  return 1;
#endif
}

void oc_sh_basis(int deg, double x, double y, double z, double* Y) { sh_basis(deg, x, y, z, Y); }

void oc_quat_rot(const double* q, double* R) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double u[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  quat_rot(u, R);
}

void oc_quat_mul(const double* a, const double* b, double* out) { quat_mul(a, b, out); }

// Per (frame-view, Gaussian) projection: out[b][i][16] =
// {valid, tz, mx, my, cov_xx, cov_xy, cov_yy, A, B, C, o, r, g, b, radius, flags}.
int oc_project(const oc_settings* s, int n, const float* params, int F, const float* res, int V, const float* cams,
               double* out) {
  Scene sc;
  if (!load_scene(sc, s, n, params, F, res, V, cams)) return -1;
#pragma omp parallel for collapse(2) schedule(static)
  for (int b = 0; b < sc.B; ++b)
    for (int i = 0; i < n; ++i) {
      double* o = out + ((size_t)b * n + i) * 16;
      std::memset(o, 0, 16 * sizeof(double));
      const int f = b / V;
      double p[kMaxC];
      compose_frame(sc.s, n, sc.P.data(), sc.res.empty() ? nullptr : sc.res.data(), f, i, p);
      if (!all_finite(sc.s, p)) continue;
      const Cam& k = sc.cams[b];
      const double tz = k.R[6] * p[0] + k.R[7] * p[1] + k.R[8] * p[2] + k.t[2];
      o[1] = tz;
      if (!(tz > sc.s.near_plane)) continue;
      Proj<double> pr;
      if (!project(p, sc.s, k, pr)) continue;
      o[0] = 1.0;
      o[2] = pr.mx; o[3] = pr.my;
      o[4] = pr.s2d[0]; o[5] = pr.s2d[1]; o[6] = pr.s2d[2];
      o[7] = pr.A; o[8] = pr.B; o[9] = pr.C; o[10] = pr.o;
      o[11] = pr.rgb[0]; o[12] = pr.rgb[1]; o[13] = pr.rgb[2];
      o[14] = pr.radius; o[15] = pr.flags;
    }
  return 0;
}

// Renders all frame-views and levels.
//   mode: 0 = bucketed candidates, 1 = brute force (every Gaussian is a candidate)
//   n_sample / sample: if sample != NULL only these pixel ids (y * W + x) are
//     rendered, in every frame-view; outputs are then [B][L][...][n_sample].
//   image   [B][L][3][npix]     colour (FP64 decisions)
//   T_final [B][L][npix]        transmittance after the last contributor (or NULL)
//   ncontrib[B][L][npix]        number of contributors (or NULL)
//   sig     [B][L][npix]        event signature for finite differences (or NULL)
//   nvar    [B][L][npix]        number of accepted alternative colours, 0 if the
//                               pixel has no ambiguous decision, -1 if excluded
//   var     [B][L][npix][16][3] accepted colours (or NULL)
int oc_render(const oc_settings* s, int n, const float* params, int F, const float* res, int V, const float* cams,
              int mode, int64_t n_sample, const int64_t* sample, double* image, double* T_final, int32_t* ncontrib,
              uint64_t* sig, int32_t* nvar, double* var) {
  Scene sc;
  if (!load_scene(sc, s, n, params, F, res, V, cams)) return -1;
  const oc_settings& S = sc.s;
  const int64_t npix = sample ? n_sample : (int64_t)S.width * S.height;
  const int L = S.n_levels;
  for (int b = 0; b < sc.B; ++b) {
    std::vector<Rec> recs = project_view(sc, b);
    Buckets bk;
    if (mode == 0) bk = make_buckets(S, recs);
    std::vector<int> all;
    if (mode == 1) { all.resize(recs.size()); for (size_t j = 0; j < recs.size(); ++j) all[j] = (int)j; }
#pragma omp parallel
    {
      std::vector<Kept> kept;
      double vbuf[kMaxVar * 3];
#pragma omp for schedule(dynamic, 64)
      for (int64_t pi = 0; pi < npix; ++pi) {
        int64_t pix = sample ? sample[pi] : pi;
        int x = (int)(pix % S.width), y = (int)(pix / S.width);
        const int* cand;
        int ncand;
        if (mode == 0) {
          const std::vector<int>& lst = bk.lists[(size_t)(y / kBucket) * bk.bw + x / kBucket];
          cand = lst.data(); ncand = (int)lst.size();
        } else {
          cand = all.data(); ncand = (int)all.size();
        }
        pixel_candidates(recs, cand, ncand, x + 0.5, y + 0.5, S, kept);
        for (int l = 0; l < L; ++l) {
          const int nl = S.level_counts[l];
          PixOut po = composite(recs, kept, nl, S, nullptr);
          size_t o = ((size_t)b * L + l);
          for (int c = 0; c < 3; ++c) image[(o * 3 + c) * npix + pi] = po.rgb[c];
          if (T_final) T_final[o * npix + pi] = po.T;
          if (ncontrib) ncontrib[o * npix + pi] = po.ncontrib;
          if (sig) sig[o * npix + pi] = po.sig;
          if (nvar) {
            int nv = pixel_variants(recs, kept, nl, S, po.stop_k, vbuf);
            nvar[o * npix + pi] = nv;
            if (var && nv > 0) std::memcpy(var + (o * npix + pi) * kMaxVar * 3, vbuf, sizeof(double) * 3 * nv);
          }
        }
      }
    }
  }
  return 0;
}

}  // extern "C"

namespace {

// The analytic FP64 backward (O7). Pixel-level compositing gradients come from
// Eq. 2 written out; the projection Jacobian comes from dual numbers through the
// projection code. d_params_abs (or NULL) receives the absolute-term sums.
int backward_impl(const oc_settings* s, int n, const float* params, int F, const float* res, int V,
                  const float* cams, int mode, const double* d_image, double* d_params, double* d_res,
                  double* grad2d_out, double* d_params_abs) {
  Scene sc;
  if (!load_scene(sc, s, n, params, F, res, V, cams)) return -1;
  if (d_params_abs && (F != 1 || sc.s.res_channels > 0)) return -1;
  const oc_settings& S = sc.s;
  const int C = n_channels(S.sh_degree);
  const int L = S.n_levels;
  const int64_t npix = (int64_t)S.width * S.height;
  const int B = sc.B;
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  // dL / d(composed params of frame f) for every Gaussian
  std::vector<double> dcomp((size_t)F * n * C, 0.0);
  std::vector<double> dabs(d_params_abs ? (size_t)n * C : 0, 0.0);
  for (int b = 0; b < B; ++b) {
    const int f = b / V;
    std::vector<Rec> recs = project_view(sc, b);
    Buckets bk;
    if (mode == 0) bk = make_buckets(S, recs);
    std::vector<int> all;
    if (mode == 1) { all.resize(recs.size()); for (size_t j = 0; j < recs.size(); ++j) all[j] = (int)j; }
    std::vector<std::vector<double>> part(nt, std::vector<double>(recs.size() * 9, 0.0));
    std::vector<std::vector<double>> part_abs(d_params_abs ? nt : 0, std::vector<double>(recs.size() * 9, 0.0));
#pragma omp parallel
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      std::vector<double>& acc = part[tid];
      double* accabs = d_params_abs ? part_abs[tid].data() : nullptr;
      std::vector<Kept> kept;
      std::vector<int> contrib;
#pragma omp for schedule(dynamic, 64)
      for (int64_t pix = 0; pix < npix; ++pix) {
        int x = (int)(pix % S.width), y = (int)(pix / S.width);
        const int* cand;
        int ncand;
        if (mode == 0) {
          const std::vector<int>& lst = bk.lists[(size_t)(y / kBucket) * bk.bw + x / kBucket];
          cand = lst.data(); ncand = (int)lst.size();
        } else {
          cand = all.data(); ncand = (int)all.size();
        }
        const double px = x + 0.5, py = y + 0.5;
        bool any_w = false;
        for (int l = 0; l < L && !any_w; ++l)
          for (int c = 0; c < 3; ++c) any_w = any_w || d_image[(((size_t)b * L + l) * 3 + c) * npix + pix] != 0.0;
        if (!any_w) continue;
        pixel_candidates(recs, cand, ncand, px, py, S, kept);
        for (int l = 0; l < L; ++l) {
          const size_t o = (size_t)b * L + l;
          double w[3];
          for (int c = 0; c < 3; ++c) w[c] = d_image[(o * 3 + c) * npix + pix];
          if (w[0] == 0.0 && w[1] == 0.0 && w[2] == 0.0) continue;
          PixOut po = composite(recs, kept, S.level_counts[l], S, &contrib);
          // transmittance before each contributor
          std::vector<double> Tb(contrib.size());
          double T = 1.0;
          for (size_t j = 0; j < contrib.size(); ++j) {
            Tb[j] = T;
            T *= 1.0 - std::min(S.alpha_max, kept[contrib[j]].araw);
          }
          // suffix colour behind contributor j, including the background
          double Sfx[3] = {po.T * S.bg[0], po.T * S.bg[1], po.T * S.bg[2]};
          for (int j = (int)contrib.size() - 1; j >= 0; --j) {
            const Kept& e = kept[contrib[j]];
            const Rec& r = recs[e.rec];
            const double a = std::min(S.alpha_max, e.araw);
            double* g = acc.data() + (size_t)e.rec * 9;
            double dLda = 0.0, dLda_abs = 0.0;
            for (int c = 0; c < 3; ++c) {
              g[6 + c] += w[c] * a * Tb[j];                               // dC/dc_i = alpha_i T_i
              dLda += w[c] * (r.rgb[c] * Tb[j] - Sfx[c] / (1.0 - a));    // dC/dalpha_i
              dLda_abs += std::fabs(w[c]) * (std::fabs(r.rgb[c]) * Tb[j] + std::fabs(Sfx[c]) / (1.0 - a));
              Sfx[c] += r.rgb[c] * a * Tb[j];
            }
            double* ga = accabs ? accabs + (size_t)e.rec * 9 : nullptr;
            if (ga)
              for (int c = 0; c < 3; ++c) ga[6 + c] += std::fabs(w[c]) * a * Tb[j];
            if (e.araw > S.alpha_max) continue;  // clamped: alpha does not depend on o, G
            g[5] += dLda * e.G;                    // d alpha / d o
            const double dpow = dLda * e.araw;    // d alpha / d power = o G
            const double dx = px - r.mx, dy = py - r.my;
            g[0] += dpow * (r.A * dx + r.B * dy);  // d power / d mx
            g[1] += dpow * (r.B * dx + r.C * dy);
            g[2] += dpow * (-0.5 * dx * dx);
            g[3] += dpow * (-dx * dy);
            g[4] += dpow * (-0.5 * dy * dy);
            if (ga) {  // the same sums of the absolute values of their terms
              const double pa = dLda_abs * e.araw;
              ga[5] += dLda_abs * e.G;
              ga[0] += pa * (std::fabs(r.A * dx) + std::fabs(r.B * dy));
              ga[1] += pa * (std::fabs(r.B * dx) + std::fabs(r.C * dy));
              ga[2] += pa * 0.5 * dx * dx;
              ga[3] += pa * std::fabs(dx * dy);
              ga[4] += pa * 0.5 * dy * dy;
            }
          }
        }
      }
    }
    // reduce thread partials
    std::vector<double> gsum(recs.size() * 9, 0.0), gabs(d_params_abs ? recs.size() * 9 : 0, 0.0);
    for (int t = 0; t < nt; ++t)
      for (size_t j = 0; j < gsum.size(); ++j) gsum[j] += part[t][j];
    for (size_t t = 0; t < part_abs.size(); ++t)
      for (size_t j = 0; j < gabs.size(); ++j) gabs[j] += part_abs[t][j];
    if (grad2d_out) {
      double* go = grad2d_out + (size_t)b * n * 9;
      std::memset(go, 0, sizeof(double) * n * 9);
      for (size_t j = 0; j < recs.size(); ++j)
        for (int c = 0; c < 9; ++c) go[(size_t)recs[j].idx * 9 + c] = gsum[j * 9 + c];
    }
    // projection Jacobian by dual numbers, per visible Gaussian
    const Cam& k = sc.cams[b];
#pragma omp parallel for schedule(dynamic, 256)
    for (int j = 0; j < (int)recs.size(); ++j) {
      const double* g = gsum.data() + (size_t)j * 9;
      bool any = false;
      for (int c = 0; c < 9; ++c) any = any || (g[c] != 0.0);
      if (!any) continue;
      const int i = recs[j].idx;
      double p[kMaxC];
      compose_frame(S, n, sc.P.data(), sc.res.empty() ? nullptr : sc.res.data(), f, i, p);
      Dual<kMaxC> pd[kMaxC];
      for (int c = 0; c < C; ++c) { pd[c] = Dual<kMaxC>(p[c]); pd[c].d[c] = 1.0; }
      Proj<Dual<kMaxC>> pr;
      if (!project(pd, S, k, pr)) continue;
      const Dual<kMaxC>* outs[9] = {&pr.mx, &pr.my, &pr.A, &pr.B, &pr.C, &pr.o, &pr.rgb[0], &pr.rgb[1], &pr.rgb[2]};
      double* dc = dcomp.data() + ((size_t)f * n + i) * C;
      for (int c = 0; c < C; ++c) {
        double v = 0.0;
        for (int m = 0; m < 9; ++m) v += g[m] * outs[m]->d[c];
        dc[c] += v;  // each (f, i) is written by one thread per view
      }
      if (d_params_abs) {
        const double* ga = gabs.data() + (size_t)j * 9;
        double* da = dabs.data() + (size_t)i * C;
        for (int c = 0; c < C; ++c)
          for (int m = 0; m < 9; ++m) da[c] += ga[m] * std::fabs(outs[m]->d[c]);
      }
    }
  }
  // frame chain backward (O1): sums are identity-Jacobian; the quaternion
  // product chain is differentiated with dual numbers.
  const int Rc = S.res_channels;
  std::memset(d_params, 0, sizeof(double) * C * n);
  if (d_res && Rc > 0) std::memset(d_res, 0, sizeof(double) * F * Rc * n);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    // quaternions of every frame, forward
    std::vector<std::array<double, 4>> qs(F + 1);
    for (int c = 0; c < 4; ++c) qs[0][c] = sc.P[(size_t)(6 + c) * n + i];
    for (int f = 0; f < F; ++f) {
      if (Rc > 0) {
        double dq[4];
        for (int c = 0; c < 4; ++c) dq[c] = sc.res[(size_t)f * Rc * n + (size_t)(3 + c) * n + i];
        quat_mul(dq, qs[f].data(), qs[f + 1].data());
      } else {
        qs[f + 1] = qs[f];
      }
    }
    std::vector<double> acc(C, 0.0);  // suffix sum over frames of d composed params
    double carry_q[4] = {0, 0, 0, 0};
    for (int f = F - 1; f >= 0; --f) {
      const double* dc = dcomp.data() + ((size_t)f * n + i) * C;
      for (int c = 0; c < C; ++c) acc[c] += dc[c];
      double gq[4];
      for (int c = 0; c < 4; ++c) gq[c] = dc[6 + c] + carry_q[c];
      const bool zero_q = gq[0] == 0.0 && gq[1] == 0.0 && gq[2] == 0.0 && gq[3] == 0.0;
      if (Rc > 0) {
        double* dr = d_res ? d_res + (size_t)f * Rc * n : nullptr;
        if (dr) {
          for (int c = 0; c < 3; ++c) dr[(size_t)c * n + i] = acc[c];
          dr[(size_t)7 * n + i] = acc[10];
          if (Rc >= 11) for (int c = 0; c < 3; ++c) dr[(size_t)(8 + c) * n + i] = acc[3 + c];
          if (Rc > 11) for (int c = 11; c < Rc && c < C; ++c) dr[(size_t)c * n + i] = acc[c];
        }
        Dual<8> a[4], bq[4], o[4];
        for (int c = 0; c < 4; ++c) {
          a[c] = Dual<8>(sc.res[(size_t)f * Rc * n + (size_t)(3 + c) * n + i]); a[c].d[c] = 1.0;
          bq[c] = Dual<8>(qs[f][c]); bq[c].d[4 + c] = 1.0;
        }
        quat_mul(a, bq, o);
        double gdq[4] = {0, 0, 0, 0}, gprev[4] = {0, 0, 0, 0};
        if (!zero_q)  // a zero cotangent gives a zero gradient, whatever the (possibly non-finite) deltas
          for (int m = 0; m < 4; ++m)
            for (int c = 0; c < 4; ++c) { gdq[c] += gq[m] * o[m].d[c]; gprev[c] += gq[m] * o[m].d[4 + c]; }
        if (dr) for (int c = 0; c < 4; ++c) dr[(size_t)(3 + c) * n + i] = gdq[c];
        for (int c = 0; c < 4; ++c) carry_q[c] = gprev[c];
      } else {
        for (int c = 0; c < 4; ++c) carry_q[c] = gq[c];
      }
    }
    for (int c = 0; c < C; ++c) d_params[(size_t)c * n + i] = acc[c];
    // the mean/logit/log-scale/SH channels of the keyframe receive the full
    // sum over frames; the quaternion receives the chain-rule carry.
    for (int c = 0; c < 4; ++c) d_params[(size_t)(6 + c) * n + i] = carry_q[c];
  }
  if (d_params_abs)
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < C; ++c) d_params_abs[(size_t)c * n + i] = dabs[(size_t)i * C + c];
  return 0;
}

}  // namespace

extern "C" {

// Analytic FP64 backward (O7) of  L = sum d_image * image  over all
// frame-views, levels, channels and pixels.
//   d_image  [B][L][3][H][W]
//   d_params [C][n]             (overwritten)
//   d_res    [F][R][n]          (overwritten; may be NULL)
//   grad2d   [B][n][9]          (overwritten; may be NULL): dL / (mx, my, A, B, C, o, r, g, b)
int oc_backward(const oc_settings* s, int n, const float* params, int F, const float* res, int V, const float* cams,
                int mode, const double* d_image, double* d_params, double* d_res, double* grad2d_out) {
  return backward_impl(s, n, params, F, res, V, cams, mode, d_image, d_params, d_res, grad2d_out, nullptr);
}

// The same sums over pixels and views as oc_backward's d_params (one frame, no
// residuals), taken of the absolute values of their terms: the scale against
// which the float32 rounding error of a gradient is bounded where its terms
// cancel.
int oc_backward_abs(const oc_settings* s, int n, const float* params, int V, const float* cams, int mode,
                    const double* d_image, double* d_params, double* d_params_abs) {
  if (!d_params_abs) return -1;
  return backward_impl(s, n, params, 1, nullptr, V, cams, mode, d_image, d_params, nullptr, nullptr, d_params_abs);
}

// Central finite differences (O8) of  L = sum d_image * image  (one frame,
// every view and level) with respect to single parameters, re-compositing only
// the pixels inside the perturbed Gaussian's footprint (the union of its discs
// at every perturbed state, plus 2 px).
//   gauss[m], chan[m]  the Gaussian and parameter channel of each request
//   h                  absolute step
//   fd_out[m]          dL/dtheta
//   status_out[m]      bit 0: some pixel-level used a one-sided difference,
//                      bit 1: some pixel-level used the step h/10,
//                      bit 2: some pixel-level was skipped (a kink on both
//                      sides at both steps), bit 3: invalid request
//   skipped_out[m]     number of skipped pixel-levels
// A pixel-level whose event signature (see composite_with) at theta + step or
// theta - step differs from the one at theta is a kink: the side that keeps
// the signature gives a one-sided difference; if neither does, the step h/10
// is tried; if that fails too the pixel-level is skipped and counted.
int oc_fd(const oc_settings* s_in, int n, const float* params, int V, const float* cams, const double* d_image,
          int64_t m, const int32_t* gauss, const int32_t* chan, double h, double* fd_out, int32_t* status_out,
          int64_t* skipped_out) {
  if (!s_in || !gauss || !chan || !fd_out || !status_out || !skipped_out || !d_image || m < 0 || !(h > 0.0))
    return -1;
  oc_settings s0 = *s_in;
  s0.band_safety = 0.0;
  s0.res_channels = 0;
  Scene sc;
  if (!load_scene(sc, &s0, n, params, 1, nullptr, V, cams)) return -1;
  const oc_settings& S = sc.s;
  const int C = n_channels(S.sh_degree);
  const int L = S.n_levels;
  const int W = S.width, H = S.height;
  const int64_t npix = (int64_t)W * H;
  std::vector<std::vector<Rec>> recs(V);
  std::vector<Buckets> bks(V);
  for (int b = 0; b < V; ++b) {
    recs[b] = project_view(sc, b);
    bks[b] = make_buckets(S, recs[b]);
  }
  // requests grouped by Gaussian
  std::vector<int> order(m);
  for (int64_t j = 0; j < m; ++j) order[j] = (int)j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return gauss[a] < gauss[b]; });
  std::vector<std::pair<int64_t, int64_t>> groups;
  for (int64_t j = 0; j < m;) {
    int64_t e = j;
    while (e < m && gauss[order[e]] == gauss[order[j]]) ++e;
    groups.push_back({j, e});
    j = e;
  }
  const double steps[2] = {h, 0.1 * h};
#pragma omp parallel
  {
    LazyKept lk;
    std::vector<int> E;
    std::vector<double> Tp, Cp, Ps, Ss;
#pragma omp for schedule(dynamic, 1)
    for (int64_t gi = 0; gi < (int64_t)groups.size(); ++gi) {
      const int64_t j0 = groups[gi].first, j1 = groups[gi].second;
      const int i = gauss[order[j0]];
      const int nreq = (int)(j1 - j0);
      std::vector<double> acc(nreq, 0.0);
      std::vector<int32_t> st(nreq, 0);
      std::vector<int64_t> skipped(nreq, 0);
      if (i < 0 || i >= n) {
        for (int r = 0; r < nreq; ++r) { fd_out[order[j0 + r]] = 0.0; status_out[order[j0 + r]] = 8; skipped_out[order[j0 + r]] = 0; }
        continue;
      }
      double p0[kMaxC];
      for (int c = 0; c < C; ++c) p0[c] = sc.P[(size_t)c * n + i];
      for (int b = 0; b < V; ++b) {
        const Cam& k = sc.cams[b];
        // states: 0 = theta, then per request r: 1 + 4 r + {0: +h, 1: -h, 2: +h/10, 3: -h/10}
        const int ns = 1 + 4 * nreq;
        std::vector<Rec> srec(ns);
        std::vector<char> svis(ns, 0);
        double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
        for (int q = 0; q < ns; ++q) {
          double p[kMaxC];
          std::memcpy(p, p0, sizeof(double) * C);
          if (q > 0) {
            const int r = (q - 1) / 4, v = (q - 1) % 4;
            const int ch = chan[order[j0 + r]];
            if (ch < 0 || ch >= C) continue;
            p[ch] += (v % 2 == 0 ? 1.0 : -1.0) * steps[v / 2];
          }
          svis[q] = make_record(S, k, p, i, 0, srec[q]) ? 1 : 0;
          if (svis[q]) {
            const Rec& e = srec[q];
            const double rad = e.radius + 2.0;
            bx0 = std::min(bx0, e.mx - rad); bx1 = std::max(bx1, e.mx + rad);
            by0 = std::min(by0, e.my - rad); by1 = std::max(by1, e.my + rad);
          }
        }
        if (bx0 > bx1) continue;  // invisible in every state
        const int u0 = std::max(0, (int)std::floor(bx0 - 0.5)), u1 = std::min(W - 1, (int)std::ceil(bx1 - 0.5));
        const int v0 = std::max(0, (int)std::floor(by0 - 0.5)), v1 = std::min(H - 1, (int)std::ceil(by1 - 0.5));
        const std::vector<Rec>& R = recs[b];
        std::vector<PixOut> po(ns);
        std::vector<char> have(ns);
        for (int y = v0; y <= v1; ++y)
          for (int x = u0; x <= u1; ++x) {
            const double px = x + 0.5, py = y + 0.5;
            const std::vector<int>& lst = bks[b].lists[(size_t)(y / kBucket) * bks[b].bw + x / kBucket];
            lk.lst = &lst; lk.R = &R; lk.skip_idx = i; lk.px = px; lk.py = py; lk.amin = S.alpha_min; lk.pos = 0;
            lk.kept.clear();
            for (int l = 0; l < L; ++l) {
              const int nl = S.level_counts[l];
              if (i >= nl) continue;
              double w[3];
              bool any = false;
              for (int c = 0; c < 3; ++c) {
                w[c] = d_image[(((size_t)b * L + l) * 3 + c) * npix + (size_t)y * W + x];
                any = any || w[c] != 0.0;
              }
              if (!any) continue;
              std::fill(have.begin(), have.end(), 0);
              // The level's kept entries E in order up to where the traversal without
              // the perturbed Gaussian stops, with prefix transmittance and colour.
              // Then for each state only the perturbed entry and the stop position
              // behind it are evaluated: behind it the colour is T' times a suffix
              // sum and the stop is where T' times a suffix product of (1 - alpha)
              // falls below t_stop (a binary search: the product does not increase).
              E.clear(); Tp.clear(); Cp.clear();
              double T = 1.0, Cc[3] = {0.0, 0.0, 0.0};
              int stop_pre = -1;
              for (size_t k = 0;; ++k) {
                if (k >= lk.kept.size() && !lk.extend()) break;
                const Kept& e = lk.kept[k];
                const Rec& r = R[e.rec];
                if (r.idx >= nl) continue;
                Tp.push_back(T);
                for (int c = 0; c < 3; ++c) Cp.push_back(Cc[c]);
                E.push_back((int)k);
                const double a = std::min(S.alpha_max, e.araw);
                const double Tn = T * (1.0 - a);
                if (Tn < S.t_stop) { stop_pre = (int)E.size() - 1; break; }
                for (int c = 0; c < 3; ++c) Cc[c] += r.rgb[c] * a * T;
                T = Tn;
              }
              const int ne = (int)E.size();
              Tp.push_back(T);
              for (int c = 0; c < 3; ++c) Cp.push_back(Cc[c]);
              const int end_pre = stop_pre >= 0 ? stop_pre : ne;  // entries composited without x
              auto ip_of = [&](const Rec& x) {
                int lo = 0, hi = ne;
                while (lo < hi) {
                  const int mid = (lo + hi) / 2;
                  if (rec_before(R[lk.kept[E[mid]].rec], x)) lo = mid + 1; else hi = mid;
                }
                return lo;
              };
              const int ip0 = svis[0] ? ip_of(srec[0]) : 0;
              // suffix products / sums from ip0 over E[ip0 .. end_pre]
              Ps.clear(); Ss.clear();
              {
                double P = 1.0, Sr[3] = {0.0, 0.0, 0.0};
                for (int k = ip0; k < ne; ++k) {
                  const Kept& e = lk.kept[E[k]];
                  const double a = std::min(S.alpha_max, e.araw);
                  for (int c = 0; c < 3; ++c) Sr[c] += R[e.rec].rgb[c] * a * P;
                  P *= 1.0 - a;
                  Ps.push_back(P);
                  for (int c = 0; c < 3; ++c) Ss.push_back(Sr[c]);
                }
              }
              auto eval = [&](int q, PixOut& o) {
                const Rec* x = svis[q] ? &srec[q] : nullptr;
                const double ax = x ? kept_araw(*x, px, py) : 0.0;
                const bool inc = x && ax >= S.alpha_min;
                int ip = inc ? ip_of(*x) : ip0;
                uint64_t h = 1469598103934665603ULL;
                if (!inc || ip > end_pre) {  // x plays no part: the traversal without it
                  for (int c = 0; c < 3; ++c) o.rgb[c] = Cp[3 * end_pre + c] + Tp[end_pre] * S.bg[c];
                  o.sig = mix(h, 0x11ULL + (uint64_t)end_pre);
                  return;
                }
                h = mix(h, 0x22ULL + (uint64_t)ip);
                const double a = std::min(S.alpha_max, ax);
                h = mix(h, (ax > S.alpha_max ? 1ULL : 0ULL) + 2ULL * (uint64_t)x->flags);
                const double T0 = Tp[ip];
                const double Tn = T0 * (1.0 - a);
                if (Tn < S.t_stop) {
                  for (int c = 0; c < 3; ++c) o.rgb[c] = Cp[3 * ip + c] + T0 * S.bg[c];
                  o.sig = mix(h, 0x33ULL);
                  return;
                }
                if (ip != ip0) {  // another order than at theta: a kink; the colour is not used
                  o.rgb[0] = o.rgb[1] = o.rgb[2] = 0.0;
                  o.sig = mix(h, 0x44ULL);
                  return;
                }
                // first k in [ip, ne) with Tn * P(k) < t_stop (P(k) includes entry k)
                int lo = ip, hi = ne;
                while (lo < hi) {
                  const int mid = (lo + hi) / 2;
                  if (Tn * Ps[mid - ip0] < S.t_stop) hi = mid; else lo = mid + 1;
                }
                const int ks = lo;  // entries ip .. ks-1 are composited behind x
                double Tf = Tn;
                for (int c = 0; c < 3; ++c) o.rgb[c] = Cp[3 * ip + c] + x->rgb[c] * a * T0;
                if (ks > ip) {
                  for (int c = 0; c < 3; ++c) o.rgb[c] += Tn * Ss[3 * (ks - 1 - ip0) + c];
                  Tf = Tn * Ps[ks - 1 - ip0];
                }
                for (int c = 0; c < 3; ++c) o.rgb[c] += Tf * S.bg[c];
                o.sig = mix(h, 0x55ULL + (uint64_t)ks);
              };
              auto get = [&](int q) -> const PixOut& {
                if (!have[q]) {
                  eval(q, po[q]);
                  have[q] = 1;
                }
                return po[q];
              };
              auto val = [&](int q) {
                const PixOut& o = get(q);
                return w[0] * o.rgb[0] + w[1] * o.rgb[1] + w[2] * o.rgb[2];
              };
              const uint64_t s0g = get(0).sig;
              for (int r = 0; r < nreq; ++r) {
                const int qb = 1 + 4 * r;
                bool done = false;
                for (int t = 0; t < 2 && !done; ++t) {
                  const int qp = qb + 2 * t, qm = qb + 2 * t + 1;
                  const bool okp = get(qp).sig == s0g, okm = get(qm).sig == s0g;
                  if (okp && okm) {
                    acc[r] += (val(qp) - val(qm)) / (2.0 * steps[t]);
                  } else if (okp) {
                    acc[r] += (val(qp) - val(0)) / steps[t];
                    st[r] |= 1;
                  } else if (okm) {
                    acc[r] += (val(0) - val(qm)) / steps[t];
                    st[r] |= 1;
                  } else {
                    continue;
                  }
                  if (t == 1) st[r] |= 2;
                  done = true;
                }
                if (!done) { st[r] |= 4; skipped[r]++; }
              }
            }
          }
      }
      for (int r = 0; r < nreq; ++r) {
        const int j = order[j0 + r];
        const int ch = chan[j];
        fd_out[j] = acc[r];
        status_out[j] = (ch < 0 || ch >= C) ? 8 : st[r];
        skipped_out[j] = skipped[r];
      }
    }
  }
  return 0;
}

}  // extern "C"

