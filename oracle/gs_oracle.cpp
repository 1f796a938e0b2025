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
//  * order: increasing camera-space depth, ties broken by lower index. The
//    depth used for the ORDER (and for the near-plane cull) is the float32
//    value fmaf(R[8], z, fmaf(R[7], y, fmaf(R[6], x, t[2]))) of float32 inputs,
//    i.e. the same precision the GPU kernel decides it in; all other
//    arithmetic is FP64;
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
  // half-widths of the bands in which an FP32 evaluation may take the other
  // outcome of a decision (see oc_render)
  double band_alpha_rel, band_tstop_abs;
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
  float Rf[9], tf[3];
};

Cam load_cam(const double* c) {
  Cam k;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) k.R[3 * i + j] = c[4 * i + j];
    k.t[i] = c[4 * i + 3];
  }
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  for (int i = 0; i < 9; ++i) k.Rf[i] = (float)k.R[i];
  for (int i = 0; i < 3; ++i) k.tf[i] = (float)k.t[i];
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

// Float32 mean of frame f (sequential float32 sums of the deltas), used only
// for the depth order and near-plane decision.
void compose_mean_f32(const oc_settings& s, int n, const float* P32, const float* res32, int f, int i, float m[3]) {
  for (int c = 0; c < 3; ++c) m[c] = P32[(size_t)c * n + i];
  if (!res32 || s.res_channels <= 0) return;
  for (int t = 0; t <= f; ++t)
    for (int c = 0; c < 3; ++c) m[c] = m[c] + res32[(size_t)t * s.res_channels * n + (size_t)c * n + i];
}

inline float depth_key_f32(const Cam& k, const float m[3]) {
  return std::fma(k.Rf[8], m[2], std::fma(k.Rf[7], m[1], std::fma(k.Rf[6], m[0], k.tf[2])));
}

// ------------------------------------------------------ projection (O2-O4)
template <class T>
struct Proj {
  T mx, my, A, B, C, o, rgb[3];
  // diagnostics (value only)
  double s2d[3], tz, radius;
  int flags;  // bit0 x-clamp, bit1 y-clamp, bit2..4 colour clamp r,g,b
};

// Projects one Gaussian with composed params p (C channels) into camera k.
// Returns false if it is culled (non-positive quaternion norm, det <= 0).
// The near-plane test is decided by the caller on the float32 depth key.
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
  float key;  // float32 depth (order key)
  double mx, my, A, B, C, o, rgb[3], radius;
};

struct Scene {
  oc_settings s;
  int n, F, V, B;
  std::vector<double> P, res;          // FP64 copies of the float32 inputs
  std::vector<float> P32, res32;
  std::vector<Cam> cams;
};

// All visible records of frame-view b, sorted by (key, index).
std::vector<Rec> project_view(const Scene& sc, int b) {
  const oc_settings& s = sc.s;
  const int n = sc.n;
  const int f = b / sc.V;
  const Cam& k = sc.cams[b];
  std::vector<Rec> out;
  out.reserve(n);
  const double* res = sc.res.empty() ? nullptr : sc.res.data();
  const float* res32 = sc.res32.empty() ? nullptr : sc.res32.data();
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
      float m32[3];
      compose_mean_f32(s, n, sc.P32.data(), res32, f, i, m32);
      float key = depth_key_f32(k, m32);
      if (!(key > (float)s.near_plane)) continue;
      compose_frame(s, n, sc.P.data(), res, f, i, p);
      Proj<double> pr;
      if (!project(p, s, k, pr)) continue;
      if (!(pr.o >= s.alpha_min)) continue;  // can never reach alpha_min
      Rec r;
      r.idx = i; r.key = key;
      r.mx = pr.mx; r.my = pr.my; r.A = pr.A; r.B = pr.B; r.C = pr.C; r.o = pr.o;
      for (int c = 0; c < 3; ++c) r.rgb[c] = pr.rgb[c];
      r.radius = pr.radius;
      part[tid].push_back(r);
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
};

// Per-pixel scan (O5): candidates with o * G >= alpha_min (or within the
// ambiguity band of it), in order.
void pixel_candidates(const std::vector<Rec>& recs, const int* cand, int ncand, double px, double py,
                      const oc_settings& s, std::vector<Kept>& out) {
  out.clear();
  const double lo = s.alpha_min * (1.0 - s.band_alpha_rel);
  for (int j = 0; j < ncand; ++j) {
    const Rec& e = recs[cand ? cand[j] : j];
    double dx = px - e.mx, dy = py - e.my;
    double power = -0.5 * (e.A * dx * dx + 2.0 * e.B * dx * dy + e.C * dy * dy);
    double G = std::exp(power);
    double araw = e.o * G;
    if (araw >= lo) out.push_back({cand ? cand[j] : j, e.idx, araw, G});
  }
}

struct PixOut {
  double rgb[3];
  double T;
  int ncontrib;
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
  o.sig = h;
  return o;
}

// Alternative outcomes. A decision whose FP64 margin is inside the band that
// a float32 evaluation can cross (alpha_min cut within band_alpha_rel of
// alpha_min, T-stop test within band_tstop_abs of t_stop) is explored both
// ways, up to kMaxBranch decisions on one path; the colours of all explored
// paths are the accepted results of the pixel. If more ambiguous decisions
// lie on one path the pixel is marked as excluded (nvar = -1).
constexpr int kMaxBranch = 4;
constexpr int kMaxVar = 1 << kMaxBranch;

struct VarCtx {
  const std::vector<Rec>* recs;
  const std::vector<Kept>* L;
  int nl;
  const oc_settings* s;
  double* out;  // [kMaxVar][3]
  int nout;
  bool overflow;
  int nflags;
};

void var_dfs(VarCtx& c, size_t k, double T, double r, double g, double b, int br);

void var_take(VarCtx& c, size_t k, bool include, double T, double r, double g, double b, int br) {
  const oc_settings& s = *c.s;
  if (!include) { var_dfs(c, k + 1, T, r, g, b, br); return; }
  const Kept& e = (*c.L)[k];
  double a = std::min(s.alpha_max, e.araw);
  double Tn = T * (1.0 - a);
  bool stop = Tn < s.t_stop;
  if (std::fabs(Tn - s.t_stop) < s.band_tstop_abs) {
    c.nflags++;
    if (br >= kMaxBranch) { c.overflow = true; return; }
    // explore the other outcome
    if (stop) {
      const Rec& q = (*c.recs)[e.rec];
      var_dfs(c, k + 1, Tn, r + q.rgb[0] * a * T, g + q.rgb[1] * a * T, b + q.rgb[2] * a * T, br + 1);
    } else {
      if (c.nout < kMaxVar) {
        double* o = c.out + 3 * c.nout++;
        o[0] = r + T * s.bg[0]; o[1] = g + T * s.bg[1]; o[2] = b + T * s.bg[2];
      }
    }
  }
  if (stop) {
    if (c.nout < kMaxVar) {
      double* o = c.out + 3 * c.nout++;
      o[0] = r + T * s.bg[0]; o[1] = g + T * s.bg[1]; o[2] = b + T * s.bg[2];
    }
    return;
  }
  const Rec& q = (*c.recs)[e.rec];
  var_dfs(c, k + 1, Tn, r + q.rgb[0] * a * T, g + q.rgb[1] * a * T, b + q.rgb[2] * a * T, br);
}

void var_dfs(VarCtx& c, size_t k, double T, double r, double g, double b, int br) {
  const oc_settings& s = *c.s;
  const std::vector<Kept>& L = *c.L;
  for (; k < L.size(); ++k) {
    const Kept& e = L[k];
    if (e.idx >= c.nl) continue;
    bool inc = e.araw >= s.alpha_min;
    if (std::fabs(e.araw - s.alpha_min) < s.band_alpha_rel * s.alpha_min) {
      c.nflags++;
      if (br >= kMaxBranch) { c.overflow = true; return; }
      var_take(c, k, !inc, T, r, g, b, br + 1);
      if (c.overflow) return;
    }
    var_take(c, k, inc, T, r, g, b, br);
    return;
  }
  if (c.nout < kMaxVar) {
    double* o = c.out + 3 * c.nout++;
    o[0] = r + T * s.bg[0]; o[1] = g + T * s.bg[1]; o[2] = b + T * s.bg[2];
  }
}

bool load_scene(Scene& sc, const oc_settings* s, int n, const float* params, int F, const float* res, int V,
                const float* cams) {
  if (!s || n < 0 || F < 1 || V < 1 || !params || !cams) return false;
  if (s->sh_degree < 0 || s->sh_degree > 3 || s->n_levels < 1 || s->n_levels > 8) return false;
  sc.s = *s;
  sc.n = n; sc.F = F; sc.V = V; sc.B = F * V;
  const int C = n_channels(s->sh_degree);
  sc.P32.assign(params, params + (size_t)C * n);
  sc.P.assign(sc.P32.begin(), sc.P32.end());
  if (res && s->res_channels > 0) {
    sc.res32.assign(res, res + (size_t)F * s->res_channels * n);
    sc.res.assign(sc.res32.begin(), sc.res32.end());
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

void oc_sh_basis(int deg, double x, double y, double z, double* Y) { sh_basis(deg, x, y, z, Y); }

void oc_quat_rot(const double* q, double* R) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double u[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  quat_rot(u, R);
}

void oc_quat_mul(const double* a, const double* b, double* out) { quat_mul(a, b, out); }

// Per (frame-view, Gaussian) projection: out[b][i][16] =
// {valid, tz(f32 key), mx, my, cov_xx, cov_xy, cov_yy, A, B, C, o, r, g, b, radius, flags}.
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
      float m32[3];
      compose_mean_f32(sc.s, n, sc.P32.data(), sc.res32.empty() ? nullptr : sc.res32.data(), f, i, m32);
      float key = depth_key_f32(sc.cams[b], m32);
      o[1] = key;
      if (!(key > (float)sc.s.near_plane)) continue;
      double p[kMaxC];
      compose_frame(sc.s, n, sc.P.data(), sc.res.empty() ? nullptr : sc.res.data(), f, i, p);
      Proj<double> pr;
      if (!project(p, sc.s, sc.cams[b], pr)) continue;
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
            VarCtx c{&recs, &kept, nl, &S, vbuf, 0, false, 0};
            var_dfs(c, 0, 1.0, 0.0, 0.0, 0.0, 0);
            int nv = c.overflow ? -1 : (c.nflags == 0 ? 0 : c.nout);
            nvar[o * npix + pi] = nv;
            if (var && nv > 0) std::memcpy(var + (o * npix + pi) * kMaxVar * 3, vbuf, sizeof(double) * 3 * nv);
          }
        }
      }
    }
  }
  return 0;
}

// Analytic FP64 backward (O7) of  L = sum d_image * image  over all
// frame-views, levels, channels and pixels.
//   d_image  [B][L][3][H][W]
//   d_params [C][n]             (overwritten)
//   d_res    [F][R][n]          (overwritten; may be NULL)
//   grad2d   [B][n][9]          (overwritten; may be NULL): dL / (mx, my, A, B, C, o, r, g, b)
// Pixel-level compositing gradients come from Eq. 2 written out; the
// projection Jacobian comes from dual numbers through the projection code.
int oc_backward(const oc_settings* s, int n, const float* params, int F, const float* res, int V, const float* cams,
                int mode, const double* d_image, double* d_params, double* d_res, double* grad2d_out) {
  Scene sc;
  if (!load_scene(sc, s, n, params, F, res, V, cams)) return -1;
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
  std::vector<double> g2((size_t)n * 9);
  for (int b = 0; b < B; ++b) {
    const int f = b / V;
    std::vector<Rec> recs = project_view(sc, b);
    Buckets bk;
    if (mode == 0) bk = make_buckets(S, recs);
    std::vector<int> all;
    if (mode == 1) { all.resize(recs.size()); for (size_t j = 0; j < recs.size(); ++j) all[j] = (int)j; }
    std::vector<std::vector<double>> part(nt, std::vector<double>(recs.size() * 9, 0.0));
#pragma omp parallel
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      std::vector<double>& acc = part[tid];
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
            double dLda = 0.0;
            for (int c = 0; c < 3; ++c) {
              g[6 + c] += w[c] * a * Tb[j];                               // dC/dc_i = alpha_i T_i
              dLda += w[c] * (r.rgb[c] * Tb[j] - Sfx[c] / (1.0 - a));    // dC/dalpha_i
              Sfx[c] += r.rgb[c] * a * Tb[j];
            }
            if (e.araw > S.alpha_max) continue;  // clamped: alpha does not depend on o, G
            g[5] += dLda * e.G;                    // d alpha / d o
            const double dpow = dLda * e.araw;    // d alpha / d power = o G
            const double dx = px - r.mx, dy = py - r.my;
            g[0] += dpow * (r.A * dx + r.B * dy);  // d power / d mx
            g[1] += dpow * (r.B * dx + r.C * dy);
            g[2] += dpow * (-0.5 * dx * dx);
            g[3] += dpow * (-dx * dy);
            g[4] += dpow * (-0.5 * dy * dy);
          }
        }
      }
    }
    // reduce thread partials
    std::vector<double> gsum(recs.size() * 9, 0.0);
    for (int t = 0; t < nt; ++t)
      for (size_t j = 0; j < gsum.size(); ++j) gsum[j] += part[t][j];
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
  return 0;
}

}  // extern "C"
