// gfx950 kernels of the differentiable Gaussian rasterizer.
//
// Pipeline of one forward (all frames, views and layers in the same launches):
//   k_compose_fwd     frame composition of a group (Sec. 3.2, pose update, Eq. 7)
//   k_project_fwd     one thread per Gaussian, looping over frames and views:
//                     activations, covariance R diag(s^2) R^T (Sec. 3.1),
//                     EWA projection, conic, footprint, tile rectangle and
//                     view-dependent SH colour; writes 48-byte records
//   k_radix_*         segmented stable LSD radix sort of float32 depth keys
//                     (one segment per frame-view, 4 passes of 8 bits)
//   k_bin_gather, k_row_bin, k_tile_bin, scans
//                     two-level stable counting scatter of the depth-sorted
//                     Gaussians into per-(view, tile) lists, the (tile, depth)
//                     order: tile rows first, then the tiles of each row
//   k_raster_fwd      one 256-thread block per (view, 16x16 tile), a wave per
//                     8x8 quadrant (or 16x4 strip): records are staged through
//                     LDS in batches of 256; every pixel composites all layers
//                     at once (Eq. 2 for each index set of Eq. 4) and stops
//                     when every layer has reached the transmittance floor.
//                     Each wave walks the staged entries it may need (a ballot
//                     mask per 64 entries, scalar find-first-set) and updates
//                     its layers with selects, skipping layers closed in all
//                     of its lanes
// Backward:
//   k_raster_bwd      reverse traversal from each layer's last contributor over
//                     the staged entries each wave can use (ballot masks walked
//                     back to front); the transmittance is recovered by
//                     division, so no per-pixel lists are stored; a
//                     permlane/DPP reduce-scatter per entry, LDS sums of the
//                     four waves, then one atomic per (record, value) and batch
// Both raster kernels have a variant that also counts their work (COUNT), used
// only while counting is switched on.
//   k_project_bwd     one thread per Gaussian, all views and frames in registers
//   k_compose_bwd     suffix sums and the quaternion-product chain over frames
#include <hip/hip_runtime.h>

#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* R) {
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// SH constants of the real orthonormal basis (Condon-Shortley phase).
constexpr float kC0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kC1 = 0.4886025119029199f;    // sqrt(3 / (4 pi))
constexpr float kC2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kC2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kC2c = 0.5462742152960396f;   // sqrt(15 / pi) / 4
constexpr float kC3a = 0.5900435899266435f;   // sqrt(35 / (2 pi)) / 4
constexpr float kC3b = 2.890611442640554f;    // sqrt(105 / pi) / 2
constexpr float kC3c = 0.4570457994644658f;   // sqrt(21 / (2 pi)) / 4
constexpr float kC3d = 0.3731763325901154f;   // sqrt(7 / pi) / 4
constexpr float kC3e = 1.445305721320277f;    // sqrt(105 / pi) / 4

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kC0;
  if constexpr (DEG >= 1) { Y[1] = -kC1 * y; Y[2] = kC1 * z; Y[3] = -kC1 * x; }
  if constexpr (DEG >= 2) {
    Y[4] = kC2a * (x * y); Y[5] = -kC2a * (y * z); Y[6] = kC2b * (3.f * z * z - 1.f);
    Y[7] = -kC2a * (x * z); Y[8] = kC2c * (x * x - y * y);
  }
  if constexpr (DEG >= 3) {
    Y[9] = -kC3a * y * (3.f * x * x - y * y);
    Y[10] = kC3b * x * y * z;
    Y[11] = -kC3c * y * (5.f * z * z - 1.f);
    Y[12] = kC3d * z * (5.f * z * z - 3.f);
    Y[13] = -kC3c * x * (5.f * z * z - 1.f);
    Y[14] = kC3e * z * (x * x - y * y);
    Y[15] = -kC3a * x * (x * x - 3.f * y * y);
  }
}

// Gradient of sum_k w_k Y_k with respect to the (unnormalised) direction components.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* w, float* g) {
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if constexpr (DEG >= 1) { gy += -kC1 * w[1]; gz += kC1 * w[2]; gx += -kC1 * w[3]; }
  if constexpr (DEG >= 2) {
    gx += kC2a * y * w[4]; gy += kC2a * x * w[4];
    gy += -kC2a * z * w[5]; gz += -kC2a * y * w[5];
    gz += 6.f * kC2b * z * w[6];
    gx += -kC2a * z * w[7]; gz += -kC2a * x * w[7];
    gx += 2.f * kC2c * x * w[8]; gy += -2.f * kC2c * y * w[8];
  }
  if constexpr (DEG >= 3) {
    gx += -6.f * kC3a * x * y * w[9]; gy += -3.f * kC3a * (x * x - y * y) * w[9];
    gx += kC3b * y * z * w[10]; gy += kC3b * x * z * w[10]; gz += kC3b * x * y * w[10];
    gy += -kC3c * (5.f * z * z - 1.f) * w[11]; gz += -10.f * kC3c * y * z * w[11];
    gz += kC3d * (15.f * z * z - 3.f) * w[12];
    gx += -kC3c * (5.f * z * z - 1.f) * w[13]; gz += -10.f * kC3c * x * z * w[13];
    gx += 2.f * kC3e * x * z * w[14]; gy += -2.f * kC3e * y * z * w[14]; gz += kC3e * (x * x - y * y) * w[14];
    gx += -3.f * kC3a * (x * x - y * y) * w[15]; gy += 6.f * kC3a * x * y * w[15];
  }
  g[0] = gx; g[1] = gy; g[2] = gz;
}

// Row a of the camera transform t = W mu + t0, in FP64 from the FP64 frame
// mean. The depth row decides the near-plane cull and, rounded once to
// float32, the depth order; the other rows give the 2D mean, which is rounded
// to float32 once.
__device__ __forceinline__ double cam_row(const gs_camera& c, int a, const double* mu) {
  const float* W = c.viewmat + 4 * a;
  return fma((double)W[2], mu[2], fma((double)W[1], mu[1], fma((double)W[0], mu[0], (double)W[3])));
}

// Per-pixel Gaussian weight. Forward and backward call this one function on
// the same inputs, so they take identical float32 decisions. The conic comes
// pre-scaled to a base-2 exponent: (a2, b2, c2) = -log2(e) (A / 2, B, C / 2), so
// that G = 2^(a2 dx^2 + b2 dx dy + c2 dy^2) = exp(-q / 2).
struct AlphaEval {
  float dx, dy, G, ga;  // ga = o * G before the alpha_max clamp
  float u, v;           // a2 dx + b2 dy and c2 dy: the exponent is u dx + v dy
};
__device__ __forceinline__ AlphaEval alpha_eval(float px, float py, float mx, float my, float a2, float b2, float c2,
                                                float o) {
  AlphaEval r;
  r.dx = px - mx;
  r.dy = py - my;
  r.u = fmaf(a2, r.dx, b2 * r.dy);
  r.v = c2 * r.dy;
  r.G = __builtin_amdgcn_exp2f(fmaf(r.u, r.dx, r.v * r.dy));
  r.ga = o * r.G;
  return r;
}
constexpr float kLn2 = 0.6931471805599453f;

// Residual channel r -> parameter channel.
__device__ __forceinline__ int res_to_param(int r) {
  if (r < 3) return r;
  if (r < 7) return r + 3;
  if (r == 7) return 10;
  if (r < 11) return r - 5;
  return r;
}

__device__ __forceinline__ void quat_mul(const float* a, const float* b, float* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// XCD-aware work mapping: consecutive work items land on the same XCD (the
// dispatcher deals blocks round-robin to the 8 XCDs), so neighbouring tiles
// of one view share that XCD's L2.
__device__ __forceinline__ int xcd_item(int bid, int per_xcd) { return (bid & 7) * per_xcd + (bid >> 3); }

// ============================================================ composition
__global__ __launch_bounds__(256) void k_compose_fwd(RenderDims d, const float* __restrict__ P,
                                                     const float* __restrict__ res, float* __restrict__ comp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const size_t n = d.n;
  const int Rc = d.Rc;
  // additive channels: everything but the quaternion (3..6)
  for (int r = 0; r < Rc; ++r) {
    if (r >= 3 && r <= 6) continue;
    float v = P[(size_t)res_to_param(r) * n + i];
    for (int f = 0; f < d.F; ++f) {
      v = v + res[((size_t)f * Rc + r) * n + i];
      comp[((size_t)f * Rc + r) * n + i] = v;
    }
  }
  float q[4] = {P[6 * n + i], P[7 * n + i], P[8 * n + i], P[9 * n + i]};
  for (int f = 0; f < d.F; ++f) {
    float dq[4], o[4];
    for (int c = 0; c < 4; ++c) dq[c] = res[((size_t)f * Rc + 3 + c) * n + i];
    quat_mul(dq, q, o);
    for (int c = 0; c < 4; ++c) {
      q[c] = o[c];
      comp[((size_t)f * Rc + 3 + c) * n + i] = o[c];
    }
  }
}

__global__ __launch_bounds__(256) void k_compose_bwd(RenderDims d, const float* __restrict__ P,
                                                     const float* __restrict__ res, const float* __restrict__ comp,
                                                     const float* __restrict__ dcomp, float* __restrict__ dP,
                                                     float* __restrict__ dres) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const size_t n = d.n;
  const int Rc = d.Rc;
  for (int r = 0; r < Rc; ++r) {
    if (r >= 3 && r <= 6) continue;
    float acc = 0.f;
    for (int f = d.F - 1; f >= 0; --f) {
      acc += dcomp[((size_t)f * Rc + r) * n + i];
      if (dres) dres[((size_t)f * Rc + r) * n + i] += acc;
    }
    dP[(size_t)res_to_param(r) * n + i] += acc;
  }
  float carry[4] = {0.f, 0.f, 0.f, 0.f};
  for (int f = d.F - 1; f >= 0; --f) {
    float g[4], a[4], b[4];
    for (int c = 0; c < 4; ++c) {
      g[c] = dcomp[((size_t)f * Rc + 3 + c) * n + i] + carry[c];
      a[c] = res[((size_t)f * Rc + 3 + c) * n + i];
      b[c] = f == 0 ? P[(size_t)(6 + c) * n + i] : comp[((size_t)(f - 1) * Rc + 3 + c) * n + i];
    }
    if (g[0] == 0.f && g[1] == 0.f && g[2] == 0.f && g[3] == 0.f) {
      // nothing flows back (a culled Gaussian): keep a non-finite delta from turning 0 into NaN
      for (int c = 0; c < 4; ++c) carry[c] = 0.f;
      continue;
    }
    // p = a (x) b; gradients of <g, p> with respect to a and b
    const float ga0 = b[0] * g[0] + b[1] * g[1] + b[2] * g[2] + b[3] * g[3];
    const float ga1 = -b[1] * g[0] + b[0] * g[1] - b[3] * g[2] + b[2] * g[3];
    const float ga2 = -b[2] * g[0] + b[3] * g[1] + b[0] * g[2] - b[1] * g[3];
    const float ga3 = -b[3] * g[0] - b[2] * g[1] + b[1] * g[2] + b[0] * g[3];
    carry[0] = a[0] * g[0] + a[1] * g[1] + a[2] * g[2] + a[3] * g[3];
    carry[1] = -a[1] * g[0] + a[0] * g[1] + a[3] * g[2] - a[2] * g[3];
    carry[2] = -a[2] * g[0] - a[3] * g[1] + a[0] * g[2] + a[1] * g[3];
    carry[3] = -a[3] * g[0] + a[2] * g[1] - a[1] * g[2] + a[0] * g[3];
    if (dres) {
      dres[((size_t)f * Rc + 3) * n + i] += ga0;
      dres[((size_t)f * Rc + 4) * n + i] += ga1;
      dres[((size_t)f * Rc + 5) * n + i] += ga2;
      dres[((size_t)f * Rc + 6) * n + i] += ga3;
    }
  }
  for (int c = 0; c < 4; ++c) dP[(size_t)(6 + c) * n + i] += carry[c];
}

// ============================================================ projection
// Frame-level quantities of one Gaussian (shared by its views).
template <int DEG>
struct GaussFrame {
  float mu[3], ls[3], q[4], logit;
  float sh[3 * (DEG + 1) * (DEG + 1)];
};

template <int DEG>
__device__ __forceinline__ void load_frame(const RenderDims& d, const float* __restrict__ P,
                                           const float* __restrict__ comp, int f, int i, GaussFrame<DEG>& g) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const size_t n = d.n;
  if (d.Rc == 0 || f < 0) {
    for (int c = 0; c < 3; ++c) g.mu[c] = P[c * n + i];
    for (int c = 0; c < 3; ++c) g.ls[c] = P[(3 + c) * n + i];
    for (int c = 0; c < 4; ++c) g.q[c] = P[(6 + c) * n + i];
    g.logit = P[10 * n + i];
#pragma unroll
    for (int c = 0; c < 3 * K; ++c) g.sh[c] = P[(11 + c) * n + i];
    return;
  }
  const float* cf = comp + (size_t)f * d.Rc * n;
  for (int c = 0; c < 3; ++c) g.mu[c] = cf[c * n + i];
  for (int c = 0; c < 4; ++c) g.q[c] = cf[(3 + c) * n + i];
  g.logit = cf[7 * n + i];
  for (int c = 0; c < 3; ++c) g.ls[c] = d.Rc >= 11 ? cf[(8 + c) * n + i] : P[(3 + c) * n + i];
#pragma unroll
  for (int c = 0; c < 3 * K; ++c) g.sh[c] = d.Rc > 11 ? cf[(11 + c) * n + i] : P[(11 + c) * n + i];
}

// The frame mean in FP64 (keyframe mean plus the translation deltas of
// frames 0..f): the depth order and the 2D mean are taken from it.
__device__ __forceinline__ void frame_mean64_init(const RenderDims& d, const float* __restrict__ P, int i,
                                                  double* mu) {
  for (int c = 0; c < 3; ++c) mu[c] = (double)P[(size_t)c * d.n + i];
}
__device__ __forceinline__ void frame_mean64_step(const RenderDims& d, const float* __restrict__ res, int f, int i,
                                                  double* mu) {
  if (d.Rc == 0) return;
  for (int c = 0; c < 3; ++c) mu[c] += (double)res[((size_t)f * d.Rc + c) * d.n + i];
}

struct FrameGeom {
  float R[9], s[3], s2[3], Sig[6];  // Sigma: xx, xy, xz, yy, yz, zz
  float o, rf;                // opacity, sqrt(2 ln(o / alpha_min))
  float qinv;                 // 1 / |q|
  float qn[4];
  bool valid;
};

// A Gaussian with a zero quaternion or any non-finite parameter is culled.
template <int DEG>
__device__ __forceinline__ FrameGeom frame_geom(const GaussFrame<DEG>& g) {
  FrameGeom fg;
  const float qq = g.q[0] * g.q[0] + g.q[1] * g.q[1] + g.q[2] * g.q[2] + g.q[3] * g.q[3];
  bool fin = isfinite(g.logit);
  for (int c = 0; c < 3; ++c) fin = fin && isfinite(g.mu[c]) && isfinite(g.ls[c]);
#pragma unroll
  for (int c = 0; c < 3 * (DEG + 1) * (DEG + 1); ++c) fin = fin && isfinite(g.sh[c]);
  fg.valid = fin && qq > 0.f && isfinite(qq);
  fg.qinv = fg.valid ? 1.0f / sqrtf(qq) : 0.f;
  for (int c = 0; c < 4; ++c) fg.qn[c] = g.q[c] * fg.qinv;
  quat_rot(fg.qn[0], fg.qn[1], fg.qn[2], fg.qn[3], fg.R);
  for (int c = 0; c < 3; ++c) {
    const float s = expf(g.ls[c]);
    fg.s[c] = s;
    fg.s2[c] = s * s;
  }
  const float* R = fg.R;
  auto sig = [&](int a, int b) {
    return R[3 * a] * fg.s2[0] * R[3 * b] + R[3 * a + 1] * fg.s2[1] * R[3 * b + 1] + R[3 * a + 2] * fg.s2[2] * R[3 * b + 2];
  };
  fg.Sig[0] = sig(0, 0); fg.Sig[1] = sig(0, 1); fg.Sig[2] = sig(0, 2);
  fg.Sig[3] = sig(1, 1); fg.Sig[4] = sig(1, 2); fg.Sig[5] = sig(2, 2);
  fg.o = 1.0f / (1.0f + expf(-g.logit));
  return fg;
}

// Opacity cull and footprint factor: a Gaussian reaches alpha_min only where
// its quadratic form is <= 2 ln(o / alpha_min).
__device__ __forceinline__ void frame_footprint(FrameGeom& fg, float alpha_min) {
  fg.valid = fg.valid && (fg.o >= alpha_min);
  fg.rf = fg.valid ? sqrtf(2.0f * logf(fg.o / alpha_min)) : 0.f;
}

// View-level projection of one Gaussian.
struct ViewProj {
  float tx, ty, tz, ux, uy;
  bool clx, cly;
  float m0[3], m1[3];  // rows of J W
  float a, b, c;       // 2D covariance (with dilation)
  float A, B, C;       // conic
  float mx, my;
  bool valid;
};

// a b - c d with one rounding error of the result (the fma recovers the
// rounding error of c d exactly).
__device__ __forceinline__ float diff_of_products(float a, float b, float c, float d) {
  const float cd = c * d;
  const float err = fmaf(-c, d, cd);
  return fmaf(a, b, -cd) + err;
}

__device__ __forceinline__ ViewProj view_proj(const RenderDims& d, const gs_camera& cam, const double* mu,
                                              const FrameGeom& fg) {
  ViewProj v;
  const double tz = cam_row(cam, 2, mu);
  const double tx = cam_row(cam, 0, mu);
  const double ty = cam_row(cam, 1, mu);
  v.valid = fg.valid && (tz > (double)d.near_plane);
  v.tz = (float)tz;
  v.tx = (float)tx;
  v.ty = (float)ty;
  const float itz = 1.0f / v.tz;
  const float limx = 1.3f * (0.5f * (float)d.W / cam.fx);
  const float limy = 1.3f * (0.5f * (float)d.H / cam.fy);
  const float rx = v.tx * itz, ry = v.ty * itz;
  v.clx = (rx > limx) || (rx < -limx);
  v.cly = (ry > limy) || (ry < -limy);
  v.ux = fminf(fmaxf(rx, -limx), limx);
  v.uy = fminf(fmaxf(ry, -limy), limy);
  const float J00 = cam.fx * itz, J02 = -cam.fx * v.ux * itz;
  const float J11 = cam.fy * itz, J12 = -cam.fy * v.uy * itz;
  const float* Wm = cam.viewmat;
  for (int k = 0; k < 3; ++k) {
    v.m0[k] = J00 * Wm[k] + J02 * Wm[8 + k];
    v.m1[k] = J11 * Wm[4 + k] + J12 * Wm[8 + k];
  }
  // Sigma2D = V V^T + dilation I with V = (J W) R diag(s) (2 x 3): the
  // diagonal entries are sums of squares, and the determinant is the sum of
  // the squared 2 x 2 minors of V plus positive dilation terms (the
  // Cauchy-Binet form), so neither suffers cancellation.
  const float* R = fg.R;
  float V0[3], V1[3];
  for (int j = 0; j < 3; ++j) {
    V0[j] = (v.m0[0] * R[j] + v.m0[1] * R[3 + j] + v.m0[2] * R[6 + j]) * fg.s[j];
    V1[j] = (v.m1[0] * R[j] + v.m1[1] * R[3 + j] + v.m1[2] * R[6 + j]) * fg.s[j];
  }
  const float a0 = V0[0] * V0[0] + V0[1] * V0[1] + V0[2] * V0[2];
  const float c0 = V1[0] * V1[0] + V1[1] * V1[1] + V1[2] * V1[2];
  v.a = a0 + d.dilation;
  v.b = V0[0] * V1[0] + V0[1] * V1[1] + V0[2] * V1[2];
  v.c = c0 + d.dilation;
  const float n01 = diff_of_products(V0[0], V1[1], V0[1], V1[0]);
  const float n02 = diff_of_products(V0[0], V1[2], V0[2], V1[0]);
  const float n12 = diff_of_products(V0[1], V1[2], V0[2], V1[1]);
  const float det = (n01 * n01 + n02 * n02 + n12 * n12) + d.dilation * (a0 + c0 + d.dilation);
  v.valid = v.valid && (det > 0.f);
  const float idet = 1.0f / det;
  v.A = v.c * idet;
  v.B = -v.b * idet;
  v.C = v.a * idet;
  const double iz = 1.0 / tz;
  v.mx = (float)fma((double)cam.fx, tx * iz, (double)cam.cx);
  v.my = (float)fma((double)cam.fy, ty * iz, (double)cam.cy);
  v.valid = v.valid && isfinite(v.mx) && isfinite(v.my) && isfinite(v.A) && isfinite(v.B) && isfinite(v.C);
  return v;
}

__device__ __forceinline__ void cam_center(const gs_camera& c, float* p) {
  const float* Wm = c.viewmat;
  for (int a = 0; a < 3; ++a) p[a] = -(Wm[a] * Wm[3] + Wm[4 + a] * Wm[7] + Wm[8 + a] * Wm[11]);
}

template <int DEG>
__device__ __forceinline__ void view_color(const gs_camera& cam, const GaussFrame<DEG>& g, float* rgb, float* raw,
                                           float* dir, float* inv_len, float* Y) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  float cp[3];
  cam_center(cam, cp);
  float v0 = g.mu[0] - cp[0], v1 = g.mu[1] - cp[1], v2 = g.mu[2] - cp[2];
  const float il = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
  dir[0] = v0 * il; dir[1] = v1 * il; dir[2] = v2 * il;
  *inv_len = il;
  sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(g.sh[3 * k + c], Y[k], acc);
    raw[c] = acc;
    rgb[c] = fmaxf(acc, 0.f);
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_fwd(RenderDims d, const float* __restrict__ P,
                                                     const float* __restrict__ res, const float* __restrict__ comp,
                                                     const gs_camera* __restrict__ cams, float4* __restrict__ rec,
                                                     uint2* __restrict__ rects, uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  GaussFrame<DEG> g;
  double mu64[3];
  frame_mean64_init(d, P, i, mu64);
  for (int f = 0; f < d.F; ++f) {
    load_frame<DEG>(d, P, comp, d.Rc ? f : -1, i, g);
    frame_mean64_step(d, res, f, i, mu64);
    FrameGeom fg = frame_geom<DEG>(g);
    frame_footprint(fg, d.alpha_min);
    for (int v = 0; v < d.V; ++v) {
      const int b = f * d.V + v;
      const gs_camera cam = cams[b];
      const size_t bi = (size_t)b * d.n + i;
      uint32_t key = 0xFFFFFFFFu;
      const ViewProj vp = view_proj(d, cam, mu64, fg);
      if (vp.valid) {
        const float mid = 0.5f * (vp.a + vp.c);
        const float hd = 0.5f * (vp.a - vp.c);
        const float lmax = mid + sqrtf(fmaxf(0.f, hd * hd + vp.b * vp.b));
        const float r = ceilf(fg.rf * sqrtf(lmax)) + 1.0f;
        const float ulo = (vp.mx - r - 0.5f) * (1.0f / kTile), uhi = (vp.mx + r - 0.5f) * (1.0f / kTile);
        const float vlo = (vp.my - r - 0.5f) * (1.0f / kTile), vhi = (vp.my + r - 0.5f) * (1.0f / kTile);
        const int x0 = (int)floorf(fmaxf(ulo, -1.f)), x1 = (int)floorf(fminf(uhi, (float)d.TX));
        const int y0 = (int)floorf(fmaxf(vlo, -1.f)), y1 = (int)floorf(fminf(vhi, (float)d.TY));
        const int cx0 = max(x0, 0), cx1 = min(x1, d.TX - 1), cy0 = max(y0, 0), cy1 = min(y1, d.TY - 1);
        if (isfinite(r) && cx0 <= cx1 && cy0 <= cy1) {
          float rgb[3], raw[3], dir[3], il, Y[K];
          view_color<DEG>(cam, g, rgb, raw, dir, &il, Y);
          rec[3 * bi + 0] = make_float4(vp.mx, vp.my, vp.A, vp.B);
          rec[3 * bi + 1] = make_float4(vp.C, fg.o, rgb[0], rgb[1]);
          // the tile rectangle also rides in the record's spare words, so that the binning gather
          // reads one contiguous 48-byte record per depth-sorted Gaussian
          const uint2 rc = make_uint2((uint32_t)cx0 | ((uint32_t)cx1 << 16), (uint32_t)cy0 | ((uint32_t)cy1 << 16));
          rec[3 * bi + 2] = make_float4(rgb[2], vp.tz, __uint_as_float(rc.x), __uint_as_float(rc.y));
          rects[bi] = rc;
          key = __float_as_uint(vp.tz);
        }
      }
      keys[bi] = key;
      vals[bi] = (uint32_t)i;
    }
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(RenderDims d, const float* __restrict__ P,
                                                     const float* __restrict__ res, const float* __restrict__ comp,
                                                     const gs_camera* __restrict__ cams,
                                                     const float* __restrict__ g2d, float* __restrict__ dP,
                                                     float* __restrict__ dcomp) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const size_t n = d.n;
  GaussFrame<DEG> g;
  float t_mu[3] = {0, 0, 0}, t_ls[3] = {0, 0, 0}, t_q[4] = {0, 0, 0, 0}, t_lg = 0.f;
  float t_sh[3 * K];
#pragma unroll
  for (int c = 0; c < 3 * K; ++c) t_sh[c] = 0.f;
  double mu64[3];
  frame_mean64_init(d, P, i, mu64);
  for (int f = 0; f < d.F; ++f) {
    load_frame<DEG>(d, P, comp, d.Rc ? f : -1, i, g);
    frame_mean64_step(d, res, f, i, mu64);
    FrameGeom fg = frame_geom<DEG>(g);
    frame_footprint(fg, d.alpha_min);
    if (!fg.valid) continue;
    float Gs[6] = {0, 0, 0, 0, 0, 0};  // (G + G^T) of dL/dSigma: xx, xy, xz, yy, yz, zz
    float dmu[3] = {0, 0, 0}, dlg = 0.f;
    float dsh[3 * K];
#pragma unroll
    for (int c = 0; c < 3 * K; ++c) dsh[c] = 0.f;
    // the gradient record of view v + 1 is loaded while view v is processed (one wave per SIMD
    // here: nothing else would hide the load)
    float4 n0, n1;
    float n8;
    auto load_rec = [&](int b) {
      const float* gp = g2d + ((size_t)b * n + i) * kGradStride;
      n0 = ((const float4*)gp)[0];
      n1 = ((const float4*)gp)[1];
      n8 = gp[8];
    };
    if (d.V > 0) load_rec(f * d.V);
    for (int v = 0; v < d.V; ++v) {
      const int b = f * d.V + v;
      float gr[9] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w, n8};
      if (v + 1 < d.V) load_rec(b + 1);
      bool any = false;
      for (int c = 0; c < 9; ++c) any = any || (gr[c] != 0.f);
      if (!any) continue;
      const gs_camera cam = cams[b];
      const ViewProj vp = view_proj(d, cam, mu64, fg);
      if (!vp.valid) continue;
      const float A = vp.A, B = vp.B, C = vp.C;
      // the record holds the moments (sum dp dx, sum dp dy); dL/dm = [[A, B], [B, C]] of them
      {
        const float mx = gr[0], my = gr[1];
        gr[0] = fmaf(A, mx, B * my);
        gr[1] = fmaf(B, mx, C * my);
      }
      // conic (A, B, C) -> covariance (a, b, c)
      const float gA = gr[2], gB = gr[3], gC = gr[4];
      const float ga = -(gA * A * A + gB * A * B + gC * B * B);
      const float gb = -(2.f * gA * A * B + gB * (A * C + B * B) + 2.f * gC * B * C);
      const float gc = -(gA * B * B + gB * B * C + gC * C * C);
      // covariance -> Sigma (symmetrised) and M = J W
      const float* S = fg.Sig;
      const float* m0 = vp.m0;
      const float* m1 = vp.m1;
      Gs[0] += 2.f * ga * m0[0] * m0[0] + 2.f * gb * m0[0] * m1[0] + 2.f * gc * m1[0] * m1[0];
      Gs[1] += 2.f * ga * m0[0] * m0[1] + gb * (m0[0] * m1[1] + m1[0] * m0[1]) + 2.f * gc * m1[0] * m1[1];
      Gs[2] += 2.f * ga * m0[0] * m0[2] + gb * (m0[0] * m1[2] + m1[0] * m0[2]) + 2.f * gc * m1[0] * m1[2];
      Gs[3] += 2.f * ga * m0[1] * m0[1] + 2.f * gb * m0[1] * m1[1] + 2.f * gc * m1[1] * m1[1];
      Gs[4] += 2.f * ga * m0[1] * m0[2] + gb * (m0[1] * m1[2] + m1[1] * m0[2]) + 2.f * gc * m1[1] * m1[2];
      Gs[5] += 2.f * ga * m0[2] * m0[2] + 2.f * gb * m0[2] * m1[2] + 2.f * gc * m1[2] * m1[2];
      float s0[3], s1[3];
      s0[0] = S[0] * m0[0] + S[1] * m0[1] + S[2] * m0[2];
      s0[1] = S[1] * m0[0] + S[3] * m0[1] + S[4] * m0[2];
      s0[2] = S[2] * m0[0] + S[4] * m0[1] + S[5] * m0[2];
      s1[0] = S[0] * m1[0] + S[1] * m1[1] + S[2] * m1[2];
      s1[1] = S[1] * m1[0] + S[3] * m1[1] + S[4] * m1[2];
      s1[2] = S[2] * m1[0] + S[4] * m1[1] + S[5] * m1[2];
      float dm0[3], dm1[3];
      for (int k = 0; k < 3; ++k) {
        dm0[k] = 2.f * ga * s0[k] + gb * s1[k];
        dm1[k] = gb * s0[k] + 2.f * gc * s1[k];
      }
      const float* Wm = cam.viewmat;
      const float dJ00 = dm0[0] * Wm[0] + dm0[1] * Wm[1] + dm0[2] * Wm[2];
      const float dJ02 = dm0[0] * Wm[8] + dm0[1] * Wm[9] + dm0[2] * Wm[10];
      const float dJ11 = dm1[0] * Wm[4] + dm1[1] * Wm[5] + dm1[2] * Wm[6];
      const float dJ12 = dm1[0] * Wm[8] + dm1[1] * Wm[9] + dm1[2] * Wm[10];
      const float itz = 1.0f / vp.tz, itz2 = itz * itz;
      float dtx = 0.f, dty = 0.f, dtz = 0.f;
      dtz += -(dJ00 * cam.fx + dJ11 * cam.fy) * itz2;
      if (!vp.clx) {
        dtx += -dJ02 * cam.fx * itz2;
        dtz += 2.f * dJ02 * cam.fx * vp.tx * itz2 * itz;
      } else {
        dtz += dJ02 * cam.fx * vp.ux * itz2;
      }
      if (!vp.cly) {
        dty += -dJ12 * cam.fy * itz2;
        dtz += 2.f * dJ12 * cam.fy * vp.ty * itz2 * itz;
      } else {
        dtz += dJ12 * cam.fy * vp.uy * itz2;
      }
      // mean2D
      dtx += gr[0] * cam.fx * itz;
      dty += gr[1] * cam.fy * itz;
      dtz += -(gr[0] * cam.fx * vp.tx + gr[1] * cam.fy * vp.ty) * itz2;
      for (int k = 0; k < 3; ++k) dmu[k] += Wm[k] * dtx + Wm[4 + k] * dty + Wm[8 + k] * dtz;
      // opacity
      dlg += gr[5] * fg.o * (1.f - fg.o);
      // colour
      float rgb[3], raw[3], dir[3], il, Y[K];
      view_color<DEG>(cam, g, rgb, raw, dir, &il, Y);
      float gcol[3];
      for (int c = 0; c < 3; ++c) gcol[c] = raw[c] < 0.f ? 0.f : gr[6 + c];
      float wk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        dsh[3 * k + 0] += gcol[0] * Y[k];
        dsh[3 * k + 1] += gcol[1] * Y[k];
        dsh[3 * k + 2] += gcol[2] * Y[k];
        wk[k] = gcol[0] * g.sh[3 * k] + gcol[1] * g.sh[3 * k + 1] + gcol[2] * g.sh[3 * k + 2];
      }
      if constexpr (DEG > 0) {
        float gd[3];
        sh_basis_grad<DEG>(dir[0], dir[1], dir[2], wk, gd);
        const float dd = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
        for (int k = 0; k < 3; ++k) dmu[k] += (gd[k] - dir[k] * dd) * il;
      }
    }
    // Sigma = R D R^T:  dL/dR = Gs R D,  dL/ds2_j = 1/2 (R^T Gs R)_jj
    const float* R = fg.R;
    const float Gm[9] = {Gs[0], Gs[1], Gs[2], Gs[1], Gs[3], Gs[4], Gs[2], Gs[4], Gs[5]};
    float dR[9];
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 3; ++j)
        dR[3 * a + j] = (Gm[3 * a] * R[j] + Gm[3 * a + 1] * R[3 + j] + Gm[3 * a + 2] * R[6 + j]) * fg.s2[j];
    float dls[3];
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int a = 0; a < 3; ++a)
        for (int b2 = 0; b2 < 3; ++b2) acc += R[3 * a + j] * Gm[3 * a + b2] * R[3 * b2 + j];
      dls[j] = acc * fg.s2[j];  // 1/2 * (R^T Gs R)_jj * d(s^2)/d(log s) = (.)_jj * s^2
    }
    const float w = fg.qn[0], x = fg.qn[1], y = fg.qn[2], z = fg.qn[3];
    float dqn[4];
    dqn[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dqn[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                    2.f * x * dR[8]);
    dqn[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                    2.f * y * dR[8]);
    dqn[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                    x * dR[6] + y * dR[7]);
    const float qd = dqn[0] * fg.qn[0] + dqn[1] * fg.qn[1] + dqn[2] * fg.qn[2] + dqn[3] * fg.qn[3];
    float dq[4];
    for (int c = 0; c < 4; ++c) dq[c] = (dqn[c] - fg.qn[c] * qd) * fg.qinv;
    if (d.Rc > 0) {
      float* df = dcomp + (size_t)f * d.Rc * n;
      for (int c = 0; c < 3; ++c) df[c * n + i] = dmu[c];
      for (int c = 0; c < 4; ++c) df[(3 + c) * n + i] = dq[c];
      df[7 * n + i] = dlg;
      if (d.Rc >= 11) {
        for (int c = 0; c < 3; ++c) df[(8 + c) * n + i] = dls[c];
      } else {
        for (int c = 0; c < 3; ++c) t_ls[c] += dls[c];
      }
      if (d.Rc > 11) {
#pragma unroll
        for (int c = 0; c < 3 * K; ++c) df[(11 + c) * n + i] = dsh[c];
      } else {
#pragma unroll
        for (int c = 0; c < 3 * K; ++c) t_sh[c] += dsh[c];
      }
    } else {
      for (int c = 0; c < 3; ++c) { t_mu[c] += dmu[c]; t_ls[c] += dls[c]; }
      for (int c = 0; c < 4; ++c) t_q[c] += dq[c];
      t_lg += dlg;
#pragma unroll
      for (int c = 0; c < 3 * K; ++c) t_sh[c] += dsh[c];
    }
  }
  if (d.Rc == 0) {
    for (int c = 0; c < 3; ++c) dP[c * n + i] += t_mu[c];
    for (int c = 0; c < 4; ++c) dP[(6 + c) * n + i] += t_q[c];
    dP[10 * n + i] += t_lg;
  }
  if (d.Rc < 11)
    for (int c = 0; c < 3; ++c) dP[(3 + c) * n + i] += t_ls[c];
  if (d.Rc <= 11) {
#pragma unroll
    for (int c = 0; c < 3 * K; ++c) dP[(11 + c) * n + i] += t_sh[c];
  }
}

// ============================================================ radix sort
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ uint32_t popc_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(RenderDims d, const uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ hist, int shift) {
  __shared__ uint32_t h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int b = blockIdx.y, chunk = blockIdx.x;
  const size_t seg = (size_t)b * d.n;
  const int start = chunk * kSortChunk;
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int e = start + it * kSortThreads + t;
    if (e < d.n) atomicAdd(&h[(keys[seg + e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[((size_t)b * 256 + t) * d.n_sort_chunks + chunk] = h[t];
}

// Stable scatter of one pass. Wave w owns the 512 consecutive keys [start + 512 w, start + 512 w
// + 512) of the block's chunk, eight rounds of 64 in order; a key's rank among the wave's keys of
// its digit is the count of that digit in the wave's earlier rounds (a running count in LDS, read by
// every peer and advanced by the round's first peer) plus its rank among this round's peers (eight
// ballots). One barrier later the block turns the four waves' counts into per-wave offsets (thread
// t for digit t), so positions follow the input order with two barriers per chunk.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(RenderDims d, const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout,
                                                               uint32_t* __restrict__ vout,
                                                               const uint32_t* __restrict__ hist, int shift) {
  static_assert(kSortThreads == 256 && kSortItems == 8, "four waves of eight rounds of 64 keys");
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int b = blockIdx.y, chunk = blockIdx.x;
  const size_t seg = (size_t)b * d.n;
  for (int k = 0; k < 4; ++k) wcnt[k][t] = 0;
  const uint32_t goff = hist[((size_t)b * 256 + t) * d.n_sort_chunks + chunk];
  __syncthreads();
  const int start = chunk * kSortChunk + w * (kSortItems * 64);
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int e = start + it * 64 + lane;
    const bool valid = e < d.n;
    key[it] = valid ? kin[seg + e] : 0u;
    val[it] = valid ? vin[seg + e] : 0u;
  }
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int e = start + it * 64 + lane;
    const bool valid = e < d.n;
    const uint32_t dg = (key[it] >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dg >> bit) & 1u;
      const unsigned long long bb = __ballot(valid && on);
      peers &= on ? bb : ~bb;
    }
    const uint32_t below = popc_below(peers);
    // LDS operations of one wave complete in order: every peer reads the count before the
    // round's first peer advances it
    const uint32_t prev = valid ? wcnt[w][dg] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) wcnt[w][dg] = prev + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[it] = prev + below;
  }
  __syncthreads();
  {
    // per-wave offsets of digit t inside the chunk's run of that digit
    uint32_t run = goff;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t c = wcnt[k][t];
      wcnt[k][t] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int e = start + it * 64 + lane;
    if (e < d.n) {
      const uint32_t pos = wcnt[w][(key[it] >> shift) & 255u] + rank[it];
      kout[seg + pos] = key[it];
      vout[seg + pos] = val[it];
    }
  }
}

// ============================================================ binning
// Binning record of one depth-sorted (frame-view, Gaussian): mean2D, conic,
// the alpha_min threshold of its quadratic form and its tile rectangle,
// gathered once after the sort so that the count and emit passes read it
// sequentially.
__global__ __launch_bounds__(256) void k_bin_gather(RenderDims d, const uint32_t* __restrict__ skeys,
                                                    const uint32_t* __restrict__ svals,
                                                    const float4* __restrict__ rec,
                                                    float4* __restrict__ brec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (k >= d.n) return;
  const size_t seg = (size_t)b * d.n;
  float4 o0 = make_float4(0.f, 0.f, 1.f, 0.f), o1 = make_float4(1.f, 1.f, 0.f, 0.f);
  float4 o2 = make_float4(-1.f, 0.f, 0.f, 0.f);
  if (skeys[seg + k] != 0xFFFFFFFFu) {
    const uint32_t i = svals[seg + k];
    const float4 r0 = rec[3 * (seg + i)], r1 = rec[3 * (seg + i) + 1], r2 = rec[3 * (seg + i) + 2];
    const uint2 rc = make_uint2(__float_as_uint(r2.z), __float_as_uint(r2.w));  // the tile rectangle
    // quadratic-form threshold of alpha >= alpha_min, with a relative margin of 1e-3 (hardware
    // log, reciprocal and square root: their ~1e-7 relative errors are far inside the margins)
    const float tau = 2.f * (__logf(r1.y) - __logf(d.alpha_min)) * 1.001f + 1e-3f;
    const float A = r0.z, B = r0.w, C = r1.x;
    const float det = A * C - B * B;
    const float idet = __builtin_amdgcn_rcpf(det);
    const float dxm = __builtin_amdgcn_sqrtf(fmaxf(tau * C * idet, 0.f));  // half-width of the ellipse
    o0 = r0;
    o1 = make_float4(det, __builtin_amdgcn_rcpf(A), -B * dxm * __builtin_amdgcn_rcpf(C),
                     __builtin_amdgcn_sqrtf(fmaxf(A * tau * idet, 0.f)));
    o2 = make_float4(tau, 0.f, __uint_as_float(rc.x), __uint_as_float(rc.y));
  }
  brec[3 * (seg + k)] = o0;
  brec[3 * (seg + k) + 1] = o1;
  brec[3 * (seg + k) + 2] = o2;
}

// Tile columns of tile row ty whose pixel centres the ellipse
// q(p) = (p - m)^T [[A, B], [B, C]] (p - m) <= tau reaches, intersected with
// [x0, x1]; false if none. The ellipse's exact x-extent over the row's band of
// pixel-centre heights is used: its right end is a concave function of the
// height with the maximum at the ellipse's rightmost point, so it is evaluated
// at that height clamped to the band (and symmetrically for the left end).
struct EllipseRows {
  float mx, my, A, B, det, iA, tau, dyr, dym;  // dyr: height of the rightmost point; dym: half-height
  __device__ __forceinline__ bool row(const RenderDims& d, int ty, int x0, int x1, int& txl, int& txh) const {
    const float Y0 = (float)(ty * kTile) + 0.5f - my;
    const float Y1 = (float)(min(ty * kTile + kTile, d.H) - 1) + 0.5f - my;
    const float lo = fmaxf(Y0, -dym), hi = fminf(Y1, dym);
    if (!(lo <= hi)) return false;
    const float dr = fminf(fmaxf(dyr, lo), hi), dl = fminf(fmaxf(-dyr, lo), hi);
    // hardware square root (about 1 ulp): far inside the 0.01-pixel and 1e-3 threshold margins
    const float xr = mx + (-B * dr + __builtin_amdgcn_sqrtf(fmaxf(A * tau - det * dr * dr, 0.f))) * iA + 0.01f;
    const float xl = mx + (-B * dl - __builtin_amdgcn_sqrtf(fmaxf(A * tau - det * dl * dl, 0.f))) * iA - 0.01f;
    // tile tx has pixel centres 16 tx + 0.5 .. 16 tx + 15.5 (clipped to the image)
    const float fl = fminf(fmaxf(ceilf((xl - 15.5f) * (1.f / kTile)), -1.f), (float)d.TX);
    const float fh = fminf(fmaxf(floorf((xr - 0.5f) * (1.f / kTile)), -1.f), (float)d.TX);
    txl = max(x0, (int)fl);
    txh = min(x1, (int)fh);
    return txl <= txh;
  }
};

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

// Tile rows [r0, r1] whose band of pixel-centre heights (16 ty + 0.5 .. min(16 ty + 16, H) - 0.5)
// meets the ellipse's vertical extent [my - dym, my + dym], widened by 0.01 pixel, intersected with
// the rectangle's rows [y0, y1]; empty when r0 > r1. A closed form, so that the counting pass needs
// no per-row work and the emitting pass visits exactly the rows it counted.
__device__ __forceinline__ void ellipse_row_span(const RenderDims& d, float my, float dym, int y0, int y1, int& r0,
                                                 int& r1) {
  const float top = my - dym - 0.01f, bot = my + dym + 0.01f;
  const float fl = ceilf((top - 15.5f) * (1.f / kTile));
  const float fh = floorf((bot - 0.5f) * (1.f / kTile));
  r0 = max(y0, (int)fminf(fmaxf(fl, -1.f), (float)d.TY));
  r1 = min(y1, (int)fminf(fmaxf(fh, -1.f), (float)d.TY));
  if (!(top <= (float)d.H - 0.5f)) r1 = r0 - 1;  // below the last row of pixel centres
}

// Level 1: rows. Each wave walks bin_chunk depth-sorted Gaussians of one frame-view, 64 at a time
// with one Gaussian per lane. Every row of a Gaussian's span (ellipse_row_span) gets one entry
// (Gaussian index, tile-column range in the row), the range packed as first column | column count
// << 16 (a count of 0 when the ellipse misses the row's pixel centres after all).
// Counting pass: the per-row counts of the chunk, as a difference array over the rows (two LDS
// atomics per Gaussian) and a prefix sum.
// Emitting pass: a lane evaluates the column ranges of the first kRowPre rows of its span up front
// (kept in LDS); the wave then visits the rows the batch reaches, and per row a ballot ranks the
// hitting lanes, so the entries of a row keep the depth order of the batch (a stable counting
// sort; the per-row write positions live in LDS). Gaussians taller than kRowPre rows evaluate
// their further rows inside the row loop.
template <bool EMIT>
__global__ __launch_bounds__(64) void k_row_bin(RenderDims d, const uint32_t* __restrict__ skeys,
                                                const uint32_t* __restrict__ svals, const float4* __restrict__ brec,
                                                uint32_t* __restrict__ hist, const uint2* __restrict__ row_ranges,
                                                uint2* __restrict__ row_lists) {
  constexpr int kRowPre = 8;
  extern __shared__ uint32_t cnt[];  // TY + 1 words
  __shared__ uint32_t s_pk[64][kRowPre + 1];  // per lane: packed column ranges of its first rows
  const int lane = threadIdx.x;
  const int b = blockIdx.y, chunk = blockIdx.x;
  const int TY = d.TY;
  uint32_t* bh = hist + ((size_t)b * d.n_bin_chunks + chunk) * TY;
  for (int t = lane; t <= TY; t += 64) cnt[t] = EMIT && t < TY ? row_ranges[(size_t)b * TY + t].x + bh[t] : 0u;
  __syncthreads();
  const size_t seg = (size_t)b * d.n;
  const int start = chunk * d.bin_chunk;
  const int end = min(start + d.bin_chunk, d.n);
  for (int base = start; base < end; base += 64) {
    const int e = base + lane;
    uint32_t gi = 0;
    bool ok = false;
    EllipseRows el{};
    int x0 = 0, x1 = -1, r0 = 0, r1 = -1;
    if (e < end) {
      ok = skeys[seg + e] != 0xFFFFFFFFu;
      if (ok) {
        gi = svals[seg + e];
        const float4 q0 = brec[3 * (seg + e)], q1 = brec[3 * (seg + e) + 1], q2 = brec[3 * (seg + e) + 2];
        el = EllipseRows{q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q2.x, q1.z, q1.w};
        const uint32_t rx = __float_as_uint(q2.z), ry = __float_as_uint(q2.w);
        x0 = (int)(rx & 0xFFFF);
        x1 = (int)(rx >> 16);
        ellipse_row_span(d, el.my, el.dym, (int)(ry & 0xFFFF), (int)(ry >> 16), r0, r1);
      }
    }
    if (__ballot(ok) == 0ull) break;  // culled keys sort last
    const bool any = r0 <= r1;
    if (!EMIT) {
      if (any) {
        atomicAdd(&cnt[r0], 1u);
        atomicAdd(&cnt[r1 + 1], 0xFFFFFFFFu);  // -1
      }
      continue;
    }
    // column ranges of the first rows of the span, as many as the wave's tallest span needs
    const int npre = min(kRowPre, wave_max_i(any ? r1 - r0 + 1 : 0));
#pragma unroll
    for (int r = 0; r < kRowPre; ++r) {
      if (r >= npre) break;
      int txl = 0, txh = 0;
      const bool h = el.row(d, r0 + r, x0, x1, txl, txh);
      s_pk[lane][r] = h ? (uint32_t)txl | ((uint32_t)(txh - txl + 1) << 16) : 0u;
    }
    const bool tall = any && r1 - r0 >= kRowPre;
    const bool any_tall = __ballot(tall) != 0ull;
    const int ylo = wave_min_i(any ? r0 : 0x7FFFFFFF);
    const int yhi = wave_max_i(any ? r1 : -1);
    for (int ty = ylo; ty <= yhi; ++ty) {
      const uint32_t r = (uint32_t)(ty - r0);
      const bool hit = any && ty >= r0 && ty <= r1;
      uint32_t rg = s_pk[lane][min(r, (uint32_t)kRowPre - 1u)];
      if (any_tall && r >= (uint32_t)kRowPre) {
        int txl = 0, txh = 0;
        const bool h = el.row(d, ty, x0, x1, txl, txh);
        rg = h ? (uint32_t)txl | ((uint32_t)(txh - txl + 1) << 16) : 0u;
      }
      const unsigned long long m = __ballot(hit);
      if (m == 0ull) continue;
      const uint32_t pos0 = cnt[ty];
      if (hit) {
        const uint32_t pos = pos0 + popc_below(m);
        if (pos < d.row_capacity) row_lists[pos] = make_uint2(gi, rg);
      }
      if (lane == 0) cnt[ty] = pos0 + (uint32_t)__popcll(m);
    }
  }
  __syncthreads();
  if (!EMIT) {  // counts = prefix sums of the difference array
    uint32_t carry = 0;
    for (int t0 = 0; t0 < TY; t0 += 64) {
      uint32_t v = t0 + lane < TY ? cnt[t0 + lane] : 0u;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
      }
      if (t0 + lane < TY) bh[t0 + lane] = carry + v;
      carry += __shfl(v, 63);
    }
  }
}

// c + bit `lane` of the wave-uniform mask m: the mask is the carry-in of an add, so a lane learns
// whether a column range given as a lane mask covers it without a compare of its own.
__device__ __forceinline__ uint32_t add_lane_bit(uint32_t c, unsigned long long m) {
  uint32_t r;
  unsigned long long carry_out;
  asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(carry_out) : "v"(c), "s"(m));
  return r;
}

// Level 2: tiles of one row. One wave takes a segment of row_seg entries of a
// (frame-view, row) list; lane l owns tile column l (and l + 64 when the image
// is 64 or more tiles wide, TWO) and appends, in list (= depth) order, every
// entry whose column range covers it, so each lane writes its own tile list
// sequentially, from the offset the counting pass (k_tile_count) and the scans give.
//
// A lane stages its tile's entries in a 32-entry ring in LDS indexed by list position. Every
// entry is written at the lane's next free slot, whether or not it covers the lane's tile; the
// lane's counter advances only if it does, so a miss is overwritten by the next hit. Every 16
// entries of the segment the wave drains, per lane, the unaligned head up to the next 16-entry
// boundary of the list and then whole aligned 16-entry runs (four 16-byte stores each): at most
// 30 entries are outstanding when one is staged, so the slot it writes never holds one.
// One column per lane (up to 63 tiles): the entries are wave-uniform loads, and an entry's range
// becomes a 64-bit lane mask (a bit field) that is the carry-in of the counter's add.
template <bool TWO>
__global__ __launch_bounds__(64) void k_tile_bin(RenderDims d, const Status* __restrict__ st,
                                                 const uint2* __restrict__ row_ranges,
                                                 const uint2* __restrict__ row_lists, const uint32_t* __restrict__ hist,
                                                 const uint2* __restrict__ ranges, uint32_t* __restrict__ lists) {
  constexpr int kRing = 32, kStride = 36;  // stride: 16-byte aligned rows, spread banks; slot 32 is a sink
  __shared__ __align__(16) uint32_t wbuf[TWO ? 2 : 1][64][kStride];
  if (st->overflow & 2u) return;
  const int lane = threadIdx.x;
  const int s = blockIdx.x, ty = blockIdx.y, b = blockIdx.z;
  const uint2 rr = row_ranges[(size_t)b * d.TY + ty];
  const uint32_t start = rr.x + (uint32_t)s * (uint32_t)d.row_seg;
  if (start >= rr.y) return;
  const uint32_t end = min(start + (uint32_t)d.row_seg, rr.y);
  const int tx0 = lane, tx1 = lane + 64;
  const uint32_t* hb = hist + (((size_t)b * d.TY + ty) * d.n_row_segs + s) * d.TX;
  uint32_t c0 = 0, c1 = 0;   // next list position to fill
  uint32_t w0 = 0, w1 = 0;   // next list position to write out
  if (tx0 < d.TX) c0 = w0 = ranges[(size_t)b * d.T + ty * d.TX + tx0].x + hb[tx0];
  if (tx1 < d.TX) c1 = w1 = ranges[(size_t)b * d.T + ty * d.TX + tx1].x + hb[tx1];
  const unsigned long long cap = d.capacity;
  auto drain = [&](int q, uint32_t c, uint32_t& w, bool last) {
    const uint32_t* ring = wbuf[q][lane];
    if (w & 15u) {  // head: up to the next aligned position
      const uint32_t bnd = (w + 15u) & ~15u;
      if (c >= bnd || last) {
        const uint32_t stop = min(bnd, c);
        for (uint32_t p = w; p < stop; ++p)
          if (p < cap) lists[p] = ring[p & (kRing - 1)];
        w = stop;
      }
    }
    while (c - w >= 16u) {  // whole aligned runs
      if ((unsigned long long)w + 16ull <= cap) {
        const uint4* src = (const uint4*)(ring + (w & (kRing - 1)));
        uint4* dst = (uint4*)(lists + w);
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[v] = src[v];
      } else {
        for (uint32_t k = 0; k < 16u; ++k)
          if (w + k < cap) lists[w + k] = ring[(w + k) & (kRing - 1)];
      }
      w += 16u;
    }
    if (last) {
      for (uint32_t p = w; p < c; ++p)
        if (p < cap) lists[p] = ring[p & (kRing - 1)];
      w = c;
    }
  };
  if constexpr (!TWO) {
    uint32_t* const ring = wbuf[0][lane];
    auto stage = [&](const uint2 en) {
      // lanes [first, first + count) of the entry's range: first < 64 is the low 6 bits of en.y
      // and the count (1..63) its high half
      const uint32_t y = __builtin_amdgcn_readfirstlane(en.y);  // wave-uniform (a no-op when scalar)
      unsigned long long m;
      asm("s_bfm_b64 %0, %1, %2" : "=s"(m) : "s"(y >> 16), "s"(y));
      ring[c0 & (kRing - 1)] = en.x;
      c0 = add_lane_bit(c0, m);
    };
    // whole blocks of 16 entries (wave-uniform loads); block k + 1 is requested once the first
    // entry of block k is staged, since waiting for any scalar load waits for all of them
    const uint32_t nfull = (end - start) >> 4;
    uint2 ea[16], eb[16];
    auto load = [&](uint2(&e)[16], uint32_t k) {
      const uint2* blk = row_lists + start + 16u * k;
#pragma unroll
      for (int u = 0; u < 16; ++u) e[u] = blk[u];
    };
    if (nfull > 0u) load(ea, 0u);
    for (uint32_t k = 0; k < nfull; k += 2u) {
      stage(ea[0]);
      if (k + 1u < nfull) load(eb, k + 1u);
#pragma unroll
      for (int u = 1; u < 16; ++u) stage(ea[u]);
      drain(0, c0, w0, false);
      if (k + 1u >= nfull) break;
      stage(eb[0]);
      if (k + 2u < nfull) load(ea, k + 2u);
#pragma unroll
      for (int u = 1; u < 16; ++u) stage(eb[u]);
      drain(0, c0, w0, false);
    }
    for (uint32_t q = start + 16u * nfull; q < end; ++q) stage(row_lists[q]);
  } else {
    for (uint32_t base = start; base < end; base += 64) {
      const uint32_t e = base + lane;
      // entries past the end of the segment get an empty column range
      const uint2 ent = e < end ? row_lists[e] : make_uint2(0u, 0u);
      const int nin = (int)min(64u, end - base);
      // blocks of 16 entries with no branch per entry: a lane whose tile the entry does not cover
      // writes the ring's spare slot kRing and does not advance; one drain per block, so that at
      // most 16 entries per lane are new since the last drain
      for (int jb = 0; jb < nin; jb += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int j = jb + u;
          const uint32_t rg = __builtin_amdgcn_readlane(ent.y, j);
          const int txl = (int)(rg & 0xFFFF), txe = txl + (int)(rg >> 16);
          const bool h0 = (tx0 >= txl) & (tx0 < txe);
          const bool h1 = (tx1 >= txl) & (tx1 < txe);
          const uint32_t gi = __builtin_amdgcn_readlane(ent.x, j);
          wbuf[0][lane][h0 ? (c0 & (kRing - 1)) : kRing] = gi;
          wbuf[TWO ? 1 : 0][lane][h1 ? (c1 & (kRing - 1)) : kRing] = gi;
          c0 += h0 ? 1u : 0u;
          c1 += h1 ? 1u : 0u;
        }
        drain(0, c0, w0, false);
        drain(TWO ? 1 : 0, c1, w1, false);
      }
    }
  }
  drain(0, c0, w0, true);
  if (TWO) drain(TWO ? 1 : 0, c1, w1, true);
}

// Level 2, counting: the number of entries of a segment of row_seg entries of a (frame-view, row)
// list whose column range covers each tile of the row, as a difference array: an entry adds 1 at
// its first column and -1 after its last (LDS atomics), and a prefix sum over the columns gives the
// counts (the same integers the emitting pass then places). One wave per segment.
__global__ __launch_bounds__(64) void k_tile_count(RenderDims d, const Status* __restrict__ st,
                                                   const uint2* __restrict__ row_ranges,
                                                   const uint2* __restrict__ row_lists, uint32_t* __restrict__ hist) {
  __shared__ int diff[kMaxTilesX + 1];
  if (st->overflow & 2u) return;
  const int lane = threadIdx.x;
  const int s = blockIdx.x, ty = blockIdx.y, b = blockIdx.z;
  const uint2 rr = row_ranges[(size_t)b * d.TY + ty];
  const uint32_t start = rr.x + (uint32_t)s * (uint32_t)d.row_seg;
  if (start >= rr.y) return;
  const uint32_t end = min(start + (uint32_t)d.row_seg, rr.y);
  for (int j = lane; j <= d.TX; j += 64) diff[j] = 0;
  __syncthreads();
  for (uint32_t e = start + lane; e < end; e += 64) {
    const uint32_t rg = row_lists[e].y;
    const int txl = (int)(rg & 0xFFFF), txe = txl + (int)(rg >> 16);  // txl < txe <= TX
    atomicAdd(&diff[txl], 1);
    atomicAdd(&diff[txe], -1);
  }
  __syncthreads();
  uint32_t* hb = hist + (((size_t)b * d.TY + ty) * d.n_row_segs + s) * d.TX;
  int carry = 0;
  for (int t0 = 0; t0 < d.TX; t0 += 64) {
    int v = t0 + lane < d.TX ? diff[t0 + lane] : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(v, off);
      if (lane >= off) v += u;
    }
    if (t0 + lane < d.TX) hb[t0 + lane] = (uint32_t)(carry + v);
    carry += __shfl(v, 63);
  }
}

// Inclusive prefix sum over the wave (every lane active).
__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  return v;
}

// Per (frame-view, bin): exclusive prefix over the chunks of level 1 (bins = rows).
// One wave per bin, 64 chunks per step.
__global__ __launch_bounds__(64) void k_chunk_scan(int nbins_total, int nbins, int nchunks,
                                                   uint32_t* __restrict__ hist, uint32_t* __restrict__ tot) {
  const int g = blockIdx.x;
  if (g >= nbins_total) return;
  const int lane = threadIdx.x;
  const int b = g / nbins, t = g - b * nbins;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nchunks; c0 += 64) {
    const int c = c0 + lane;
    const size_t o = ((size_t)b * nchunks + c) * nbins + t;
    const uint32_t v = c < nchunks ? hist[o] : 0u;
    const uint32_t incl = (uint32_t)wave_incl_scan_u64(v, lane);
    if (c < nchunks) hist[o] = carry + incl - v;
    carry += (uint32_t)__shfl(incl, 63);
  }
  if (lane == 0) tot[g] = carry;
}

// Exclusive scan of count values by one 1024-thread block, 4 consecutive values per thread
// per pass (coalesced 16-byte loads); emit(i, prefix, value) is called for every element, and
// the returned value is the total. All threads of the block must call it.
template <class Emit>
__device__ unsigned long long block_scan_u32(const uint32_t* __restrict__ in, int count, Emit emit) {
  __shared__ unsigned long long s_w[16];
  __shared__ unsigned long long s_tile;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  unsigned long long carry = 0;
  for (int base = 0; base < count; base += 4096) {
    const int i0 = base + 4 * t;
    uint32_t v[4];
    if (i0 + 3 < count && ((reinterpret_cast<uintptr_t>(in + i0) & 15) == 0)) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + i0);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = i0 + k < count ? in[i0 + k] : 0u;
    }
    const unsigned long long tsum = (unsigned long long)v[0] + v[1] + v[2] + v[3];
    const unsigned long long wincl = wave_incl_scan_u64(tsum, lane);
    if (lane == 63) s_w[w] = wincl;
    __syncthreads();
    if (w == 0) {
      const unsigned long long x = lane < 16 ? s_w[lane] : 0ull;
      const unsigned long long xi = wave_incl_scan_u64(x, lane);
      if (lane < 16) s_w[lane] = xi - x;
      if (lane == 15) s_tile = xi;
    }
    __syncthreads();
    unsigned long long run = carry + s_w[w] + wincl - tsum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < count) emit(i0 + k, run, v[k]);
      run += v[k];
    }
    carry += s_tile;
    __syncthreads();
  }
  return carry;
}

// Per (frame-view, tile): exclusive prefix over the level-2 segments of its row.
__global__ __launch_bounds__(256) void k_seg_scan(RenderDims d, const Status* __restrict__ st,
                                                  const uint2* __restrict__ row_ranges, uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ tot) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.B * d.T) return;
  const int b = g / d.T, tile = g - b * d.T;
  const int ty = tile / d.TX, tx = tile - ty * d.TX;
  uint32_t run = 0;
  if (!(st->overflow & 2u)) {
    const uint2 rr = row_ranges[(size_t)b * d.TY + ty];
    const int nseg = (int)((rr.y - rr.x + d.row_seg - 1) / d.row_seg);
    for (int sgi = 0; sgi < nseg; ++sgi) {
      const size_t o = (((size_t)b * d.TY + ty) * d.n_row_segs + sgi) * d.TX + tx;
      const uint32_t v = hist[o];
      hist[o] = run;
      run += v;
    }
  }
  tot[g] = run;
}

// Exclusive scan of `count` totals into [start, end) ranges. level 0 (rows):
// flags overflow bit 2 if the row pairs exceed their capacity; level 1 (tiles):
// flags bit 1 for the tile pairs and records the pairs needed.
// Per frame-view: exclusive scan of the (digit-major, chunk-minor) radix histogram.
__global__ __launch_bounds__(1024) void k_radix_scan(RenderDims d, uint32_t* __restrict__ hist) {
  uint32_t* h = hist + (size_t)blockIdx.x * 256 * d.n_sort_chunks;
  block_scan_u32(h, 256 * d.n_sort_chunks, [&](int j, unsigned long long run, uint32_t) { h[j] = (uint32_t)run; });
}

__global__ __launch_bounds__(1024) void k_scan_ranges(int count, int level, unsigned long long cap,
                                                      const uint32_t* __restrict__ tot, uint2* __restrict__ ranges,
                                                      Status* __restrict__ st) {
  const unsigned long long total =
      block_scan_u32(tot, count, [&](int j, unsigned long long run, uint32_t v) {
        const unsigned long long e = run + v;
        ranges[j] = make_uint2((uint32_t)min(run, 0xFFFFFFFFull), (uint32_t)min(e, 0xFFFFFFFFull));
      });
  if (threadIdx.x == 0) {
    if (level == 0) {
      st->overflow = total > cap ? 2u : 0u;
      st->needed_pairs = 2ull * total;  // a lower bound of the tile pairs while the rows overflow
      st->fwd_evals = 0;
      st->fwd_contribs = 0;
    } else if (!(st->overflow & 2u)) {
      st->overflow = total > cap ? 1u : 0u;
      st->needed_pairs = max(total, st->needed_pairs);
    }
  }
}

// ============================================================ rasterization
struct TileCtx {
  int b, tile, px, py, ox, oy;  // ox, oy: pixel origin of the tile
  bool inside;
  uint2 range;
};

__device__ __forceinline__ bool tile_ctx(const RenderDims& d, const uint2* ranges, TileCtx& c) {
  const int per = (d.B * d.T + 7) / 8;
  const int wid = xcd_item(blockIdx.x, per);
  if (wid >= d.B * d.T) return false;
  c.b = wid / d.T;
  c.tile = wid - c.b * d.T;
  const int tx = c.tile % d.TX, ty = c.tile / d.TX;
  c.ox = tx * kTile;
  c.oy = ty * kTile;
  // layout 1: wave w covers the 8x8 quadrant (w & 1, w >> 1) of the tile, lane l its pixel
  // (l & 7, l >> 3); layout 2: wave w covers rows 4w..4w+3, lane l pixel (l & 15, l >> 4)
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (d.wave_layout == 2) {
    c.px = tx * kTile + (l & 15);
    c.py = ty * kTile + 4 * w + (l >> 4);
  } else {
    c.px = tx * kTile + (w & 1) * 8 + (l & 7);
    c.py = ty * kTile + (w >> 1) * 8 + (l >> 3);
  }
  c.inside = c.px < d.W && c.py < d.H;
  c.range = ranges[(size_t)c.b * d.T + c.tile];
  return true;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
  return v;
}

// Adds the per-thread work counters of a block to the status word (one atomic per wave).
__device__ __forceinline__ void flush_counters(uint32_t evals, uint32_t contribs, unsigned long long* e,
                                               unsigned long long* c) {
  evals = wave_sum_u(evals);
  contribs = wave_sum_u(contribs);
  if ((threadIdx.x & 63) == 0) {
    if (evals) atomicAdd(e, (unsigned long long)evals);
    if (contribs) atomicAdd(c, (unsigned long long)contribs);
  }
}

// Smallest layer a Gaussian of index gi belongs to (layers are nested prefixes).
__device__ __forceinline__ uint32_t first_layer(const RenderDims& d, uint32_t gi) {
  uint32_t l = 0;
#pragma unroll
  for (int q = 0; q < kMaxLevels - 1; ++q) l += (q < d.L - 1 && gi >= (uint32_t)d.lv[q]) ? 1u : 0u;
  return l;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within each 16 lanes

// Unsigned maximum over the wave, in every lane (all 64 lanes active).
__device__ __forceinline__ uint32_t wave_max_u(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppXor1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppXor2, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppHalfMirror, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppMirror, 0xF, 0xF, false));
  const auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = max(r16[0], r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return __builtin_amdgcn_readfirstlane(max(r32[0], r32[1]));
}

// Sub-tiles of the 16x16 tile with origin (x0, y0) whose pixel centres the
// ellipse q(p) <= tau of alpha >= alpha_min may reach: bit w for the pixels of
// wave w (layout 1: the 8x8 quadrant (w & 1, w >> 1); layout 2: rows 4w..4w+3).
// The same exact row-extent test (and margins) as the binning, on the sub-tiles'
// bands of pixel-centre rows; a wave skips every entry whose bit is clear.
__device__ __forceinline__ uint32_t quad_mask(const RenderDims& d, float mx, float my, float A, float B, float C,
                                              float o, int x0, int y0) {
  // hardware log / reciprocal / square root: their relative errors (~1e-7) are far inside the
  // 1e-3 threshold margin and the 0.01-pixel margin
  const float tau = 2.f * (__logf(o) - __logf(d.alpha_min)) * 1.001f + 1e-3f;
  const float det = A * C - B * B;
  if (!(tau > 0.f) || !(det > 0.f) || !(A > 0.f) || !(C > 0.f)) return 0xFu;
  const float iA = __builtin_amdgcn_rcpf(A), idet = __builtin_amdgcn_rcpf(det);
  const float dxm = __builtin_amdgcn_sqrtf(tau * C * idet);
  const float dyr = -B * dxm * __builtin_amdgcn_rcpf(C), dym = __builtin_amdgcn_sqrtf(A * tau * idet);
  const bool strips = d.wave_layout == 2;
  const int nb = strips ? 4 : 2;           // bands of pixel-centre rows
  const float bh = strips ? 3.f : 7.f;     // band height - 1
  uint32_t m = 0;
  for (int q = 0; q < nb; ++q) {
    const float Y0 = (float)(y0 + (strips ? 4 : 8) * q) + 0.5f - my;
    const float lo = fmaxf(Y0, -dym), hi = fminf(Y0 + bh, dym);
    if (!(lo <= hi)) continue;
    const float dr = fminf(fmaxf(dyr, lo), hi), dl = fminf(fmaxf(-dyr, lo), hi);
    const float xr = mx + (-B * dr + __builtin_amdgcn_sqrtf(fmaxf(A * tau - det * dr * dr, 0.f))) * iA + 0.01f;
    const float xl = mx + (-B * dl - __builtin_amdgcn_sqrtf(fmaxf(A * tau - det * dl * dl, 0.f))) * iA - 0.01f;
    if (strips) {
      const float X0 = (float)x0 + 0.5f;
      if (xl <= X0 + 15.f && xr >= X0) m |= 1u << q;
    } else {
#pragma unroll
      for (int qx = 0; qx < 2; ++qx) {
        const float X0 = (float)(x0 + 8 * qx) + 0.5f;
        if (xl <= X0 + 7.f && xr >= X0) m |= 1u << (2 * q + qx);
      }
    }
  }
  return m;
}

// Block-wide stable compaction of one candidate per thread: returns the slot of
// this thread's candidate (if `keep`) and the number kept in *total.
__device__ __forceinline__ int compact_slot(bool keep, uint32_t* s_wcnt, int* total) {
  const int t = threadIdx.x, w = t >> 6;
  const unsigned long long m = __ballot(keep);
  if ((t & 63) == 0) s_wcnt[w] = (uint32_t)__popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < kTilePix / 64; ++q) {
    const int c = (int)s_wcnt[q];
    off += q < w ? c : 0;
    tot += c;
  }
  *total = tot;
  return off + (int)popc_below(m);
}

// Open-layer state of the forward compositor, read from the signs of Tr (a closed layer holds
// -T): nlhi = bound of the lane's highest open layer (0 if none), wopen = the layers open in
// some lane of the wave and whi = the bound of the highest of them (both wave-uniform). Called
// with every lane of the wave active. The state only shrinks, so a stale copy is a superset of
// the true one: it costs evaluations, never a contribution.
template <int MAXL>
__device__ __forceinline__ void open_state(const RenderDims& d, const float* Tr, uint32_t& nlhi, uint32_t& wopen,
                                           uint32_t& whi) {
  nlhi = 0;
  wopen = 0;
  whi = 0;
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    if (l >= d.L) break;
    const bool open = Tr[l] > 0.f;
    nlhi = open ? (uint32_t)d.lv[l] : nlhi;
    if (__ballot(open) != 0ull) {
      wopen |= 1u << l;
      whi = (uint32_t)d.lv[l];
    }
  }
}

// at least 7 waves per SIMD for up to 6 layers (72 VGPRs; one value spilled before the walk and
// reloaded for the output): the walk has long LDS and exp latencies, and a seventh wave hid more
// of them than the registers it costs (eight waves need spills inside the walk and are slower)
template <int MAXL, bool COUNT>
__global__ __launch_bounds__(kTilePix) __attribute__((amdgpu_waves_per_eu(MAXL <= 6 ? 7 : 1))) void k_raster_fwd(RenderDims d, Status* __restrict__ st,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ lists,
                                                         const float4* __restrict__ rec, float* __restrict__ image,
                                                         float* __restrict__ t_final, uint32_t* __restrict__ n_last) {
  if (st->overflow) return;
  TileCtx c;
  if (!tile_ctx(d, ranges, c)) return;
  __shared__ float4 s_a[kTilePix];  // mx, my, o, index bits
  __shared__ float4 s_b[kTilePix];  // scaled conic a2, b2, c2, (first layer | quadrant mask << 8) bits
  __shared__ float4 s_c[kTilePix];  // r, g, b, list position bits
  __shared__ uint32_t s_wcnt[kTilePix / 64];
  __shared__ uint32_t s_hi;
  const float fpx = (float)c.px + 0.5f, fpy = (float)c.py + 0.5f;
  const int t = threadIdx.x;
  const uint32_t qbit = 1u << (8 + __builtin_amdgcn_readfirstlane(t >> 6));
  // Tr[l] > 0: open layer and its transmittance; a closed layer keeps -T (its final
  // transmittance, negated), so that T (1 - alpha) < t_stop rejects it with no extra test
  float Tr[MAXL], Cr[MAXL], Cg[MAXL], Cb[MAXL];
  uint32_t last[MAXL];
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    Tr[l] = (c.inside && l < d.L) ? 1.f : -1.f;
    Cr[l] = Cg[l] = Cb[l] = 0.f;
    last[l] = 0;
  }
  uint32_t nlhi, wopen, whi;
  const size_t recbase = (size_t)c.b * d.n;
  uint32_t n_eval = 0, n_contrib = 0;
  // the list entry of the next batch is read while this batch is walked
  // entries staged per round (d.batch <= kTilePix, threads t < d.batch stage one each)
  const uint32_t nb = (uint32_t)d.batch;
  const bool stager = (uint32_t)t < nb;
  uint32_t gnext = stager && c.range.x + t < c.range.y ? lists[c.range.x + t] : 0xFFFFFFFFu;
  for (uint32_t base = c.range.x; base < c.range.y; base += nb) {
    const uint32_t gi = gnext;
    gnext = stager && base + nb + t < c.range.y ? lists[base + nb + t] : 0xFFFFFFFFu;
    open_state<MAXL>(d, Tr, nlhi, wopen, whi);
    // entries of index >= every pixel's highest open layer bound are useless to the whole tile
    if (t == 0) s_hi = 0;
    __syncthreads();
    if (nlhi) atomicMax(&s_hi, nlhi);
    __syncthreads();
    const uint32_t hib = s_hi;
    if (hib == 0) break;
    const uint32_t k = base + t;
    int cnt;
    const int slot = compact_slot(gi < hib, s_wcnt, &cnt);
    if (gi < hib) {
      const float4* r = rec + 3 * (recbase + gi);
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      const uint32_t qm = quad_mask(d, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, c.ox, c.oy);
      s_a[slot] = make_float4(r0.x, r0.y, r1.y, __uint_as_float(gi));
      s_b[slot] = make_float4(-0.5f * kLog2e * r0.z, -kLog2e * r0.w, -0.5f * kLog2e * r1.x,
                              __uint_as_float(first_layer(d, gi) | (qm << 8)));
      s_c[slot] = make_float4(r1.z, r1.w, r2.x, __uint_as_float(k - c.range.x + 1));
    }
    __syncthreads();
    // the staged entries this wave may need (ellipse reaching its pixels, index below the bound
    // of its highest open layer), one ballot mask per 64 staged entries walked in order with
    // scalar find-first-set; per lane, the layer updates are selects, a layer closed in every
    // lane of the wave is skipped, and the open-layer state is refreshed after each 64 entries
    for (int q = 0; q * 64 < cnt && wopen; ++q) {
      uint64_t m;
      {
        const int e = q * 64 + (t & 63);
        bool need = false;
        if (e < cnt) need = (__float_as_uint(s_b[e].w) & qbit) && __float_as_uint(s_a[e].w) < whi;
        m = __ballot(need);
      }
      while (m != 0) {
        const int bit = (int)__builtin_ctzll(m);
        m &= ~(1ull << bit);
        const int e = (q << 6) + bit;
        // all three staged vectors are read up front, so that the colour and first layer are at hand
        // when some lane contributes
        const float4 a = s_a[e];
        const float4 cb = s_b[e];
        const float4 col = s_c[e];
        const uint32_t lmin = __builtin_amdgcn_readfirstlane(__float_as_uint(cb.w)) & 0xFFu;
        const AlphaEval ev = alpha_eval(fpx, fpy, a.x, a.y, cb.x, cb.y, cb.z, a.z);
        const bool cand = __float_as_uint(a.w) < nlhi;
        if (COUNT) n_eval += cand ? 1u : 0u;
        // keeps the colour read here, ahead of the branch (the compiler would sink it into it)
        asm volatile("" ::"v"(col.x), "v"(col.y), "v"(col.z), "v"(col.w));
        if (cand && ev.ga >= d.alpha_min) {
          const float al = __builtin_amdgcn_fmed3f(ev.ga, 0.f, d.alpha_max);  // min(alpha_max, ga), ga >= 0
          const float oma = 1.f - al;
          const uint32_t pos = __float_as_uint(col.w);
          // the entry's layers (lmin and above) that are open in some lane of the wave (uniform)
          const uint32_t lmask = wopen & (0xFFu << lmin);
#pragma unroll
          for (int l = 0; l < MAXL; ++l) {
            if (!((lmask >> l) & 1u)) continue;
            const float Tn = Tr[l] * oma;
            // false for a closed layer; for an open one, this Gaussian would take the layer below
            // the floor: it closes the layer and does not contribute
            const bool ok = Tn >= d.t_stop;
            const float wgt = ok ? al * Tr[l] : 0.f;
            Cr[l] = fmaf(col.x, wgt, Cr[l]);
            Cg[l] = fmaf(col.y, wgt, Cg[l]);
            Cb[l] = fmaf(col.z, wgt, Cb[l]);
            Tr[l] = ok ? Tn : -fabsf(Tr[l]);
            last[l] = ok ? pos : last[l];
            if (COUNT) n_contrib += ok ? 1u : 0u;
          }
        }
      }
      open_state<MAXL>(d, Tr, nlhi, wopen, whi);
    }
  }
  if (COUNT) flush_counters(n_eval, n_contrib, &st->fwd_evals, &st->fwd_contribs);
  if (!c.inside) return;
  const size_t HW = (size_t)d.W * d.H;
  const size_t pix = (size_t)c.py * d.W + c.px;
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    if (l >= d.L) break;
    const size_t o = (size_t)c.b * d.L + l;
    const float T = fabsf(Tr[l]);
    image[(o * 3 + 0) * HW + pix] = fmaf(T, d.bg[0], Cr[l]);
    image[(o * 3 + 1) * HW + pix] = fmaf(T, d.bg[1], Cg[l]);
    image[(o * 3 + 2) * HW + pix] = fmaf(T, d.bg[2], Cb[l]);
    t_final[o * HW + pix] = T;
    n_last[o * HW + pix] = last[l];
  }
}

// The nine per-entry sums of the backward are moments of dp = dL/dalpha * o * G over the pixels
// (dp dx, dp dy, dp dx^2, dp dx dy, dp dy^2, dp), with dx, dy the offset of the pixel from the
// mean, and the colour gradients (r, g, b); their constant factors are applied once to each sum:
// dL/d(A, B, C) = -(1/2, 1, 1/2) (sum dp dx^2, sum dp dx dy, sum dp dy^2), dL/do = sum dp / o (the
// flush divides by o). The gradient record keeps the first two as moments: the mean gradient,
// dL/dm = [[A, B], [B, C]] (sum dp dx, sum dp dy), is formed by the projection backward, which has
// the conic at hand, once per (view, Gaussian).
constexpr float kGradScale[9] = {1.f, 1.f, -0.5f, -1.f, -0.5f, 1.f, 1.f, 1.f, 1.f};

// A float in LDS, addressed with 32-bit offsets.
typedef __attribute__((address_space(3))) float lds_float;

// Wave reduction of nine per-lane values. Values 0..7 are reduce-scattered:
// each halving step pairs two values and exchanges the halves of the wave
// that keep them (v_permlane32_swap, then v_permlane16_swap across rows, then a
// row mirror), so that every aligned group of 8 lanes ends with the sum of one
// value over all 64 lanes, which a butterfly inside the group completes. Value
// 8 is only summed inside each aligned group of 8 lanes (the same butterfly);
// the caller adds the eight group sums. On return g[0] holds the group's value
// and g[8] the group's sum of value 8.
__device__ __forceinline__ void reduce_scatter9(float* g, int lane) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[q]), __float_as_uint(g[q + 4]), false, false);
    g[q] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(g[q]), __float_as_uint(g[q + 2]), false, false);
    g[q] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool hi = lane & 8;
    const float send = hi ? g[0] : g[1];
    const float keep = hi ? g[1] : g[0];
    g[0] = keep + dpp<kDppMirror>(send);
  }
  g[0] += dpp<kDppHalfMirror>(g[0]);
  g[0] += dpp<kDppXor2>(g[0]);
  g[0] += dpp<kDppXor1>(g[0]);
  float v = g[8];
  v += dpp<kDppHalfMirror>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppXor1>(v);
  g[8] = v;
}

// Deterministic accumulation: a float x is added to a 128-bit two's-complement fixed-point sum
// (low word: the fraction, 2^-64 units; high word: the integer part) with two 64-bit integer
// atomics, the carry out of the low word going into the high word. Integer addition does not
// depend on the order, so the sum is the same on every run; bits of x below 2^-64 are dropped and
// |x| is saturated at 2^62.
__device__ __forceinline__ void fx_add(unsigned long long* p, float x) {
  double a = fabs((double)x);
  if (!(a < 0x1p62)) a = 0x1p62;
  const double ip = floor(a);
  unsigned long long lo = (unsigned long long)((a - ip) * 0x1p64);  // a - ip is exact and < 1
  unsigned long long hi = (unsigned long long)ip;
  if (x < 0.f) {  // negate the 128-bit value
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const unsigned long long old = atomicAdd(p, lo);
  atomicAdd(p + 1, hi + (old + lo < old ? 1ull : 0ull));
}

__device__ __forceinline__ float fx_value(const unsigned long long* p) {
  return (float)((double)(long long)p[1] + (double)p[0] * 0x1p-64);
}

// at least 7 waves per SIMD for up to 6 layers (72 VGPRs, the layer bounds in scalar registers):
// a seventh wave hides more of the walk's LDS and exp latencies than six waves with 78 registers
template <int MAXL, bool COUNT, bool DET>
__global__ __launch_bounds__(kTilePix) __attribute__((amdgpu_waves_per_eu(MAXL <= 6 ? 7 : 1))) void k_raster_bwd(RenderDims d, Status* __restrict__ st,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ lists,
                                                         const float4* __restrict__ rec,
                                                         const float* __restrict__ t_final,
                                                         const uint32_t* __restrict__ n_last,
                                                         const float* __restrict__ image,
                                                         const float* __restrict__ d_image,
                                                         const float* __restrict__ target,
                                                         float* __restrict__ g2d, float* __restrict__ loss_out,
                                                         unsigned long long* __restrict__ g2d_fx,
                                                         unsigned long long* __restrict__ loss_fx) {
  if (st->overflow) return;
  TileCtx c;
  if (!tile_ctx(d, ranges, c)) return;
  __shared__ float4 s_a[kTilePix];  // mx, my, o, index bits
  __shared__ float4 s_b[kTilePix];  // scaled conic a2, b2, c2, (first layer | quadrant mask << 8) bits
  __shared__ float4 s_c[kTilePix];  // r, g, b, list position bits
  __shared__ float s_g[kTilePix][kGradLds];  // per-entry gradient sums of the four waves
  __shared__ uint32_t s_wcnt[kTilePix / 64];
  __shared__ uint32_t s_lmax[kMaxLevels];
  __shared__ float s_loss;
  const int t = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const uint32_t qbit = 1u << (8 + wv);
  if (t < kMaxLevels) s_lmax[t] = 0;
  if (t == 0) s_loss = 0.f;
  for (int v = 0; v < kGradLds; ++v) s_g[t][v] = 0.f;
  __syncthreads();
  const float fpx = (float)c.px + 0.5f, fpy = (float)c.py + 0.5f;
  const size_t HW = (size_t)d.W * d.H;
  const size_t pix = (size_t)c.py * d.W + c.px;
  // Q[l]: the colour composited behind the current entry (background included), weighted by
  // dL/dC of the layer and summed over the channels; it is all the backward needs of it
  float Tr[MAXL], wr[MAXL], wg[MAXL], wb[MAXL], Q[MAXL];
  uint32_t last[MAXL];
  float loss = 0.f;
  const float inv3hw = 1.0f / (3.0f * (float)HW);
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    Tr[l] = 0.f; wr[l] = wg[l] = wb[l] = 0.f; last[l] = 0;
    if (c.inside && l < d.L) {
      const size_t o = (size_t)c.b * d.L + l;
      Tr[l] = t_final[o * HW + pix];
      last[l] = n_last[o * HW + pix];
      float w3[3];
      for (int ch = 0; ch < 3; ++ch) {
        if (d_image) {
          w3[ch] = d_image[(o * 3 + ch) * HW + pix];
        } else {
          const float diff = image[(o * 3 + ch) * HW + pix] - target[((size_t)c.b * 3 + ch) * HW + pix];
          const float sgn = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
          w3[ch] = d.lw[l] * sgn * inv3hw;
          loss += d.lw[l] * fabsf(diff) * inv3hw;
        }
      }
      wr[l] = w3[0]; wg[l] = w3[1]; wb[l] = w3[2];
      if (last[l]) atomicMax(&s_lmax[l], last[l]);
    }
    Q[l] = Tr[l] * (wr[l] * d.bg[0] + wg[l] * d.bg[1] + wb[l] * d.bg[2]);
  }
  if (loss_out) {
    loss = wave_sum(loss);
    if ((t & 63) == 0) {
      if (DET)
        fx_add(loss_fx, loss);
      else
        atomicAdd(&s_loss, loss);
    }
  }
  __syncthreads();
  if (!DET && loss_out && t == 0) unsafeAtomicAdd(loss_out, s_loss);
  uint32_t lmax[MAXL];
  uint32_t ktop = 0;
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    lmax[l] = __builtin_amdgcn_readfirstlane(l < d.L ? s_lmax[l] : 0u);  // block-uniform: scalar registers
    ktop = max(ktop, lmax[l]);
  }
  // per wave: lw[m] = the largest last-contributor position over its pixels and the layers l >= m,
  // so that an entry of first layer m at position kk can matter to the wave only if kk < lw[m]
  uint32_t lw[MAXL];
  {
    uint32_t run = 0;
#pragma unroll
    for (int l = MAXL - 1; l >= 0; --l) {
      run = max(run, wave_max_u(l < d.L ? last[l] : 0u));
      lw[l] = __builtin_amdgcn_readfirstlane(run);  // wave-uniform
    }
  }
  const size_t recbase = (size_t)c.b * d.n;
  const int lane = t & 63;
  uint32_t n_eval = 0, n_contrib = 0;
  // the value index an aligned 8-lane group holds after reduce_scatter9: reduce the one-hot
  // pattern g[q] = q (every lane), which leaves 64 * index in each lane
  int vid;
  {
    float pr[9] = {0.f, 1.f, 2.f, 3.f, 4.f, 5.f, 6.f, 7.f, 0.f};
    reduce_scatter9(pr, lane);
    vid = (int)(pr[0] * (1.f / 64.f) + 0.5f);
  }
  // after the reduction lane 8k adds value vid and lane 8k + 1 the group's sum of value 8 to the
  // entry's LDS sums (an LDS atomic each; the eight value-8 adds meet on one address)
  const bool adder = (lane & 7) < 2;
  lds_float* const g_slot = (lds_float*)&s_g[0][0] + ((lane & 7) == 0 ? vid : 8);
  const int nb = d.batch;  // entries staged per round (<= kTilePix, threads t < nb stage one each)
  for (int top = (int)ktop; top > 0; top -= nb) {
    const int lo = max(0, top - nb);
    __syncthreads();
    // stage the entries some pixel of the tile still needs (position before that layer's last
    // contributor, index inside the layer), keeping their order
    const uint32_t k = (uint32_t)(lo + t);
    uint32_t gi = 0xFFFFFFFFu;
    bool need = false;
    if (t < nb && (int)k < top) {
      gi = lists[c.range.x + k];
#pragma unroll
      for (int l = 0; l < MAXL; ++l) need = need || (k < lmax[l] && gi < (uint32_t)d.lv[l]);
    }
    int cnt;
    const int slot = compact_slot(need, s_wcnt, &cnt);
    if (need) {
      const float4* r = rec + 3 * (recbase + gi);
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      const uint32_t qm = quad_mask(d, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, c.ox, c.oy);
      s_a[slot] = make_float4(r0.x, r0.y, r1.y, __uint_as_float(gi));
      s_b[slot] = make_float4(-0.5f * kLog2e * r0.z, -kLog2e * r0.w, -0.5f * kLog2e * r1.x,
                              __uint_as_float(first_layer(d, gi) | (qm << 8)));
      s_c[slot] = make_float4(r1.z, r1.w, r2.x, __uint_as_float(k));
    }
    __syncthreads();
    // this wave's entries: staged entries whose ellipse reaches its quadrant and that lie before the
    // last contributor of some layer they belong to, for some pixel of the wave; one ballot mask
    // per 64 staged entries, walked back to front with scalar find-last-set
    for (int q = (cnt - 1) >> 6; q >= 0; --q) {
      uint64_t m;
      {
        const int e = q * 64 + lane;
        bool keep = false;
        if (e < cnt) {
          const uint32_t meta = __float_as_uint(s_b[e].w);
          const uint32_t lm = meta & 0xFFu;
          uint32_t lim = 0;
#pragma unroll
          for (int l = 0; l < MAXL; ++l) lim = lm == (uint32_t)l ? lw[l] : lim;
          keep = (meta & qbit) && __float_as_uint(s_c[e].w) < lim;
        }
        m = __ballot(keep);
      }
      while (m != 0) {
        const int bit = 63 - (int)__builtin_clzll(m);
        m &= ~(1ull << bit);
        const int j = (q << 6) + bit;
        const float4 cb = s_b[j];
        const float4 a = s_a[j];
        const float4 col = s_c[j];
        const uint32_t kk = __float_as_uint(col.w);
        const uint32_t lmin = __builtin_amdgcn_readfirstlane(__float_as_uint(cb.w)) & 0xFFu;
        // some lane of the wave may use the entry (the mask holds no other entries); lanes that
        // cannot compute the evaluation and discard it
        const AlphaEval ev = alpha_eval(fpx, fpy, a.x, a.y, cb.x, cb.y, cb.z, a.z);
        const bool hit = ev.ga >= d.alpha_min;
        const float al = __builtin_amdgcn_fmed3f(ev.ga, 0.f, d.alpha_max);  // min(alpha_max, ga), ga >= 0
        const float oma = 1.f - al;
        const float ioma = __builtin_amdgcn_rcpf(oma);
        float gr = 0.f, gg = 0.f, gb = 0.f, dal = 0.f;
        // cand: the pixel lies before the last contributor of some layer the entry belongs to; the
        // per-layer comparisons serve both the count and the layer updates (bitwise, no branches)
        bool cand = false;
        // the entry's layers are lmin and above: walked from the top down to a uniform exit, so
        // that the layers below lmin cost nothing (a uniform test per layer is turned into lane
        // masking, a compare and a handful of scalar operations per skipped layer)
#pragma unroll
        for (int l = MAXL - 1; l >= 0; --l) {
          if ((uint32_t)l < lmin) break;
          const bool before = kk < last[l];
          if (COUNT) cand |= before;
          if (!(hit & before)) continue;
          const float Tb = Tr[l] * ioma;  // transmittance in front of this Gaussian
          const float wT = al * Tb;
          gr = fmaf(wr[l], wT, gr);
          gg = fmaf(wg[l], wT, gg);
          gb = fmaf(wb[l], wT, gb);
          const float wc = fmaf(wr[l], col.x, fmaf(wg[l], col.y, wb[l] * col.z));
          dal = fmaf(Tb, wc, fmaf(-Q[l], ioma, dal));
          Q[l] = fmaf(wT, wc, Q[l]);
          Tr[l] = Tb;
          if (COUNT) ++n_contrib;
        }
        if (COUNT) n_eval += cand ? 1u : 0u;
        // the reduction runs for every walked entry: one with no contributing lane is rare, and
        // testing for it cost more than it saved
        {
          // the clamp at alpha_max has zero derivative; dal is zero without a contribution
          const float dl = ev.ga <= d.alpha_max ? dal : 0.f;
          const float dp = dl * ev.ga;
          // the moments of dp and the colour gradients (kGradScale)
          const float pdx = dp * ev.dx, pdy = dp * ev.dy;
          float g[9] = {pdx, pdy, pdx * ev.dx, pdx * ev.dy, pdy * ev.dy, dp, gr, gg, gb};
          reduce_scatter9(g, lane);
          if (DET) {
            // value 8 summed over the eight groups too (every lane of a group holds the same value)
            float v8 = g[8];
            {
              const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v8), __float_as_uint(v8), false, false);
              v8 = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            }
            {
              const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v8), __float_as_uint(v8), false, false);
              v8 = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            }
            v8 += dpp<kDppMirror>(v8);
            // this wave's sums of the entry, scaled as in the flush below, into the fixed-point sums
            const int v = (lane & 7) == 0 ? vid : 8;
            const float x = (lane & 7) == 0 ? g[0] : v8;
            if ((lane & 7) == 0 || lane == 1) {
              const float sc = v == 5 ? __builtin_amdgcn_rcpf(a.z) : kGradScale[v];
              if (x != 0.f) fx_add(g2d_fx + (((recbase + __float_as_uint(a.w)) * 9 + v) << 1), x * sc);
            }
          } else {
            const float x = (lane & 7) == 0 ? g[0] : g[8];
            if (adder && x != 0.f)
              __hip_atomic_fetch_add(g_slot + j * kGradLds, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
    __syncthreads();
    if (!DET && t < cnt) {
      const uint32_t g_i = __float_as_uint(s_a[t].w);
      float* dst = g2d + (recbase + g_i) * kGradStride;
      const float inv_o = __builtin_amdgcn_rcpf(s_a[t].z);
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        const float x = s_g[t][v];
        if (x != 0.f) {
          unsafeAtomicAdd(dst + v, x * (v == 5 ? inv_o : kGradScale[v]));
          s_g[t][v] = 0.f;
        }
      }
    }
  }
  if (COUNT) flush_counters(n_eval, n_contrib, &st->bwd_evals, &st->bwd_contribs);
}

// Block-wide stable compaction for a block of NW waves (see compact_slot).
template <int NW>
__device__ __forceinline__ int compact_slot_w(bool keep, uint32_t* s_wcnt, int* total) {
  const int t = threadIdx.x, w = t >> 6;
  const unsigned long long m = __ballot(keep);
  if ((t & 63) == 0) s_wcnt[w] = (uint32_t)__popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int c = (int)s_wcnt[q];
    off += q < w ? c : 0;
    tot += c;
  }
  *total = tot;
  return off + (int)popc_below(m);
}

// The backward with two pixels per lane: a block of 128 threads (two waves) per 16x16 tile, wave w
// holding rows 8w..8w+7 (the quadrants 2w and 2w + 1), lane l the pixels (l & 15, 8w + (l >> 4))
// and (l & 15, 8w + 4 + (l >> 4)). Per walked entry the LDS reads, the per-entry bookkeeping and
// the nine-value wave reduction are shared by the lane's two pixels, whose gradient terms are
// added in the lane first. Per pixel the arithmetic is that of k_raster_bwd, so the gradients
// agree up to the order of the float additions.
constexpr int kBwd2Threads = 128;

template <int MAXL, bool COUNT>
__global__ __launch_bounds__(kBwd2Threads) void k_raster_bwd2(RenderDims d, Status* __restrict__ st,
                                                              const uint2* __restrict__ ranges,
                                                              const uint32_t* __restrict__ lists,
                                                              const float4* __restrict__ rec,
                                                              const float* __restrict__ t_final,
                                                              const uint32_t* __restrict__ n_last,
                                                              const float* __restrict__ image,
                                                              const float* __restrict__ d_image,
                                                              const float* __restrict__ target,
                                                              float* __restrict__ g2d, float* __restrict__ loss_out) {
  if (st->overflow) return;
  const int per = (d.B * d.T + 7) / 8;
  const int wid = xcd_item(blockIdx.x, per);
  if (wid >= d.B * d.T) return;
  const int bv = wid / d.T, tile = wid - bv * d.T;
  const int tx = tile % d.TX, ty = tile / d.TX;
  const int ox = tx * kTile, oy = ty * kTile;
  const uint2 range = ranges[(size_t)bv * d.T + tile];
  __shared__ float4 s_a[kTilePix];  // mx, my, o, index bits
  __shared__ float4 s_b[kTilePix];  // scaled conic a2, b2, c2, (first layer | quadrant mask << 8) bits
  __shared__ float4 s_c[kTilePix];  // r, g, b, list position bits
  __shared__ float s_g[kTilePix][kGradLds];  // per-entry gradient sums of the two waves
  __shared__ uint32_t s_wcnt[kBwd2Threads / 64];
  __shared__ uint32_t s_lmax[kMaxLevels];
  __shared__ float s_loss;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const uint32_t qbits = 3u << (8 + 2 * wv);
  if (t < kMaxLevels) s_lmax[t] = 0;
  if (t == 0) s_loss = 0.f;
  for (int e = t; e < kTilePix; e += kBwd2Threads)
    for (int v = 0; v < kGradLds; ++v) s_g[e][v] = 0.f;
  __syncthreads();
  const int px = ox + (lane & 15);
  const int py0 = oy + 8 * wv + (lane >> 4);
  const float fpx = (float)px + 0.5f;
  const float fpy[2] = {(float)py0 + 0.5f, (float)(py0 + 4) + 0.5f};
  const size_t HW = (size_t)d.W * d.H;
  // per pixel p of the lane, as in k_raster_bwd
  float Tr[2][MAXL], wr[2][MAXL], wg[2][MAXL], wb[2][MAXL], Q[2][MAXL];
  uint32_t last[2][MAXL];
  float loss = 0.f;
  const float inv3hw = 1.0f / (3.0f * (float)HW);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int py = py0 + 4 * p;
    const bool inside = px < d.W && py < d.H;
    const size_t pix = (size_t)py * d.W + px;
#pragma unroll
    for (int l = 0; l < MAXL; ++l) {
      Tr[p][l] = 0.f; wr[p][l] = wg[p][l] = wb[p][l] = 0.f; last[p][l] = 0;
      if (inside && l < d.L) {
        const size_t o = (size_t)bv * d.L + l;
        Tr[p][l] = t_final[o * HW + pix];
        last[p][l] = n_last[o * HW + pix];
        float w3[3];
        for (int ch = 0; ch < 3; ++ch) {
          if (d_image) {
            w3[ch] = d_image[(o * 3 + ch) * HW + pix];
          } else {
            const float diff = image[(o * 3 + ch) * HW + pix] - target[((size_t)bv * 3 + ch) * HW + pix];
            const float sgn = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
            w3[ch] = d.lw[l] * sgn * inv3hw;
            loss += d.lw[l] * fabsf(diff) * inv3hw;
          }
        }
        wr[p][l] = w3[0]; wg[p][l] = w3[1]; wb[p][l] = w3[2];
        if (last[p][l]) atomicMax(&s_lmax[l], last[p][l]);
      }
      Q[p][l] = Tr[p][l] * (wr[p][l] * d.bg[0] + wg[p][l] * d.bg[1] + wb[p][l] * d.bg[2]);
    }
  }
  if (loss_out) {
    loss = wave_sum(loss);
    if (lane == 0) atomicAdd(&s_loss, loss);
  }
  __syncthreads();
  if (loss_out && t == 0) unsafeAtomicAdd(loss_out, s_loss);
  uint32_t lmax[MAXL];
  uint32_t ktop = 0;
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    lmax[l] = l < d.L ? s_lmax[l] : 0u;
    ktop = max(ktop, lmax[l]);
  }
  uint32_t lw[MAXL];
  {
    uint32_t run = 0;
#pragma unroll
    for (int l = MAXL - 1; l >= 0; --l) {
      run = max(run, wave_max_u(l < d.L ? max(last[0][l], last[1][l]) : 0u));
      lw[l] = run;
    }
  }
  const size_t recbase = (size_t)bv * d.n;
  uint32_t n_eval = 0, n_contrib = 0;
  int vid;
  {
    float pr[9] = {0.f, 1.f, 2.f, 3.f, 4.f, 5.f, 6.f, 7.f, 0.f};
    reduce_scatter9(pr, lane);
    vid = (int)(pr[0] * (1.f / 64.f) + 0.5f);
  }
  const bool adder = (lane & 7) < 2;
  lds_float* const g_slot = (lds_float*)&s_g[0][0] + ((lane & 7) == 0 ? vid : 8);
  const int nb = d.batch;
  for (int top = (int)ktop; top > 0; top -= nb) {
    const int lo = max(0, top - nb);
    __syncthreads();
    // stage the needed entries of [lo, top) in order, kBwd2Threads list positions per sub-round
    int cnt = 0;
    for (int sub = 0; sub * kBwd2Threads < nb; ++sub) {
      const int off = sub * kBwd2Threads + t;
      const uint32_t k = (uint32_t)(lo + off);
      uint32_t gi = 0xFFFFFFFFu;
      bool need = false;
      if (off < nb && (int)k < top) {
        gi = lists[range.x + k];
#pragma unroll
        for (int l = 0; l < MAXL; ++l) need = need || (k < lmax[l] && gi < (uint32_t)d.lv[l]);
      }
      int csub;
      const int slot = cnt + compact_slot_w<kBwd2Threads / 64>(need, s_wcnt, &csub);
      if (need) {
        const float4* r = rec + 3 * (recbase + gi);
        const float4 r0 = r[0], r1 = r[1], r2 = r[2];
        const uint32_t qm = quad_mask(d, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, ox, oy);
        s_a[slot] = make_float4(r0.x, r0.y, r1.y, __uint_as_float(gi));
        s_b[slot] = make_float4(-0.5f * kLog2e * r0.z, -kLog2e * r0.w, -0.5f * kLog2e * r1.x,
                                __uint_as_float(first_layer(d, gi) | (qm << 8)));
        s_c[slot] = make_float4(r1.z, r1.w, r2.x, __uint_as_float(k));
      }
      cnt += csub;
      __syncthreads();
    }
    for (int q = (cnt - 1) >> 6; q >= 0; --q) {
      uint64_t m;
      {
        const int e = q * 64 + lane;
        bool keep = false;
        if (e < cnt) {
          const uint32_t meta = __float_as_uint(s_b[e].w);
          const uint32_t lm = meta & 0xFFu;
          uint32_t lim = 0;
#pragma unroll
          for (int l = 0; l < MAXL; ++l) lim = lm == (uint32_t)l ? lw[l] : lim;
          keep = (meta & qbits) && __float_as_uint(s_c[e].w) < lim;
        }
        m = __ballot(keep);
      }
      while (m != 0) {
        const int bit = 63 - (int)__builtin_clzll(m);
        m &= ~(1ull << bit);
        const int j = (q << 6) + bit;
        const float4 cb = s_b[j];
        const float4 a = s_a[j];
        const float4 col = s_c[j];
        const uint32_t kk = __float_as_uint(col.w);
        const uint32_t lmin = __builtin_amdgcn_readfirstlane(__float_as_uint(cb.w)) & 0xFFu;
        float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const AlphaEval ev = alpha_eval(fpx, fpy[p], a.x, a.y, cb.x, cb.y, cb.z, a.z);
          const bool hit = ev.ga >= d.alpha_min;
          const float al = __builtin_amdgcn_fmed3f(ev.ga, 0.f, d.alpha_max);  // min(alpha_max, ga), ga >= 0
          const float oma = 1.f - al;
          const float ioma = __builtin_amdgcn_rcpf(oma);
          float gr = 0.f, gg = 0.f, gb = 0.f, dal = 0.f;
          bool cand = false;
          // the entry's layers, lmin and above, from the top down to a uniform exit (as in
          // k_raster_bwd)
#pragma unroll
          for (int l = MAXL - 1; l >= 0; --l) {
            if ((uint32_t)l < lmin) break;
            const bool before = kk < last[p][l];
            if (COUNT) cand |= before;
            if (!(hit & before)) continue;
            const float Tb = Tr[p][l] * ioma;  // transmittance in front of this Gaussian
            const float wT = al * Tb;
            gr = fmaf(wr[p][l], wT, gr);
            gg = fmaf(wg[p][l], wT, gg);
            gb = fmaf(wb[p][l], wT, gb);
            const float wc = fmaf(wr[p][l], col.x, fmaf(wg[p][l], col.y, wb[p][l] * col.z));
            dal = fmaf(Tb, wc, fmaf(-Q[p][l], ioma, dal));
            Q[p][l] = fmaf(wT, wc, Q[p][l]);
            Tr[p][l] = Tb;
            if (COUNT) ++n_contrib;
          }
          if (COUNT) n_eval += cand ? 1u : 0u;
          // the clamp at alpha_max has zero derivative; dal is zero without a contribution
          const float dl = ev.ga <= d.alpha_max ? dal : 0.f;
          const float dp = dl * ev.ga;
          const float pdx = dp * ev.dx, pdy = dp * ev.dy;
          g[0] += pdx;
          g[1] += pdy;
          g[2] += pdx * ev.dx;
          g[3] += pdx * ev.dy;
          g[4] += pdy * ev.dy;
          g[5] += dp;
          g[6] += gr;
          g[7] += gg;
          g[8] += gb;
        }
        reduce_scatter9(g, lane);
        const float x = (lane & 7) == 0 ? g[0] : g[8];
        if (adder && x != 0.f)
            __hip_atomic_fetch_add(g_slot + j * kGradLds, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    __syncthreads();
    for (int e = t; e < cnt; e += kBwd2Threads) {
      const uint32_t g_i = __float_as_uint(s_a[e].w);
      float* dst = g2d + (recbase + g_i) * kGradStride;
      const float inv_o = __builtin_amdgcn_rcpf(s_a[e].z);
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        const float x = s_g[e][v];
        if (x != 0.f) {
          unsafeAtomicAdd(dst + v, x * (v == 5 ? inv_o : kGradScale[v]));
          s_g[e][v] = 0.f;
        }
      }
    }
  }
  if (COUNT) flush_counters(n_eval, n_contrib, &st->bwd_evals, &st->bwd_contribs);
}

// Order-sensitive checksum: sum over i of word_i * (2 i + 1) (mod 2^64).
__global__ __launch_bounds__(256) void k_checksum(const uint32_t* __restrict__ p, size_t n,
                                                  unsigned long long* __restrict__ out) {
  unsigned long long acc = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    acc += (unsigned long long)p[i] * (2ull * i + 1ull);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

__global__ void k_zero(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = i; j < n; j += stride) p[j] = 0u;
}

}  // namespace

// ============================================================ launchers
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  {
    ProfScope ps_(K_ZERO, st);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, n);
  }
  return hipGetLastError();
}

hipError_t launch_checksum(const uint32_t* p, size_t n, unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (uint32_t*)out, (size_t)2);
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  if (blocks > 0) hipLaunchKernelGGL(k_checksum, dim3(blocks), dim3(256), 0, st, p, n, out);
  return hipGetLastError();
}

hipError_t launch_compose_fwd(const RenderDims& d, const float* params, const float* res, float* composed,
                              hipStream_t st) {
  {
    ProfScope ps_(K_COMPOSE_FWD, st);
    hipLaunchKernelGGL(k_compose_fwd, dim3((d.n + 255) / 256), dim3(256), 0, st, d, params, res, composed);
  }
  return hipGetLastError();
}

hipError_t launch_compose_bwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const float* d_composed, float* d_params, float* d_res, hipStream_t st) {
  {
    ProfScope ps_(K_COMPOSE_BWD, st);
    hipLaunchKernelGGL(k_compose_bwd, dim3((d.n + 255) / 256), dim3(256), 0, st, d, params, res, composed, d_composed,
                     d_params, d_res);
  }
  return hipGetLastError();
}

hipError_t launch_project_fwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const gs_camera* cams, char* ws, const Layout& lo, hipStream_t st) {
  dim3 grid((d.n + 255) / 256), block(256);
  float4* rec = (float4*)(ws + lo.records);
  uint2* rects = (uint2*)(ws + lo.rects);
  uint32_t* keys = (uint32_t*)(ws + lo.keys0);
  uint32_t* vals = (uint32_t*)(ws + lo.vals0);
  ProfScope ps_(K_PROJECT_FWD, st);
  switch (d.deg) {
    case 0: hipLaunchKernelGGL(k_project_fwd<0>, grid, block, 0, st, d, params, res, composed, cams, rec, rects, keys, vals); break;
    case 1: hipLaunchKernelGGL(k_project_fwd<1>, grid, block, 0, st, d, params, res, composed, cams, rec, rects, keys, vals); break;
    case 2: hipLaunchKernelGGL(k_project_fwd<2>, grid, block, 0, st, d, params, res, composed, cams, rec, rects, keys, vals); break;
    default: hipLaunchKernelGGL(k_project_fwd<3>, grid, block, 0, st, d, params, res, composed, cams, rec, rects, keys, vals); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_bwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const gs_camera* cams, char* ws, const Layout& lo, float* d_params, hipStream_t st) {
  dim3 grid((d.n + 255) / 256), block(256);
  const float* g2d = (const float*)(ws + lo.grad2d);
  float* dcomp = (float*)(ws + lo.d_composed);
  ProfScope ps_(K_PROJECT_BWD, st);
  switch (d.deg) {
    case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, block, 0, st, d, params, res, composed, cams, g2d, d_params, dcomp); break;
    case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, block, 0, st, d, params, res, composed, cams, g2d, d_params, dcomp); break;
    case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, block, 0, st, d, params, res, composed, cams, g2d, d_params, dcomp); break;
    default: hipLaunchKernelGGL(k_project_bwd<3>, grid, block, 0, st, d, params, res, composed, cams, g2d, d_params, dcomp); break;
  }
  return hipGetLastError();
}

// Stable LSD radix sort (four 8-bit passes) of B segments of n (key, value) pairs, ping-ponging
// between k[0]/v[0] (the input) and k[1]/v[1]; returns the buffers that hold the result.
static hipError_t radix_passes(const RenderDims& d, uint32_t* k[2], uint32_t* v[2], uint32_t* hist, uint32_t** keys_out,
                               uint32_t** vals_out, hipStream_t st) {
  dim3 grid(d.n_sort_chunks, d.B);
  int cur = 0;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    {
      ProfScope ps_(K_RADIX_HIST, st);
      hipLaunchKernelGGL(k_radix_hist, grid, dim3(kSortThreads), 0, st, d, k[cur], hist, shift);
    }
    {
      ProfScope ps_(K_RADIX_SCAN, st);
      hipLaunchKernelGGL(k_radix_scan, dim3(d.B), dim3(1024), 0, st, d, hist);
    }
    {
      ProfScope ps_(K_RADIX_SCATTER, st);
      hipLaunchKernelGGL(k_radix_scatter, grid, dim3(kSortThreads), 0, st, d, k[cur], v[cur], k[cur ^ 1], v[cur ^ 1],
                         hist, shift);
    }
    cur ^= 1;
  }
  *keys_out = k[cur];
  *vals_out = v[cur];
  return hipGetLastError();
}

hipError_t launch_sort(const RenderDims& d, char* ws, const Layout& lo, uint32_t** keys_out, uint32_t** vals_out,
                       hipStream_t st) {
  uint32_t* k[2] = {(uint32_t*)(ws + lo.keys0), (uint32_t*)(ws + lo.keys1)};
  uint32_t* v[2] = {(uint32_t*)(ws + lo.vals0), (uint32_t*)(ws + lo.vals1)};
  return radix_passes(d, k, v, (uint32_t*)(ws + lo.sort_hist), keys_out, vals_out, st);
}

size_t radix_hist_words(int n) { return (size_t)256 * ((n + kSortChunk - 1) / kSortChunk); }

hipError_t launch_radix_sort(int n, uint32_t* keys[2], uint32_t* vals[2], uint32_t* hist, uint32_t** keys_out,
                             uint32_t** vals_out, hipStream_t st) {
  RenderDims d{};
  d.n = n;
  d.B = 1;
  d.n_sort_chunks = (n + kSortChunk - 1) / kSortChunk;
  return radix_passes(d, keys, vals, hist, keys_out, vals_out, st);
}

hipError_t launch_bin(const RenderDims& d, const uint32_t* skeys, const uint32_t* svals, char* ws, const Layout& lo,
                      hipStream_t st) {
  const float4* rec = (const float4*)(ws + lo.records);
  float4* brec = (float4*)(ws + lo.bin_rec);
  uint32_t* rhist = (uint32_t*)(ws + lo.bin_hist);
  uint32_t* rtot = (uint32_t*)(ws + lo.row_tot);
  uint2* rranges = (uint2*)(ws + lo.row_ranges);
  uint2* rlists = (uint2*)(ws + lo.row_lists);
  uint32_t* thist = (uint32_t*)(ws + lo.tile_hist);
  uint2* ranges = (uint2*)(ws + lo.ranges);
  uint32_t* lists = (uint32_t*)(ws + lo.lists);
  uint32_t* tot = (uint32_t*)(ws + lo.tile_tot);
  Status* status = (Status*)(ws + lo.status);
  dim3 grid1(d.n_bin_chunks, d.B);
  const size_t lds1 = (size_t)(d.TY + 1) * sizeof(uint32_t);
  dim3 grid2(d.n_row_segs, d.TY, d.B);
  if (d.n_bin_chunks > 0) {
    {
      ProfScope ps_(K_BIN_GATHER, st);
      hipLaunchKernelGGL(k_bin_gather, dim3((d.n + 255) / 256, d.B), dim3(256), 0, st, d, skeys, svals, rec,
                         brec);
    }
    ProfScope ps_(K_ROW_COUNT, st);
    hipLaunchKernelGGL(k_row_bin<false>, grid1, dim3(64), lds1, st, d, skeys, svals, brec, rhist, rranges, rlists);
  }
  {
    ProfScope ps_(K_BIN_CHUNK_SCAN, st);
    hipLaunchKernelGGL(k_chunk_scan, dim3(d.B * d.TY), dim3(64), 0, st, d.B * d.TY, d.TY,
                       d.n_bin_chunks, rhist, rtot);
    hipLaunchKernelGGL(k_scan_ranges, dim3(1), dim3(1024), 0, st, d.B * d.TY, 0, d.row_capacity, rtot, rranges,
                       status);
  }
  if (d.n_bin_chunks > 0) {
    ProfScope ps_(K_ROW_EMIT, st);
    hipLaunchKernelGGL(k_row_bin<true>, grid1, dim3(64), lds1, st, d, skeys, svals, brec, rhist, rranges, rlists);
  }
  if (d.n_row_segs > 0) {
    ProfScope ps_(K_BIN_COUNT, st);
    hipLaunchKernelGGL(k_tile_count, grid2, dim3(64), 0, st, d, status, rranges, rlists, thist);
  }
  {
    ProfScope ps_(K_TILE_RANGES, st);
    hipLaunchKernelGGL(k_seg_scan, dim3((d.B * d.T + 255) / 256), dim3(256), 0, st, d, status, rranges, thist, tot);
    hipLaunchKernelGGL(k_scan_ranges, dim3(1), dim3(1024), 0, st, d.B * d.T, 1, d.capacity, tot, ranges, status);
  }
  if (d.n_row_segs > 0) {
    ProfScope ps_(K_BIN_EMIT, st);
    if (d.TX > 63)  // one column per lane needs column counts below 64
      hipLaunchKernelGGL((k_tile_bin<true>), grid2, dim3(64), 0, st, d, status, rranges, rlists, thist, ranges,
                         lists);
    else
      hipLaunchKernelGGL((k_tile_bin<false>), grid2, dim3(64), 0, st, d, status, rranges, rlists, thist, ranges,
                         lists);
  }
  return hipGetLastError();
}

hipError_t launch_raster_fwd(const RenderDims& d, char* ws, const Layout& lo, float* image, hipStream_t st) {
  Status* status = (Status*)(ws + lo.status);
  const uint2* ranges = (const uint2*)(ws + lo.ranges);
  const uint32_t* lists = (const uint32_t*)(ws + lo.lists);
  const float4* rec = (const float4*)(ws + lo.records);
  float* tf = (float*)(ws + lo.t_final);
  uint32_t* nl = (uint32_t*)(ws + lo.n_last);
  const int per = (d.B * d.T + 7) / 8;
  dim3 grid(per * 8), block(kTilePix);
  ProfScope ps_(K_RASTER_FWD, st);
  const bool cnt = work_counting();
#define GS_FWD(L_)                                                                                             \
  do {                                                                                                         \
    if (cnt)                                                                                                   \
      hipLaunchKernelGGL((k_raster_fwd<L_, true>), grid, block, 0, st, d, status, ranges, lists, rec, image, tf, nl);  \
    else                                                                                                       \
      hipLaunchKernelGGL((k_raster_fwd<L_, false>), grid, block, 0, st, d, status, ranges, lists, rec, image, tf, nl); \
  } while (0)
  if (d.L == 1)
    GS_FWD(1);
  else if (d.L == 2)
    GS_FWD(2);
  else if (d.L <= 4)
    GS_FWD(4);
  else if (d.L <= 6)
    GS_FWD(6);
  else
    GS_FWD(8);
#undef GS_FWD
  return hipGetLastError();
}

hipError_t launch_raster_bwd(const RenderDims& d, char* ws, const Layout& lo, const float* image,
                             const float* d_image, const float* target, float* loss_out, hipStream_t st) {
  Status* status = (Status*)(ws + lo.status);
  const uint2* ranges = (const uint2*)(ws + lo.ranges);
  const uint32_t* lists = (const uint32_t*)(ws + lo.lists);
  const float4* rec = (const float4*)(ws + lo.records);
  const float* tf = (const float*)(ws + lo.t_final);
  const uint32_t* nl = (const uint32_t*)(ws + lo.n_last);
  float* g2d = (float*)(ws + lo.grad2d);
  const int per = (d.B * d.T + 7) / 8;
  dim3 grid(per * 8), block(kTilePix), block2(kBwd2Threads);
  // the deterministic variant: one pixel per lane, no counting, fixed-point sums (launch_fx_finish)
  const bool det = d.det != 0;
  const bool cnt = work_counting() && !det;
  const bool two = d.bwd_pixels == 2 && !det;
  unsigned long long* gfx = det ? (unsigned long long*)(ws + lo.grad2d_fx) : nullptr;
  unsigned long long* lfx = det ? (unsigned long long*)(ws + lo.loss_fx) : nullptr;
#define GS_BWD(L_)                                                                                          \
  do {                                                                                                      \
    if (two && cnt)                                                                                         \
      hipLaunchKernelGGL((k_raster_bwd2<L_, true>), grid, block2, 0, st, d, status, ranges, lists, rec, tf, nl, \
                         image, d_image, target, g2d, loss_out);                                            \
    else if (two)                                                                                           \
      hipLaunchKernelGGL((k_raster_bwd2<L_, false>), grid, block2, 0, st, d, status, ranges, lists, rec, tf,  \
                         nl, image, d_image, target, g2d, loss_out);                                        \
    else if (det)                                                                                           \
      hipLaunchKernelGGL((k_raster_bwd<L_, false, true>), grid, block, 0, st, d, status, ranges, lists, rec, tf, \
                         nl, image, d_image, target, g2d, loss_out, gfx, lfx);                              \
    else if (cnt)                                                                                           \
      hipLaunchKernelGGL((k_raster_bwd<L_, true, false>), grid, block, 0, st, d, status, ranges, lists, rec, tf, \
                         nl, image, d_image, target, g2d, loss_out, gfx, lfx);                              \
    else                                                                                                    \
      hipLaunchKernelGGL((k_raster_bwd<L_, false, false>), grid, block, 0, st, d, status, ranges, lists, rec, \
                         tf, nl, image, d_image, target, g2d, loss_out, gfx, lfx);                          \
  } while (0)
  ProfScope ps_(K_RASTER_BWD, st);
  if (d.L == 1) GS_BWD(1);
  else if (d.L == 2) GS_BWD(2);
  else if (d.L <= 4) GS_BWD(4);
  else if (d.L <= 6) GS_BWD(6);
  else GS_BWD(8);
#undef GS_BWD
  return hipGetLastError();
}

// The deterministic backward's fixed-point sums into the gradient records (and the loss).
__global__ __launch_bounds__(256) void k_fx_finish(size_t count, const unsigned long long* __restrict__ g2d_fx,
                                                   float* __restrict__ g2d, const unsigned long long* __restrict__ loss_fx,
                                                   float* __restrict__ loss_out) {
  const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;  // (view, Gaussian) * 9 + value
  if (k < count) g2d[(k / 9) * kGradStride + k % 9] = fx_value(g2d_fx + 2 * k);
  if (k == 0 && loss_out) loss_out[0] += fx_value(loss_fx);
}

hipError_t launch_fx_finish(const RenderDims& d, char* ws, const Layout& lo, float* loss_out, hipStream_t st) {
  const size_t count = (size_t)d.B * d.n * 9;
  hipLaunchKernelGGL(k_fx_finish, dim3((unsigned)((count + 255) / 256 > 0 ? (count + 255) / 256 : 1)), dim3(256), 0,
                     st, count, (const unsigned long long*)(ws + lo.grad2d_fx), (float*)(ws + lo.grad2d),
                     (const unsigned long long*)(ws + lo.loss_fx), loss_out);
  return hipGetLastError();
}

}  // namespace gs
