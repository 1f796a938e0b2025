// Colour loss of the rendered layers with its D-SSIM term (Sec. 3.3: L_color of every layer,
// weighted by lambda^l as in App. A) and its gradient with respect to the rendered colours.
//
// SSIM is taken per colour channel with an 11 x 11 Gaussian window (sigma 1.5) that sees zeros
// outside the image; the window is separable, so every windowed mean is one 11-tap pass along the
// rows and one along the columns. With mu_x = G*x, E_xx = G*(x x), E_xy = G*(x y):
//   S = (2 mu_x mu_y + C1)(2 (E_xy - mu_x mu_y) + C2) / ((mu_x^2 + mu_y^2 + C1)(E_xx - mu_x^2 + E_yy - mu_y^2 + C2))
// and the gradient of sum_p w S(p) with respect to x(q) is
//   (G*a)(q) + 2 x(q) (G*b)(q) + y(q) (G*c)(q),  a = w dS/dmu_x, b = w dS/dE_xx, c = w dS/dE_xy
// (the window is symmetric, so the zero-padded G* is its own adjoint).
//
// Two kernels, both bound by their VALU work:
//  ssim_fwd  one block per (view, channel, 64 x 24 tile), looping over the layers: the target's
//            windowed moments are made once per tile, each layer stages its tile (with a 5-pixel
//            halo) in LDS, runs the row pass of x, x^2, x y and the column pass, and writes the
//            three gradient maps a, b, c (already scaled by the loss weight) and adds its loss.
//  ssim_bwd  one block per (view, layer, channel, 64 x 32 tile): the row and column passes of a,
//            b and c, combined with the L1 term into dL/dC.
// Both fetch the next region (layer or map) into registers while the current one is processed.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kWinR = 5;                    // window radius: 11 taps
constexpr int kWinN = 2 * kWinR + 1;
constexpr int kLossTW = 64;                 // tile columns: one per lane
constexpr int kRegW = kLossTW + 2 * kWinR;  // staged columns (74)
constexpr int kRegStride = 76;              // LDS row stride in floats: 16-byte aligned rows
// tile rows of the two kernels; each of the four waves of a block owns a quarter of them
constexpr int kFwdTH = 24;
constexpr int kBwdTH = 32;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct LossArgs {
  const float* image;   // [B][L][3][H][W]
  const float* target;  // [B][3][H][W]
  float* maps;          // [3][B][L][3][H][W] gradient maps a, b, c, or NULL (loss only)
  float* d_image;       // [B][L][3][H][W]
  float* loss_out;      // one float (+=), or NULL
  size_t map_stride;    // floats per gradient map (B L 3 H W)
  int W, H, B, L, tiles_x, tiles, per_xcd;  // tiles (per image plane) and per_xcd: set per launch
  float lambda_ssim, inv_n;  // inv_n = 1 / (3 H W): the means run over pixels and channels
  float lw[kMaxLevels];
  float g[kWinN];
};

// Consecutive blocks land on the same XCD, so tiles that share halo rows share that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int per_xcd) { return (bid & 7) * per_xcd + (bid >> 3); }

// The (TH + 10) x 74 region around a tile is fetched into registers (kRegion<TH> values per
// thread) and stored to LDS later, so that the loads of the next region are in flight while the
// current one is processed. Where each value comes from and goes to depends only on the thread
// and the tile, so it is worked out once per block: the offset in the image plane (-1 outside
// the image, which reads as zero) and the LDS offset.
template <int TH>
constexpr int kRegion = ((TH + 2 * kWinR) * kRegW + 255) / 256;

template <int TH>
struct RegionMap {
  int src[kRegion<TH>];
  int lds[kRegion<TH>];  // -1: no value for this thread
};

template <int TH>
__device__ __forceinline__ void region_map(RegionMap<TH>& m, int x0, int y0, int W, int H) {
  constexpr int N = (TH + 2 * kWinR) * kRegW;
#pragma unroll
  for (int k = 0; k < kRegion<TH>; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int r = idx / kRegW, c = idx - r * kRegW;
    const int gy = y0 - kWinR + r, gx = x0 - kWinR + c;
    const bool in = idx < N && gy >= 0 && gy < H && gx >= 0 && gx < W;
    m.src[k] = in ? gy * W + gx : -1;
    m.lds[k] = idx < N ? r * kRegStride + c : -1;
  }
}

template <int TH>
__device__ __forceinline__ void fetch_region(float (&v)[kRegion<TH>], const RegionMap<TH>& m,
                                             const float* __restrict__ src) {
#pragma unroll
  for (int k = 0; k < kRegion<TH>; ++k) v[k] = m.src[k] >= 0 ? src[m.src[k]] : 0.f;
}

template <int TH>
__device__ __forceinline__ void store_region(float* __restrict__ s, const float (&v)[kRegion<TH>],
                                             const RegionMap<TH>& m) {
#pragma unroll
  for (int k = 0; k < kRegion<TH>; ++k)
    if (m.lds[k] >= 0) s[m.lds[k]] = v[k];
}

// The 14 staged values row r, columns 4j .. 4j + 13: the inputs of four row-pass outputs.
__device__ __forceinline__ void load_window(const float* __restrict__ s, int r, int j, float (&w)[14]) {
  const float* p = s + r * kRegStride + 4 * j;
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  const float4 c = *reinterpret_cast<const float4*>(p + 8);
  const float2 d = *reinterpret_cast<const float2*>(p + 12);
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
  w[8] = c.x; w[9] = c.y; w[10] = c.z; w[11] = c.w;
  w[12] = d.x; w[13] = d.y;
}

// Row pass: four consecutive outputs of the 11-tap window, stored as one float4.
__device__ __forceinline__ void row_pass(const float (&w)[14], const float (&g)[kWinN], float* __restrict__ out) {
  float o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kWinN; ++k) acc = fmaf(g[k], w[i + k], acc);
    o[i] = acc;
  }
  *reinterpret_cast<float4*>(out) = make_float4(o[0], o[1], o[2], o[3]);
}

// Column pass: the MR outputs of column c from rows r0 .. r0 + MR + 9 of a row-pass buffer.
template <int MR>
__device__ __forceinline__ void col_pass(const float* __restrict__ h, int c, int r0, const float (&g)[kWinN],
                                         float (&o)[MR]) {
  float w[MR + 2 * kWinR];
#pragma unroll
  for (int k = 0; k < MR + 2 * kWinR; ++k) w[k] = h[(r0 + k) * kLossTW + c];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kWinN; ++k) acc = fmaf(g[k], w[i + k], acc);
    o[i] = acc;
  }
}

template <int TH>
__global__ __launch_bounds__(256) void k_ssim_fwd(const LossArgs a) {
  constexpr int RH = TH + 2 * kWinR;
  constexpr int MR = TH / 4;
  __shared__ __align__(16) float s_y[RH * kRegStride];
  __shared__ __align__(16) float s_x[RH * kRegStride];
  __shared__ __align__(16) float s_h[3][RH * kLossTW];
  __shared__ float s_red[4];
  const int wid = xcd_block(blockIdx.x, a.per_xcd);
  if (wid >= a.B * 3 * a.tiles) return;
  const int bc = wid / a.tiles, tile = wid - bc * a.tiles;  // bc = view * 3 + channel
  const int b = bc / 3, ch = bc - 3 * b;
  const int x0 = (tile % a.tiles_x) * kLossTW, y0 = (tile / a.tiles_x) * TH;
  const size_t HW = (size_t)a.W * a.H;
  const int t = threadIdx.x, c = t & 63, r0 = (t >> 6) * MR;
  float g[kWinN];
#pragma unroll
  for (int k = 0; k < kWinN; ++k) g[k] = a.g[k];

  // windowed moments of the target, shared by every layer
  RegionMap<TH> rm;
  region_map<TH>(rm, x0, y0, a.W, a.H);
  float pre[kRegion<TH>];
  fetch_region<TH>(pre, rm, a.target + (size_t)bc * HW);
  store_region<TH>(s_y, pre, rm);
  const size_t plane0 = (size_t)b * a.L * 3 + ch;  // plane of layer l: plane0 + 3 l
  fetch_region<TH>(pre, rm, a.image + plane0 * HW);
  __syncthreads();
  for (int it = t; it < RH * 16; it += 256) {
    const int r = it >> 4, j = it & 15;
    float w[14], w2[14];
    load_window(s_y, r, j, w);
#pragma unroll
    for (int k = 0; k < 14; ++k) w2[k] = w[k] * w[k];
    row_pass(w, g, &s_h[0][r * kLossTW + 4 * j]);
    row_pass(w2, g, &s_h[1][r * kLossTW + 4 * j]);
  }
  __syncthreads();
  float mu2[MR], eyy[MR], yv[MR];
  col_pass<MR>(s_h[0], c, r0, g, mu2);
  col_pass<MR>(s_h[1], c, r0, g, eyy);
#pragma unroll
  for (int i = 0; i < MR; ++i) yv[i] = s_y[(r0 + i + kWinR) * kRegStride + c + kWinR];
  const int px = x0 + c;
  const float lam = a.lambda_ssim;
  float loss = 0.f;

  for (int l = 0; l < a.L; ++l) {
    __syncthreads();  // the previous layer's row-pass buffers and staged tile are consumed
    const size_t plane = plane0 + 3 * (size_t)l;
    store_region<TH>(s_x, pre, rm);
    if (l + 1 < a.L) fetch_region<TH>(pre, rm, a.image + (plane + 3) * HW);
    __syncthreads();
    for (int it = t; it < RH * 16; it += 256) {
      const int r = it >> 4, j = it & 15;
      float wx[14], wy[14], wxx[14], wxy[14];
      load_window(s_x, r, j, wx);
      load_window(s_y, r, j, wy);
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        wxx[k] = wx[k] * wx[k];
        wxy[k] = wx[k] * wy[k];
      }
      row_pass(wx, g, &s_h[0][r * kLossTW + 4 * j]);
      row_pass(wxx, g, &s_h[1][r * kLossTW + 4 * j]);
      row_pass(wxy, g, &s_h[2][r * kLossTW + 4 * j]);
    }
    __syncthreads();
    float mu1[MR], exx[MR], exy[MR];
    col_pass<MR>(s_h[0], c, r0, g, mu1);
    col_pass<MR>(s_h[1], c, r0, g, exx);
    col_pass<MR>(s_h[2], c, r0, g, exy);
    const float wl = a.lw[l] * a.inv_n;
    const float coef = -wl * lam;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const int py = y0 + r0 + i;
      if (px >= a.W || py >= a.H) continue;
      const float xv = s_x[(r0 + i + kWinR) * kRegStride + c + kWinR];
      const float m1 = mu1[i], m2 = mu2[i];
      const float m11 = m1 * m1, m22 = m2 * m2, m12 = m1 * m2;
      const float A1 = 2.f * m12 + kC1;
      const float A2 = 2.f * (exy[i] - m12) + kC2;
      const float B1 = m11 + m22 + kC1;
      const float B2 = (exx[i] - m11) + (eyy[i] - m22) + kC2;
      const float rB1 = __builtin_amdgcn_rcpf(B1), rB2 = __builtin_amdgcn_rcpf(B2);  // 1 ulp
      const float S = A1 * A2 * rB1 * rB2;
      loss += wl * ((1.f - lam) * fabsf(xv - yv[i]) + lam * (1.f - S));
      if (a.maps) {
        const float d_mu = 2.f * m2 * (A2 - A1) * rB1 * rB2 - 2.f * m1 * S * (rB1 - rB2);
        const float d_exx = -S * rB2;
        const float d_exy = 2.f * A1 * rB1 * rB2;
        const size_t o = plane * HW + (size_t)py * a.W + px;
        a.maps[o] = coef * d_mu;
        a.maps[o + a.map_stride] = coef * d_exx;
        a.maps[o + 2 * a.map_stride] = coef * d_exy;
      }
    }
  }
  if (a.loss_out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
    if ((t & 63) == 0) s_red[t >> 6] = loss;
    __syncthreads();
    if (t == 0) unsafeAtomicAdd(a.loss_out, (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
  }
}

template <int TH>
__global__ __launch_bounds__(256) void k_ssim_bwd(const LossArgs a) {
  constexpr int RH = TH + 2 * kWinR;
  constexpr int MR = TH / 4;
  __shared__ __align__(16) float s_r[RH * kRegStride];
  __shared__ __align__(16) float s_h[RH * kLossTW];
  const int wid = xcd_block(blockIdx.x, a.per_xcd);
  if (wid >= a.B * a.L * 3 * a.tiles) return;
  const int plane = wid / a.tiles, tile = wid - plane * a.tiles;  // plane = (view * L + layer) * 3 + channel
  const int ch = plane % 3, bl = plane / 3;
  const int b = bl / a.L, l = bl - b * a.L;
  const int x0 = (tile % a.tiles_x) * kLossTW, y0 = (tile / a.tiles_x) * TH;
  const size_t HW = (size_t)a.W * a.H;
  const int t = threadIdx.x, c = t & 63, r0 = (t >> 6) * MR;
  const int px = x0 + c;
  float g[kWinN];
#pragma unroll
  for (int k = 0; k < kWinN; ++k) g[k] = a.g[k];
  const float* img = a.image + (size_t)plane * HW;
  const float* tgt = a.target + ((size_t)b * 3 + ch) * HW;
  float xv[MR], yv[MR], acc[MR];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int py = y0 + r0 + i;
    const bool in = px < a.W && py < a.H;
    xv[i] = in ? img[(size_t)py * a.W + px] : 0.f;
    yv[i] = in ? tgt[(size_t)py * a.W + px] : 0.f;
    acc[i] = 0.f;
  }
  auto rows = [&]() {
    for (int it = t; it < RH * 16; it += 256) {
      const int r = it >> 4, j = it & 15;
      float w[14];
      load_window(s_r, r, j, w);
      row_pass(w, g, &s_h[r * kLossTW + 4 * j]);
    }
  };
  const float* maps = a.maps + (size_t)plane * HW;
  RegionMap<TH> rm;
  region_map<TH>(rm, x0, y0, a.W, a.H);
  float pre[kRegion<TH>];
  fetch_region<TH>(pre, rm, maps);
  store_region<TH>(s_r, pre, rm);
  fetch_region<TH>(pre, rm, maps + a.map_stride);
  __syncthreads();
  rows();
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    // the staged map is consumed by the row pass: store the next one (fetched during the row
    // pass) and fetch the one after while the columns run
    if (q < 2) store_region<TH>(s_r, pre, rm);
    if (q < 1) fetch_region<TH>(pre, rm, maps + 2 * a.map_stride);
    float o[MR];
    col_pass<MR>(s_h, c, r0, g, o);
#pragma unroll
    for (int i = 0; i < MR; ++i) acc[i] = fmaf(q == 0 ? 1.f : (q == 1 ? 2.f * xv[i] : yv[i]), o[i], acc[i]);
    __syncthreads();
    if (q < 2) {
      rows();
      __syncthreads();
    }
  }
  const float w1 = a.lw[l] * a.inv_n * (1.f - a.lambda_ssim);
  float* out = a.d_image + (size_t)plane * HW;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int py = y0 + r0 + i;
    if (px >= a.W || py >= a.H) continue;
    const float d = xv[i] - yv[i];
    const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    out[(size_t)py * a.W + px] = fmaf(w1, sgn, acc[i]);
  }
}

int loss_dims(const gs_settings* s, int32_t F, int32_t V, LossArgs& a) {
  if (!s) return report_arg("settings is NULL");
  if (F < 1 || V < 1) return report_arg("n_frames and n_views must be >= 1");
  if (s->width < 1 || s->height < 1) return report_arg("width and height must be >= 1");
  if (s->n_levels < 1 || s->n_levels > kMaxLevels) return report_arg("n_levels must be in 1..8");
  if ((int64_t)s->width * s->height >= ((int64_t)1 << 31)) return report_arg("image plane of 2^31 pixels or more");
  a.W = s->width;
  a.H = s->height;
  a.B = F * V;
  a.L = s->n_levels;
  a.tiles_x = (a.W + kLossTW - 1) / kLossTW;
  const int min_th = kFwdTH < kBwdTH ? kFwdTH : kBwdTH;
  if ((int64_t)F * V * a.L * 3 * a.tiles_x * ((a.H + min_th - 1) / min_th) > (int64_t)0x7FFFFFF0)
    return report_arg("image batch too large");
  for (int l = 0; l < kMaxLevels; ++l) a.lw[l] = l < a.L ? s->level_weights[l] : 0.f;
  a.map_stride = (size_t)a.B * a.L * 3 * a.W * a.H;
  a.inv_n = (float)(1.0 / (3.0 * (double)a.W * (double)a.H));
  double gd[kWinN], sum = 0.0;
  for (int k = 0; k < kWinN; ++k) {
    const double x = k - kWinR;
    gd[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
    sum += gd[k];
  }
  for (int k = 0; k < kWinN; ++k) a.g[k] = (float)(gd[k] / sum);
  return GS_OK;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int gs_color_loss_workspace_size(const gs_settings* s, int32_t n_frames, int32_t n_views, size_t* bytes_out) {
  LossArgs a;
  int rc = loss_dims(s, n_frames, n_views, a);
  if (rc) return rc;
  if (!bytes_out) return report_arg("bytes_out is NULL");
  *bytes_out = 3 * a.map_stride * sizeof(float);
  return GS_OK;
}

int gs_color_loss(const gs_settings* s, int32_t n_frames, int32_t n_views, const float* image, const float* target,
                  float lambda_ssim, float* d_image, float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  LossArgs a;
  int rc = loss_dims(s, n_frames, n_views, a);
  if (rc) return rc;
  if (!image || !target) return report_arg("NULL image or target");
  if (!d_image && !loss_out) return report_arg("nothing to compute: d_image and loss_out are NULL");
  if (!(lambda_ssim >= 0.f && lambda_ssim <= 1.f)) return report_arg("lambda_ssim must be in [0, 1]");
  if (d_image) {
    if (!ws) return report_arg("the gradient needs a workspace");
    if (ws_bytes < 3 * a.map_stride * sizeof(float)) {
      report_arg("workspace too small");
      return GS_ERR_WORKSPACE;
    }
  }
  if ((rc = require_device())) return rc;
  a.image = image;
  a.target = target;
  a.maps = d_image ? (float*)ws : nullptr;
  a.d_image = d_image;
  a.loss_out = loss_out;
  a.lambda_ssim = lambda_ssim;
  hipStream_t st = (hipStream_t)stream;
  {
    ProfScope ps_(K_SSIM_FWD, st);
    a.tiles = a.tiles_x * ((a.H + kFwdTH - 1) / kFwdTH);
    const int n_blocks = a.B * 3 * a.tiles;
    a.per_xcd = (n_blocks + 7) / 8;
    hipLaunchKernelGGL(k_ssim_fwd<kFwdTH>, dim3(8 * a.per_xcd), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e, "ssim_fwd");
  }
  if (d_image) {
    ProfScope ps_(K_SSIM_BWD, st);
    a.tiles = a.tiles_x * ((a.H + kBwdTH - 1) / kBwdTH);
    const int n_blocks = a.B * a.L * 3 * a.tiles;
    a.per_xcd = (n_blocks + 7) / 8;
    hipLaunchKernelGGL(k_ssim_bwd<kBwdTH>, dim3(8 * a.per_xcd), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e, "ssim_bwd");
  }
  return GS_OK;
}

}  // extern "C"
