// Rigid-motion module of inter-frame training (Sec. 3.2, rigid transformation; Eq. 5-6): the
// previous frame's Gaussian positions are encoded by a multi-resolution hash grid and two small
// MLPs predict each Gaussian's translation and rotation, written as the frame's residual
// channels 0..6 (the translation, and the quaternion (1 + o0, o1, o2, o3) that multiplies the
// previous rotation).
//
// Encoding (the published multi-resolution hash encoding): 16 levels of 2 features, 2^15
// entries each, resolutions 16 .. 1024 geometric; trilinear interpolation of the 8 corners of the
// point's cell, corners indexed densely while the level's grid fits the table, else by the
// spatial hash (i * 1 ^ j * 2654435761 ^ k * 805459861) mod 2^15.
// MLPs: 32 -> 64 -> 64 -> 3 (translation) and 32 -> 64 -> 64 -> 4 (rotation), ReLU, FP32.
//
//  motion_fwd    one thread per Gaussian: the 16 x 8 corner gathers (the table stays in L2) and
//                both MLPs with their weights broadcast from LDS
//  motion_bwd    one thread per Gaussian: the forward again, the MLP backward, the feature
//                gradients scattered into the table with float atomics, and the per-Gaussian
//                activations and gradients staged for the weight gradients
//  motion_wgrad  the weight gradients, sums over Gaussians of outer products: a block takes one
//                weight matrix (with its bias as a column against a constant 1) and a range of
//                Gaussians, 64 at a time through LDS, and adds its sums with one atomic per entry
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kLevels = 16, kFeats = 2, kLog2T = 15, kT = 1 << kLog2T;
constexpr int kIn = kLevels * kFeats, kHid = 64;
// weights of one head: W1 [64][32], b1, W2 [64][64], b2, W3 [out][64], b3
constexpr int head_size(int out) { return kHid * kIn + kHid + kHid * kHid + kHid + out * kHid + out; }
constexpr int kWMu = 0, kWR = head_size(3), kNW = head_size(3) + head_size(4);
// staging fields per Gaussian: h, then per head a1, dz1, a2, dz2, dy
constexpr int kFH = 0;
constexpr int head_fields(int head) { return kIn + head * (4 * kHid + 3); }
constexpr int kNF = kIn + 2 * 4 * kHid + 3 + 4;

struct MotionDims {
  int n;
  double lo[3], inv_ext[3];
  int res[kLevels];
  int dense[kLevels];
  int row;  // row stride of the means, output and d_out arrays (floats)
};

__device__ __forceinline__ uint32_t corner_entry(const MotionDims& d, int l, uint32_t i, uint32_t j, uint32_t k) {
  const uint32_t N1 = (uint32_t)d.res[l] + 1u;
  if (d.dense[l]) return i + j * N1 + k * N1 * N1;
  return (i * 1u ^ j * 2654435761u ^ k * 805459861u) & (uint32_t)(kT - 1);
}

// Unit-cube position of a Gaussian and, per level, its cell corner and fractions. The position
// and the grid coordinate are FP64: at the finest level (1024 cells) an FP32 coordinate would
// move the interpolation weights by ~1e-4 of a cell.
__device__ __forceinline__ void cell(const MotionDims& d, const double p[3], int l, uint32_t c[3], float f[3]) {
  const double N = (double)d.res[l];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double x = p[a] * N;
    const double fl = fmin(floor(x), N - 1.0);
    c[a] = (uint32_t)fl;
    f[a] = (float)(x - fl);
  }
}

__device__ __forceinline__ void position(const MotionDims& d, const float* __restrict__ means, int i, double p[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    p[a] = fmin(fmax(((double)means[(size_t)a * d.row + i] - d.lo[a]) * d.inv_ext[a], 0.0), 1.0);
}

// The level loop is not unrolled (8 corner loads in flight, not 128): each level's two features
// are shifted in at the end of h, so after the 16 levels h[2 l] and h[2 l + 1] are level l's and
// every index into h is a compile-time constant.
__device__ __forceinline__ void encode(const MotionDims& d, const float* __restrict__ table, const double p[3],
                                       float (&h)[kIn]) {
  for (int l = 0; l < kLevels; ++l) {
    uint32_t c[3];
    float f[3];
    cell(d, p, l, c, f);
    float h0 = 0.f, h1 = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t di = k & 1, dj = (k >> 1) & 1, dk = (k >> 2) & 1;
      const float w = (di ? f[0] : 1.f - f[0]) * (dj ? f[1] : 1.f - f[1]) * (dk ? f[2] : 1.f - f[2]);
      const uint32_t e = corner_entry(d, l, c[0] + di, c[1] + dj, c[2] + dk);
      const float2 v = *reinterpret_cast<const float2*>(table + ((size_t)l * kT + e) * kFeats);
      h0 = fmaf(w, v.x, h0);
      h1 = fmaf(w, v.y, h1);
    }
#pragma unroll
    for (int j = 0; j < kIn - 2; ++j) h[j] = h[j + 2];
    h[kIn - 2] = h0;
    h[kIn - 1] = h1;
  }
}

// Weights in LDS, per head: W1 [64][32], b1, W2 transposed [64 in][64 out], b2, W3 [out][64], b3
// (the same offsets as the weight vector; only W2 is stored transposed, so that both passes read
// contiguous rows). A first-layer unit is made one at a time and folded straight into the 64
// second-layer sums, so no activation vector is ever indexed at run time.
__device__ __forceinline__ void load_weights(float* sw, const float* __restrict__ weights) {
  for (int k = threadIdx.x; k < kNW; k += blockDim.x) {
    const int head = k >= kWR;
    const int base = head ? kWR : kWMu;
    const int r = k - base;
    const int w2 = kHid * kIn + kHid;
    int dst = k;
    if (r >= w2 && r < w2 + kHid * kHid) {
      const int e = r - w2, o = e / kHid, j = e % kHid;  // W2[o][j] -> W2T[j][o]
      dst = base + w2 + j * kHid + o;
    }
    sw[dst] = weights[k];
  }
  __syncthreads();
}

struct HeadW {
  const float *W1, *b1, *W2T, *b2, *W3, *b3;
};

template <int OUT>
__device__ __forceinline__ HeadW head_weights(const float* w) {
  HeadW h;
  h.W1 = w;
  h.b1 = h.W1 + kHid * kIn;
  h.W2T = h.b1 + kHid;
  h.b2 = h.W2T + kHid * kHid;
  h.W3 = h.b2 + kHid;
  h.b3 = h.W3 + OUT * kHid;
  return h;
}

__device__ __forceinline__ float unit1(const HeadW& w, const float (&h)[kIn], int o) {
  float acc = w.b1[o];
#pragma unroll
  for (int j = 0; j < kIn; ++j) acc = fmaf(w.W1[o * kIn + j], h[j], acc);
  return acc;  // z1[o]
}

// a2 = relu(W2 relu(W1 h + b1) + b2)
__device__ __forceinline__ void hidden2(const HeadW& w, const float (&h)[kIn], float (&a2)[kHid]) {
#pragma unroll
  for (int o = 0; o < kHid; ++o) a2[o] = w.b2[o];
  for (int o1 = 0; o1 < kHid; ++o1) {
    const float a = fmaxf(unit1(w, h, o1), 0.f);
#pragma unroll
    for (int o = 0; o < kHid; ++o) a2[o] = fmaf(w.W2T[o1 * kHid + o], a, a2[o]);
  }
#pragma unroll
  for (int o = 0; o < kHid; ++o) a2[o] = fmaxf(a2[o], 0.f);
}

template <int OUT>
__device__ __forceinline__ void head_out(const HeadW& w, const float (&a2)[kHid], float (&y)[OUT]) {
#pragma unroll
  for (int k = 0; k < OUT; ++k) {
    float acc = w.b3[k];
#pragma unroll
    for (int j = 0; j < kHid; ++j) acc = fmaf(w.W3[k * kHid + j], a2[j], acc);
    y[k] = acc;
  }
}

__global__ __launch_bounds__(256) void k_motion_fwd(MotionDims d, const float* __restrict__ means,
                                                    const float* __restrict__ table, const float* __restrict__ weights,
                                                    float* __restrict__ out) {
  __shared__ float sw[kNW];
  load_weights(sw, weights);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  double p[3];
  float h[kIn], a2[kHid];
  position(d, means, i, p);
  encode(d, table, p, h);
  float y3[3], y4[4];
  const HeadW wm = head_weights<3>(sw + kWMu), wr = head_weights<4>(sw + kWR);
  hidden2(wm, h, a2);
  head_out<3>(wm, a2, y3);
#pragma unroll
  for (int k = 0; k < 3; ++k) out[(size_t)k * d.row + i] = y3[k];
  // one head at a time: keeps the compiler from interleaving the two heads' 64 accumulators
  // (165 registers, three waves per SIMD, instead of more than 256)
  asm volatile("" ::: "memory");
  hidden2(wr, h, a2);
  head_out<4>(wr, a2, y4);
  out[(size_t)3 * d.row + i] = 1.f + y4[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) out[(size_t)(3 + k) * d.row + i] = y4[k];
}

// Backward of one head for one Gaussian: stages a1, dz1, a2, dz2, dy and adds W1^T dz1 to d_h.
template <int OUT>
__device__ __forceinline__ void head_backward(const HeadW& w, const float (&h)[kIn], const float (&dy)[OUT],
                                              float (&d_h)[kIn], float* __restrict__ stage, int n, int i, int f0) {
  float a2[kHid];
  hidden2(w, h, a2);
  // dz2 = (W3^T dy) where z2 > 0 (a2 > 0 exactly there)
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < OUT; ++k) acc = fmaf(w.W3[k * kHid + j], dy[k], acc);
    stage[(size_t)(f0 + 2 * kHid + j) * n + i] = a2[j];
    a2[j] = a2[j] > 0.f ? acc : 0.f;  // now dz2
    stage[(size_t)(f0 + 3 * kHid + j) * n + i] = a2[j];
  }
  // per first-layer unit: dz1 = (W2^T dz2)[o1] where z1 > 0; d_h += W1[o1] dz1
  for (int o1 = 0; o1 < kHid; ++o1) {
    const float z1 = unit1(w, h, o1);
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < kHid; ++o) s = fmaf(w.W2T[o1 * kHid + o], a2[o], s);
    const float dz1 = z1 > 0.f ? s : 0.f;
    stage[(size_t)(f0 + o1) * n + i] = fmaxf(z1, 0.f);
    stage[(size_t)(f0 + kHid + o1) * n + i] = dz1;
#pragma unroll
    for (int j = 0; j < kIn; ++j) d_h[j] = fmaf(w.W1[o1 * kIn + j], dz1, d_h[j]);
  }
#pragma unroll
  for (int k = 0; k < OUT; ++k) stage[(size_t)(f0 + 4 * kHid + k) * n + i] = dy[k];
}

__global__ __launch_bounds__(256) void k_motion_bwd(MotionDims d, const float* __restrict__ means,
                                                    const float* __restrict__ table, const float* __restrict__ weights,
                                                    const float* __restrict__ d_out, float* __restrict__ d_table,
                                                    float* __restrict__ stage) {
  __shared__ float sw[kNW];
  load_weights(sw, weights);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  double p[3];
  float h[kIn], d_h[kIn];
  position(d, means, i, p);
  encode(d, table, p, h);
#pragma unroll
  for (int j = 0; j < kIn; ++j) {
    d_h[j] = 0.f;
    stage[(size_t)(kFH + j) * d.n + i] = h[j];
  }
  float dy3[3], dy4[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) dy3[k] = d_out[(size_t)k * d.row + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) dy4[k] = d_out[(size_t)(3 + k) * d.row + i];
  head_backward<3>(head_weights<3>(sw + kWMu), h, dy3, d_h, stage, d.n, i, head_fields(0));
  head_backward<4>(head_weights<4>(sw + kWR), h, dy4, d_h, stage, d.n, i, head_fields(1));
  // feature gradients into the table: corner weight times the level's two feature gradients
#pragma unroll
  for (int l = 0; l < kLevels; ++l) {
    uint32_t c[3];
    float f[3];
    cell(d, p, l, c, f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t di = k & 1, dj = (k >> 1) & 1, dk = (k >> 2) & 1;
      const float wgt = (di ? f[0] : 1.f - f[0]) * (dj ? f[1] : 1.f - f[1]) * (dk ? f[2] : 1.f - f[2]);
      const uint32_t e = corner_entry(d, l, c[0] + di, c[1] + dj, c[2] + dk);
      float* t = d_table + ((size_t)l * kT + e) * kFeats;
      unsafeAtomicAdd(t, wgt * d_h[2 * l]);
      unsafeAtomicAdd(t + 1, wgt * d_h[2 * l + 1]);
    }
  }
}

// Weight gradients: d W[o][c] = sum_g A[o][g] B[c][g] and d b[o] = sum_g A[o][g], with A the
// layer's output gradients and B its inputs, both staged per Gaussian. A block takes one layer of
// one head (blockIdx.y) and a range of Gaussians, 64 at a time through LDS stored Gaussian-major,
// so that four consecutive rows are one 16-byte read; each thread owns a 4 x 4 tile of d W
// (2 reads per 16 FMAs) and, for the tiles in column 0, the 4 bias sums.
constexpr int kWTile = 64;     // Gaussians per LDS tile
constexpr int kWPad = kHid + 4;  // LDS row: 64 values + pad (16-byte aligned rows)

__global__ __launch_bounds__(256) void k_motion_wgrad(int n, int per_block, const float* __restrict__ stage,
                                                      float* __restrict__ d_weights) {
  __shared__ __align__(16) float sa[kWTile][kWPad];  // [g][o]
  __shared__ __align__(16) float sb[kWTile][kWPad];  // [g][c]
  const int task = blockIdx.y;
  const int head = task / 3, layer = task % 3;
  const int f0 = head_fields(head);
  const int out = head == 0 ? 3 : 4;
  const int wbase = head == 0 ? kWMu : kWR;
  int a_field, a_rows, b_field, b_rows, w_off;
  if (layer == 0) {         // W1: A = dz1, B = h
    a_field = f0 + kHid; a_rows = kHid; b_field = kFH; b_rows = kIn; w_off = wbase;
  } else if (layer == 1) {  // W2: A = dz2, B = a1
    a_field = f0 + 3 * kHid; a_rows = kHid; b_field = f0; b_rows = kHid; w_off = wbase + kHid * kIn + kHid;
  } else {                  // W3: A = dy, B = a2
    a_field = f0 + 4 * kHid; a_rows = out; b_field = f0 + 2 * kHid; b_rows = kHid;
    w_off = wbase + kHid * kIn + kHid + kHid * kHid + kHid;
  }
  const int bias_off = w_off + a_rows * b_rows;
  const int tiles_c = b_rows / 4, tiles_o = (a_rows + 3) / 4;
  const int t = threadIdx.x;
  const bool owner = t < tiles_o * tiles_c;
  const int o0 = 4 * (t / tiles_c), c0 = 4 * (t % tiles_c);
  float acc[4][4], bacc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bacc[r] = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
  }
  const int g0 = blockIdx.x * per_block, g1 = min(g0 + per_block, n);
  for (int t0 = g0; t0 < g1; t0 += kWTile) {
    __syncthreads();
    // rows beyond a_rows (the 3-row head) and Gaussians beyond the range read as zero
    for (int e = t; e < kHid * kWTile; e += 256) {
      const int r = e / kWTile, g = e % kWTile;
      const bool in = t0 + g < g1;
      sa[g][r] = in && r < a_rows ? stage[(size_t)(a_field + r) * n + t0 + g] : 0.f;
      sb[g][r] = in && r < b_rows ? stage[(size_t)(b_field + r) * n + t0 + g] : 0.f;
    }
    __syncthreads();
    if (owner) {
      for (int g = 0; g < kWTile; ++g) {
        const float4 av = *reinterpret_cast<const float4*>(&sa[g][o0]);
        const float4 bv = *reinterpret_cast<const float4*>(&sb[g][c0]);
        const float ar[4] = {av.x, av.y, av.z, av.w}, br[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(ar[r], br[c], acc[r][c]);
          bacc[r] += ar[r];
        }
      }
    }
  }
  if (!owner) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (o0 + r >= a_rows) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) unsafeAtomicAdd(d_weights + w_off + (o0 + r) * b_rows + c0 + c, acc[r][c]);
    if (c0 == 0) unsafeAtomicAdd(d_weights + bias_off + o0 + r, bacc[r]);
  }
}

int motion_dims(const gs_motion_desc* desc, int32_t row_stride, MotionDims& d) {
  if (!desc) return report_arg("desc is NULL");
  if (desc->n < 0) return report_arg("n < 0");
  if (row_stride < desc->n) return report_arg("row_stride < n");
  d.n = desc->n;
  d.row = row_stride;
  for (int a = 0; a < 3; ++a) {
    const double ext = (double)desc->box_hi[a] - (double)desc->box_lo[a];
    if (!(ext > 0.0) || std::isinf(ext)) return report_arg("the scene box must have positive finite extent");
    d.lo[a] = desc->box_lo[a];
    d.inv_ext[a] = 1.0 / ext;
  }
  const double b = std::exp((std::log(1024.0) - std::log(16.0)) / (kLevels - 1));
  for (int l = 0; l < kLevels; ++l) {
    d.res[l] = (int)std::floor(16.0 * std::pow(b, l) + 1e-9);
    const long long N1 = d.res[l] + 1;
    d.dense[l] = N1 * N1 * N1 <= kT;
  }
  return GS_OK;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int gs_motion_sizes(int64_t* table_floats, int64_t* n_weights) {
  if (table_floats) *table_floats = (int64_t)kLevels * kT * kFeats;
  if (n_weights) *n_weights = kNW;
  return GS_OK;
}

int gs_motion_workspace_size(int32_t n, size_t* bytes_out) {
  if (n < 0 || !bytes_out) return report_arg("n < 0 or bytes_out NULL");
  *bytes_out = (size_t)kNF * (size_t)(n > 0 ? n : 1) * sizeof(float);
  return GS_OK;
}

int gs_motion_forward(const gs_motion_desc* desc, const float* means, int32_t row_stride, const float* table,
                      const float* weights, float* out, void* stream) {
  MotionDims d;
  int rc = motion_dims(desc, row_stride, d);
  if (rc) return rc;
  if (d.n == 0) return GS_OK;
  if (!means || !table || !weights || !out) return report_arg("NULL buffer");
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  {
    ProfScope ps_(K_MOTION_FWD, st);
    hipLaunchKernelGGL(k_motion_fwd, dim3((d.n + 255) / 256), dim3(256), 0, st, d, means, table, weights, out);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "motion forward");
}

int gs_motion_backward(const gs_motion_desc* desc, const float* means, int32_t row_stride, const float* table,
                       const float* weights, const float* d_out, float* d_table, float* d_weights, void* ws,
                       size_t ws_bytes, void* stream) {
  MotionDims d;
  int rc = motion_dims(desc, row_stride, d);
  if (rc) return rc;
  if (d.n == 0) return GS_OK;
  if (!means || !table || !weights || !d_out || !d_table || !d_weights || !ws) return report_arg("NULL buffer");
  size_t need = 0;
  gs_motion_workspace_size(d.n, &need);
  if (ws_bytes < need) {
    report_arg("workspace too small");
    return GS_ERR_WORKSPACE;
  }
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  float* stage = (float*)ws;
  {
    ProfScope ps_(K_MOTION_BWD, st);
    hipLaunchKernelGGL(k_motion_bwd, dim3((d.n + 255) / 256), dim3(256), 0, st, d, means, table, weights, d_out,
                       d_table, stage);
  }
  {
    ProfScope ps_(K_MOTION_WGRAD, st);
    const int per_block = 2048;
    hipLaunchKernelGGL(k_motion_wgrad, dim3((d.n + per_block - 1) / per_block, 6), dim3(256), 0, st, d.n, per_block,
                       stage, d_weights);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "motion backward");
}

}  // extern "C"
