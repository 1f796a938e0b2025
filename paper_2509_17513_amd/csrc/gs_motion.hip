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
// The MLP layers run on the FP32 matrix cores (v_mfma_f32_32x32x2_f32, FP32 products and sums):
// a wave takes 32 Gaussians at a time, with the activations held transposed (hidden units as
// rows, the 32 Gaussians as columns), so that each layer's accumulator is the next layer's B
// operand with no data movement (T layout: lane l holds Gaussian l & 31, accumulator element r
// the unit 8 (r / 4) + 4 (l >> 5) + (r & 3) of its 32-unit tile; the contraction index of each
// product is permuted to match). The two lanes of a Gaussian each gather 4 of the 8 corners of
// every level and add their halves across the wave halves.
//
//  motion_fwd    both MLPs per 32-Gaussian task, weights in LDS (rows padded to an odd length so
//                that both orientations read them without bank conflicts)
//  motion_bwd    one block per group of tasks, both MLPs: the forward again, dZ2 = W3^T dy on the
//                VALU, dZ1 = W2^T dZ2 and dL/dh = W1^T dZ1 on the matrix cores, dL/dh staged per
//                Gaussian; the weight gradients dW = dZ^T X are sums over Gaussians, so the wave
//                transposes dZ and X through its own LDS scratch and contracts over the 32
//                Gaussians on the matrix cores, accumulating over its tasks; each wave writes its
//                partial weight gradients once
//  motion_wgrad  d_weights += the sum of the waves' partial weight gradients (16 partial sums per
//                weight, added with float atomics)
//  motion_table  the table gradient without memory-side atomics: a block owns one feature of one
//                level (the whole 2^15-entry column in LDS) and one chunk of the Gaussians, adds
//                the chunk's corner terms into it (LDS atomics, every lane active), and writes it
//                to its chunk's partial table; motion_table_sum adds the chunks' partial tables
//                into d_table. (Device-scope float atomics into the table are
//                performed past the L2 at about 2e10 per second on this part, and the 16 x 8 x 2
//                per Gaussian took 90% of the backward.)
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kLevels = 16, kFeats = 2, kLog2T = 15, kT = 1 << kLog2T;
constexpr int kIn = kLevels * kFeats, kHid = 64;
// weights of one head in the flat vector: W1 [64][32], b1, W2 [64][64], b2, W3 [out][64], b3
constexpr int head_size(int out) { return kHid * kIn + kHid + kHid * kHid + kHid + out * kHid + out; }
constexpr int kWMu = 0, kWR = head_size(3), kNW = head_size(3) + head_size(4);
constexpr int kFW1 = 0, kFB1 = kFW1 + kHid * kIn, kFW2 = kFB1 + kHid, kFB2 = kFW2 + kHid * kHid, kFW3 = kFB2 + kHid;
// one head in LDS: W1 rows of 33, b1, W2 rows of 65, b2, W3 [out][64], b3 (16-byte aligned biases)
constexpr int kW1S = kIn + 1, kW2S = kHid + 1;
constexpr int kLW1 = 0, kLB1 = kHid * kW1S, kLW2 = kLB1 + kHid, kLB2 = kLW2 + kHid * kW2S, kLW3 = kLB2 + kHid;
constexpr int kHeadLds = kLW3 + 4 * kHid + 8;
// backward: waves per block, blocks per head, the wave's transpose scratch (two [64][33] arrays and
// dy [4][32]) and the record of one wave's partial weight gradients (a 32 x 32 tile of dW2 and of
// dW1, a row of dW3, 16 entries of db1 and db2, one of db3)
constexpr int kBwdWaves = 4, kBwdBlocks = 256;
constexpr int kScrS = 33, kScr = 2 * kHid * kScrS + 4 * 32;
constexpr int kPW2 = 0, kPW1 = 1024, kPW3 = 2048, kPB1 = kPW3 + kHid, kPB2 = kPB1 + 16, kPB3 = kPB2 + 16;
constexpr int kPart = kPB3 + 16;
// table-gradient pass: Gaussian chunks (partial tables), Gaussians in flight per thread, block size
constexpr int kChunks = 8, kTabILP = 4, kTabThreads = 1024;

typedef __attribute__((ext_vector_type(16))) float f32x16;

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

// Row of accumulator element r in wave half hf (the T layout's unit within a 32-unit tile):
// trow = tro(r) + 4 hf. Addresses below fold the lane's part into one base pointer and leave
// tro(r) (a compile-time constant) to the instruction's offset.
__device__ __forceinline__ constexpr int tro(int r) { return 8 * (r >> 2) + (r & 3); }
__device__ __forceinline__ int trow(int r, int hf) { return tro(r) + 4 * hf; }

__device__ __forceinline__ f32x16 mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// One head's weights from the flat vector into LDS (layout kLW*).
__device__ __forceinline__ void load_head(float* sw, const float* __restrict__ w, int out) {
  for (int k = threadIdx.x; k < head_size(out); k += blockDim.x) {
    int dst;
    if (k < kFB1) dst = kLW1 + (k / kIn) * kW1S + k % kIn;
    else if (k < kFW2) dst = kLB1 + (k - kFB1);
    else if (k < kFB2) dst = kLW2 + ((k - kFW2) / kHid) * kW2S + (k - kFW2) % kHid;
    else if (k < kFW3) dst = kLB2 + (k - kFB2);
    else dst = kLW3 + (k - kFW3);  // W3 [out][64] then b3, contiguous
    sw[dst] = w[k];
  }
}

// The encoding of the task's Gaussian for this lane: hv[s] = feature 2 s + hf (level s, feature hf)
// of Gaussian l & 31. Each lane gathers corners 4 hf .. 4 hf + 3 of every level; the two halves'
// partial sums are exchanged with v_permlane32_swap.
__device__ __forceinline__ void encode_half(const MotionDims& d, const float* __restrict__ table, const double p[3],
                                            int hf, float (&hv)[kLevels]) {
  for (int l = 0; l < kLevels; ++l) {
    uint32_t c[3];
    float f[3];
    cell(d, p, l, c, f);
    float h0 = 0.f, h1 = 0.f;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint32_t k = 4u * (uint32_t)hf + (uint32_t)kk;
      const uint32_t di = k & 1u, dj = (k >> 1) & 1u, dk = (k >> 2) & 1u;
      const float w = (di ? f[0] : 1.f - f[0]) * (dj ? f[1] : 1.f - f[1]) * (dk ? f[2] : 1.f - f[2]);
      const uint32_t e = corner_entry(d, l, c[0] + di, c[1] + dj, c[2] + dk);
      const float2 v = *reinterpret_cast<const float2*>(table + ((size_t)l * kT + e) * kFeats);
      h0 = fmaf(w, v.x, h0);
      h1 = fmaf(w, v.y, h1);
    }
    // lanes 0..31 end with feature 0 of the level, lanes 32..63 with feature 1, each summed over
    // the 8 corners
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(h0), __float_as_uint(h1), false, false);
#pragma unroll
    for (int j = 0; j < kLevels - 1; ++j) hv[j] = hv[j + 1];
    hv[kLevels - 1] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// Hidden layers of one head in the T layout: a1 = relu(W1 h + b1), a2 = relu(W2 a1 + b2) (two
// 32-unit tiles each). Layer 1 contracts over the input features in the order of hv (step s,
// half hf: feature 2 s + hf); layer 2 over the hidden units in the order of a1's accumulator.
__device__ __forceinline__ void hidden_layers(const float* sw, const float (&hv)[kLevels], int lrow, int hf,
                                              f32x16 (&a1)[2], f32x16 (&a2)[2]) {
  const float* b1 = sw + kLB1 + 4 * hf;                 // + 32 t + tro(r)
  const float* w1 = sw + kLW1 + lrow * kW1S + hf;       // + 32 t kW1S + 2 s
  const float* b2 = sw + kLB2 + 4 * hf;
  const float* w2 = sw + kLW2 + lrow * kW2S + 4 * hf;   // + 32 t2 kW2S + 32 t + tro(r)
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) a1[t][r] = b1[32 * t + tro(r)];
#pragma unroll
  for (int s = 0; s < kLevels; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) a1[t] = mfma(w1[32 * t * kW1S + 2 * s], hv[s], a1[t]);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      a1[t][r] = fmaxf(a1[t][r], 0.f);
      a2[t][r] = b2[32 * t + tro(r)];
    }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2) a2[t2] = mfma(w2[32 * t2 * kW2S + 32 * t + tro(r)], a1[t][r], a2[t2]);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) a2[t][r] = fmaxf(a2[t][r], 0.f);
}

// Output layer: y_k = b3[k] + W3[k] . a2 for the lane's Gaussian. Each half sums over its 32
// units; v_permlane32_swap then leaves y[2 m] complete in lanes 0..31 and y[2 m + 1] in lanes
// 32..63 (returned as pair m).
template <int OUT>
__device__ __forceinline__ void out_layer(const float* sw, const f32x16 (&a2)[2], int hf, float (&y)[2]) {
  float part[4] = {0.f, 0.f, 0.f, 0.f};
  const float* w3 = sw + kLW3 + 4 * hf;  // + k 64 + 32 t + tro(r)
#pragma unroll
  for (int k = 0; k < OUT; ++k)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[k] = fmaf(w3[k * kHid + 32 * t + tro(r)], a2[t][r], part[k]);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[2 * m]), __float_as_uint(part[2 * m + 1]),
                                                    false, false);
    const int k = 2 * m + hf;
    y[m] = __uint_as_float(r[0]) + __uint_as_float(r[1]) + (k < OUT ? sw[kLW3 + OUT * kHid + k] : 0.f);
  }
}

__global__ __launch_bounds__(256) void k_motion_fwd(MotionDims d, const float* __restrict__ means,
                                                    const float* __restrict__ table, const float* __restrict__ weights,
                                                    float* __restrict__ out) {
  __shared__ __align__(16) float sw[2 * kHeadLds];
  load_head(sw, weights + kWMu, 3);
  load_head(sw + kHeadLds, weights + kWR, 4);
  __syncthreads();
  const int lane = threadIdx.x & 63, lrow = lane & 31, hf = lane >> 5;
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task * 32 >= d.n) return;
  const int i = task * 32 + lrow;
  const bool valid = i < d.n;
  double p[3];
  position(d, means, valid ? i : d.n - 1, p);
  float hv[kLevels];
  encode_half(d, table, p, hf, hv);
  f32x16 a1[2], a2[2];
  float y[2];
  // translation: rows 0..2
  hidden_layers(sw, hv, lrow, hf, a1, a2);
  out_layer<3>(sw, a2, hf, y);
  if (valid) {
    out[(size_t)hf * d.row + i] = y[0];
    if (hf == 0) out[(size_t)2 * d.row + i] = y[1];
  }
  // rotation: rows 3..6, the quaternion (1 + o0, o1, o2, o3)
  hidden_layers(sw + kHeadLds, hv, lrow, hf, a1, a2);
  out_layer<4>(sw + kHeadLds, a2, hf, y);
  if (valid) {
    out[(size_t)(3 + hf) * d.row + i] = hf == 0 ? 1.f + y[0] : y[0];
    out[(size_t)(5 + hf) * d.row + i] = y[1];
  }
}

// Backward. The block's waves take one task each per round; each wave encodes its 32 Gaussians
// once and, per head, runs the chain (forward again, dZ2, dZ1, dL/dh) and then puts the factors of
// the weight gradients into its LDS scratch (rows [unit][Gaussian], stride 33: the T layout writes
// along a row, the transposed operands read along a column); after a barrier the weight gradients
// are contracted over all the block's 128 Gaussians with the work split over the waves: wave w
// owns the dW2 tile (w >> 1, w & 1), half w >> 1 of the Gaussians for the dW1 tile w & 1, row w of
// dW3 (if w < OUT), and units 16 w .. 16 w + 15 of db1 and db2.
struct WGrad {
  f32x16 w2, w1;
  float w3, b1, b2, b3;
};

template <int OUT>
__device__ __forceinline__ void bwd_head_round(const MotionDims& d, const float* sw, const float (&hv)[kLevels], int i,
                                               bool valid, const float* __restrict__ d_out,
                                               float* __restrict__ dh_out, float (*scr)[kScr], WGrad& G) {
  const int lane = threadIdx.x & 63, lrow = lane & 31, hf = lane >> 5;
  const int w = threadIdx.x >> 6;
  float* SX = scr[w];
  float* SD = SX + 2 * kHid * kScrS;
  const int dy_row = OUT == 3 ? 0 : 3;
  // per-lane base pointers (the constant parts of the addresses go to the instruction offsets)
  const float* w3 = sw + kLW3 + 4 * hf;                  // W3[k][32 t + trow]: + k 64 + 32 t + tro(r)
  const float* w2t = sw + kLW2 + 4 * hf * kW2S + lrow;   // W2[32 t2 + trow][32 t1 + lrow]
  const float* w1t = sw + kLW1 + 4 * hf * kW1S + lrow;   // W1[32 t1 + trow][lrow]
  float* sxw = SX + 4 * hf * kScrS + lrow;               // T-layout writes: + (32 t + tro(r)) 33
  float* syw = sxw + kHid * kScrS;
  float* syh = SX + kHid * kScrS + hf * kScrS + lrow;    // H rows 2 s + hf
  const int ta = w >> 1, tb = w & 1;
  f32x16 a1[2], a2[2];
  hidden_layers(sw, hv, lrow, hf, a1, a2);
  float dy[OUT];
#pragma unroll
  for (int k = 0; k < OUT; ++k) dy[k] = valid ? d_out[(size_t)(dy_row + k) * d.row + i] : 0.f;
  // dZ2 = (W3^T dy) where a2 > 0 (T layout)
  f32x16 dz2[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < OUT; ++k) s = fmaf(w3[k * kHid + 32 * t + tro(r)], dy[k], s);
      dz2[t][r] = a2[t][r] > 0.f ? s : 0.f;
    }
  // dZ1 = (W2^T dZ2) where a1 > 0: A = W2^T (row o1, contraction o2 = W2 read along a row)
  f32x16 dz1[2];
#pragma unroll
  for (int r = 0; r < 16; ++r) dz1[0][r] = dz1[1][r] = 0.f;
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int t1 = 0; t1 < 2; ++t1) dz1[t1] = mfma(w2t[(32 * t2 + tro(r)) * kW2S + 32 * t1], dz2[t2][r], dz1[t1]);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) dz1[t][r] = a1[t][r] > 0.f ? dz1[t][r] : 0.f;
  // dL/dh = W1^T dZ1 (one 32-feature tile), staged as [level][n][2] for the table pass
  {
    f32x16 dh;
#pragma unroll
    for (int r = 0; r < 16; ++r) dh[r] = 0.f;
#pragma unroll
    for (int t1 = 0; t1 < 2; ++t1)
#pragma unroll
      for (int r = 0; r < 16; ++r) dh = mfma(w1t[(32 * t1 + tro(r)) * kW1S], dz1[t1][r], dh);
    // elements (r, r + 1), r even, are the two features of level 4 (r >> 2) + 2 hf + ((r & 3) >> 1)
    float* dhp = dh_out + ((size_t)2 * hf * d.n + i) * 2;
    if (valid)
#pragma unroll
      for (int r = 0; r < 16; r += 2)
        *reinterpret_cast<float2*>(dhp + (size_t)(4 * (r >> 2) + ((r & 3) >> 1)) * 2 * d.n) =
            make_float2(dh[r], dh[r + 1]);
  }
  // (1) dW3 = dy^T A2, db3: SX = A2, SD = dy
  __syncthreads();  // the previous phase's reads of the scratch are done
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) sxw[(32 * t + tro(r)) * kScrS] = a2[t][r];
  if (hf == 0)
#pragma unroll
    for (int k = 0; k < OUT; ++k) SD[k * 32 + lrow] = dy[k];
  __syncthreads();
  if (w < OUT) {
    // row w of dW3: lane = unit, summed over the block's 128 Gaussians
    for (int v = 0; v < kBwdWaves; ++v) {
      const float* x = scr[v] + lane * kScrS;
      const float* y = scr[v] + 2 * kHid * kScrS + w * 32;
#pragma unroll 8
      for (int g = 0; g < 32; ++g) G.w3 = fmaf(y[g], x[g], G.w3);
      if (lane == 0)
#pragma unroll 8
        for (int g = 0; g < 32; ++g) G.b3 += y[g];
    }
  }
  __syncthreads();
  // (2) dW2 = dZ2^T A1, db2: SX = dZ2, SY = A1
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      sxw[(32 * t + tro(r)) * kScrS] = dz2[t][r];
      syw[(32 * t + tro(r)) * kScrS] = a1[t][r];
    }
  __syncthreads();
  for (int v = 0; v < kBwdWaves; ++v) {
    const float* xr = scr[v] + (32 * ta + lrow) * kScrS + hf;
    const float* yr = scr[v] + kHid * kScrS + (32 * tb + lrow) * kScrS + hf;
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) G.w2 = mfma(xr[2 * s2], yr[2 * s2], G.w2);
  }
  if (lane < 16)
    for (int v = 0; v < kBwdWaves; ++v) {
      const float* x = scr[v] + (16 * w + lane) * kScrS;
#pragma unroll 8
      for (int g = 0; g < 32; ++g) G.b2 += x[g];
    }
  __syncthreads();
  // (3) dW1 = dZ1^T H, db1: SX = dZ1, SY rows 0..31 = H
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) sxw[(32 * t + tro(r)) * kScrS] = dz1[t][r];
#pragma unroll
  for (int s2 = 0; s2 < kLevels; ++s2) syh[2 * s2 * kScrS] = hv[s2];
  __syncthreads();
  for (int v = 2 * ta; v < 2 * ta + 2; ++v) {  // this wave's half of the Gaussians
    const float* xr = scr[v] + (32 * tb + lrow) * kScrS + hf;
    const float* yr = scr[v] + kHid * kScrS + lrow * kScrS + hf;
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) G.w1 = mfma(xr[2 * s2], yr[2 * s2], G.w1);
  }
  if (lane < 16)
    for (int v = 0; v < kBwdWaves; ++v) {
      const float* x = scr[v] + (16 * w + lane) * kScrS;
#pragma unroll 8
      for (int g = 0; g < 32; ++g) G.b1 += x[g];
    }
}

// One wave's partial weight gradients of one head (accumulator layouts; motion_wgrad maps them back).
__device__ __forceinline__ void write_wgrad(const WGrad& G, float* __restrict__ q) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    q[kPW2 + r * 64 + lane] = G.w2[r];
    q[kPW1 + r * 64 + lane] = G.w1[r];
  }
  q[kPW3 + lane] = G.w3;
  if (lane < 16) {
    q[kPB1 + lane] = G.b1;
    q[kPB2 + lane] = G.b2;
  }
  if (lane == 0) q[kPB3] = G.b3;
}

__global__ __launch_bounds__(kBwdWaves * 64) void k_motion_bwd(MotionDims d, const float* __restrict__ means,
                                                                const float* __restrict__ table,
                                                                const float* __restrict__ weights,
                                                                const float* __restrict__ d_out,
                                                                float* __restrict__ dh_out, float* __restrict__ part) {
  __shared__ __align__(16) float sw[2 * kHeadLds];
  __shared__ __align__(16) float scr[kBwdWaves][kScr];
  load_head(sw, weights + kWMu, 3);
  load_head(sw + kHeadLds, weights + kWR, 4);
  __syncthreads();
  const int lane = threadIdx.x & 63, lrow = lane & 31, hf = lane >> 5;
  const int w = threadIdx.x >> 6;
  WGrad G0, G1;
#pragma unroll
  for (int r = 0; r < 16; ++r) G0.w2[r] = G0.w1[r] = G1.w2[r] = G1.w1[r] = 0.f;
  G0.w3 = G0.b1 = G0.b2 = G0.b3 = G1.w3 = G1.b1 = G1.b2 = G1.b3 = 0.f;
  const int ntasks = (d.n + 31) / 32;
  // every wave of the block runs the same number of rounds (the phases synchronise the block)
  const int rounds = (ntasks + kBwdWaves * gridDim.x - 1) / (kBwdWaves * gridDim.x);
  for (int round = 0; round < rounds; ++round) {
    const int task = (round * gridDim.x + blockIdx.x) * kBwdWaves + w;
    const int i = task * 32 + lrow;
    const bool valid = i < d.n;
    double p[3];
    position(d, means, valid ? i : max(d.n - 1, 0), p);
    float hv[kLevels];
    encode_half(d, table, p, hf, hv);
    bwd_head_round<3>(d, sw, hv, i, valid, d_out, dh_out, scr, G0);
    bwd_head_round<4>(d, sw + kHeadLds, hv, i, valid, d_out, dh_out + (size_t)kIn * d.n, scr, G1);
  }
  write_wgrad(G0, part + ((size_t)blockIdx.x * kBwdWaves + w) * kPart);
  write_wgrad(G1, part + (((size_t)gridDim.x + blockIdx.x) * kBwdWaves + w) * kPart);
}

// d_weights += the sum over the blocks of their waves' partial weight gradients: one thread per
// weight of head blockIdx.y finds the wave and record field that hold it (see bwd_head_round).
__global__ __launch_bounds__(256) void k_motion_wgrad(int nblocks, const float* __restrict__ part,
                                                      float* __restrict__ d_weights) {
  const int head = blockIdx.y, out = head ? 4 : 3;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= head_size(out)) return;
  // (wave, field) of the weight; dW1 has a second wave (the other half of the Gaussians)
  int w0 = -1, w1 = -1, f = 0;
  auto field = [](int row, int col) {  // accumulator element of (row, col) inside a 32 x 32 tile
    const int hf = (row >> 2) & 1, r = 4 * (row >> 3) + (row & 3);
    return r * 64 + 32 * hf + col;
  };
  if (k < kFB1) {
    const int o1 = k / kIn, i = k % kIn;
    w0 = o1 >> 5;
    w1 = 2 + (o1 >> 5);
    f = kPW1 + field(o1 & 31, i);
  } else if (k < kFW2) {
    w0 = (k - kFB1) / 16;
    f = kPB1 + (k - kFB1) % 16;
  } else if (k < kFB2) {
    const int o2 = (k - kFW2) / kHid, o1 = (k - kFW2) % kHid;
    w0 = 2 * (o2 >> 5) + (o1 >> 5);
    f = kPW2 + field(o2 & 31, o1 & 31);
  } else if (k < kFW3) {
    w0 = (k - kFB2) / 16;
    f = kPB2 + (k - kFB2) % 16;
  } else if (k < kFW3 + out * kHid) {
    w0 = (k - kFW3) / kHid;
    f = kPW3 + (k - kFW3) % kHid;
  } else {
    w0 = k - kFW3 - out * kHid;
    f = kPB3;
  }
  const float* src = part + (size_t)head * nblocks * kBwdWaves * kPart;
  // blockIdx.z takes every gridDim.z-th block record; the splits meet in one float atomic each
  float s = 0.f;
  for (int b = blockIdx.z; b < nblocks; b += gridDim.z) {
    s += src[((size_t)b * kBwdWaves + w0) * kPart + f];
    if (w1 >= 0) s += src[((size_t)b * kBwdWaves + w1) * kPart + f];
  }
  unsafeAtomicAdd(d_weights + (head ? kWR : kWMu) + k, s);
}

// Table gradient, one (level, feature) x one chunk of the Gaussians per block: the corner terms
// w_k dL/dh_f of the chunk's Gaussians are added into an LDS copy of the level's column of feature
// f (2^15 floats, 128 KB), which is then written, whole, to the chunk's partial table
// [chunk][level][feature][entry].
__global__ __launch_bounds__(kTabThreads) void k_motion_table(MotionDims d, const float* __restrict__ means,
                                                              const float* __restrict__ dh, float* __restrict__ partial) {
  __shared__ float acc[kT];
  const int chunk = blockIdx.x, l = blockIdx.y >> 1, feat = blockIdx.y & 1;
  const int used = d.dense[l] ? (d.res[l] + 1) * (d.res[l] + 1) * (d.res[l] + 1) : kT;
  for (int j = threadIdx.x; j < used; j += kTabThreads) acc[j] = 0.f;
  __syncthreads();
  const int per = (d.n + kChunks - 1) / kChunks;
  const int g0 = chunk * per, g1 = min(g0 + per, d.n);
  // kTabILP Gaussians per thread per round, their loads issued together
  for (int i0 = g0 + (int)threadIdx.x; i0 < g1; i0 += kTabThreads * kTabILP) {
    float mu[kTabILP][3], gh[kTabILP];
#pragma unroll
    for (int u = 0; u < kTabILP; ++u) {
      const int i = min(i0 + kTabThreads * u, g1 - 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) mu[u][a] = means[(size_t)a * d.row + i];
      // the feature gradients of the two MLPs, each [16 levels][n][2]
      gh[u] = dh[((size_t)l * d.n + i) * 2 + feat] + dh[((size_t)(kLevels + l) * d.n + i) * 2 + feat];
    }
#pragma unroll
    for (int u = 0; u < kTabILP; ++u) {
      if (i0 + kTabThreads * u >= g1) break;
      double p[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) p[a] = fmin(fmax(((double)mu[u][a] - d.lo[a]) * d.inv_ext[a], 0.0), 1.0);
      uint32_t c[3];
      float f[3];
      cell(d, p, l, c, f);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t di = k & 1, dj = (k >> 1) & 1, dk = (k >> 2) & 1;
        const uint32_t e = corner_entry(d, l, c[0] + di, c[1] + dj, c[2] + dk);
        const float wgt = (di ? f[0] : 1.f - f[0]) * (dj ? f[1] : 1.f - f[1]) * (dk ? f[2] : 1.f - f[2]);
        atomicAdd(&acc[e], wgt * gh[u]);
      }
    }
  }
  __syncthreads();
  float* out = partial + (((size_t)chunk * kLevels + l) * kFeats + feat) * kT;
  for (int j = threadIdx.x; j < used; j += kTabThreads) out[j] = acc[j];
}

// d_table += the sum of the chunks' partial tables, over the entries each level uses.
__global__ __launch_bounds__(256) void k_motion_table_sum(MotionDims d, const float* __restrict__ partial,
                                                          float* __restrict__ d_table) {
  const int l = blockIdx.y;
  const int used = d.dense[l] ? (d.res[l] + 1) * (d.res[l] + 1) * (d.res[l] + 1) : kT;
  const int j = blockIdx.x * 256 + threadIdx.x;  // table float (entry j >> 1, feature j & 1) of level l
  if (j >= used * kFeats) return;
  const size_t src = ((size_t)l * kFeats + (j & 1)) * kT + (j >> 1);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) s += partial[(size_t)c * kLevels * kFeats * kT + src];
  d_table[(size_t)l * kT * kFeats + j] += s;
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
  // the two MLPs' feature gradients [2][32][n], the waves' partial weight gradients, the chunks'
  // partial tables
  *bytes_out = ((size_t)2 * kIn * (size_t)(n > 0 ? n : 1) + (size_t)2 * kBwdBlocks * kBwdWaves * kPart +
                (size_t)kChunks * kLevels * kT * kFeats) *
               sizeof(float);
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
    hipLaunchKernelGGL(k_motion_fwd, dim3((d.n + 127) / 128), dim3(256), 0, st, d, means, table, weights, out);
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
  float* dh = (float*)ws;
  float* part = dh + (size_t)2 * kIn * d.n;
  float* partial = part + (size_t)2 * kBwdBlocks * kBwdWaves * kPart;
  {
    ProfScope ps_(K_MOTION_BWD, st);
    hipLaunchKernelGGL(k_motion_bwd, dim3(kBwdBlocks), dim3(kBwdWaves * 64), 0, st, d, means, table, weights, d_out,
                       dh, part);
  }
  {
    ProfScope ps_(K_MOTION_WGRAD, st);
    hipLaunchKernelGGL(k_motion_wgrad, dim3((head_size(4) + 255) / 256, 2, 16), dim3(256), 0, st, kBwdBlocks, part,
                       d_weights);
  }
  {
    ProfScope ps_(K_MOTION_TABLE, st);
    hipLaunchKernelGGL(k_motion_table, dim3(kChunks, kLevels * kFeats), dim3(kTabThreads), 0, st, d, means, dh, partial);
    hipLaunchKernelGGL(k_motion_table_sum, dim3((kT * kFeats + 255) / 256, kLevels), dim3(256), 0, st, d, partial,
                       d_table);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "motion backward");
}

}  // extern "C"
