// Rate terms of the quantised Gaussian attributes (Sec. 3.3: quantisation
// simulated with additive uniform noise, rate = -sum log2 PMF with the PMF
// taken from CDF differences one quantisation step apart).
//
//   k_rate_ctx        16 context features per Gaussian, BF16, [n][16]
//   k_rate_mlp        per-attribute MLP 16 -> 64 -> 64 -> 2 on MFMA (BF16 in,
//                     FP32 accumulate) giving a discretised Laplace per symbol,
//                     its bits, and the backward to the weights and (training
//                     mode) to the attributes; activations never leave the chip
//   k_hist_*          empirical-histogram rate: symbol range, LDS-privatised
//                     counts, FP64 entropy sum
//   k_adam            Adam update of FP32 masters with an optional BF16 copy
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include <stdint.h>

#include <algorithm>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kCtx = 16;
constexpr int kHid = 64;
constexpr int kW1 = kHid * kCtx;  // 1024
constexpr int kW2 = kHid * kHid;  // 4096
constexpr int kW3 = 2 * kHid;     // 128
constexpr int kWPerAttr = kW1 + kW2 + kW3;
constexpr int kBPerAttr = kHid + kHid + 2;
constexpr float kPFloor = 1e-9f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2e = 1.4426950408889634f;

// FP32 -> BF16, round to nearest even, on the hardware converter (v_cvt_pk_bf16_f32)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f32_to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float lo, float hi) {
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Stores the two BF16 halves of a packed pair at p[i0] and p[i1]. The empty asm makes the pair
// opaque, so the halves are taken from its bits instead of being converted from float again.
__device__ __forceinline__ void store_pair(uint16_t* p, int i0, int i1, uint32_t hp) {
  asm("" : "+v"(hp));
  p[i0] = (uint16_t)hp;
  p[i1] = (uint16_t)(hp >> 16);
}

// ------------------------------------------------------------------ context
// x = [mu / extent (3), sin / cos(pi 2^k mu / extent) for k = 0, 1 (12), (layer - 1) / 5 (1)]
__global__ __launch_bounds__(256) void k_rate_ctx(int n, const float* __restrict__ means, float extent, int n_levels,
                                                  int4 lv_lo, int4 lv_hi, uint16_t* __restrict__ ctx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lv[8] = {lv_lo.x, lv_lo.y, lv_lo.z, lv_lo.w, lv_hi.x, lv_hi.y, lv_hi.z, lv_hi.w};
  int layer = 1;
  for (int l = 0; l < n_levels; ++l)
    if (i >= lv[l]) layer = l + 2;
  layer = min(layer, n_levels);
  float f[kCtx];
  for (int c = 0; c < 3; ++c) {
    const float u = means[(size_t)c * n + i] / extent;
    f[c] = u;
    f[3 + c] = sinf(3.14159265358979f * u);
    f[6 + c] = cosf(3.14159265358979f * u);
    f[9 + c] = sinf(6.28318530717959f * u);
    f[12 + c] = cosf(6.28318530717959f * u);
  }
  f[15] = (float)(layer - 1) / 5.0f;
  uint16_t* o = ctx + (size_t)i * kCtx;
  for (int c = 0; c < kCtx; ++c) o[c] = f32_to_bf16(f[c]);
}

// ---------------------------------------------------------------- histogram
__global__ void k_hist_init(int n_attr, int* __restrict__ mm) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < n_attr) {
    mm[2 * a] = 0x7FFFFFFF;
    mm[2 * a + 1] = (int)0x80000000;
  }
}

__device__ __forceinline__ int symbol_of(float y, float step) { return (int)rintf(y / step); }

__global__ __launch_bounds__(256) void k_hist_minmax(int n, const float* __restrict__ attrs, float step,
                                                     int* __restrict__ mm) {
  const int a = blockIdx.y;
  const float* y = attrs + (size_t)a * n;
  int lo = 0x7FFFFFFF, hi = (int)0x80000000;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = symbol_of(y[i], step);
    lo = min(lo, k);
    hi = max(hi, k);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off));
    hi = max(hi, __shfl_xor(hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&mm[2 * a], lo);
    atomicMax(&mm[2 * a + 1], hi);
  }
}

constexpr int kHistBins = 1 << 16;      // per attribute, in the workspace
constexpr int kHistLdsBins = 1 << 14;   // LDS-privatised when the range fits

__global__ __launch_bounds__(256) void k_hist_count(int n, const float* __restrict__ attrs, float step,
                                                    const int* __restrict__ mm, uint32_t* __restrict__ hist,
                                                    uint32_t* __restrict__ err) {
  __shared__ uint32_t lh[kHistLdsBins];
  const int a = blockIdx.y;
  const int kmin = mm[2 * a], kmax = mm[2 * a + 1];
  const long long range = (long long)kmax - kmin + 1;
  if (range > kHistBins) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(err, 1u);
    return;
  }
  const float* y = attrs + (size_t)a * n;
  uint32_t* gh = hist + (size_t)a * kHistBins;
  const bool use_lds = range <= kHistLdsBins;
  if (use_lds) {
    for (int j = threadIdx.x; j < range; j += blockDim.x) lh[j] = 0;
    __syncthreads();
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = symbol_of(y[i], step) - kmin;
    if (use_lds) atomicAdd(&lh[k], 1u);
    else atomicAdd(&gh[k], 1u);
  }
  if (use_lds) {
    __syncthreads();
    for (int j = threadIdx.x; j < range; j += blockDim.x)
      if (lh[j]) atomicAdd(&gh[j], lh[j]);
  }
}

// bits_a = N log2 N - sum_k n_k log2 n_k  (= -sum_i log2(n(k_i) / N)), in FP64
__global__ __launch_bounds__(256) void k_hist_bits(int n, const int* __restrict__ mm, const uint32_t* __restrict__ hist,
                                                   double* __restrict__ bits) {
  __shared__ double part[256];
  const int a = blockIdx.x;
  const long long range = (long long)mm[2 * a + 1] - mm[2 * a] + 1;
  const uint32_t* gh = hist + (size_t)a * kHistBins;
  double s = 0.0;
  if (range <= kHistBins)
    for (int j = threadIdx.x; j < range; j += blockDim.x) {
      const double c = (double)gh[j];
      if (c > 0) s += c * log2(c);
    }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bits[a] = (n > 0 ? (double)n * log2((double)n) : 0.0) - part[0];
}


// ------------------------------------------------------- output-bias initialisation
// Per attribute: sum of y (pass 0) and of |y - mean| (pass 1) in FP64, then the
// output bias of the Laplace head set to (mean, softplus^-1(max(MAD - step/16, step/4))).
__global__ __launch_bounds__(256) void k_rate_init_sum(int n, const float* __restrict__ attrs,
                                                       double* __restrict__ acc, int pass) {
  const int a = blockIdx.y;
  const float* y = attrs + (size_t)a * n;
  const double mean = pass ? acc[2 * a] / (double)n : 0.0;
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s += pass ? fabs((double)y[i] - mean) : (double)y[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(&acc[2 * a + pass], s);
}

__global__ void k_rate_init_bias(int n, int n_attr, const double* __restrict__ acc, float step,
                                 float* __restrict__ b) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_attr) return;
  const double mean = acc[2 * a] / (double)n, mad = acc[2 * a + 1] / (double)n;
  const double target = fmax(mad - step / 16.0, step / 4.0);
  float* ba = b + (size_t)a * kBPerAttr + 2 * kHid;
  ba[0] = (float)mean;
  ba[1] = (float)log(expm1(target));
}

// ---------------------------------------------------------------------- MLP
// One wave handles 32 symbols of one attribute at a time. MFMA operand layout
// (v_mfma_f32_32x32x16_bf16): lane l holds row / column (l & 31) and 8 values
// of the contraction index; accumulator element r of lane l is row
// 8 (r / 4) + 4 (l >> 5) + (r & 3), column (l & 31). Products are computed
// transposed (hidden units as rows, symbols as columns), so the accumulator
// of one layer, after bias + GELU + BF16 rounding, is directly the B operand
// of the next layer: its 8 values per K-step are the hidden units
// 16 ks + 8 (j / 4) + 4 (l >> 5) + (j & 3), and the weight (A) operand is
// gathered with the same permutation of the contraction index.
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;

struct RateArgs {
  int n, n_attr, mode, n_levels;
  float step;
  unsigned long long seed, offset;
  const unsigned long long* offset_dev;  // if set, the counter offset is read here at run time
  int lv[8];
  float wsym[8];  // per-symbol loss weight of each layer: lambda_rate lambda^l / |G^l|
  float wfit;     // per-symbol weight of the maximum-likelihood fit of the MLP weights
};

__device__ __forceinline__ bf16x8 pack8(const uint16_t* h) {
  uint4 u;
  u.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
  u.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  u.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
  u.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {  // 16-byte aligned
  return __builtin_bit_cast(bf16x8, *(const uint4*)p);
}
// W2 in LDS: row o2 padded to kW2Row BF16 (144 bytes: 16-byte reads of consecutive rows, and
// 16-bit reads of a column by two row groups 4 apart, touch distinct banks), column i at
// position w2_pos(i), i.e. bits 2 and 3 of i swapped, so that the eight contraction values a lane
// holds for one layer-2 K-step (i = 16 ks + 4 g + {0..3} and 16 ks + 8 + 4 g + {0..3}) are one
// contiguous 16-byte run.
constexpr int kW2Row = 72;
__device__ __forceinline__ int w2_pos(int i) { return (i & ~12) | ((i & 4) << 1) | ((i & 8) >> 1); }
// Eight values of column p of W2 (pointer at row 0 of the group): rows 0..3 and 8..11.
__device__ __forceinline__ bf16x8 load_col8(const uint16_t* p) {
  uint32_t u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r0 = 2 * j < 4 ? 2 * j : 2 * j + 4;
    u[j] = (uint32_t)p[r0 * kW2Row] | ((uint32_t)p[(r0 + 1) * kW2Row] << 16);
  }
  return __builtin_bit_cast(bf16x8, make_uint4(u[0], u[1], u[2], u[3]));
}

// tanh-approximated GELU, 0.5 x (1 + tanh(u)) with u = c (x + 0.044715 x^3), c = sqrt(2 / pi),
// evaluated as x * s with s = 0.5 (1 + tanh(u)) = 1 / (1 + e^{-2u}) on the hardware exp2 and
// reciprocal (absolute error ~1e-7, far below the BF16 rounding that follows).
constexpr float kGeluC = 0.7978845608028654f;
constexpr float kGeluE0 = -2.f * kGeluC * 1.4426950408889634f;  // e^{-2u} = 2^{x (E0 + E1 x^2)}
constexpr float kGeluE1 = kGeluE0 * 0.044715f;
__device__ __forceinline__ float gelu_s(float x) {
  const float e = __builtin_amdgcn_exp2f(x * fmaf(x * x, kGeluE1, kGeluE0));
  return __builtin_amdgcn_rcpf(1.f + e);
}
// d/dx [x s] = s + x s (1 - s) 2 u', with 2 u' = 2 c (1 + 3 * 0.044715 x^2), from s = gelu_s(x)
// (the training forward evaluates the sigmoid once for GELU and its derivative)
__device__ __forceinline__ float gelu_grad_s(float x, float s) {
  const float du2 = fmaf(x * x, 2.f * kGeluC * 3.f * 0.044715f, 2.f * kGeluC);
  return fmaf(x * du2, fmaf(-s, s, s), s);
}

// Staging slot (in BF16 elements) of row r, symbol s of a per-wave [R rows][32 symbols] tile kept
// chunk-major: the 16-byte chunk of symbols 8c..8c+7 of row r sits at chunk index R c + (r ^ c)
// (c < 4). An MFMA operand read (consecutive rows, one chunk) is then one contiguous run of
// 16-byte chunks, and a staging write (rows r and r + 4, all 32 symbols) spreads over distinct
// banks.
template <int R>
__device__ __forceinline__ int stg(int r, int s) {
  const int c = s >> 3;
  return (R * c + (r ^ c)) * 8 + (s & 7);
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// e^x and ln x on the hardware exp2 and log2 (about 1 ulp each), and 1 - e^{-x}, e^x - 1 for
// x >= 0 with a three-term series below 2^-5, where the difference would cancel (relative error
// below 2e-6 throughout): far inside the per-symbol accuracy the rate needs.
__device__ __forceinline__ float hw_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float hw_log(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ __forceinline__ float one_minus_exp_neg(float x) {
  return x < 0.03125f ? x * fmaf(x, fmaf(x, 1.f / 6.f, -0.5f), 1.f) : 1.f - hw_exp(-x);
}
__device__ __forceinline__ float exp_minus_one(float x) {
  return x < 0.03125f ? x * fmaf(x, fmaf(x, 1.f / 6.f, 0.5f), 1.f) : hw_exp(x) - 1.f;
}

// -log2 max(F(y + q/2) - F(y - q/2), 1e-9) for a Laplace(m, b) CDF F, and its
// derivatives with respect to y and b (zero where the floor binds).
__device__ __forceinline__ void laplace_bits(float y, float m, float b, float q, float& bits, float& dy, float& db) {
  const float h = 0.5f * q;
  const float d = y - m;
  const float t = fabsf(d);
  // divisions by b, b^2 and P as products with hardware reciprocals (b >= q/16 > 0, P >= 1e-9 where
  // used): their ~1 ulp is far inside the per-symbol accuracy the rate needs
  const float rb = __builtin_amdgcn_rcpf(b);
  const float qb = q * rb;
  float lp, dlt, dlb;
  if (t >= h) {
    const float th = (t - h) * rb;
    lp = -kLn2 - th + hw_log(one_minus_exp_neg(qb));
    dlt = -rb;
    dlb = rb * (th - qb * __builtin_amdgcn_rcpf(exp_minus_one(qb)));
  } else {
    const float ea = hw_exp(-(h + t) * rb), eb = hw_exp(-(h - t) * rb);
    const float P = 1.f - 0.5f * ea - 0.5f * eb;
    lp = hw_log(P);
    const float rP = __builtin_amdgcn_rcpf(P);
    dlt = 0.5f * rb * (ea - eb) * rP;
    dlb = -0.5f * rb * rb * (ea * (h + t) + eb * (h - t)) * rP;
  }
  const float lfloor = -20.723265836946411f;  // ln 1e-9
  if (!(lp >= lfloor)) {
    bits = -lfloor * kLog2e;
    dy = 0.f;
    db = 0.f;
    return;
  }
  bits = -lp * kLog2e;
  const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
  dy = -dlt * sg * kLog2e;
  db = -dlb * kLog2e;
}

// Accumulator rows of the lane (o = 32 h + 8 (r / 4) + 4 g + (r & 3), r = 0..15) of a bias vector,
// so that a layer's MFMA starts from its bias: four 16-byte LDS reads.
__device__ __forceinline__ f32x16 bias_rows(const float* b, int h, int g) {
  f32x16 v;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 x = *(const float4*)&b[32 * h + 8 * q + 4 * g];
    v[4 * q] = x.x;
    v[4 * q + 1] = x.y;
    v[4 * q + 2] = x.z;
    v[4 * q + 3] = x.w;
  }
  return v;
}

struct RateShared {
  uint16_t w2[kHid * kW2Row];  // [o2][w2_pos(i)], rows padded
  float w3[2 * kHid];
  float b1[kHid], b2[kHid], b3[2];
};
struct RateWaveTmp {           // transposed per-wave staging for the weight gradients (slots: stg)
  uint16_t h1[kHid * 32];      // rows i, 32 symbols
  uint16_t h2[kHid * 32];      // rows o2
  uint16_t d2[kHid * 32];      // rows o2
  uint16_t d1[kHid * 32];      // rows i
  uint16_t x[kCtx * 32];       // rows f
  uint16_t dout[2 * 32];       // [r][s], BF16 (the operand of the layer-3 weight gradient)
};

// Two waves per SIMD (two blocks per CU): at most 256 registers per lane and 80 KB of LDS per block.
template <bool GRAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rate_mlp(RateArgs ra, const float* __restrict__ attrs,
                                                  const uint16_t* __restrict__ ctx, const uint16_t* __restrict__ W,
                                                  const float* __restrict__ Bv, double* __restrict__ bits_out,
                                                  double* __restrict__ loss_out, float* __restrict__ sym_bits,
                                                  float* __restrict__ d_attrs, float* __restrict__ d_w,
                                                  float* __restrict__ d_b) {
  // the weights in a static LDS array of their own, the staging in the dynamic one: the compiler
  // then knows that staging stores leave the weights unchanged, and schedules weight reads early
  __shared__ __align__(16) RateShared sh;
  extern __shared__ __align__(16) char smem[];
  RateWaveTmp* wt = (RateWaveTmp*)smem;
  const int a = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sl = lane & 31, g = lane >> 5;
  const uint16_t* Wa = W + (size_t)a * kWPerAttr;
  const float* Ba = Bv + (size_t)a * kBPerAttr;
  for (int j = tid; j < kW2; j += 256) sh.w2[(j >> 6) * kW2Row + w2_pos(j & 63)] = Wa[kW1 + j];
  // the layer-1 weight operand (rows 32 h + sl of W1, contraction slots 8 g ..): in registers when
  // training (the staging area leaves no LDS for it), else in LDS after the shared weights
  bf16x8 w1f[2];
  uint16_t* w1s = (uint16_t*)wt;
  if constexpr (GRAD) {
    w1f[0] = load8(Wa + sl * kCtx + 8 * g);
    w1f[1] = load8(Wa + (32 + sl) * kCtx + 8 * g);
  } else {
    for (int j = tid; j < kW1; j += 256) w1s[j] = Wa[j];
  }
  for (int j = tid; j < kW3; j += 256) sh.w3[j] = bf16_to_f32(Wa[kW1 + kW2 + j]);
  if (tid < kHid) {
    sh.b1[tid] = Ba[tid];
    sh.b2[tid] = Ba[kHid + tid];
  }
  if (tid < 2) sh.b3[tid] = Ba[2 * kHid + tid];
  __syncthreads();

  const int n = ra.n;
  const float q = ra.step;
  const float* ya = attrs + (size_t)a * n;
  const int nchunks = (n + 31) / 32;
  const int per_iter = gridDim.x * 4;
  const int iters = (nchunks + per_iter - 1) / per_iter;
  float bits_acc = 0.f, loss_acc = 0.f;
  // Weight gradients are split over the block's four waves: wave w accumulates rows 16w..16w+15
  // of dW2 and dW1 and columns 16w..16w+15 of dW3, over the symbols of all four waves (their
  // staged activations are read from LDS), so each wave holds 24 accumulators instead of 96.
  f32x4 acc2[4], acc1, acc3, accb1, accb2;  // accb: bias sums (every column holds them)
  float db30 = 0.f, db31 = 0.f;
  if constexpr (GRAD) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc2[u][r] = 0.f;
      acc1[r] = 0.f;
      acc3[r] = 0.f;
      accb1[r] = 0.f;
      accb2[r] = 0.f;
    }
  }
  RateWaveTmp& T = wt[wave];
  float* gp1s = (float*)T.d2;  // spans d2 and d1
  const f32x16 zero16 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

  // the context features and the attribute value of a chunk's symbol, loaded one chunk ahead
  auto fetch = [&](int it, bf16x8& x, float& y) {
    const int s = ((it * gridDim.x + blockIdx.x) * 4 + wave) * 32 + sl;
    const bool v = it < iters && s < n;
    x = v ? load8(ctx + (size_t)s * kCtx + 8 * g) : __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    y = v ? ya[s] : 0.f;
  };
  bf16x8 bx_next;
  float y_next;
  fetch(0, bx_next, y_next);
  for (int it = 0; it < iters; ++it) {
    // Weights, biases and operand fragments are re-read from LDS every chunk rather than held in
    // registers across the loop (holding all of them would exceed the register file).
    asm volatile("" ::: "memory");
    const int chunk = (it * gridDim.x + blockIdx.x) * 4 + wave;
    const int sidx = chunk * 32 + sl;
    const bool valid = sidx < n;
    const bf16x8 bx = bx_next;
    const float y_sym = y_next;
    fetch(it + 1, bx_next, y_next);
    // ---- layer 1: Z1^T (64 x 32) = W1 (64 x 16) X^T (16 x 32)
    f32x16 c1[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
      c1[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(GRAD ? w1f[h] : load8(&w1s[(32 * h + sl) * kCtx + 8 * g]), bx,
                                                      bias_rows(sh.b1, h, g), 0, 0, 0);
    // GELU + BF16 (the MFMA started from the bias), packed straight into the B operand of layer 2
    uint32_t b2[4][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int o = 32 * h + 8 * (r >> 2) + 4 * g + (r & 3);  // o + 1 for r + 1
        const float x0 = c1[h][r], x1 = c1[h][r + 1];
        const float s0 = gelu_s(x0), s1 = gelu_s(x1);
        const uint32_t hp = f32x2_to_bf16x2(x0 * s0, x1 * s1);
        if constexpr (GRAD) {
          // GELU'(Z1) from the same sigmoid, kept in the wave's d2 | d1 staging area (8 KB, unused
          // until the backward) as [value r][lane] until dZ1 is formed
          gp1s[(16 * h + r) * 64 + lane] = gelu_grad_s(x0, s0);
          gp1s[(16 * h + r + 1) * 64 + lane] = gelu_grad_s(x1, s1);
          store_pair(T.h1, stg<kHid>(o, sl), stg<kHid>(o + 1, sl), hp);
        }
        b2[2 * h + (r >> 3)][(r & 7) >> 1] = hp;
      }
    // ---- layer 2: Z2^T (64 x 32) = W2 (64 x 64) H1^T (64 x 32), K in 4 steps of 16
    // (the two row halves alternate, so that consecutive MFMAs are independent)
    f32x16 c2[2] = {bias_rows(sh.b2, 0, g), bias_rows(sh.b2, 1, g)};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2)
        c2[h2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            load8(&sh.w2[(32 * h2 + sl) * kW2Row + 16 * ks + 8 * g]),
            __builtin_bit_cast(bf16x8, make_uint4(b2[ks][0], b2[ks][1], b2[ks][2], b2[ks][3])), c2[h2], 0, 0, 0);
    // ---- GELU; layer 3 (2 outputs) on the VALU, each lane holds half the hidden units
    float o0 = 0.f, o1 = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int o2 = 32 * h + 8 * (r >> 2) + 4 * g + (r & 3);  // o2 + 1 for r + 1
        const float z0 = c2[h][r], z1 = c2[h][r + 1];
        const float s0 = gelu_s(z0), s1 = gelu_s(z1);
        if constexpr (GRAD) {  // keep GELU'(Z2) for the backward
          c2[h][r] = gelu_grad_s(z0, s0);
          c2[h][r + 1] = gelu_grad_s(z1, s1);
        }
        const uint32_t hp = f32x2_to_bf16x2(z0 * s0, z1 * s1);
        if constexpr (GRAD) {
          store_pair(T.h2, stg<kHid>(o2, sl), stg<kHid>(o2 + 1, sl), hp);
        }
        o0 = fmaf(sh.w3[o2], __uint_as_float(hp << 16), o0);
        o1 = fmaf(sh.w3[kHid + o2], __uint_as_float(hp << 16), o1);
        o0 = fmaf(sh.w3[o2 + 1], __uint_as_float(hp & 0xFFFF0000u), o0);
        o1 = fmaf(sh.w3[kHid + o2 + 1], __uint_as_float(hp & 0xFFFF0000u), o1);
      }
    o0 += __shfl_xor(o0, 32);
    o1 += __shfl_xor(o1, 32);
    o0 += sh.b3[0];
    o1 += sh.b3[1];
    // ---- discretised Laplace rate of the symbol
    const float m = o0;
    const float sp = fmaxf(o1, 0.f) + hw_log(1.f + hw_exp(-fabsf(o1)));  // softplus
    const float bsc = sp + q * (1.f / 16.f);
    float bits = 0.f, dby = 0.f, dbb = 0.f, wsym = 0.f;
    if (valid) {
      const float y = y_sym;
      float yh;
      if (ra.mode == 0) {
        yh = rintf(y / q) * q;
      } else {
        const unsigned long long off = ra.offset_dev ? *ra.offset_dev : ra.offset;
        const unsigned long long ctr = off + (unsigned long long)a * (unsigned long long)n +
                                       (unsigned long long)sidx + 1ull;
        const unsigned long long zz = splitmix64(ra.seed + ctr * 0x9E3779B97F4A7C15ull);
        const float u = (float)(uint32_t)(zz >> 40) * (1.0f / 16777216.0f) - 0.5f;
        yh = y + u * q;
      }
      laplace_bits(yh, m, bsc, q, bits, dby, dbb);
      int layer = 0;
      for (int l = 0; l < ra.n_levels - 1; ++l)
        if (sidx >= ra.lv[l]) layer = l + 1;
      wsym = ra.wsym[layer];
      if (g == 0) {
        bits_acc += bits;
        loss_acc += wsym * bits;
        if (sym_bits) sym_bits[(size_t)a * n + sidx] = bits;
        if (ra.mode == 1 && d_attrs) d_attrs[(size_t)a * n + sidx] += wsym * dby;
      }
    }
    if constexpr (GRAD) {
      const float dout0 = valid ? -ra.wfit * dby : 0.f;
      const float sig1 = __builtin_amdgcn_rcpf(1.f + __expf(-o1));
      const float dout1 = valid ? ra.wfit * dbb * sig1 : 0.f;
      // dH2^T (64 x 32) = W3^T (64 x 2) dout (2 x 32) on the FP32 MFMA (v_mfma_f32_32x32x2_f32: lane l
      // gives A row l & 31 and B column l & 31 at K = l >> 5, i.e. W3 row g and dout_g of the lane's
      // symbol; the accumulator has the rows of c2), then dZ2 = dH2 * GELU'(Z2), packed into the B
      // operand of dH1^T = W2^T dZ2^T
      f32x16 dh[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
        dh[h] = __builtin_amdgcn_mfma_f32_32x32x2f32(sh.w3[g * kHid + 32 * h + sl], g ? dout1 : dout0, zero16, 0, 0, 0);
      uint32_t bd[4][4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          bd[2 * h + (r >> 3)][(r & 7) >> 1] = f32x2_to_bf16x2(dh[h][r] * c2[h][r], dh[h][r + 1] * c2[h][r + 1]);
        }
      f32x16 c3[2];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
        for (int hi = 0; hi < 2; ++hi) {
          // W2^T rows i, K = o2 in the order 16 ks + 4 g + {0..3, 8..11}: a column of W2
          const uint16_t* col = &sh.w2[(16 * ks + 4 * g) * kW2Row + 32 * hi + w2_pos(sl)];
          c3[hi] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              load_col8(col), __builtin_bit_cast(bf16x8, make_uint4(bd[ks][0], bd[ks][1], bd[ks][2], bd[ks][3])),
              ks == 0 ? zero16 : c3[hi], 0, 0, 0);
        }
      }
      // dZ1 = dH1 * GELU'(Z1): every stashed value is read before the d1 and d2 staging writes
      // that reuse its memory (LDS operations of a wave complete in order)
      float gp1[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) gp1[j] = gp1s[j * 64 + lane];
      asm volatile("" ::: "memory");
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int u = 32 * h + 8 * (r >> 2) + 4 * g + (r & 3);  // u + 1 for r + 1
          const uint32_t dp = f32x2_to_bf16x2(c3[h][r] * gp1[16 * h + r], c3[h][r + 1] * gp1[16 * h + r + 1]);
          store_pair(T.d1, stg<kHid>(u, sl), stg<kHid>(u + 1, sl), dp);
        }
      // dZ2 into its staging rows (the B operand above holds it packed)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int o2 = 32 * h + 8 * (r >> 2) + 4 * g + (r & 3);
          const uint32_t dp = bd[2 * h + (r >> 3)][(r & 7) >> 1];
          store_pair(T.d2, stg<kHid>(o2, sl), stg<kHid>(o2 + 1, sl), dp);
        }
      {
        const uint4 xv = __builtin_bit_cast(uint4, bx);
        const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) T.x[stg<kCtx>(8 * g + j, sl)] = (uint16_t)(xs[j >> 1] >> (16 * (j & 1)));
      }
      if (g == 0) {
        T.dout[sl] = f32_to_bf16(dout0);
        T.dout[32 + sl] = f32_to_bf16(dout1);
        db30 += dout0;
        db31 += dout1;
      }
      __syncthreads();
      // This wave's slices of the weight gradients over the 4 x 32 symbols of the block
      // (v_mfma_f32_16x16x32_bf16: lane l holds A row / B column l & 15 and K slots 8 (l >> 4) ..).
      //   dW2 rows 16w.. (16 x 64) += dZ2^T (16 x 32 s) H1 (32 s x 64)
      //   dW1 rows 16w.. (16 x 16) += dZ1^T (16 x 32 s) X (32 s x 16)
      //   dW3 columns 16w.. (2 x 16, rows padded to 16) += dout^T (2 x 32 s) H2 (32 s x 16)
      //   db2, db1 rows 16w.. += dZ2^T, dZ1^T (16 x 32 s) times a matrix of ones (32 s x 16)
      {
        const int r16 = lane & 15, g16 = lane >> 4;
        const int row = 16 * wave + r16;
        const bf16x8 ones = __builtin_bit_cast(bf16x8, make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u));
#pragma unroll
        for (int src = 0; src < 4; ++src) {
          const RateWaveTmp& S = wt[src];
          const bf16x8 a2 = load8(&S.d2[stg<kHid>(row, 8 * g16)]);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
            acc2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, load8(&S.h1[stg<kHid>(16 * nt + r16, 8 * g16)]),
                                                                acc2[nt], 0, 0, 0);
          accb2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, ones, accb2, 0, 0, 0);
          const bf16x8 a1 = load8(&S.d1[stg<kHid>(row, 8 * g16)]);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, load8(&S.x[stg<kCtx>(r16, 8 * g16)]), acc1, 0, 0, 0);
          accb1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, ones, accb1, 0, 0, 0);
          const bf16x8 ad = r16 < 2 ? load8(&S.dout[r16 * 32 + 8 * g16])
                                    : __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
          acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ad, load8(&S.h2[stg<kHid>(row, 8 * g16)]), acc3, 0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  // ---- block reductions
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    bits_acc += __shfl_xor(bits_acc, off);
    loss_acc += __shfl_xor(loss_acc, off);
  }
  __shared__ float red[2][4];
  if (lane == 0) {
    red[0][wave] = bits_acc;
    red[1][wave] = loss_acc;
  }
  __syncthreads();
  if (tid == 0) {
    const float bsum = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const float lsum = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    atomicAdd(bits_out + a, (double)bsum);
    if (loss_out) atomicAdd(loss_out, (double)lsum);
  }
  if constexpr (GRAD) {
    // the waves' slices are disjoint (the output-layer bias sums of the four waves are added in
    // LDS, reusing the staging area), then one atomic per value
    float* acc = (float*)wt;
    for (int j = tid; j < kWPerAttr + kBPerAttr; j += 256) acc[j] = 0.f;
    __syncthreads();
    {
      const int r16 = lane & 15, g16 = lane >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * wave + 4 * g16 + r;  // output row of this accumulator value
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[kW1 + o * kHid + 16 * nt + r16] = acc2[nt][r];
        acc[o * kCtx + r16] = acc1[r];
        if (4 * g16 + r < 2) acc[kW1 + kW2 + (4 * g16 + r) * kHid + 16 * wave + r16] = acc3[r];
        if (r16 == 0) {
          acc[kWPerAttr + o] = accb1[r];
          acc[kWPerAttr + kHid + o] = accb2[r];
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      db30 += __shfl_xor(db30, off);
      db31 += __shfl_xor(db31, off);
    }
    if (lane == 0) {
      atomicAdd(&acc[kWPerAttr + 2 * kHid], db30);
      atomicAdd(&acc[kWPerAttr + 2 * kHid + 1], db31);
    }
    __syncthreads();
    if (d_w)
      for (int j = tid; j < kWPerAttr; j += 256)
        if (acc[j] != 0.f) unsafeAtomicAdd(d_w + (size_t)a * kWPerAttr + j, acc[j]);
    if (d_b)
      for (int j = tid; j < kBPerAttr; j += 256)
        if (acc[kWPerAttr + j] != 0.f) unsafeAtomicAdd(d_b + (size_t)a * kBPerAttr + j, acc[kWPerAttr + j]);
  }
}

// --------------------------------------------------------------------- Adam
__global__ __launch_bounds__(256) void k_adam(long long n, float* __restrict__ p, float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              uint16_t* __restrict__ bf16_copy, float lr, float b1, float b2,
                                              float eps, float c1, float c2, const int* __restrict__ step_dev) {
  if (step_dev) {  // the bias corrections of the step number held on the device
    const float t = (float)*step_dev;
    c1 = 1.f - powf(b1, t);
    c2 = 1.f - powf(b2, t);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    g[i] = 0.f;
    if (bf16_copy) bf16_copy[i] = f32_to_bf16(pi);
  }
}

// Step number += 1 and noise counter offset += delta, on the device (for captured steps).
__global__ void k_advance(int* __restrict__ step, unsigned long long* __restrict__ offset, unsigned long long delta) {
  if (threadIdx.x == 0) {
    if (step) *step += 1;
    if (offset) *offset += delta;
  }
}

}  // namespace
}  // namespace gs

using namespace gs;

// ------------------------------------------------ histogram without allocation
// Scratch for gs_rate_histogram_noalloc: the same layout as the workspace of
// gs_rate_histogram for up to kNoAllocMaxAttr attributes. Each GPU the library
// runs on holds its own copy until the process ends. Host code never passes
// the array's name to a kernel (on the host it is only a stand-in): it uses
// the device address hipGetSymbolAddress returns, looked up once per device
// with that device current and kept in g_noalloc_ptr.
constexpr int kNoAllocMaxAttr = 64;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocMaxAttr * 8 + (size_t)kNoAllocMaxAttr * kHistBins * 4;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of this device's scratch, set up on the first call on the device.
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return GS_ERR_NO_DEVICE;
  if (dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GS_ERR_HIP;
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return GS_OK;
}
}  // namespace

namespace {

// The histogram rate on a workspace w laid out as gs_rate_histogram_workspace_size states:
// status word, per-attribute symbol range, per-attribute bins.
int hist_launch(int32_t n, int32_t n_attr, const float* attrs, float step, double* bits_out, char* w,
                hipStream_t st) {
  uint32_t* err = (uint32_t*)w;
  int* mm = (int*)(w + 256);
  uint32_t* hist = (uint32_t*)(w + 256 + (size_t)n_attr * 8);
  if (launch_zero(w, 256, st) != hipSuccess) return GS_ERR_HIP;
  if (launch_zero(hist, (size_t)n_attr * kHistBins * 4, st) != hipSuccess) return GS_ERR_HIP;
  {
    ProfScope ps_(K_RATE_HIST_MINMAX, st);
    hipLaunchKernelGGL(k_hist_init, dim3((n_attr + 63) / 64), dim3(64), 0, st, n_attr, mm);
    if (n > 0)
      hipLaunchKernelGGL(k_hist_minmax, dim3(std::min(64, (n + 255) / 256), n_attr), dim3(256), 0, st, n, attrs,
                         step, mm);
  }
  if (n > 0) {
    ProfScope ps_(K_RATE_HIST_COUNT, st);
    hipLaunchKernelGGL(k_hist_count, dim3(std::min(32, (n + 255) / 256), n_attr), dim3(256), 0, st, n, attrs, step,
                       mm, hist, err);
  }
  {
    ProfScope ps_(K_RATE_HIST_BITS, st);
    hipLaunchKernelGGL(k_hist_bits, dim3(n_attr), dim3(256), 0, st, n, mm, hist, bits_out);
  }
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
}  // namespace


extern "C" {

int gs_rate_context(int32_t n, const float* means, float extent, int32_t n_levels, const int32_t* level_counts,
                    uint16_t* ctx_out, void* stream) {
  if (n < 0 || !means || !ctx_out || !(extent > 0.f) || n_levels < 1 || n_levels > 8 || !level_counts)
    return GS_ERR_INVALID_ARG;
  if (n == 0) return GS_OK;
  int lv[8];
  for (int l = 0; l < 8; ++l) lv[l] = l < n_levels ? level_counts[l] : n;
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps_(K_RATE_CTX, st);
  hipLaunchKernelGGL(k_rate_ctx, dim3((n + 255) / 256), dim3(256), 0, st, n, means, extent, n_levels,
                     make_int4(lv[0], lv[1], lv[2], lv[3]), make_int4(lv[4], lv[5], lv[6], lv[7]), ctx_out);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_rate_histogram_workspace_size(int32_t n_attr, size_t* bytes_out) {
  if (n_attr < 1 || !bytes_out) return GS_ERR_INVALID_ARG;
  *bytes_out = 256 + (size_t)n_attr * 8 + (size_t)n_attr * kHistBins * 4;
  return GS_OK;
}


int gs_rate_histogram(int32_t n, int32_t n_attr, const float* attrs, float step, double* bits_out, void* ws,
                      size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (n < 0 || n_attr < 1 || !attrs || !bits_out || !ws || !(step > 0.f)) return GS_ERR_INVALID_ARG;
  gs_rate_histogram_workspace_size(n_attr, &need);
  if (ws_bytes < need) return GS_ERR_WORKSPACE;
  return hist_launch(n, n_attr, attrs, step, bits_out, (char*)ws, (hipStream_t)stream);
}


int gs_rate_histogram_noalloc(int32_t n, int32_t n_attr, const float* attrs, float step, double* bits_out,
                              void* stream) {
  if (n < 0 || n_attr < 1 || !attrs || !bits_out || !(step > 0.f)) return GS_ERR_INVALID_ARG;
  if (n_attr > kNoAllocMaxAttr) return GS_ERR_INVALID_ARG;
  void* w = nullptr;
  const int rc = noalloc_scratch(&w);
  if (rc != GS_OK) return rc;
  return hist_launch(n, n_attr, attrs, step, bits_out, (char*)w, (hipStream_t)stream);
}


int gs_rate_init_output_bias(int32_t n, int32_t n_attr, const float* attrs, float step, float* b_f32, double* acc,
                             void* stream) {
  if (n < 1 || n_attr < 1 || !attrs || !b_f32 || !acc || !(step > 0.f)) return GS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (launch_zero(acc, (size_t)n_attr * 2 * sizeof(double), st) != hipSuccess) return GS_ERR_HIP;
  const dim3 grid(std::min(64, (n + 255) / 256), n_attr);
  for (int pass = 0; pass < 2; ++pass) hipLaunchKernelGGL(k_rate_init_sum, grid, dim3(256), 0, st, n, attrs, acc, pass);
  hipLaunchKernelGGL(k_rate_init_bias, dim3((n_attr + 63) / 64), dim3(64), 0, st, n, n_attr, acc, step, b_f32);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_rate_model(const gs_rate_desc* desc, const float* attrs, const uint16_t* ctx, const uint16_t* w_bf16,
                  const float* b_f32, double* bits_out, double* loss_out, float* sym_bits, float* d_attrs, float* d_w,
                  float* d_b, void* stream) {
  if (!desc || !attrs || !ctx || !w_bf16 || !b_f32 || !bits_out) return GS_ERR_INVALID_ARG;
  const gs_rate_desc& d = *desc;
  if (d.n < 0 || d.n_attr < 1 || !(d.step > 0.f) || (d.mode != 0 && d.mode != 1)) return GS_ERR_INVALID_ARG;
  if (d.n_levels < 1 || d.n_levels > 8 || d.level_counts[d.n_levels - 1] != d.n) return GS_ERR_INVALID_ARG;
  for (int l = 1; l < d.n_levels; ++l)
    if (d.level_counts[l] < d.level_counts[l - 1] || d.level_counts[l - 1] < 0) return GS_ERR_INVALID_ARG;
  if (d.n == 0) return GS_OK;
  RateArgs ra;
  ra.n = d.n; ra.n_attr = d.n_attr; ra.mode = d.mode; ra.n_levels = d.n_levels; ra.step = d.step;
  ra.seed = d.seed; ra.offset = d.offset; ra.offset_dev = (const unsigned long long*)d.offset_dev;
  ra.wfit = d.fit_scale;
  int prev = 0;
  for (int l = 0; l < 8; ++l) {
    ra.lv[l] = l < d.n_levels ? d.level_counts[l] : d.n;
    const int cnt = l < d.n_levels ? d.level_counts[l] - prev : 0;
    ra.wsym[l] = cnt > 0 ? d.lambda_rate * d.level_weights[l] / (float)cnt : 0.f;
    if (l < d.n_levels) prev = d.level_counts[l];
  }
  const bool grad = d_w || d_b;
  const int nchunks = (d.n + 31) / 32;
  const int nb = std::max(1, std::min(d.blocks_per_attr > 0 ? d.blocks_per_attr : 64, (nchunks + 3) / 4));
  const size_t lds = grad ? 4 * sizeof(RateWaveTmp) : (size_t)kW1 * sizeof(uint16_t);
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps_(K_RATE_MLP, st);
  if (grad)
    hipLaunchKernelGGL(k_rate_mlp<true>, dim3(nb, d.n_attr), dim3(256), lds, st, ra, attrs, ctx, w_bf16, b_f32,
                       bits_out, loss_out, sym_bits, d_attrs, d_w, d_b);
  else
    hipLaunchKernelGGL(k_rate_mlp<false>, dim3(nb, d.n_attr), dim3(256), lds, st, ra, attrs, ctx, w_bf16, b_f32,
                       bits_out, loss_out, sym_bits, d_attrs, d_w, d_b);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_adam_step(int64_t n, float* params, float* grads, float* m, float* v, uint16_t* bf16_copy, float lr,
                 float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (n < 0 || !params || !grads || !m || !v || step < 1) return GS_ERR_INVALID_ARG;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  ProfScope ps_(K_ADAM, st);
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, st, (long long)n, params, grads, m, v, bf16_copy, lr, beta1,
                     beta2, eps, c1, c2, (const int*)nullptr);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_adam_step_dev(int64_t n, float* params, float* grads, float* m, float* v, uint16_t* bf16_copy, float lr,
                     float beta1, float beta2, float eps, const int32_t* step_dev, void* stream) {
  if (n < 0 || !params || !grads || !m || !v || !step_dev) return GS_ERR_INVALID_ARG;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  ProfScope ps_(K_ADAM, st);
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, st, (long long)n, params, grads, m, v, bf16_copy, lr, beta1,
                     beta2, eps, 1.f, 1.f, (const int*)step_dev);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_advance_counters(int32_t* step_dev, uint64_t* offset_dev, uint64_t offset_delta, void* stream) {
  if (!step_dev && !offset_dev) return GS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, (hipStream_t)stream, (int*)step_dev,
                     (unsigned long long*)offset_dev, (unsigned long long)offset_delta);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"

int gs_rate_autotune(const gs_rate_desc* desc, const float* attrs, const uint16_t* ctx, const uint16_t* w_bf16,
                     const float* b_f32, double* bits_scratch, float* d_attrs, float* d_w, float* d_b, void* stream,
                     int32_t* best_blocks, float* times_ms) {
  constexpr int kCand = 5;
  static const int32_t cand[kCand] = {16, 32, 64, 128, 256};
  if (!desc || !bits_scratch || !best_blocks) return GS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int A = desc->n_attr;
  if (A < 1) return GS_ERR_INVALID_ARG;
  std::vector<double> ref(A), got(A);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GS_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);  // clean-up: the creation error is the one reported
    return GS_ERR_HIP;
  }
  int rc = GS_OK;
  float best_t = -1.f;
  int32_t best = 0;
  for (int c = 0; c < kCand && rc == GS_OK; ++c) {
    gs_rate_desc dc = *desc;
    dc.blocks_per_attr = cand[c];
    double* bits = bits_scratch + (size_t)c * A;
    if (hipMemsetAsync(bits, 0, sizeof(double) * A, st) != hipSuccess) { rc = GS_ERR_HIP; break; }
    rc = gs_rate_model(&dc, attrs, ctx, w_bf16, b_f32, bits, nullptr, nullptr, d_attrs, d_w, d_b, stream);
    if (rc != GS_OK) break;
    if (hipMemcpyAsync(got.data(), bits, sizeof(double) * A, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) { rc = GS_ERR_HIP; break; }
    bool agree = true;
    if (c == 0) {
      ref = got;
    } else {
      for (int a = 0; a < A; ++a)
        if (!(std::fabs(got[a] - ref[a]) <= 1e-5 * std::fabs(ref[a]) + 1e-6)) agree = false;
    }
    if (hipEventRecord(e0, st) != hipSuccess) { rc = GS_ERR_HIP; break; }
    for (int r = 0; r < 3 && rc == GS_OK; ++r)
      rc = gs_rate_model(&dc, attrs, ctx, w_bf16, b_f32, bits, nullptr, nullptr, d_attrs, d_w, d_b, stream);
    if (rc != GS_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = GS_ERR_HIP; break; }
    ms /= 3.f;
    if (times_ms) times_ms[c] = agree ? ms : -1.f;
    if (agree && (best_t < 0.f || ms < best_t)) {
      best_t = ms;
      best = cand[c];
    }
  }
  // clean-up of the timing events; the trials' own status is what this call reports
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == GS_OK) *best_blocks = best;
  return rc;
}
