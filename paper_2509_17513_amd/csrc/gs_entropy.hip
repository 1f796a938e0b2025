// The paper's entropy models of the quantised attributes (Sec. 3.3): the KDE rate of keyframe
// attributes (Silverman bandwidth, the CDF through a convolution of the binned symbols with the
// kernel's CDF, the PMF as CDF differences one step apart) and the Gaussian rate (mean and
// variance of the symbols) with the temporal L1 term of residual attributes.
//
// Work is split into (layer, attribute) segments, each cut into chunks of kChunk symbols:
//  stats     per chunk: min, max, sum and sum of squares of the symbols (FP64) -> partials
//  setup     per segment, summing its chunks in order (deterministic): bandwidth and grid (KDE),
//            or mean and standard deviation (Gaussian)
//  hist      (KDE) per chunk: linear binning into an LDS histogram of fixed-point weights
//            (2^-16 of a symbol, the two weights of a symbol summing to exactly one), flushed with
//            integer atomics, so the counts do not depend on the order of the atomics
//  cdf       (KDE) per segment: prefix sums of the counts and the windowed convolution with the
//            kernel's CDF (FP64; the kernel is 0 or 1 to FP64 precision beyond 8 bandwidths)
//  eval      per symbol: bits, the gradient, per-chunk partial sums
//  finalize  per attribute bits and the loss, summed in a fixed order
//  grad      (Gaussian) per symbol: the gradient terms through the mean and deviation, and the
//            sign of the temporal L1 term
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kChunk = 8192;      // symbols per block
constexpr int kGridMax = 16384;   // CDF grid points per segment
constexpr int kKernMax = 3071;    // kernel half-width in grid points (its CDF table fits LDS)
constexpr double kFloor = 1e-9;   // PMF floor
constexpr double kLn2 = 0.69314718055994530942;
constexpr uint32_t kFix = 65536;  // fixed-point units per symbol in the histogram

struct EntDims {
  int n, A, L, kind, mode;
  float q;
  unsigned long long seed, offset;
  int lv[kMaxLevels + 1];          // symbol ranges of the layers
  int cb[kMaxLevels + 1];          // first chunk of each layer (per attribute); cb[L] = chunks
  float lw[kMaxLevels];
  float lambda_rate, lambda_reg;
};

struct Seg {
  double h, lo, delta;  // KDE grid
  double mu, sd, sigma; // Gaussian
  double w;             // symbol weight lambda_rate lambda^l / m
  double d_mu, d_sig;   // Gaussian: sum_i w dbits_i/dmu, sum_i w dbits_i/dsigma
  int G, K, m, pad;
};

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Symbol of attribute a of Gaussian i: quantised (mode 0) or with uniform noise of one step
// (mode 1, counter offset + a n + i + 1), rounded like the attributes (FP32, no contraction).
__device__ __forceinline__ float symbol(const EntDims& d, const float* __restrict__ attrs, int a, int i) {
  const float y = attrs[(size_t)a * d.n + i];
  if (d.mode == 0) return __fmul_rn(rintf(y / d.q), d.q);
  const unsigned long long ctr = d.offset + (unsigned long long)a * (unsigned long long)d.n + (unsigned long long)i + 1ull;
  const unsigned long long z = splitmix64(d.seed + ctr * 0x9E3779B97F4A7C15ull);
  const float u = (float)(uint32_t)(z >> 40) * (1.0f / 16777216.0f) - 0.5f;
  return __fadd_rn(y, __fmul_rn(u, d.q));
}

// Layer of a chunk and the chunk's symbol range.
__device__ __forceinline__ bool chunk_range(const EntDims& d, int c, int& l, int& i0, int& i1) {
  l = -1;
  for (int k = 0; k < d.L; ++k)
    if (c >= d.cb[k] && c < d.cb[k + 1]) l = k;
  if (l < 0) return false;
  i0 = d.lv[l] + (c - d.cb[l]) * kChunk;
  i1 = min(i0 + kChunk, d.lv[l + 1]);
  return true;
}

template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T r = sh[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = op(r, sh[k]);
  return r;
}

struct Max {
  __device__ double operator()(double a, double b) const { return a > b ? a : b; }
};
struct Min {
  __device__ double operator()(double a, double b) const { return a < b ? a : b; }
};
struct Add {
  __device__ double operator()(double a, double b) const { return a + b; }
};

// partials [A][chunks][4]
__global__ __launch_bounds__(256) void k_ent_stats(EntDims d, const float* __restrict__ attrs,
                                                   double* __restrict__ part) {
  __shared__ double sh[4];
  const int c = blockIdx.x, a = blockIdx.y;
  int l, i0, i1;
  if (!chunk_range(d, c, l, i0, i1)) return;
  double mn = 1e300, mx = -1e300, s1 = 0.0, s2 = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double y = symbol(d, attrs, a, i);
    mn = fmin(mn, y);
    mx = fmax(mx, y);
    s1 += y;
    s2 += y * y;
  }
  mn = block_reduce(mn, Min(), sh);
  mx = block_reduce(mx, Max(), sh);
  s1 = block_reduce(s1, Add(), sh);
  s2 = block_reduce(s2, Add(), sh);
  if (threadIdx.x == 0) {
    double* p = part + ((size_t)a * d.cb[d.L] + c) * 4;
    p[0] = mn;
    p[1] = mx;
    p[2] = s1;
    p[3] = s2;
  }
}

// Sum over a segment's chunks by one wave: lane j takes chunks j, j + 64, ..., then a fixed
// butterfly, so the result does not depend on scheduling.
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per (layer, attribute) segment.
__global__ __launch_bounds__(64) void k_ent_setup(EntDims d, const double* __restrict__ part, Seg* __restrict__ seg) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int l = s / d.A, a = s - l * d.A;
  double mn = 1e300, mx = -1e300, s1 = 0.0, s2 = 0.0;
  for (int c = d.cb[l] + lane; c < d.cb[l + 1]; c += 64) {
    const double* p = part + ((size_t)a * d.cb[d.L] + c) * 4;
    mn = fmin(mn, p[0]);
    mx = fmax(mx, p[1]);
    s1 += p[2];
    s2 += p[3];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
  }
  s1 = wave_sum_d(s1);
  s2 = wave_sum_d(s2);
  if (lane != 0) return;
  Seg g{};
  g.m = d.lv[l + 1] - d.lv[l];
  if (g.m > 0) {
    const double m = g.m, q = d.q;
    g.w = (double)d.lambda_rate * d.lw[l] / m;
    const double ss = fmax(s2 - s1 * s1 / m, 0.0);  // sum of squared deviations
    if (d.kind == 0) {
      const double sd = g.m > 1 ? sqrt(ss / (m - 1.0)) : 0.0;
      g.h = fmax(sd * pow(0.75 * m, -0.2), q / 4.0);
      const double pad = 8.0 * g.h + q;
      g.lo = mn - pad;
      const double hi = mx + pad;
      g.delta = fmax(fmax(fmin(q, g.h) / 4.0, (hi - g.lo) / (kGridMax - 1)), 8.0 * g.h / kKernMax);
      g.G = min((int)ceil((hi - g.lo) / g.delta) + 1, kGridMax);
      g.K = min((int)ceil(8.0 * g.h / g.delta), kKernMax);
    } else {
      g.mu = s1 / m;
      g.sd = sqrt(ss / m);
      g.sigma = fmax(g.sd, q * 1e-3);
    }
  }
  seg[s] = g;
}

// (KDE) linear binning of a chunk into the LDS histogram of its segment, then into the counts.
__global__ __launch_bounds__(256) void k_ent_hist(EntDims d, const float* __restrict__ attrs,
                                                  const Seg* __restrict__ seg,
                                                  unsigned long long* __restrict__ counts) {
  __shared__ uint32_t h[kGridMax];
  const int c = blockIdx.x, a = blockIdx.y;
  int l, i0, i1;
  if (!chunk_range(d, c, l, i0, i1)) return;
  const Seg g = seg[l * d.A + a];
  for (int k = threadIdx.x; k < g.G; k += 256) h[k] = 0u;
  __syncthreads();
  const double inv = 1.0 / g.delta;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double t = ((double)symbol(d, attrs, a, i) - g.lo) * inv;
    int k = (int)floor(t);
    k = min(max(k, 0), g.G - 2);
    const double f = fmin(fmax(t - k, 0.0), 1.0);
    const uint32_t w1 = (uint32_t)rint(f * kFix);
    atomicAdd(&h[k], kFix - w1);
    atomicAdd(&h[k + 1], w1);
  }
  __syncthreads();
  unsigned long long* dst = counts + (size_t)(l * d.A + a) * kGridMax;
  for (int k = threadIdx.x; k < g.G; k += 256)
    if (h[k]) atomicAdd(&dst[k], (unsigned long long)h[k]);
}

// (KDE) one block per segment: prefix sums of the counts, then
// F_k = (C_{k-K-1} + sum_{|j-k| <= K} c_j Phi((k - j) Delta / h)) / (kFix m).
__global__ __launch_bounds__(1024) void k_ent_cdf(EntDims d, const Seg* __restrict__ seg,
                                                  const unsigned long long* __restrict__ counts,
                                                  double* __restrict__ prefix, double* __restrict__ F) {
  __shared__ double phi[2 * kKernMax + 1];
  __shared__ unsigned long long tot[1024];
  const int s = blockIdx.x;
  const Seg g = seg[s];
  if (g.m == 0) return;
  const unsigned long long* c = counts + (size_t)s * kGridMax;
  double* C = prefix + (size_t)s * kGridMax;
  double* out = F + (size_t)s * kGridMax;
  const int t = threadIdx.x;
  for (int j = t; j <= 2 * g.K; j += 1024) phi[j] = 0.5 * erfc(-((j - g.K) * g.delta / g.h) * 0.70710678118654752440);
  // inclusive prefix of the counts: contiguous runs per thread, then a scan of the run totals
  const int per = (g.G + 1023) / 1024;
  const int k0 = t * per, k1 = min(k0 + per, g.G);
  unsigned long long run = 0;
  for (int k = k0; k < k1; ++k) run += c[k];
  tot[t] = run;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned long long v = t >= off ? tot[t - off] : 0ull;
    __syncthreads();
    tot[t] += v;
    __syncthreads();
  }
  unsigned long long acc = t > 0 ? tot[t - 1] : 0ull;
  for (int k = k0; k < k1; ++k) {
    acc += c[k];
    C[k] = (double)acc;
  }
  __syncthreads();
  const double norm = 1.0 / ((double)kFix * g.m);
  for (int k = t; k < g.G; k += 1024) {
    double v = k - g.K - 1 >= 0 ? C[k - g.K - 1] : 0.0;
    const int j0 = max(k - g.K, 0), j1 = min(k + g.K, g.G - 1);
    for (int j = j0; j <= j1; ++j) v += (double)c[j] * phi[k - j + g.K];
    out[k] = v * norm;
  }
}

__device__ __forceinline__ void interp(const double* __restrict__ F, const Seg& g, double x, double& val,
                                       double& slope) {
  const double t = (x - g.lo) / g.delta;
  int k = (int)floor(t);
  k = min(max(k, 0), g.G - 2);
  const double f = t - k;
  const double f0 = F[k], f1 = F[k + 1];
  val = f0 + f * (f1 - f0);
  slope = (f1 - f0) / g.delta;
}

// Gaussian model: P = Phi(a) - Phi(b) from the accurate tail; returns bits and the partials of
// bits in y (direct) and sigma.
__device__ __forceinline__ double gauss_bits(const Seg& g, double y, double q, double& db_dy, double& db_dsig) {
  const double a = (y - g.mu + 0.5 * q) / g.sigma, b = (y - g.mu - 0.5 * q) / g.sigma;
  const double r = 0.70710678118654752440;
  const double P = b > 0.0 ? 0.5 * (erfc(b * r) - erfc(a * r)) : 0.5 * (erfc(-a * r) - erfc(-b * r));
  if (!(P >= kFloor)) {
    db_dy = db_dsig = 0.0;
    return -log2(kFloor);
  }
  const double c = 0.39894228040143267794;  // 1 / sqrt(2 pi)
  const double pa = c * exp(-0.5 * a * a), pb = c * exp(-0.5 * b * b);
  const double gP = -1.0 / (P * kLn2);
  db_dy = gP * (pa - pb) / g.sigma;
  db_dsig = gP * (-(a * pa - b * pb) / g.sigma);
  return -log2(P);
}

// partials [A][chunks][4]: bits, |y|, sum w dbits/dmu, sum w dbits/dsigma
__global__ __launch_bounds__(256) void k_ent_eval(EntDims d, const float* __restrict__ attrs, const Seg* __restrict__ seg,
                                                  const double* __restrict__ F, double* __restrict__ part,
                                                  float* __restrict__ sym_bits, float* __restrict__ d_attrs) {
  __shared__ double sh[4];
  const int c = blockIdx.x, a = blockIdx.y;
  int l, i0, i1;
  if (!chunk_range(d, c, l, i0, i1)) return;
  const int s = l * d.A + a;
  const Seg g = seg[s];
  const double* Fs = F + (size_t)s * kGridMax;
  const double q = d.q;
  double sb = 0.0, sy = 0.0, smu = 0.0, ssig = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double y = symbol(d, attrs, a, i);
    double bits, dby;
    if (d.kind == 0) {
      double fp, sp, fm, sm;
      interp(Fs, g, y + 0.5 * q, fp, sp);
      interp(Fs, g, y - 0.5 * q, fm, sm);
      const double P = fp - fm;
      if (P >= kFloor) {
        bits = -log2(P);
        dby = -(sp - sm) / (P * kLn2);
      } else {
        bits = -log2(kFloor);
        dby = 0.0;
      }
      if (d_attrs && d.mode == 1) d_attrs[(size_t)a * d.n + i] += (float)(g.w * dby);
    } else {
      double dsig;
      bits = gauss_bits(g, y, q, dby, dsig);
      smu -= g.w * dby;
      ssig += g.w * dsig;
      sy += fabs(y);
    }
    sb += bits;
    if (sym_bits) sym_bits[(size_t)a * d.n + i] = (float)bits;
  }
  sb = block_reduce(sb, Add(), sh);
  sy = block_reduce(sy, Add(), sh);
  smu = block_reduce(smu, Add(), sh);
  ssig = block_reduce(ssig, Add(), sh);
  if (threadIdx.x == 0) {
    double* p = part + ((size_t)a * d.cb[d.L] + c) * 4;
    p[0] = sb;
    p[1] = sy;
    p[2] = smu;
    p[3] = ssig;
  }
}

// One wave per segment: its chunk sums (bits, |y|, and the Gaussian model's mean / deviation
// gradient sums, kept in the segment).
__global__ __launch_bounds__(64) void k_ent_segsum(EntDims d, const double* __restrict__ part, Seg* __restrict__ seg,
                                                   double* __restrict__ segsum) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int l = s / d.A, a = s - l * d.A;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = d.cb[l] + lane; c < d.cb[l + 1]; c += 64) {
    const double* p = part + ((size_t)a * d.cb[d.L] + c) * 4;
    for (int k = 0; k < 4; ++k) v[k] += p[k];
  }
  for (int k = 0; k < 4; ++k) v[k] = wave_sum_d(v[k]);
  if (lane == 0) {
    segsum[2 * s] = v[0];
    segsum[2 * s + 1] = v[1];
    seg[s].d_mu = v[2];
    seg[s].d_sig = v[3];
  }
}

// One block: per attribute bits (layers in order) and the loss (attributes in order).
__global__ __launch_bounds__(256) void k_ent_finalize(EntDims d, const Seg* __restrict__ seg,
                                                      const double* __restrict__ segsum, double* __restrict__ bits_out,
                                                      double* __restrict__ loss_out) {
  __shared__ double la[256];
  double lsum = 0.0;
  for (int a0 = 0; a0 < d.A; a0 += 256) {
    const int a = a0 + threadIdx.x;
    double ba = 0.0, lo = 0.0;
    if (a < d.A) {
      for (int l = 0; l < d.L; ++l) {
        const int s = l * d.A + a;
        ba += segsum[2 * s];
        lo += seg[s].w * segsum[2 * s];
        if (d.kind == 1) lo += (double)d.lw[l] * d.lambda_reg * segsum[2 * s + 1];
      }
      if (bits_out) bits_out[a] = ba;
    }
    la[threadIdx.x] = lo;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < 256 && a0 + k < d.A; ++k) lsum += la[k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_out) *loss_out += lsum;
}

// (Gaussian) d_attrs += w dbits/dy + (sum w dbits/dmu) / m + (sum w dbits/dsigma) (y - mu) / (m sd)
//                      + lambda^l lambda_reg sign(y)
__global__ __launch_bounds__(256) void k_ent_grad(EntDims d, const float* __restrict__ attrs, const Seg* __restrict__ seg,
                                                  float* __restrict__ d_attrs) {
  const int c = blockIdx.x, a = blockIdx.y;
  int l, i0, i1;
  if (!chunk_range(d, c, l, i0, i1)) return;
  const Seg g = seg[l * d.A + a];
  const double q = d.q;
  const double through_sd = g.sd > q * 1e-3 ? g.d_sig / (g.m * g.sd) : 0.0;
  const double reg = (double)d.lw[l] * d.lambda_reg;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double y = symbol(d, attrs, a, i);
    double dby, dsig;
    gauss_bits(g, y, q, dby, dsig);
    const double sgn = y > 0.0 ? 1.0 : (y < 0.0 ? -1.0 : 0.0);
    const double v = g.w * dby + g.d_mu / g.m + through_sd * (y - g.mu) + reg * sgn;
    d_attrs[(size_t)a * d.n + i] += (float)v;
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int ent_dims(const gs_entropy_desc* desc, EntDims& d) {
  if (!desc) return report_arg("desc is NULL");
  const gs_entropy_desc& s = *desc;
  if (s.n < 0 || s.n_attr < 1) return report_arg("n < 0 or n_attr < 1");
  if (!(s.step > 0.f) || std::isinf(s.step)) return report_arg("step must be finite and > 0");
  if (s.mode != 0 && s.mode != 1) return report_arg("mode must be 0 or 1");
  if (s.kind != 0 && s.kind != 1) return report_arg("kind must be 0 (KDE) or 1 (Gaussian)");
  if (s.n_levels < 1 || s.n_levels > kMaxLevels) return report_arg("n_levels must be in 1..8");
  if (s.level_counts[s.n_levels - 1] != s.n) return report_arg("the last level count must equal n");
  if (!(s.lambda_rate >= 0.f) || !(s.lambda_reg >= 0.f)) return report_arg("lambda_rate and lambda_reg must be >= 0");
  d.n = s.n;
  d.A = s.n_attr;
  d.L = s.n_levels;
  d.kind = s.kind;
  d.mode = s.mode;
  d.q = s.step;
  d.seed = s.seed;
  d.offset = s.offset;
  d.lambda_rate = s.lambda_rate;
  d.lambda_reg = s.lambda_reg;
  d.lv[0] = 0;
  d.cb[0] = 0;
  for (int l = 0; l < d.L; ++l) {
    d.lv[l + 1] = s.level_counts[l];
    if (d.lv[l + 1] < d.lv[l]) return report_arg("level_counts must be ascending and >= 0");
    d.lw[l] = s.level_weights[l];
    d.cb[l + 1] = d.cb[l] + (d.lv[l + 1] - d.lv[l] + kChunk - 1) / kChunk;
  }
  for (int l = d.L; l < kMaxLevels; ++l) {
    d.lv[l + 1] = d.lv[d.L];
    d.cb[l + 1] = d.cb[d.L];
    d.lw[l] = 0.f;
  }
  if ((int64_t)d.A * d.cb[d.L] > 0x7FFFFFFF) return report_arg("too many symbols");
  return GS_OK;
}

struct EntLayout {
  size_t part, seg, segsum, counts, prefix, F, total;
};

EntLayout ent_layout(const EntDims& d) {
  EntLayout lo{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t segs = (size_t)d.L * d.A;
  lo.part = take((size_t)d.A * (d.cb[d.L] > 0 ? d.cb[d.L] : 1) * 4 * sizeof(double));
  lo.seg = take(segs * sizeof(Seg));
  lo.segsum = take(segs * 2 * sizeof(double));
  if (d.kind == 0) {
    lo.counts = take(segs * kGridMax * sizeof(unsigned long long));
    lo.prefix = take(segs * kGridMax * sizeof(double));
    lo.F = take(segs * kGridMax * sizeof(double));
  }
  lo.total = off;
  return lo;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int gs_entropy_workspace_size(const gs_entropy_desc* desc, size_t* bytes_out) {
  EntDims d;
  int rc = ent_dims(desc, d);
  if (rc) return rc;
  if (!bytes_out) return report_arg("bytes_out is NULL");
  *bytes_out = ent_layout(d).total;
  return GS_OK;
}

int gs_entropy_model(const gs_entropy_desc* desc, const float* attrs, double* bits_out, double* loss_out,
                     float* sym_bits, float* d_attrs, void* ws, size_t ws_bytes, void* stream) {
  EntDims d;
  int rc = ent_dims(desc, d);
  if (rc) return rc;
  if (!ws || (d.n > 0 && !attrs)) return report_arg("NULL buffer");
  const EntLayout lo = ent_layout(d);
  if (ws_bytes < lo.total) {
    report_arg("workspace too small");
    return GS_ERR_WORKSPACE;
  }
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  double* part = (double*)(w + lo.part);
  Seg* seg = (Seg*)(w + lo.seg);
  double* segsum = (double*)(w + lo.segsum);
  const int chunks = d.cb[d.L];
  const dim3 grid(chunks > 0 ? chunks : 1, d.A);
  const int segs = d.L * d.A;
  hipError_t e;
  {
    ProfScope ps_(K_ENT_STATS, st);
    if (chunks > 0) hipLaunchKernelGGL(k_ent_stats, grid, dim3(256), 0, st, d, attrs, part);
    hipLaunchKernelGGL(k_ent_setup, dim3(segs), dim3(64), 0, st, d, part, seg);
  }
  double* F = nullptr;
  if (d.kind == 0 && chunks > 0) {
    unsigned long long* counts = (unsigned long long*)(w + lo.counts);
    if ((e = launch_zero(counts, (size_t)segs * kGridMax * sizeof(unsigned long long), st)) != hipSuccess)
      return report_hip(e, "zero");
    F = (double*)(w + lo.F);
    {
      ProfScope ps_(K_ENT_HIST, st);
      hipLaunchKernelGGL(k_ent_hist, grid, dim3(256), 0, st, d, attrs, seg, counts);
    }
    {
      ProfScope ps_(K_ENT_CDF, st);
      hipLaunchKernelGGL(k_ent_cdf, dim3(segs), dim3(1024), 0, st, d, seg, counts, (double*)(w + lo.prefix), F);
    }
  }
  {
    ProfScope ps_(K_ENT_EVAL, st);
    if (chunks > 0)
      hipLaunchKernelGGL(k_ent_eval, grid, dim3(256), 0, st, d, attrs, seg, F, part, sym_bits, d_attrs);
    hipLaunchKernelGGL(k_ent_segsum, dim3(segs), dim3(64), 0, st, d, part, seg, segsum);
    hipLaunchKernelGGL(k_ent_finalize, dim3(1), dim3(256), 0, st, d, seg, segsum, bits_out, loss_out);
    if (d.kind == 1 && d_attrs && d.mode == 1 && chunks > 0)
      hipLaunchKernelGGL(k_ent_grad, grid, dim3(256), 0, st, d, attrs, seg, d_attrs);
  }
  e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "entropy model");
}

}  // extern "C"
