// Significance ordering (Sec. 3.1: Psi = opacity + lambda_psi (4/3) pi a b c, Gaussians sorted by
// Psi descending and split into nested layers) and the quantise-to-2D-maps step of progressive
// bitstream generation (Sec. 3.3): per layer and channel, min/max quantisation to 16 bits for
// positions and 8 bits for the other attributes, each channel flattened into a 2D map.
//
// Map layout: a layer's Gaussians are ordered by the Morton code of their quantised position (top
// 10, 10, 9 bits of x, y, z; ties by significance rank) and written 256 at a time into 16 x 16
// blocks; the blocks snake row by row and the 256 Gaussians of a block follow the 2D Morton curve
// inside it, so Gaussians close in space land close in the map. Pixels past the layer's last
// Gaussian repeat it. The codec that compresses the maps is outside this library.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

constexpr int kPosChannels = 3;  // channels 0..2 (the mean) take 16-bit codes, the rest 8-bit

// The part of the layout the kernels need (built from gs_maps_layout on the host).
struct MapsDims {
  int n, C, L;
  int lv[kMaxLevels + 1];   // lv[0] = 0, lv[l + 1] = level_counts[l]
  int w[kMaxLevels], h[kMaxLevels];
  long long pix[kMaxLevels + 1];  // prefix sums of w * h over the layers
  long long off[kMaxLevels];      // byte offset of each layer's first plane
};

// Float <-> unsigned key whose unsigned order is the float order (for atomic min / max).
__device__ __forceinline__ uint32_t ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unordered(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// order[] comes from the caller and must be a permutation of 0..n-1; an index outside it is
// clamped so that a bad order gives wrong codes, never a read outside params.
__device__ __forceinline__ int gaussian(const MapsDims& d, const int32_t* order, int r) {
  return min(max(order[r], 0), d.n - 1);
}

__device__ __forceinline__ int level_of(const MapsDims& d, int r) {
  int l = 0;
#pragma unroll
  for (int k = 1; k < kMaxLevels; ++k)
    if (k < d.L && r >= d.lv[k]) l = k;
  return l;
}

// Byte offset of plane (l, c): three 16-bit planes, then the 8-bit ones.
__device__ __forceinline__ long long plane_offset(const MapsDims& d, int l, int c) {
  const long long wh = (long long)d.w[l] * d.h[l];
  return d.off[l] + (c < kPosChannels ? 2 * wh * c : 2 * wh * kPosChannels + wh * (c - kPosChannels));
}

__device__ __forceinline__ uint32_t quantise(float v, float mn, float mx, float top) {
  if (!(mx > mn)) return 0u;
  const float scale = top / (mx - mn);
  const float q = rintf((v - mn) * scale);
  return (uint32_t)fminf(fmaxf(q, 0.f), top);
}

__device__ __forceinline__ uint32_t spread3(uint32_t x) {  // bit k -> bit 3k (10 bits)
  x &= 0x3FFu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Pixel of sequence position p in a map w pixels wide.
__device__ __forceinline__ void block_pixel(int p, int w, int& x, int& y) {
  const int blk = p >> 8, q = p & 255;
  const int nbx = w >> 4;
  const int by = blk / nbx;
  int bx = blk - by * nbx;
  if (by & 1) bx = nbx - 1 - bx;
  const int u = (q & 1) | ((q >> 1) & 2) | ((q >> 2) & 4) | ((q >> 3) & 8);
  const int v = ((q >> 1) & 1) | ((q >> 2) & 2) | ((q >> 3) & 4) | ((q >> 4) & 8);
  x = 16 * bx + u;
  y = 16 * by + v;
}

__global__ __launch_bounds__(256) void k_psi_keys(int n, const float* __restrict__ params, float lambda_psi,
                                                  uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                  float* __restrict__ psi_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float opacity = 1.f / (1.f + expf(-params[(size_t)10 * n + i]));
  const float volume = (4.f / 3.f) * 3.14159265358979f * expf(params[(size_t)3 * n + i]) *
                       expf(params[(size_t)4 * n + i]) * expf(params[(size_t)5 * n + i]);
  const float psi = opacity + lambda_psi * volume;
  keys[i] = ~__float_as_uint(psi);  // Psi > 0: descending Psi = ascending key
  vals[i] = (uint32_t)i;
  if (psi_out) psi_out[i] = psi;
}

__global__ __launch_bounds__(256) void k_copy_u32(int n, const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_range_init(int count, uint32_t* __restrict__ mm) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) mm[i] = (i & 1) ? 0u : 0xFFFFFFFFu;  // (min, max) pairs
}

// Per (layer, channel) minimum and maximum; grid (rank blocks of 2048, channels). A thread keeps
// the extremes of the block's first layer in registers (reduced across the wave before one LDS
// atomic); ranks of later layers in the same block go to LDS directly.
__global__ __launch_bounds__(256) void k_range(MapsDims d, const float* __restrict__ params,
                                               const int32_t* __restrict__ order, uint32_t* __restrict__ mm) {
  __shared__ uint32_t s_mm[kMaxLevels][2];
  const int t = threadIdx.x, c = blockIdx.y;
  if (t < 2 * kMaxLevels) s_mm[t >> 1][t & 1] = (t & 1) ? 0u : 0xFFFFFFFFu;
  __syncthreads();
  const int r0 = blockIdx.x * 2048;
  const int l0 = level_of(d, r0);
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  for (int k = 0; k < 8; ++k) {
    const int r = r0 + k * 256 + t;
    if (r >= d.n) break;
    const uint32_t key = ordered(params[(size_t)c * d.n + gaussian(d, order, r)]);
    const int l = level_of(d, r);
    if (l == l0) {
      lo = min(lo, key);
      hi = max(hi, key);
    } else {
      atomicMin(&s_mm[l][0], key);
      atomicMax(&s_mm[l][1], key);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
  }
  if ((t & 63) == 0) {
    atomicMin(&s_mm[l0][0], lo);
    atomicMax(&s_mm[l0][1], hi);
  }
  __syncthreads();
  if (t < d.L) {
    if (s_mm[t][0] != 0xFFFFFFFFu) atomicMin(&mm[((size_t)t * d.C + c) * 2], s_mm[t][0]);
    if (s_mm[t][1] != 0u) atomicMax(&mm[((size_t)t * d.C + c) * 2 + 1], s_mm[t][1]);
  }
}

// (min, max) pairs as floats; a layer with no Gaussians gets (0, 0).
__global__ __launch_bounds__(256) void k_range_out(int pairs, const uint32_t* __restrict__ mm,
                                                   float* __restrict__ ranges) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= pairs) return;
  const uint32_t lo = mm[2 * i], hi = mm[2 * i + 1];
  const bool empty = lo == 0xFFFFFFFFu && hi == 0u;
  ranges[2 * i] = empty ? 0.f : unordered(lo);
  ranges[2 * i + 1] = empty ? 0.f : unordered(hi);
}

// Sort key of every rank: layer (3 bits) above the Morton code (29 bits) of its quantised position.
__global__ __launch_bounds__(256) void k_maps_keys(MapsDims d, const float* __restrict__ params,
                                                   const int32_t* __restrict__ order, const float* __restrict__ ranges,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= d.n) return;
  const int l = level_of(d, r), i = gaussian(d, order, r);
  uint32_t q[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* rg = ranges + ((size_t)l * d.C + c) * 2;
    q[c] = quantise(params[(size_t)c * d.n + i], rg[0], rg[1], 65535.f);
  }
  const uint32_t m = spread3(q[0] >> 6) | (spread3(q[1] >> 6) << 1) | (spread3(q[2] >> 7) << 2);
  keys[r] = ((uint32_t)l << 29) | m;
  vals[r] = (uint32_t)r;
}

// One thread per map pixel of every layer: the codes of all channels of the Gaussian at that
// pixel (the layer's last one past its end), and the Gaussian index of each sequence position.
__global__ __launch_bounds__(256) void k_maps_write(MapsDims d, const float* __restrict__ params,
                                                    const int32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ sorted_rank,
                                                    const float* __restrict__ ranges, uint8_t* __restrict__ maps,
                                                    int32_t* __restrict__ seq) {
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= d.pix[d.L]) return;
  int l = 0;
#pragma unroll
  for (int k = 1; k < kMaxLevels; ++k)
    if (k < d.L && g >= d.pix[k]) l = k;
  const int p = (int)(g - d.pix[l]);
  const int m = d.lv[l + 1] - d.lv[l];
  int x, y;
  block_pixel(p, d.w[l], x, y);
  const long long px = (long long)y * d.w[l] + x;
  if (m == 0) {  // a layer with no Gaussians: zero maps
    for (int c = 0; c < d.C; ++c) {
      uint8_t* plane = maps + plane_offset(d, l, c);
      if (c < kPosChannels)
        reinterpret_cast<uint16_t*>(plane)[px] = 0;
      else
        plane[px] = 0;
    }
    return;
  }
  const int j = d.lv[l] + min(p, m - 1);
  const int i = gaussian(d, order, (int)sorted_rank[j]);
  if (seq && p < m) seq[j] = i;
  for (int c = 0; c < d.C; ++c) {
    const float* rg = ranges + ((size_t)l * d.C + c) * 2;
    const float v = params[(size_t)c * d.n + i];
    uint8_t* plane = maps + plane_offset(d, l, c);
    if (c < kPosChannels)
      reinterpret_cast<uint16_t*>(plane)[px] = (uint16_t)quantise(v, rg[0], rg[1], 65535.f);
    else
      plane[px] = (uint8_t)quantise(v, rg[0], rg[1], 255.f);
  }
}

// One thread per sequence position: dequantised parameters in map order.
__global__ __launch_bounds__(256) void k_maps_decode(MapsDims d, const uint8_t* __restrict__ maps,
                                                     const float* __restrict__ ranges, float* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= d.n) return;
  const int l = level_of(d, j);
  int x, y;
  block_pixel(j - d.lv[l], d.w[l], x, y);
  const long long px = (long long)y * d.w[l] + x;
  for (int c = 0; c < d.C; ++c) {
    const float* rg = ranges + ((size_t)l * d.C + c) * 2;
    const uint8_t* plane = maps + plane_offset(d, l, c);
    const float code = c < kPosChannels ? (float)reinterpret_cast<const uint16_t*>(plane)[px] : (float)plane[px];
    const float top = c < kPosChannels ? 65535.f : 255.f;
    const float step = (rg[1] - rg[0]) / top;
    out[(size_t)c * d.n + j] = fmaf(code, step, rg[0]);
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int maps_dims(const gs_maps_layout* lo, MapsDims& d) {
  if (!lo) return report_arg("layout is NULL");
  if (lo->n_levels < 1 || lo->n_levels > kMaxLevels) return report_arg("n_levels must be in 1..8");
  if (lo->n_channels < 11) return report_arg("n_channels must be >= 11 (mean, scale, rotation, opacity)");
  d.C = lo->n_channels;
  d.L = lo->n_levels;
  d.lv[0] = 0;
  d.pix[0] = 0;
  long long end = 0;
  for (int l = 0; l < d.L; ++l) {
    d.lv[l + 1] = lo->level_counts[l];
    d.w[l] = lo->width[l];
    d.h[l] = lo->height[l];
    d.off[l] = lo->offset[l];
    d.pix[l + 1] = d.pix[l] + (long long)d.w[l] * d.h[l];
    // every write of the kernels stays inside the layer's planes, which must fit the buffer
    const long long wh = (long long)d.w[l] * d.h[l];
    if (d.lv[l + 1] < d.lv[l]) return report_arg("level_counts must be ascending and >= 0");
    if (d.w[l] < 16 || d.h[l] < 16 || d.w[l] % 16 || d.h[l] % 16 || wh < d.lv[l + 1] - d.lv[l] ||
        wh > ((long long)1 << 31))
      return report_arg("map sizes must be multiples of 16 that hold the layer");
    if (d.off[l] < end) return report_arg("layer offsets overlap");
    end = d.off[l] + wh * (2 * kPosChannels + (d.C - kPosChannels));
  }
  if (end > lo->total_bytes) return report_arg("layers exceed total_bytes");
  for (int l = d.L; l < kMaxLevels; ++l) {
    d.lv[l + 1] = d.lv[d.L];
    d.w[l] = d.h[l] = 16;
    d.off[l] = 0;
    d.pix[l + 1] = d.pix[d.L];
  }
  d.n = d.lv[d.L];
  return GS_OK;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int gs_maps_describe(int32_t n_channels, int32_t n_levels, const int32_t* level_counts, gs_maps_layout* out) {
  if (!level_counts || !out) return report_arg("NULL argument");
  if (n_levels < 1 || n_levels > kMaxLevels) return report_arg("n_levels must be in 1..8");
  if (n_channels < 11 || n_channels > 1024) return report_arg("n_channels must be in 11..1024");
  gs_maps_layout lo{};
  lo.n_channels = n_channels;
  lo.n_levels = n_levels;
  size_t off = 0;
  int prev = 0;
  for (int l = 0; l < n_levels; ++l) {
    const int c = level_counts[l];
    if (c < prev) return report_arg("level_counts must be ascending and >= 0");
    const int m = c - prev;
    int w = 16, h = 16;
    if (m > 0) {
      const int side = (int)std::ceil(std::sqrt((double)m));
      w = 16 * ((side + 15) / 16);
      h = 16 * (((m + w - 1) / w + 15) / 16);
    }
    lo.level_counts[l] = c;
    lo.width[l] = w;
    lo.height[l] = h;
    lo.offset[l] = (int64_t)off;
    off = align256(off + (size_t)w * h * (2 * kPosChannels + (n_channels - kPosChannels)));
    prev = c;
  }
  lo.total_bytes = (int64_t)off;
  *out = lo;
  return GS_OK;
}

int gs_significance_workspace_size(int32_t n, size_t* bytes_out) {
  if (n < 0 || !bytes_out) return report_arg("n < 0 or bytes_out NULL");
  *bytes_out = 4 * align256((size_t)n * 4) + align256(radix_hist_words(n) * 4);
  return GS_OK;
}

int gs_significance_order(int32_t n, const float* params, int32_t n_channels, float lambda_psi, int32_t* order,
                          float* psi, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n_channels < 11) return report_arg("n < 0 or n_channels < 11");
  if (!(lambda_psi >= 0.f) || std::isinf(lambda_psi)) return report_arg("lambda_psi must be finite and >= 0");
  if (n == 0) return GS_OK;
  if (!params || !order || !ws) return report_arg("NULL buffer");
  size_t need = 0;
  gs_significance_workspace_size(n, &need);
  if (ws_bytes < need) {
    report_arg("workspace too small");
    return GS_ERR_WORKSPACE;
  }
  int rc;
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t a = align256((size_t)n * 4);
  uint32_t* k[2] = {(uint32_t*)w, (uint32_t*)(w + a)};
  uint32_t* v[2] = {(uint32_t*)(w + 2 * a), (uint32_t*)(w + 3 * a)};
  uint32_t* hist = (uint32_t*)(w + 4 * a);
  const int blocks = (n + 255) / 256;
  {
    ProfScope ps_(K_PSI, st);
    hipLaunchKernelGGL(k_psi_keys, dim3(blocks), dim3(256), 0, st, n, params, lambda_psi, k[0], v[0], psi);
  }
  uint32_t *sk, *sv;
  hipError_t e = launch_radix_sort(n, k, v, hist, &sk, &sv, st);
  if (e != hipSuccess) return report_hip(e, "significance sort");
  hipLaunchKernelGGL(k_copy_u32, dim3(blocks), dim3(256), 0, st, n, sv, (uint32_t*)order);
  e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "significance order");
}

int gs_encode_workspace_size(const gs_maps_layout* lo, size_t* bytes_out) {
  MapsDims d;
  int rc = maps_dims(lo, d);
  if (rc) return rc;
  if (!bytes_out) return report_arg("bytes_out is NULL");
  *bytes_out = align256((size_t)d.L * d.C * 8) + 4 * align256((size_t)d.n * 4) + align256(radix_hist_words(d.n) * 4);
  return GS_OK;
}

int gs_encode_maps(const gs_maps_layout* lo, const float* params, const int32_t* order, float* ranges, uint8_t* maps,
                   int32_t* seq, void* ws, size_t ws_bytes, void* stream) {
  MapsDims d;
  int rc = maps_dims(lo, d);
  if (rc) return rc;
  if (!ranges || !maps || !ws || (d.n > 0 && (!params || !order))) return report_arg("NULL buffer");
  size_t need = 0;
  gs_encode_workspace_size(lo, &need);
  if (ws_bytes < need) {
    report_arg("workspace too small");
    return GS_ERR_WORKSPACE;
  }
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  uint32_t* mm = (uint32_t*)w;
  const size_t b0 = align256((size_t)d.L * d.C * 8);
  const size_t a = align256((size_t)d.n * 4);
  uint32_t* k[2] = {(uint32_t*)(w + b0), (uint32_t*)(w + b0 + a)};
  uint32_t* v[2] = {(uint32_t*)(w + b0 + 2 * a), (uint32_t*)(w + b0 + 3 * a)};
  uint32_t* hist = (uint32_t*)(w + b0 + 4 * a);
  const int cnt = d.L * d.C * 2;
  {
    ProfScope ps_(K_MAPS_RANGE, st);
    hipLaunchKernelGGL(k_range_init, dim3((cnt + 255) / 256), dim3(256), 0, st, cnt, mm);
    if (d.n > 0)
      hipLaunchKernelGGL(k_range, dim3((d.n + 2047) / 2048, d.C), dim3(256), 0, st, d, params, order, mm);
    hipLaunchKernelGGL(k_range_out, dim3((cnt / 2 + 255) / 256), dim3(256), 0, st, cnt / 2, mm, ranges);
  }
  uint32_t *sk = k[0], *sv = v[0];
  if (d.n > 0) {
    {
      ProfScope ps_(K_MAPS_KEYS, st);
      hipLaunchKernelGGL(k_maps_keys, dim3((d.n + 255) / 256), dim3(256), 0, st, d, params, order, ranges, k[0], v[0]);
    }
    hipError_t e = launch_radix_sort(d.n, k, v, hist, &sk, &sv, st);
    if (e != hipSuccess) return report_hip(e, "maps sort");
  }
  {
    ProfScope ps_(K_MAPS_WRITE, st);
    const long long total = d.pix[d.L];
    hipLaunchKernelGGL(k_maps_write, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, d, params, order, sv,
                         ranges, maps, seq);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "maps write");
}

int gs_decode_maps(const gs_maps_layout* lo, const uint8_t* maps, const float* ranges, float* params_out,
                   void* stream) {
  MapsDims d;
  int rc = maps_dims(lo, d);
  if (rc) return rc;
  if (d.n == 0) return GS_OK;
  if (!maps || !ranges || !params_out) return report_arg("NULL buffer");
  if ((rc = require_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  {
    ProfScope ps_(K_MAPS_DECODE, st);
    hipLaunchKernelGGL(k_maps_decode, dim3((d.n + 255) / 256), dim3(256), 0, st, d, maps, ranges, params_out);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : report_hip(e, "maps decode");
}

}  // extern "C"
