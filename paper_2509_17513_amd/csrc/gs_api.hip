// Host side of the C ABI: argument validation, workspace layout and the
// launch sequence of the forward and backward render.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gs4d.h"
#include "gs_internal.h"
#include "gs_prof.h"

namespace gs {
namespace {

thread_local std::string g_last_error;

int fail_hip(hipError_t e, const char* where) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
  g_last_error = buf;
  return GS_ERR_HIP;
}

int fail_arg(const char* msg) {
  g_last_error = msg;
  return GS_ERR_INVALID_ARG;
}

// Checks once per process that the current device is a gfx950.
int check_device() {
  static std::once_flag once;
  static int status = GS_OK;
  std::call_once(once, [] {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
      status = GS_ERR_NO_DEVICE;
      return;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      status = GS_ERR_NO_DEVICE;
      return;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) status = GS_ERR_NO_DEVICE;
  });
  if (status != GS_OK) g_last_error = "no gfx950 device visible";
  return status;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int make_dims(const gs_settings* s, int32_t n, int32_t F, int32_t V, int64_t cap, RenderDims& d) {
  if (!s) return fail_arg("settings is NULL");
  if (n < 0) return fail_arg("n < 0");
  if (F < 1 || V < 1) return fail_arg("n_frames and n_views must be >= 1");
  if (s->width < 1 || s->height < 1) return fail_arg("width and height must be >= 1");
  if (s->sh_degree < 0 || s->sh_degree > 3) return fail_arg("sh_degree must be in 0..3");
  if (s->n_levels < 1 || s->n_levels > kMaxLevels) return fail_arg("n_levels must be in 1..8");
  for (int l = 0; l < s->n_levels; ++l) {
    if (s->level_counts[l] < 0 || s->level_counts[l] > n) return fail_arg("level_counts out of range");
    if (l > 0 && s->level_counts[l] < s->level_counts[l - 1]) return fail_arg("level_counts not ascending");
  }
  if (s->level_counts[s->n_levels - 1] != n) return fail_arg("last level count must equal n");
  const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  const int C = 11 + 3 * K;
  if (!(s->res_channels == 0 || s->res_channels == 8 || s->res_channels == 11 || s->res_channels == C))
    return fail_arg("res_channels must be 0, 8, 11 or 11 + 3 (d+1)^2");
  if ((s->tile_w != 0 || s->tile_h != 0) && (s->tile_w != kTile || s->tile_h != kTile)) {
    g_last_error = "only 16x16 tiles are implemented";
    return GS_ERR_UNSUPPORTED;
  }
  // alpha_max < 1: the backward recovers the transmittance in front of a
  // Gaussian by dividing by 1 - alpha
  if (!(s->alpha_min > 0.f) || !(s->alpha_max < 1.f) || !(s->alpha_min <= s->alpha_max))
    return fail_arg("need 0 < alpha_min <= alpha_max < 1");
  if (!(s->t_stop >= 0.f) || !(s->near_plane > 0.f) || !(s->dilation >= 0.f))
    return fail_arg("need t_stop >= 0, near_plane > 0, dilation >= 0");
  if (cap < 0 || cap > 0xFFFFFFFFll) return fail_arg("pair_capacity must be in [0, 2^32)");
  d.n = n; d.F = F; d.V = V; d.B = F * V; d.W = s->width; d.H = s->height;
  d.TX = (d.W + kTile - 1) / kTile;
  d.TY = (d.H + kTile - 1) / kTile;
  d.T = d.TX * d.TY;
  if (d.TX > kMaxTilesX) {
    g_last_error = "images wider than 2048 pixels are not implemented";
    return GS_ERR_UNSUPPORTED;
  }
  if (d.TY > 4096) return fail_arg("image taller than 65536 pixels");
  if ((int64_t)d.B * n > (int64_t)1 << 31) return fail_arg("n_frames * n_views * n too large");
  d.deg = s->sh_degree; d.K = K; d.C = C; d.L = s->n_levels; d.Rc = s->res_channels;
  for (int l = 0; l < kMaxLevels; ++l) {
    d.lv[l] = l < d.L ? s->level_counts[l] : n;
    d.lw[l] = l < d.L ? s->level_weights[l] : 0.f;
  }
  d.near_plane = s->near_plane; d.dilation = s->dilation; d.alpha_min = s->alpha_min;
  d.alpha_max = s->alpha_max; d.t_stop = s->t_stop;
  for (int c = 0; c < 3; ++c) d.bg[c] = s->bg[c];
  d.bin_chunk = s->bin_chunk == 0 ? kBinChunk : s->bin_chunk;
  d.row_seg = s->row_seg == 0 ? kRowSeg : s->row_seg;
  d.wave_layout = s->wave_layout == 0 ? 1 : s->wave_layout;
  if (d.bin_chunk != 512 && d.bin_chunk != 1024 && d.bin_chunk != 2048)
    return fail_arg("bin_chunk must be 0, 512, 1024 or 2048");
  if (d.row_seg != 1024 && d.row_seg != 2048 && d.row_seg != 4096)
    return fail_arg("row_seg must be 0, 1024, 2048 or 4096");
  if (d.wave_layout != 1 && d.wave_layout != 2) return fail_arg("wave_layout must be 0, 1 or 2");
  d.batch = s->lds_batch == 0 ? kTilePix : s->lds_batch;
  if (d.batch != 64 && d.batch != 128 && d.batch != 256) return fail_arg("lds_batch must be 0, 64, 128 or 256");
  d.bwd_pixels = s->bwd_pixels == 0 ? 1 : s->bwd_pixels;
  if (d.bwd_pixels != 1 && d.bwd_pixels != 2) return fail_arg("bwd_pixels must be 0, 1 or 2");
  d.det = deterministic() ? 1 : 0;
  d.n_sort_chunks = (n + kSortChunk - 1) / kSortChunk;
  d.n_bin_chunks = (n + d.bin_chunk - 1) / d.bin_chunk;
  d.n_row_segs = (n + d.row_seg - 1) / d.row_seg;
  d.n_bin_chunks_max = (n + kBinChunkMin - 1) / kBinChunkMin;
  d.n_row_segs_max = (n + kRowSegMin - 1) / kRowSegMin;
  d.capacity = (unsigned long long)cap;
  d.row_capacity = d.capacity / 2;
  return GS_OK;
}

}  // namespace

int report_arg(const char* msg) { return fail_arg(msg); }

std::atomic<int> g_work_counting{0};
bool work_counting() { return g_work_counting.load(std::memory_order_relaxed) != 0; }
std::atomic<int> g_deterministic{0};
bool deterministic() { return g_deterministic.load(std::memory_order_relaxed) != 0; }
int report_hip(hipError_t e, const char* where) { return fail_hip(e, where); }
int require_device() { return check_device(); }


// ------------------------------------------------------------ profiling
namespace {
struct ProfRec {
  int id;
  hipEvent_t a, b;
  bool ended;  // the end event was recorded
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

const char* kKernelNames[K_COUNT] = {
    "compose_fwd", "project_fwd", "radix_hist", "radix_scan", "radix_scatter", "bin_count", "bin_chunk_scan",
    "tile_ranges", "bin_emit", "raster_fwd", "zero", "raster_bwd", "project_bwd", "compose_bwd", "rate_ctx",
    "rate_mlp", "rate_hist_minmax", "rate_hist_count", "rate_hist_bits", "adam", "bin_gather", "row_count", "row_emit",
    "ssim_fwd", "ssim_bwd", "psi", "maps_range", "maps_keys", "maps_write", "maps_decode", "ent_stats", "ent_hist", "ent_cdf", "ent_eval", "motion_fwd", "motion_bwd",
    "motion_wgrad", "motion_table"};
}  // namespace

int prof_begin(int id, hipStream_t st) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on) return -1;
  ProfRec r{id, prof_event(), prof_event(), false};
  // a record whose events cannot be made or started is dropped (its events go back to the pool)
  if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {
    if (r.a) g_prof_pool.push_back(r.a);
    if (r.b) g_prof_pool.push_back(r.b);
    return -1;
  }
  g_prof_recs.push_back(r);
  return (int)g_prof_recs.size() - 1;
}

void prof_end(int slot, hipStream_t st) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (slot < (int)g_prof_recs.size()) g_prof_recs[slot].ended = hipEventRecord(g_prof_recs[slot].b, st) == hipSuccess;
}

Layout make_layout(const RenderDims& d) {
  Layout lo;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t Bn = (size_t)d.B * d.n;
  const size_t HW = (size_t)d.W * d.H;
  lo.status = take(256);
  lo.records = take(Bn * 48);
  lo.rects = take(Bn * 8);
  lo.keys0 = take(Bn * 4);
  lo.vals0 = take(Bn * 4);
  lo.keys1 = take(Bn * 4);
  lo.vals1 = take(Bn * 4);
  lo.sort_hist = take((size_t)d.B * 256 * d.n_sort_chunks * 4);
  lo.bin_rec = take(Bn * 48);
  lo.bin_hist = take((size_t)d.B * d.n_bin_chunks_max * d.TY * 4);
  lo.row_tot = take((size_t)d.B * d.TY * 4);
  lo.row_ranges = take((size_t)d.B * d.TY * 8);
  lo.tile_hist = take((size_t)d.B * d.TY * d.n_row_segs_max * d.TX * 4);
  lo.tile_tot = take((size_t)d.B * d.T * 4);
  lo.ranges = take((size_t)d.B * d.T * 8);
  lo.t_final = take((size_t)d.B * d.L * HW * 4);
  lo.n_last = take((size_t)d.B * d.L * HW * 4);
  lo.grad2d = take(Bn * kGradStride * 4);
  lo.composed = take((size_t)d.F * d.Rc * d.n * 4);
  lo.d_composed = take((size_t)d.F * d.Rc * d.n * 4);
  lo.check = take(256);  // the autotuner's image checksum
  // deterministic backward: 128-bit fixed-point sums of the nine gradient values per (view,
  // Gaussian) and of the loss
  lo.grad2d_fx = take(d.det ? Bn * 9 * 16 : 0);
  lo.loss_fx = take(d.det ? 16 : 0);
  // the pair lists are last, so every other offset is independent of their capacity
  lo.lists = take((size_t)d.capacity * 4);
  lo.row_lists = take((size_t)d.row_capacity * 8);
  lo.total = off;
  return lo;
}

// The largest pair capacity whose layout fits in ws_bytes (4 bytes of tile list and 4 bytes of
// row list, half as many 8-byte entries, per unit of capacity).
void set_capacity(RenderDims& d, const Layout& lo0, size_t ws_bytes) {
  unsigned long long cap = std::min<unsigned long long>((ws_bytes - lo0.total) / 8, 0xFFFFFFFFull);
  for (;;) {
    d.capacity = cap;
    d.row_capacity = cap / 2;
    const size_t tot = make_layout(d).total;
    if (tot <= ws_bytes || cap == 0) break;
    cap -= std::min<unsigned long long>(cap, (tot - ws_bytes + 7) / 8);
  }
}

}  // namespace gs

using namespace gs;

// ------------------------------------------------------ attainable peaks
// Eight independent FMA chains per thread (enough to hide the FMA latency),
// iters rounds each; the result is stored so that nothing is dead code.
__global__ __launch_bounds__(256) void k_peak_fma(int iters, float x, float y, float* __restrict__ out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (float)(gid + k) * 1e-7f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], x, y);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[gid] = s;
}

// A plain device copy in 16-byte vectors (grid-stride).
__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

extern "C" {

int gs_workspace_size(const gs_settings* s, int32_t n, int32_t n_frames, int32_t n_views, int64_t pair_capacity,
                      size_t* bytes_out) {
  if (!bytes_out) return fail_arg("bytes_out is NULL");
  RenderDims d;
  int rc = make_dims(s, n, n_frames, n_views, pair_capacity, d);
  if (rc) return rc;
  *bytes_out = make_layout(d).total;
  return GS_OK;
}

int gs_workspace_describe(const gs_settings* s, int32_t n, int32_t n_frames, int32_t n_views,
                          int64_t pair_capacity, gs_workspace_layout* out) {
  if (!out) return fail_arg("out is NULL");
  RenderDims d;
  int rc = make_dims(s, n, n_frames, n_views, pair_capacity, d);
  if (rc) return rc;
  Layout lo = make_layout(d);
  out->status = lo.status;
  out->records = lo.records;
  out->rects = lo.rects;
  out->keys = lo.keys0;
  out->vals = lo.vals0;
  out->ranges = lo.ranges;
  out->lists = lo.lists;
  out->t_final = lo.t_final;
  out->n_last = lo.n_last;
  out->grad2d = lo.grad2d;
  out->composed = lo.composed;
  out->total = lo.total;
  out->tiles_x = d.TX;
  out->tiles_y = d.TY;
  out->pair_capacity = (int64_t)d.capacity;
  return GS_OK;
}

int gs_render_forward(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                      const float* residuals, int32_t n_views, const gs_camera* cams, float* image, void* ws,
                      size_t ws_bytes, void* stream) {
  RenderDims d;
  // the pair capacity is whatever the workspace holds after the fixed regions
  int rc = make_dims(s, n, n_frames, n_views, 0, d);
  if (rc) return rc;
  if ((n > 0 && !params) || !cams || !image || !ws) return fail_arg("NULL buffer");
  if (d.Rc > 0 && !residuals) return fail_arg("res_channels > 0 needs residuals");
  if (!d.Rc && residuals) return fail_arg("residuals given but res_channels == 0");
  Layout lo0 = make_layout(d);
  if (ws_bytes < lo0.total) {
    g_last_error = "workspace too small";
    return GS_ERR_WORKSPACE;
  }
  set_capacity(d, lo0, ws_bytes);
  const Layout lo = make_layout(d);
  if ((rc = check_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  hipError_t e;
  if (d.Rc > 0 && n > 0) {
    if ((e = launch_compose_fwd(d, params, residuals, (float*)(w + lo.composed), st)) != hipSuccess)
      return fail_hip(e, "compose_fwd");
  }
  if (n > 0) {
    if ((e = launch_project_fwd(d, params, d.Rc > 0 ? residuals : nullptr, (const float*)(w + lo.composed), cams, w, lo, st)) != hipSuccess)
      return fail_hip(e, "project_fwd");
    uint32_t *sk, *sv;
    if ((e = launch_sort(d, w, lo, &sk, &sv, st)) != hipSuccess) return fail_hip(e, "sort");
    if ((e = launch_bin(d, sk, sv, w, lo, st)) != hipSuccess) return fail_hip(e, "bin");
  } else {
    if ((e = launch_bin(d, nullptr, nullptr, w, lo, st)) != hipSuccess) return fail_hip(e, "bin");
  }
  if ((e = launch_raster_fwd(d, w, lo, image, st)) != hipSuccess) return fail_hip(e, "raster_fwd");
  return GS_OK;
}

int gs_render_backward(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                       const float* residuals, int32_t n_views, const gs_camera* cams, const float* image,
                       const float* d_image, const float* target, float* d_params, float* d_residuals,
                       float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  RenderDims d;
  int rc = make_dims(s, n, n_frames, n_views, 0, d);
  if (rc) return rc;
  if ((n > 0 && (!params || !d_params)) || !cams || !ws) return fail_arg("NULL buffer");
  if ((d_image == nullptr) == (target == nullptr)) return fail_arg("exactly one of d_image and target");
  if (target && !image) return fail_arg("the fused L1 gradient needs the forward image");
  if (d.Rc > 0 && !residuals) return fail_arg("res_channels > 0 needs residuals");
  if (!d.Rc && (residuals || d_residuals)) return fail_arg("residuals given but res_channels == 0");
  Layout lo0 = make_layout(d);
  if (ws_bytes < lo0.total) {
    g_last_error = "workspace too small";
    return GS_ERR_WORKSPACE;
  }
  set_capacity(d, lo0, ws_bytes);
  const Layout lo = make_layout(d);
  if ((rc = check_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  hipError_t e;
  if ((e = launch_zero(w + lo.status + offsetof(Status, bwd_evals), 16, st)) != hipSuccess) return fail_hip(e, "zero");
  if (d.det && (e = launch_zero(w + lo.loss_fx, 16, st)) != hipSuccess) return fail_hip(e, "zero");
  if (n == 0) {
    if (loss_out || target) {
      // the loss of an empty scene still depends on the background; run the raster backward for it
      if ((e = launch_raster_bwd(d, w, lo, image, d_image, target, loss_out, st)) != hipSuccess)
        return fail_hip(e, "raster_bwd");
      if (d.det && (e = launch_fx_finish(d, w, lo, loss_out, st)) != hipSuccess) return fail_hip(e, "fx_finish");
    }
    return GS_OK;
  }
  if ((e = launch_zero(w + lo.grad2d, (size_t)d.B * d.n * kGradStride * 4, st)) != hipSuccess) return fail_hip(e, "zero");
  if (d.det && (e = launch_zero(w + lo.grad2d_fx, (size_t)d.B * d.n * 9 * 16, st)) != hipSuccess)
    return fail_hip(e, "zero");
  if (d.Rc > 0 && (e = launch_zero(w + lo.d_composed, (size_t)d.F * d.Rc * d.n * 4, st)) != hipSuccess)
    return fail_hip(e, "zero");
  if ((e = launch_raster_bwd(d, w, lo, image, d_image, target, loss_out, st)) != hipSuccess)
    return fail_hip(e, "raster_bwd");
  if (d.det && (e = launch_fx_finish(d, w, lo, loss_out, st)) != hipSuccess) return fail_hip(e, "fx_finish");
  if ((e = launch_project_bwd(d, params, d.Rc > 0 ? residuals : nullptr, (const float*)(w + lo.composed), cams, w, lo, d_params,
                              st)) != hipSuccess)
    return fail_hip(e, "project_bwd");
  if (d.Rc > 0) {
    if ((e = launch_compose_bwd(d, params, residuals, (const float*)(w + lo.composed),
                                (const float*)(w + lo.d_composed), d_params, d_residuals, st)) != hipSuccess)
      return fail_hip(e, "compose_bwd");
  }
  return GS_OK;
}

int gs_check_status(void* ws, void* stream, int64_t* needed_pairs) {
  if (!ws) return fail_arg("ws is NULL");
  int rc = check_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Status h;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof(Status), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return fail_hip(e, "check_status copy");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_hip(e, "check_status sync");
  if (needed_pairs) *needed_pairs = (int64_t)h.needed_pairs;
  return h.overflow ? GS_ERR_PAIR_OVERFLOW : GS_OK;
}

int gs_autotune_render(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                       const float* residuals, int32_t n_views, const gs_camera* cams, float* image, float* d_params,
                       float* d_residuals, void* ws, size_t ws_bytes, void* stream, gs_settings* best,
                       float* times_ms) {
  if (!s || !best || !image || !ws) return fail_arg("NULL argument");
  RenderDims d;
  int rc = make_dims(s, n, n_frames, n_views, 0, d);
  if (rc) return rc;
  if (n > 0 && !d_params) return fail_arg("the timed backward needs d_params scratch");
  Layout lo0 = make_layout(d);
  if (ws_bytes < lo0.total) {
    g_last_error = "workspace too small";
    return GS_ERR_WORKSPACE;
  }
  set_capacity(d, lo0, ws_bytes);
  const Layout lo = make_layout(d);
  if ((rc = check_device())) return rc;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* chk = (unsigned long long*)((char*)ws + lo.check);
  const size_t img_words = (size_t)d.B * d.L * 3 * d.W * d.H;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);  // clean-up: the creation error is the one reported
    return fail_hip(hipErrorUnknown, "autotune events");
  }
  gs_settings cur = *s;
  cur.bin_chunk = d.bin_chunk;
  cur.row_seg = d.row_seg;
  cur.wave_layout = d.wave_layout;
  cur.lds_batch = d.batch;
  cur.bwd_pixels = d.bwd_pixels;
  unsigned long long ref = 0;
  bool have_ref = false;
  // one trial: forward, parity check of the image against the first trial, then two timed
  // forward + backward passes; *ms = -1 if the image differs
  auto trial = [&](const gs_settings& t, float* ms) -> int {
    int r = gs_render_forward(&t, n, params, n_frames, residuals, n_views, cams, image, ws, ws_bytes, stream);
    if (r) return r;
    hipError_t e = launch_checksum((const uint32_t*)image, img_words, chk, st);
    if (e != hipSuccess) return fail_hip(e, "checksum");
    if ((r = gs_check_status(ws, stream, nullptr))) return r;
    unsigned long long h = 0;
    if ((e = hipMemcpyAsync(&h, chk, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return fail_hip(e, "checksum copy");
    if (!have_ref) {
      ref = h;
      have_ref = true;
    } else if (h != ref) {
      *ms = -1.f;
      return GS_OK;
    }
    if ((e = hipEventRecord(e0, st)) != hipSuccess) return fail_hip(e, "event");
    for (int k = 0; k < 2; ++k) {
      if ((r = gs_render_forward(&t, n, params, n_frames, residuals, n_views, cams, image, ws, ws_bytes, stream)))
        return r;
      if ((r = gs_render_backward(&t, n, params, n_frames, residuals, n_views, cams, image, image, nullptr, d_params,
                                  d_residuals, nullptr, ws, ws_bytes, stream)))
        return r;
    }
    if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
      return fail_hip(e, "event");
    float el = 0.f;
    if ((e = hipEventElapsedTime(&el, e0, e1)) != hipSuccess) return fail_hip(e, "event");
    *ms = 0.5f * el;
    return GS_OK;
  };
  // greedy: the wave layout, then the binning chunk, then the row segment, then the LDS batch, then
  // the backward's pixels per lane
  static const int32_t kLayouts[2] = {1, 2}, kChunks[3] = {512, 1024, 2048}, kSegs[3] = {1024, 2048, 4096},
                       kBatches[3] = {64, 128, 256}, kBwdPix[2] = {1, 2};
  int ti = 0;
  auto field = [](gs_settings& g, int phase) -> int32_t& {
    return phase == 0 ? g.wave_layout : phase == 1 ? g.bin_chunk : phase == 2 ? g.row_seg
                      : phase == 3 ? g.lds_batch : g.bwd_pixels;
  };
  for (int phase = 0; phase < 5 && rc == GS_OK; ++phase) {
    const int32_t* vals = phase == 0 ? kLayouts : phase == 1 ? kChunks : phase == 2 ? kSegs
                        : phase == 3 ? kBatches : kBwdPix;
    const int nv = (phase == 0 || phase == 4) ? 2 : 3;
    float best_ms = -1.f;
    int32_t best_v = field(cur, phase);
    for (int k = 0; k < nv && rc == GS_OK; ++k) {
      gs_settings t = cur;
      field(t, phase) = vals[k];
      float ms = -1.f;
      rc = trial(t, &ms);
      if (times_ms) times_ms[ti] = ms;
      ++ti;
      if (rc == GS_OK && ms >= 0.f && (best_ms < 0.f || ms < best_ms)) {
        best_ms = ms;
        best_v = vals[k];
      }
    }
    field(cur, phase) = best_v;
  }
  // clean-up of the timing events; the trials' own status is what this call reports
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == GS_OK) *best = cur;
  return rc;
}

int gs_set_work_counters(int enable) { return g_work_counting.exchange(enable ? 1 : 0); }

int gs_set_deterministic(int enable) { return g_deterministic.exchange(enable ? 1 : 0); }

int gs_workspace_stats(void* ws, void* stream, gs_stats* out) {
  if (!ws || !out) return fail_arg("NULL argument");
  int rc = check_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Status h;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof(Status), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_hip(e, "workspace_stats");
  out->overflow = (int32_t)h.overflow;
  out->needed_pairs = (int64_t)h.needed_pairs;
  out->fwd_evals = (int64_t)h.fwd_evals;
  out->fwd_contribs = (int64_t)h.fwd_contribs;
  out->bwd_evals = (int64_t)h.bwd_evals;
  out->bwd_contribs = (int64_t)h.bwd_contribs;
  return GS_OK;
}

const char* gs_error_string(int code) {
  switch (code) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID_ARG: return "invalid argument";
    case GS_ERR_WORKSPACE: return "workspace too small";
    case GS_ERR_PAIR_OVERFLOW: return "pair list capacity exceeded";
    case GS_ERR_HIP: return "HIP runtime error";
    case GS_ERR_NO_DEVICE: return "no gfx950 device";
    case GS_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

const char* gs_last_error(void) { return g_last_error.c_str(); }

int gs_zero(void* p, size_t bytes, void* stream) {
  if (!p && bytes) return fail_arg("NULL buffer");
  if (bytes % 4) return fail_arg("bytes must be a multiple of 4");
  hipError_t e = launch_zero(p, bytes, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : fail_hip(e, "zero");
}

int gs_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return GS_OK;
}

int gs_profile_collect(int32_t max_ids, double* total_ms, int32_t* counts) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (int k = 0; k < max_ids; ++k) {
    if (total_ms) total_ms[k] = 0.0;
    if (counts) counts[k] = 0;
  }
  int rc = GS_OK;
  for (auto& r : g_prof_recs) {
    hipError_t e = r.ended ? hipEventSynchronize(r.b) : hipErrorNotReady;
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) rc = fail_hip(e, r.ended ? "profile" : "profile: a kernel's end event was not recorded");
    if (r.id < max_ids) {
      if (total_ms) total_ms[r.id] += ms;
      if (counts) counts[r.id] += 1;
    }
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return rc;
}

const char* gs_kernel_name(int32_t id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : "?"; }

int gs_peak_fma(int32_t blocks, int32_t iters, float x, float y, float* out, void* stream) {
  if (blocks < 1 || iters < 1 || !out) return fail_arg("gs_peak_fma: need blocks >= 1, iters >= 1, out");
  hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, x, y, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : fail_hip(e, "peak_fma");
}

int gs_peak_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes % 16) return fail_arg("gs_peak_copy: need src, dst and bytes a multiple of 16");
  const size_t n = bytes / 16;
  if (n == 0) return GS_OK;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(k_peak_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src, (float4*)dst,
                     n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : fail_hip(e, "peak_copy");
}


}  // extern "C"
