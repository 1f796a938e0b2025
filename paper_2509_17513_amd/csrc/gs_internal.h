// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs4d.h"

namespace gs {

constexpr int kTile = 16;            // screen tile edge (pixels); one tile = one 256-thread block
constexpr int kTilePix = kTile * kTile;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortChunk = kSortThreads * kSortItems;  // keys per radix block
// Launch shapes of the binning (gs_settings bin_chunk / row_seg): defaults and the smallest
// values, for which the workspace histograms are sized.
constexpr int kBinChunk = 1024;      // depth-sorted Gaussians per row-binning wave
constexpr int kBinChunkMin = 512;
constexpr int kRowSeg = 2048;        // row-list entries per tile-binning wave
constexpr int kRowSegMin = 1024;
constexpr int kMaxTilesX = 128;      // tile columns one tile-binning wave covers (two per lane)
constexpr int kMaxTilesPerView = 16384;
constexpr int kMaxLevels = 8;
constexpr int kGradStride = 16;      // floats per (view, Gaussian) gradient record (9 used, 64-byte aligned)
constexpr int kGradLds = 10;         // LDS row stride of the per-entry gradient sums

// Status word at the start of the workspace.
struct Status {
  uint32_t overflow;      // 1 if the pair list did not fit
  uint32_t pad;
  unsigned long long needed_pairs;
  // work counters of the last forward / backward raster pass:
  // evals = (pixel, list entry) pairs whose Gaussian weight was evaluated,
  // contribs = (pixel, entry, layer) compositing updates
  unsigned long long fwd_evals, fwd_contribs, bwd_evals, bwd_contribs;
};

// Everything a kernel needs to know about one render call.
struct RenderDims {
  int n, F, V, B, W, H, TX, TY, T;  // T = tiles per view
  int deg, C, K, L, Rc;
  int lv[kMaxLevels];
  float lw[kMaxLevels];
  float near_plane, dilation, alpha_min, alpha_max, t_stop;
  float bg[3];
  int n_sort_chunks, n_bin_chunks, n_row_segs;
  int bin_chunk, row_seg;             // launch shapes of the binning
  int wave_layout;                    // 1: 8x8 quadrant per wave, 2: 16x4 strip per wave
  int batch;                          // list entries staged in LDS per round of the raster passes
  int bwd_pixels;                     // pixels per lane of the backward raster: 1 or 2
  int det;                            // deterministic backward (gs_set_deterministic)
  int n_bin_chunks_max, n_row_segs_max;  // at the smallest shapes (workspace sizing)
  unsigned long long capacity;      // (tile, Gaussian) pairs
  unsigned long long row_capacity;  // (tile row, Gaussian) pairs
};

// Byte offsets inside the workspace.
struct Layout {
  size_t status, records, rects, keys0, vals0, keys1, vals1, sort_hist, bin_rec, bin_hist, row_tot, row_ranges,
      tile_hist, tile_tot, ranges, t_final, n_last, grad2d, composed, d_composed, check, grad2d_fx, loss_fx, lists,
      row_lists, total;
};

Layout make_layout(const RenderDims& d);

// Whether the raster passes count their work (gs_set_work_counters; off by default).
bool work_counting();
// Whether the backward runs its deterministic variant (gs_set_deterministic; off by default).
bool deterministic();

// ---- launchers (gs_render.hip) ----
hipError_t launch_compose_fwd(const RenderDims& d, const float* params, const float* res, float* composed,
                              hipStream_t st);
hipError_t launch_project_fwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const gs_camera* cams, char* ws, const Layout& lo, hipStream_t st);
hipError_t launch_sort(const RenderDims& d, char* ws, const Layout& lo, uint32_t** keys_out, uint32_t** vals_out,
                       hipStream_t st);
hipError_t launch_bin(const RenderDims& d, const uint32_t* skeys, const uint32_t* svals, char* ws, const Layout& lo,
                      hipStream_t st);
hipError_t launch_raster_fwd(const RenderDims& d, char* ws, const Layout& lo, float* image, hipStream_t st);
hipError_t launch_raster_bwd(const RenderDims& d, char* ws, const Layout& lo, const float* image,
                             const float* d_image, const float* target, float* loss_out, hipStream_t st);
// deterministic backward: the fixed-point sums of the raster backward into grad2d (and loss_out +=)
hipError_t launch_fx_finish(const RenderDims& d, char* ws, const Layout& lo, float* loss_out, hipStream_t st);
hipError_t launch_project_bwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const gs_camera* cams, char* ws, const Layout& lo, float* d_params, hipStream_t st);
hipError_t launch_compose_bwd(const RenderDims& d, const float* params, const float* res, const float* composed,
                              const float* d_composed, float* d_params, float* d_res, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// Stable radix sort of n 32-bit (key, value) pairs (one segment): the input is in keys[0]/vals[0],
// keys[1]/vals[1] and hist (radix_hist_words(n) words) are scratch; *_out name the result.
size_t radix_hist_words(int n);
hipError_t launch_radix_sort(int n, uint32_t* keys[2], uint32_t* vals[2], uint32_t* hist, uint32_t** keys_out,
                             uint32_t** vals_out, hipStream_t st);
// order-sensitive 64-bit checksum of n words (written to *out, which it zeroes first)
hipError_t launch_checksum(const uint32_t* p, size_t n, unsigned long long* out, hipStream_t st);

// ---- error reporting shared by the entry points of every source file (gs_api.hip) ----
int report_arg(const char* msg);                      // sets gs_last_error, returns GS_ERR_INVALID_ARG
int report_hip(hipError_t e, const char* where);      // sets gs_last_error, returns GS_ERR_HIP
int require_device();                                 // GS_OK or GS_ERR_NO_DEVICE (checked once)

}  // namespace gs
