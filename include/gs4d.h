/* gs4d.h - C ABI of the MI355X (gfx950) differentiable Gaussian-splatting library.
 *
 * The library implements the rendering hot path of 4DGCPro (arXiv 2509.17513):
 * projection of anisotropic 3D Gaussians with spherical-harmonic colour
 * (Sec. 3.1, Eq. 1 and the covariance factorisation), front-to-back alpha
 * compositing of depth-ordered Gaussians (Eq. 2) for every nested layer
 * (progressive rendering, Eq. 4), frame composition of a group from its
 * keyframe and residuals (Sec. 3.2, pose update and Eq. 7), and the backward of
 * all of these (with the layer-weighted L1 colour loss fused, Sec. 3.3);
 * around it: the colour loss with its D-SSIM term (gs_color_loss), the rate of
 * the quantised attributes (a learned Laplace model, gs_rate_model; the empirical
 * histogram, gs_rate_histogram; the paper's KDE and Gaussian entropy models,
 * gs_entropy_model), the rigid-motion module of inter-frame training
 * (gs_motion_*), and the significance ranking and quantised 2D feature maps of
 * the progressive bitstream (gs_significance_order, gs_*_maps).
 *
 * General rules
 *  - Every buffer pointer is a DEVICE pointer owned by the caller, unless a
 *    parameter says "host". The library never allocates device memory; all
 *    scratch state lives in the caller's workspace `ws`.
 *  - Every launch is asynchronous on `stream` (a hipStream_t; NULL = the
 *    default stream). Only gs_check_status synchronises.
 *  - Functions return GS_OK (0) or a negative GS_ERR_* code. Argument checks
 *    happen on the host before any launch. HIP launch errors are reported as
 *    GS_ERR_HIP with a message available from gs_last_error().
 *  - Floating-point layouts are float32, planar ("[C][N]" = C rows of N).
 *  - Concurrent calls that share a workspace race; calls on different
 *    workspaces are independent.
 */
#ifndef GS4D_H
#define GS4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = -1,   /* bad size, pointer, degree or level layout */
  GS_ERR_WORKSPACE = -2,     /* ws_bytes smaller than gs_workspace_size() */
  GS_ERR_PAIR_OVERFLOW = -3, /* more (tile, Gaussian) pairs than pair_capacity */
  GS_ERR_HIP = -4,           /* a HIP runtime call or launch failed */
  GS_ERR_NO_DEVICE = -5,     /* no gfx950 device is visible */
  GS_ERR_UNSUPPORTED = -6    /* a valid request this build does not implement */
};

/* One pinhole camera (64 bytes). Cameras are passed as a DEVICE array of
 * F * V entries, frame-major (camera of frame f, view v at f * V + v).
 * viewmat is the row-major world-to-camera [R | t] (3 x 4) with OpenCV axes
 * (x right, y down, z forward). Pixel (u, v) is sampled at (u + 0.5, v + 0.5). */
typedef struct {
  float viewmat[12];
  float fx, fy, cx, cy;
} gs_camera;

/* Render settings (host struct, read at call time).
 *  sh_degree     0..3; the parameter array has C = 11 + 3 (sh_degree + 1)^2 rows.
 *  n_levels      1..8 nested layers; level_counts ascending, the last == n.
 *                Layer l renders the Gaussians with index < level_counts[l]
 *                (progressive rendering over the index sets N^l, Eq. 4).
 *  level_weights lambda^l of the layer-weighted loss (App. A uses 0.5 / l for
 *                l < L and 1 for l = L); used by the fused L1 gradient.
 *  res_channels  0 (no residuals), 8 (translation 3, rotation quaternion 4,
 *                opacity logit 1), 11 (+ log-scale 3) or 11 + 3 (d+1)^2 (+ SH).
 *  near_plane    Gaussians whose camera depth is <= near_plane are culled. The
 *                depth is computed in FP64 from the frame mean composed in FP64;
 *                its float32 rounding is the depth-order key (ties by index).
 *  dilation      added to the diagonal of every 2D covariance (pixels^2).
 *  alpha_min     a Gaussian contributes to a pixel iff min(alpha_max, o G) >= alpha_min.
 *  alpha_max     upper clamp of the per-pixel alpha; must be < 1 (the backward
 *                divides by 1 - alpha), else GS_ERR_INVALID_ARG.
 *  t_stop        compositing stops before a Gaussian that would bring the
 *                transmittance below t_stop (that Gaussian is not included).
 *  bg            background colour added with the final transmittance.
 *  tile_w/tile_h screen tile in pixels; 0/0 selects 16 x 16, the only shape
 *                this build implements.
 *  bin_chunk, row_seg, wave_layout   launch shapes; every value renders the same
 *                images bit for bit (gs_autotune_render picks them for a workload):
 *    bin_chunk   depth-sorted Gaussians per row-binning wave: 0 (= 1024), 512, 1024, 2048
 *    row_seg     row-list entries per tile-binning wave: 0 (= 2048), 1024, 2048, 4096
 *    wave_layout pixels of the four waves of a 16 x 16 tile: 0 or 1 = 8 x 8 quadrants,
 *                2 = 16 x 4 strips
 *    lds_batch   list entries the raster passes stage in LDS per round: 0 (= 256), 64, 128, 256
 *    bwd_pixels  pixels per lane of the backward raster: 0 or 1 (a 256-thread block per 16 x 16
 *                tile), 2 (a 128-thread block, two rows apart per lane); gradients agree up to
 *                the order of float additions
 *                The workspace size does not depend on them. */
typedef struct {
  int32_t width, height;
  int32_t sh_degree;
  int32_t n_levels;
  int32_t level_counts[8];
  float level_weights[8];
  int32_t res_channels;
  float near_plane, dilation, alpha_min, alpha_max, t_stop;
  float bg[3];
  int32_t tile_w, tile_h;
  int32_t bin_chunk, row_seg, wave_layout;
  int32_t lds_batch;
  int32_t bwd_pixels;
} gs_settings;

/* Bytes of workspace needed for a render of n Gaussians, n_frames frames of
 * n_views views each, with room for pair_capacity (tile, Gaussian) pairs.
 * A forward that needs more pairs flags GS_ERR_PAIR_OVERFLOW, reported by
 * gs_check_status together with the number it needed. */
int gs_workspace_size(const gs_settings* s, int32_t n, int32_t n_frames, int32_t n_views,
                      int64_t pair_capacity, size_t* bytes_out);

/* Byte offsets of the workspace regions (for inspection by tests). */
typedef struct {
  size_t status, records, rects, keys, vals, ranges, lists, t_final, n_last, grad2d, composed;
  size_t total;
  int32_t tiles_x, tiles_y;
  int64_t pair_capacity;
} gs_workspace_layout;
int gs_workspace_describe(const gs_settings* s, int32_t n, int32_t n_frames, int32_t n_views,
                          int64_t pair_capacity, gs_workspace_layout* out);

/* Forward render (Eq. 2 for every layer of Eq. 4, every view and frame).
 *  params     [C][n] keyframe parameters: 0..2 mean, 3..5 log-scale,
 *             6..9 rotation quaternion (w, x, y, z; need not be unit),
 *             10 opacity logit, 11 + 3k + c SH coefficient k of colour c.
 *             Activations: scale = exp, opacity = sigmoid, rotation = R(q/|q|).
 *  residuals  [n_frames][res_channels][n] per-frame deltas, or NULL (then
 *             every frame renders the keyframe). Frame f composes the
 *             keyframe with the deltas of frames 0..f: means, logit,
 *             log-scales and SH add; rotation q_f = dq_f (x) q_{f-1}.
 *  cams       DEVICE [n_frames * n_views] cameras.
 *  image      [n_frames][n_views][n_levels][3][height][width] output.
 *  ws         workspace of at least gs_workspace_size() bytes; it keeps the
 *             state the backward needs, so do not reuse it in between. */
int gs_render_forward(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                      const float* residuals, int32_t n_views, const gs_camera* cams, float* image,
                      void* ws, size_t ws_bytes, void* stream);

/* Backward of the last gs_render_forward made with the same arguments and ws.
 *  d_image    dL/d image in the image layout, or NULL when target != NULL.
 *  target     [n_frames][n_views][3][height][width]: fuse the gradient of
 *             L = sum_{f,v,l} lambda^l mean_{pixel,channel} |C^l - target|
 *             (needs image = the forward's output); NULL when d_image != NULL.
 *  d_params   [C][n], accumulated (+=).
 *  d_residuals[n_frames][res_channels][n], accumulated (+=), or NULL.
 *  loss_out   one float, accumulated (+=) with L in the fused mode, or NULL. */
int gs_render_backward(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                       const float* residuals, int32_t n_views, const gs_camera* cams, const float* image,
                       const float* d_image, const float* target, float* d_params, float* d_residuals,
                       float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* Colour loss of a render with its D-SSIM term, and its gradient (Sec. 3.3: the colour loss of
 * every layer, L^l = (1 - lambda_ssim) L1 + lambda_ssim D-SSIM, weighted by lambda^l):
 *   L = sum_{f,v,l} lambda^l [ (1 - lambda_ssim) mean |C^l - target|
 *                              + lambda_ssim (1 - mean SSIM(C^l, target)) ]
 * with the means over pixels and channels. SSIM is computed per channel with an 11 x 11
 * Gaussian window (sigma 1.5) that sees zeros outside the image, C1 = 0.01^2, C2 = 0.03^2.
 * lambda_ssim = 0 gives the L1 loss of gs_render_backward's fused mode.
 *  s          width, height, n_levels and level_weights are used; the rest is ignored.
 *  image      [n_frames][n_views][n_levels][3][height][width] (gs_render_forward's output)
 *  target     [n_frames][n_views][3][height][width]
 *  lambda_ssim in [0, 1] (the paper pre-trains with 0.2)
 *  d_image    dL/dC in the image layout (overwritten), to pass to gs_render_backward; or NULL
 *             for the loss alone (then ws may be NULL)
 *  loss_out   one float, accumulated (+=) with L, or NULL
 *  ws         workspace of gs_color_loss_workspace_size() bytes (three floats per image
 *             element: the per-pixel SSIM derivatives); independent of the render workspace.
 * Errors: GS_ERR_INVALID_ARG for sizes, NULL buffers or lambda_ssim outside [0, 1];
 * GS_ERR_WORKSPACE when ws_bytes is too small. */
int gs_color_loss_workspace_size(const gs_settings* s, int32_t n_frames, int32_t n_views, size_t* bytes_out);
int gs_color_loss(const gs_settings* s, int32_t n_frames, int32_t n_views, const float* image, const float* target,
                  float lambda_ssim, float* d_image, float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* Significance order (Sec. 3.1): Psi_i = sigmoid(logit_i) + lambda_psi (4/3) pi a_i b_i c_i with
 * a, b, c = exp(log-scales), in FP32; Gaussians ranked by Psi descending, ties by lower index
 * (App. A uses lambda_psi = 1e5). Layer l of the hierarchy is then ranks [N_{l-1}, N_l).
 *  params     [n_channels][n] (rows 3..5 log-scale and 10 opacity logit are read)
 *  order      [n] int32 output: order[r] = index of the Gaussian of rank r
 *  psi        [n] float output (Psi of every Gaussian, by index), or NULL
 *  ws         gs_significance_workspace_size(n) bytes (sort keys, values and histograms)
 * Errors: GS_ERR_INVALID_ARG (n < 0, n_channels < 11, lambda_psi negative or not finite, NULL
 * buffers), GS_ERR_WORKSPACE. */
int gs_significance_workspace_size(int32_t n, size_t* bytes_out);
int gs_significance_order(int32_t n, const float* params, int32_t n_channels, float lambda_psi, int32_t* order,
                          float* psi, void* ws, size_t ws_bytes, void* stream);

/* 2D feature maps of a layered Gaussian set, up to the video codec (Sec. 3.3, progressive
 * bitstream: per layer, differential quantisation with 16-bit positions and 8-bit other
 * attributes, each channel flattened into one 2D image).
 * Layer l holds the Gaussians of ranks [level_counts[l-1], level_counts[l]). Every channel of a
 * layer is quantised with that layer's minimum and maximum,
 *   code = rint((v - min) * ((2^b - 1) / (max - min)))   (FP32, half to even; 0 if max == min)
 * with b = 16 for channels 0..2 (the mean) and 8 for the others; decoding is
 *   min + code * ((max - min) / (2^b - 1)).
 * A layer's m Gaussians are ordered by the Morton code of their position codes (top 10, 10, 9
 * bits of x, y, z; ties by rank) and written 256 at a time into 16 x 16 pixel blocks, the blocks
 * snaking row by row (odd block rows right to left) and the Gaussians of a block following the 2D
 * Morton curve inside it; the layer's maps are width = 16 ceil(ceil(sqrt m) / 16) by
 * height = 16 ceil(ceil(m / width) / 16) pixels and pixels past its m-th Gaussian repeat it.
 * Maps buffer: layer l at offset[l] holds its three 16-bit planes (channels 0..2) and then one
 * 8-bit plane per other channel, each plane row-major height x width. */
typedef struct {
  int32_t n_channels, n_levels;
  int32_t level_counts[8];
  int32_t width[8], height[8];
  int64_t offset[8];
  int64_t total_bytes;
} gs_maps_layout;

/* Fills the layout (host only; no device work). level_counts ascending, n_levels 1..8,
 * n_channels 11..1024. */
int gs_maps_describe(int32_t n_channels, int32_t n_levels, const int32_t* level_counts, gs_maps_layout* out);

/* Encodes params [n_channels][n] (n = the last level count), ranked by `order` (a permutation of
 * 0..n-1, as written by gs_significance_order), into the maps.
 *  ranges     [n_levels][n_channels][2] float output: (min, max) per layer and channel
 *  maps       output of layout->total_bytes bytes
 *  seq        [n] int32 output, or NULL: the Gaussian index at each layer's sequence position
 *             (layer l's positions at level_counts[l-1] + p, in map order)
 *  ws         gs_encode_workspace_size() bytes
 * The layout is re-validated (sizes and offsets must hold every layer). */
int gs_encode_workspace_size(const gs_maps_layout* layout, size_t* bytes_out);
int gs_encode_maps(const gs_maps_layout* layout, const float* params, const int32_t* order, float* ranges,
                   uint8_t* maps, int32_t* seq, void* ws, size_t ws_bytes, void* stream);

/* Decodes the maps into params_out [n_channels][n] in map order (layer by layer, sequence
 * position by position): the Gaussian set a client renders, with the same level_counts. */
int gs_decode_maps(const gs_maps_layout* layout, const uint8_t* maps, const float* ranges, float* params_out,
                   void* stream);

/* The paper's entropy models of the quantised attributes (Sec. 3.3), per layer and attribute:
 *  kind 0, keyframe attributes: a Gaussian KDE of the layer's symbols with Silverman's bandwidth
 *          h = sigma (3 m / 4)^(-1/5) (sigma the sample standard deviation of its m symbols; at
 *          least step / 4); its CDF on a grid of spacing min(step, h) / 4 from lo = min - 8 h - step
 *          to max + 8 h + step (at most 16384 points and 3071 a kernel side, widening the spacing),
 *          made by linearly binning the symbols and convolving the counts with the kernel's CDF,
 *          and taken between grid points by linear interpolation. The gradient holds the binned
 *          density fixed (binning has no derivative).
 *  kind 1, residual attributes: a normal CDF with the layer's symbol mean and standard deviation
 *          (1/m, at least step 1e-3); the gradient includes the mean's and deviation's dependence
 *          on every symbol. Adds the temporal term lambda^l lambda_reg |y| per symbol.
 * Symbols: mode 0 rint(y / step) step; mode 1 y + u step with u uniform in [-1/2, 1/2) from the
 * counter-based SplitMix64 generator of gs_rate_model (counter = offset + a n + i + 1). A symbol
 * costs -log2 max(F(y + step/2) - F(y - step/2), 1e-9) bits (the PMF as CDF differences), weighted
 * by w = lambda_rate lambda^l / |G^l| in the loss.
 *  attrs     [n_attr][n] (n = level_counts[n_levels-1]; layer l = symbols [N_{l-1}, N_l))
 *  bits_out  [n_attr] float64 per attribute bit totals (written), or NULL
 *  loss_out  one float64 (+= L), or NULL
 *  sym_bits  [n_attr][n] float per-symbol bits, or NULL
 *  d_attrs   [n_attr][n] (+= dL/dy, mode 1 only), or NULL
 *  ws        gs_entropy_workspace_size() bytes (about 130 MB per 336 (layer, attribute) pairs
 *            for the KDE, which keeps a full-size grid per pair)
 * All sums are taken in a fixed order: results do not depend on scheduling. */
typedef struct {
  int32_t n, n_attr;
  float step;
  int32_t mode;
  uint64_t seed, offset;
  int32_t n_levels;
  int32_t level_counts[8];
  float level_weights[8];
  float lambda_rate;
  int32_t kind;
  float lambda_reg;
} gs_entropy_desc;
int gs_entropy_workspace_size(const gs_entropy_desc* desc, size_t* bytes_out);
int gs_entropy_model(const gs_entropy_desc* desc, const float* attrs, double* bits_out, double* loss_out,
                     float* sym_bits, float* d_attrs, void* ws, size_t ws_bytes, void* stream);

/* Rigid-motion module of inter-frame training (Sec. 3.2, rigid transformation; Eq. 5-6): the
 * previous frame's positions are encoded by a multi-resolution hash grid (16 levels of 2
 * features, 2^15 entries per level, resolutions floor(16 b^l) from 16 to 1024; trilinear
 * interpolation of the cell corners, indexed densely while (N + 1)^3 <= 2^15, else by the
 * spatial hash (i ^ j 2654435761 ^ k 805459861) mod 2^15) inside the scene box, and two MLPs
 * (32 -> 64 -> 64 -> 3 and 32 -> 64 -> 64 -> 4, ReLU, FP32 on the matrix cores) predict each
 * Gaussian's translation d_mu and rotation quaternion dq = (1 + o0, o1, o2, o3), written as the
 * residual channels 0..6
 * of a frame (mu_t = mu_{t-1} + d_mu, q_t = dq (x) q_{t-1} in gs_render_forward's composition).
 *  table    [16][2^15][2] float features (gs_motion_sizes gives the float count)
 *  weights  W1 [64][32], b1, W2 [64][64], b2, W3 [3][64], b3 of the translation MLP, then the
 *           rotation MLP's with W3 [4][64], b3 (row-major [out][in]; gs_motion_sizes gives the
 *           count)
 *  means    rows 0..2 of an array of row stride row_stride (the previous frame's positions)
 *  out      rows 0..6 of an array of row stride row_stride (a frame's residual block)
 *  d_out    rows 0..6 of dL/d(those residuals), row stride row_stride
 *  d_table, d_weights   accumulated (+=): d_table from per-chunk partial tables summed in a
 *           second pass (no atomics into it), d_weights from per-wave partial sums added with
 *           float atomics
 *  ws       gs_motion_workspace_size(n) bytes (the feature gradients of the Gaussians, the
 *           waves' partial weight gradients and 8 partial tables of 4 MB)
 * Errors: GS_ERR_INVALID_ARG for n < 0, row_stride < n, a degenerate box or NULL buffers. */
typedef struct {
  int32_t n;
  float box_lo[3], box_hi[3];
} gs_motion_desc;
int gs_motion_sizes(int64_t* table_floats, int64_t* n_weights);
int gs_motion_workspace_size(int32_t n, size_t* bytes_out);
int gs_motion_forward(const gs_motion_desc* desc, const float* means, int32_t row_stride, const float* table,
                      const float* weights, float* out, void* stream);
int gs_motion_backward(const gs_motion_desc* desc, const float* means, int32_t row_stride, const float* table,
                       const float* weights, const float* d_out, float* d_table, float* d_weights, void* ws,
                       size_t ws_bytes, void* stream);

/* Autotuner of the render launch shapes (bin_chunk, row_seg, wave_layout, lds_batch, bwd_pixels
 * of gs_settings) for one workload: shapes picked by timed trials that must pass parity. Starting
 * from *s, it tries the wave layouts, then the binning chunk sizes, then the row-segment sizes,
 * then the LDS batch sizes, then the backward's pixels per lane, keeping the best of each before
 * moving on (13 trials). A trial renders the
 * forward once, requires an image bit-identical to the first trial's (checksum on the device)
 * and no pair-list overflow, then times two forward + backward passes between HIP events on
 * `stream` (the backward takes the image itself as dL/dC and accumulates into the scratch
 * d_params [C][n] and d_residuals [F][R][n] or NULL). Synchronises the stream.
 * *best receives *s with the five fields set; times_ms[13] (or NULL) each trial's time per
 * forward + backward, or -1 for a rejected trial. Returns GS_ERR_PAIR_OVERFLOW if the workspace
 * is too small for the pairs (grow it first: render once and check gs_check_status), and the
 * errors of gs_render_forward otherwise. */
int gs_autotune_render(const gs_settings* s, int32_t n, const float* params, int32_t n_frames,
                       const float* residuals, int32_t n_views, const gs_camera* cams, float* image, float* d_params,
                       float* d_residuals, void* ws, size_t ws_bytes, void* stream, gs_settings* best,
                       float* times_ms);

/* Synchronises `stream` and reports the status of the last forward on ws:
 * GS_ERR_PAIR_OVERFLOW (and *needed_pairs) if its pair list did not fit. */
int gs_check_status(void* ws, void* stream, int64_t* needed_pairs);

/* Work counters of the last forward and backward on ws (synchronises stream).
 *  fwd_evals / bwd_evals       (pixel, list entry) pairs whose Gaussian weight
 *                              was evaluated by the raster pass
 *  fwd_contribs / bwd_contribs (pixel, entry, layer) compositing updates
 * The raster passes count only while counting is enabled (gs_set_work_counters);
 * otherwise these four read 0. */
typedef struct {
  int32_t overflow, pad;
  int64_t needed_pairs, fwd_evals, fwd_contribs, bwd_evals, bwd_contribs;
} gs_stats;
int gs_workspace_stats(void* ws, void* stream, gs_stats* out);

/* Process-wide switch of the raster work counters (off at load): raster passes launched
 * while it is on run an instrumented variant of their kernels that also counts its work
 * (meant for measurement runs: on the 300k-Gaussian, 24-view workload its forward takes
 * about 1.8x and its backward 1.1x the time; images and gradients are identical up to
 * the order of float atomics). Host-only, thread-safe; takes effect at the next launch (a
 * captured graph keeps the variant it captured). Returns the previous setting. */
int gs_set_work_counters(int enable);

/* Process-wide switch of the deterministic backward (off at load), a debug aid: while it is on,
 * gs_workspace_size includes 144 bytes per (view, Gaussian) more and gs_render_backward runs a
 * variant whose gradients and loss are the same bits on every run with the same inputs. The raster
 * backward then adds each wave's per-entry sums into 128-bit fixed-point accumulators (the value
 * times 2^64, saturated at 2^62, bits below 2^-64 dropped) with integer atomics, whose result does
 * not depend on the order, and converts them once; every later sum of the backward already has a
 * fixed order. It uses one pixel per lane (bwd_pixels is ignored) and no work counters, and is
 * slower than the default, whose float atomics leave ulp-level run-to-run differences. Set it
 * before sizing the workspace and before the forward whose state the backward uses. Host-only,
 * thread-safe. Returns the previous setting. */
int gs_set_deterministic(int enable);

/* Text of an error code, and the last HIP error message of this thread. */
const char* gs_error_string(int code);
const char* gs_last_error(void);

/* ---------------------------------------------------------------- rate terms
 * The attributes whose rate is estimated are the non-position channels of the
 * parameter array (rotation, scale, opacity and SH: the set the keyframe rate
 * of Sec. 3.3 sums over), stored [n_attr][n]. Symbols are k = rint(y / step). */

/* 16 context features per Gaussian, written BF16 [n][16]:
 * mean / extent (3), sin and cos of pi 2^k mean / extent for k = 0, 1 (12),
 * (layer - 1) / 5 (1), where layer l holds the indices [level_counts[l-1], level_counts[l]).
 *  means  [3][n] float32 (the first three parameter rows). */
int gs_rate_context(int32_t n, const float* means, float extent, int32_t n_levels, const int32_t* level_counts,
                    uint16_t* ctx_out, void* stream);

/* Learned rate. For attribute a and symbol i a per-attribute MLP
 * 16 -> 64 -> 64 -> 2 (tanh-GELU; BF16 weights and activations on MFMA, FP32
 * accumulation and biases) maps the context to a Laplace location m = out0 and
 * scale b = softplus(out1) + step / 16; the symbol costs
 * -log2 max(F(y + step/2) - F(y - step/2), 1e-9) bits (the PMF of Sec. 3.3 as
 * CDF differences one step apart). mode 0 evaluates at y = rint(y/step) step;
 * mode 1 at y + u with u uniform in [-step/2, step/2) from the counter-based
 * SplitMix64 generator, counter = offset + a n + i + 1, state = seed + counter *
 * 0x9E3779B97F4A7C15, u = (mix >> 40) 2^-24 - 1/2 (quantisation simulated by
 * uniform noise, Sec. 3.3). The training loss is
 * L = sum_i w_i sum_a bits_{a,i}, w_i = lambda_rate lambda^l / |layer l| for
 * the layer of Gaussian i (per-layer rate weighted by the layer weight).
 *  attrs   [n_attr][n] float32;  ctx [n][16] BF16 (gs_rate_context)
 *  w_bf16  [n_attr][5248] BF16: W1 [64][16], W2 [64][64], W3 [2][64] row-major
 *  b_f32   [n_attr][130]: b1 [64], b2 [64], b3 [2]
 *  bits_out[n_attr] float64, accumulated (+=) with the unweighted bits per attribute
 *  loss_out[1] float64 (+= L) or NULL
 *  sym_bits[n_attr][n] float32 bits of every symbol (overwritten) or NULL
 *  d_attrs [n_attr][n] (+= dL/dy, mode 1 only) or NULL
 *  d_w, d_b same layouts as the weights (+=) or NULL: the gradient of the maximum-likelihood
 *          fit of the entropy model, L_fit = fit_scale sum_i sum_a bits_{a,i} (the entropy model
 *          is fitted to the attributes whatever lambda_rate is). No workspace. */
typedef struct {
  int32_t n, n_attr;
  float step;
  int32_t mode;
  uint64_t seed, offset;
  int32_t n_levels;
  int32_t level_counts[8];
  float level_weights[8];
  float lambda_rate;
  float fit_scale;
  int32_t blocks_per_attr; /* launch blocks per attribute; 0 = the library default (64, fewer when
                              n is small); gs_rate_autotune picks one for a given workload */
  const uint64_t* offset_dev; /* device word holding the noise counter offset, read when the kernel
                                 runs (then `offset` is ignored), or NULL: lets a captured graph
                                 draw new noise on every replay (gs_advance_counters) */
} gs_rate_desc;
int gs_rate_model(const gs_rate_desc* desc, const float* attrs, const uint16_t* ctx, const uint16_t* w_bf16,
                  const float* b_f32, double* bits_out, double* loss_out, float* sym_bits, float* d_attrs, float* d_w,
                  float* d_b, void* stream);

/* Launch-shape autotuner of gs_rate_model (the rate MLP's only free parameter: how many
 * blocks share an attribute's symbols; it changes the summation order, not the result).
 * Runs desc with blocks_per_attr in {16, 32, 64, 128, 256} (clamped to the work available) on
 * the caller's inputs, once untimed and then 3 times between HIP events on `stream`; a
 * candidate qualifies if its bits agree with the first candidate's to 1e-5 relative.
 * Synchronises the stream. bits_scratch [5][n_attr] float64 (overwritten); d_attrs, d_w, d_b
 * as in gs_rate_model (accumulated into; pass the buffers of the calls being tuned, or NULL, so
 * that the timed work is the same). *best_blocks receives the fastest qualifying value;
 * times_ms [5] (or NULL) the mean time of each candidate, or -1 for one that disagreed.
 * Returns GS_ERR_INVALID_ARG as gs_rate_model does, GS_ERR_HIP on a launch or event error. */
int gs_rate_autotune(const gs_rate_desc* desc, const float* attrs, const uint16_t* ctx, const uint16_t* w_bf16,
                     const float* b_f32, double* bits_scratch, float* d_attrs, float* d_w, float* d_b, void* stream,
                     int32_t* best_blocks, float* times_ms);

/* Initial output bias of the learned rate's Laplace head from the attributes themselves (a
 * starting point for training, Sec. 3.3 fits the entropy model jointly): for each attribute a,
 * b[a][128] = mean(y) and b[a][129] = softplus^-1(max(MAD - step/16, step/4)) with MAD the mean
 * absolute deviation, so that the untrained network starts at the context-free Laplace fit.
 * Other entries of b are left as they are. attrs [n_attr][n] float32, b_f32 [n_attr][130],
 * acc [2 n_attr] float64 device scratch (overwritten). n >= 1. */
int gs_rate_init_output_bias(int32_t n, int32_t n_attr, const float* attrs, float step, float* b_f32, double* acc,
                             void* stream);

/* Empirical-histogram rate (the reference the learned rate is checked against): per attribute
 * bits = -sum_i log2(count(k_i) / n) = n H over its symbol histogram, in FP64.
 * bits_out [n_attr] float64 (overwritten). The symbol range of one attribute
 * must span at most 65536 symbols (else bits_out is left undefined and the
 * status word of ws is non-zero). ws holds gs_rate_histogram_workspace_size bytes. */
int gs_rate_histogram_workspace_size(int32_t n_attr, size_t* bytes_out);
int gs_rate_histogram(int32_t n, int32_t n_attr, const float* attrs, float step, double* bits_out, void* ws,
                      size_t ws_bytes, void* stream);

/* gs_rate_histogram for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same kernels and result,
 * with the workspace in a fixed scratch array of the library (16.8 MB per GPU, held until the
 * process ends) instead of a caller's buffer. The caller passes device attrs [n_attr][n] and
 * bits_out [n_attr] float64 (overwritten). n_attr may be at most 64, else GS_ERR_INVALID_ARG;
 * the symbol range rule of gs_rate_histogram applies. The call allocates nothing and does not
 * synchronise. Every call on one GPU shares that GPU's scratch (it starts each call by clearing
 * it): calls that overlap on one GPU, on different streams or threads, race. Returns
 * GS_ERR_NO_DEVICE without a current device, GS_ERR_HIP on a launch error. */
int gs_rate_histogram_noalloc(int32_t n, int32_t n_attr, const float* attrs, float step, double* bits_out,
                              void* stream);

/* Adam step on float32 masters (bias-corrected, t = step >= 1); grads are
 * zeroed after use; bf16_copy (or NULL) receives the BF16 rounding of the
 * updated parameters (the MFMA copy of the MLP weights). */
int gs_adam_step(int64_t n, float* params, float* grads, float* m, float* v, uint16_t* bf16_copy, float lr,
                 float beta1, float beta2, float eps, int32_t step, void* stream);

/* gs_adam_step with the step number read from the device word step_dev when the kernel runs,
 * so that a captured training step replays with the right bias corrections; and the kernel that
 * advances such counters (step_dev += 1, offset_dev += offset_delta; either may be NULL) at the
 * end of a captured step. */
int gs_adam_step_dev(int64_t n, float* params, float* grads, float* m, float* v, uint16_t* bf16_copy, float lr,
                     float beta1, float beta2, float eps, const int32_t* step_dev, void* stream);
int gs_advance_counters(int32_t* step_dev, uint64_t* offset_dev, uint64_t offset_delta, void* stream);

/* Zero-fills bytes (a multiple of 4) of device memory with a kernel (no memset node, so it is
 * safe inside captured graphs). */
int gs_zero(void* p, size_t bytes, void* stream);

/* Measurement kernels for the attainable peaks the hot kernels are compared with (not part of
 * the method). gs_peak_fma: blocks x 256 threads, each running 8 independent float32 FMA chains
 * of iters rounds (16 iters flops per thread), writing one float per thread to out [blocks x 256].
 * gs_peak_copy: a plain copy of bytes (a multiple of 16) from src to dst in 16-byte vectors
 * (also the reference kernel for calibrating HBM byte counters). Both asynchronous. */
int gs_peak_fma(int32_t blocks, int32_t iters, float x, float y, float* out, void* stream);
int gs_peak_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Per-kernel timing. While enabled, every kernel launch of the library is
 * bracketed by HIP events recorded on its launch stream (do not enable it
 * during hipGraph capture). gs_profile_collect waits for the recorded events,
 * writes the summed milliseconds and launch counts per kernel id
 * (0 <= id < max_ids; gs_kernel_name gives the names) and clears the record. */
int gs_profile_enable(int on);
int gs_profile_collect(int32_t max_ids, double* total_ms, int32_t* counts);
const char* gs_kernel_name(int32_t id);

#ifdef __cplusplus
}
#endif
#endif /* GS4D_H */
