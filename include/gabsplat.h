/*
 * gabsplat.h -- C ABI of the MI355X (gfx950) 3D Gabor splatting rasterizer.
 *
 * The library implements the tile-based differentiable rasterizer for 3D Gabor
 * primitives: each primitive is a 3D Gaussian envelope (Sec. 3.1, Eq.
 * 3d_gaussian) modulated by a bank of K directional cosine terms (Sec. 3.2,
 * the 3D Gabor-based primitive), projected to the image plane with the EWA
 * covariance (Sec. 3.1) and the frequency projection + z-integration of
 * Sec. 3.3.1-3.3.2 (derived in supplementary A.1-A.2), and alpha-blended front
 * to back (Sec. 3.3.3).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers unless stated otherwise; the
 *    struct arguments themselves (gabsplat_scene, gabsplat_camera,
 *    gabsplat_geom) live in HOST memory.
 *  - The caller owns every buffer.  The library never allocates, frees or
 *    synchronises; every call only enqueues work on `stream` (a hipStream_t,
 *    passed as void*; NULL = the default stream) and returns.
 *  - Calls return a gabsplat_status; no C++ exception crosses the ABI.  On an
 *    error status nothing has been enqueued unless stated otherwise.
 *  - Attribute values are ACTIVATED: scales > 0, opacities in (0,1), weights
 *    >= 0 (the paper applies exp / sigmoid before rasterizing, Sec. 3.4.1).
 *    Quaternions are normalised inside and gradients are taken w.r.t. the
 *    unnormalised input.
 *  - Layouts are fp32.  Attributes that every call reads for every primitive
 *    (means, scales, quaternions, opacities, frequencies, weights) are planar
 *    structure-of-arrays, attribute-major: element (attribute a, primitive i)
 *    of an array with A attributes is at a*n + i.  Colour coefficients (sh or
 *    colors), which only the visible primitives need, are stored per
 *    primitive: element (a, i) of a colour array with A values per primitive
 *    is at i*A + a, so that reading a visible primitive's colour touches only
 *    its own row.
 *  - An "item" is a (view, primitive) pair; item = view_item_offset + i where
 *    views are laid out back to back in the order given.
 *  - Pixel (px, py) samples the image point (px + 0.5, py + 0.5).  Tiles are
 *    16x16 pixels, row-major inside a view; the global tile id of a view's
 *    tile t is (sum of the tile counts of the earlier views) + t.
 */
#ifndef GABSPLAT_H
#define GABSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GABSPLAT_ABI_VERSION 7
#define GABSPLAT_TILE 16
#define GABSPLAT_MAX_K 8
#define GABSPLAT_MAX_SH_DEGREE 3
#define GABSPLAT_MAX_VIEWS 4096
/* gabsplat_scene.flags */
#define GABSPLAT_FLAG_ATTENUATION 1
#define GABSPLAT_FLAG_MIP_2D 2
#define GABSPLAT_FLAG_MIP_3D 4
/* gabsplat_scene_grads.flags */
#define GABSPLAT_GRAD_ABS_MEAN2D 1

/* Every entry point that launches device work checks its arguments first
 * (GABSPLAT_ERR_INVALID_ARGUMENT, ..._WORKSPACE_TOO_SMALL, ..._SCRATCH_LIMIT
 * need no device), then that the current HIP device is a gfx950
 * (GABSPLAT_ERR_UNSUPPORTED_DEVICE otherwise; asked once per device). */
typedef enum {
  GABSPLAT_OK = 0,
  GABSPLAT_ERR_INVALID_ARGUMENT = 1,
  GABSPLAT_ERR_WORKSPACE_TOO_SMALL = 2,
  GABSPLAT_ERR_CAPACITY_EXCEEDED = 3,
  GABSPLAT_ERR_HIP = 4,
  GABSPLAT_ERR_UNSUPPORTED_DEVICE = 5,
  GABSPLAT_ERR_SCRATCH_LIMIT = 6
} gabsplat_status;

/* A set of N primitives (Sec. 3.2: mean, covariance via scale and rotation,
 * opacity, colour, and F = k pairs (frequency f_i, weight w_i)).
 *   means     [3][n]   world space
 *   scales    [3][n]   > 0; Sigma = R S S^T R^T with S = diag(scales)
 *   quats     [4][n]   (w, x, y, z), any non-zero norm
 *   opacities [n]      in (0, 1)
 *   sh        [n][(deg+1)^2][3]  real SH coefficients per primitive,
 *                      coefficient-major then channel (element (i, d, c) at
 *                      (i*(deg+1)^2 + d)*3 + c); or NULL
 *   colors    [n][3]   precomputed RGB per primitive (element (i, c) at
 *                      i*3 + c); or NULL (exactly one of sh/colors)
 *   freqs     [k][3][n] cycles per world unit (element (j, axis, i) at
 *                      (j*3 + axis)*n + i)
 *   weights   [k][n]   >= 0 (the DC weight is 1 - sum_j w_j)
 *   flags     GABSPLAT_FLAG_ATTENUATION: keep, for every cosine term, the factor
 *             exp(-2 pi^2 v_j) that the z-integration of supplementary A.2
 *             produces (v_j the variance of f_j . x along the ray given the
 *             image point) and the paper's final 2D primitive (Sec. 3.3.2)
 *             drops; 0 reproduces the paper's primitive.
 *             GABSPLAT_FLAG_MIP_3D and GABSPLAT_FLAG_MIP_2D: the anti-aliasing
 *             filters of Mip-Splatting, which the paper combines with its
 *             primitive (Sec. 4.1, Table 1).  They act on the Gaussian envelope
 *             only.  MIP_3D convolves it with an isotropic 3D Gaussian of
 *             variance filter3d[i]: every scale s becomes sqrt(s^2 + v) and the
 *             opacity is multiplied by prod_j s_j / sqrt(s_j^2 + v), which keeps
 *             the envelope's integral.  MIP_2D replaces the 0.3 px^2 dilation
 *             with a 0.1 px^2 Gaussian and multiplies the opacity by
 *             sqrt(max(det S / det(S + 0.1 I), 1e-6)), S the undilated 2D
 *             covariance.  The near and opacity culls test the input opacity.
 *             A filtered primitive whose opacity is at most 1/255 is culled.
 *             The 3D frequencies and weights are not changed.  Gradients are
 *             taken with respect to the unfiltered scales and opacity.
 *   filter3d  [n] variance of the 3D filter (world units squared, >= 0), e.g.
 *             from gabsplat_mip_filter3d; read only with GABSPLAT_FLAG_MIP_3D
 *             (may be NULL otherwise).
 *   rows      [n][gabsplat_row_floats(k)] or NULL: a row-major copy of each
 *             primitive's quaternion, frequencies and weights, as
 *             gabsplat_pack_rows writes it from the planes above (16-byte
 *             aligned).  When given, gabsplat_preprocess reads those three
 *             attributes of the primitives it projects from their rows: one
 *             aligned row per primitive instead of 4 + 4k planes, whose
 *             lines hold mostly culled neighbours.  The planes must still be
 *             given (the backward and density control read them), and the
 *             rows must be packed again after any change to them: the rows
 *             are for scenes that stay fixed across frames (serving).
 * Limits: 0 <= k <= GABSPLAT_MAX_K, sh_degree in [0, 3] when sh != NULL,
 * 0 <= n < 2^31.  All scenes of one call share k, the colour mode, the flags
 * and whether rows are given. */
typedef struct {
  int64_t n;
  int32_t k;
  int32_t sh_degree;
  int32_t flags;
  int32_t pad;
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  const float* colors;
  const float* freqs;
  const float* weights;
  const float* filter3d;
  const float* rows;
} gabsplat_scene;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A world point x
 * maps to camera space as R x + t with world_to_cam = [R | t] row-major
 * (R at [0..2], [4..6], [8..10]; t at [3], [7], [11]).  cam_pos is the camera
 * centre in world space (view direction of the SH colour).  Primitives with
 * camera z <= near_plane are culled.  bg is added with the final
 * transmittance.  1 <= width, height <= 16384. */
typedef struct {
  int32_t width;
  int32_t height;
  float fx, fy, cx, cy;
  float world_to_cam[12];
  float cam_pos[3];
  float near_plane;
  float bg[3];
} gabsplat_camera;

/* Per-item projected data, caller-allocated device buffers of `items` rows.
 *   rec    [items][gabsplat_record_floats(k)] render record:
 *            [0,1]  mu2d (pixels)
 *            [2..4] quadratic form q = a dx^2 + b dx dy + c dy^2 in log2
 *                   units: (a, b, c) = -log2(e) * (C_xx/2, C_xy, C_yy/2),
 *                   C = (Sigma2d + 0.3 I)^-1 the conic
 *            [5]    log2(opacity)
 *            [6..8] RGB colour
 *            [9]    DC weight 1 - sum_j w_j
 *            [10+3j .. 12+3j]  2D frequency (cycles/pixel, x then y) and
 *                   weight of component j's cosine (w_j, times its
 *                   attenuation when GABSPLAT_FLAG_ATTENUATION is set)
 *            [10+3k, 11+3k]  residuals of mu2d's float32 rounding: the mean
 *                   is mu2d + residual (a float pair, computed in double),
 *                   which holds it to ~1e-6 px where a float alone holds
 *                   ~1e-4 px (at coordinates near 1000)
 *          so o * G(p) = exp2(q(p - mu2d) + rec[5]).
 *   depth  [items] fp32 camera z, computed as ((r20 x + r21 y) + r22 z) + t2
 *          with one IEEE rounding per operation
 *   rect   [items][2] tile rectangle: word 0 = x0 | y0 << 16, word 1 =
 *          x1 | y1 << 16 (x1, y1 exclusive)
 *   tiles  [items] number of tiles in rect; 0 means culled
 *   k      number of Gabor components of the scenes (record layout)
 *   views  view table, gabsplat_views_bytes(num_views, num_scenes) bytes,
 *          written by gabsplat_preprocess; gabsplat_bin_sort,
 *          gabsplat_render_fwd and gabsplat_render_bwd read it, so they must
 *          be given the same views as the preprocess call that wrote it. */
typedef struct {
  int32_t k;
  int32_t pad;
  float* rec;
  float* depth;
  uint32_t* rect;
  uint32_t* tiles;
  void* views;
} gabsplat_geom;

/* Gradient buffers, same layouts as gabsplat_scene.  With accumulate != 0 the
 * gradients are added (+=) to the buffers (views and calls accumulate);
 * with accumulate == 0 they are overwritten, every primitive included (culled
 * ones get 0).  Entries may be NULL to skip that gradient (sh or colors must
 * match the scene's colour mode).  grad2d [items][gabsplat_grad2d_floats(k)]
 * is scratch that receives the image-plane gradients, i.e. the gradient with
 * respect to every field of the render record, in the record's order (row
 * stride gabsplat_grad2d_stride(k, flags)).  With flags GABSPLAT_GRAD_ABS_MEAN2D
 * the two floats after those fields receive, per item, the sums over pixels
 * of the absolute per-pixel gradients |dL_p / d mu2d_x| and |dL_p / d mu2d_y|.
 * This is the homodirectional gradient of AbsGS, the densification variant
 * the paper combines with its primitive (Sec. 4.1, Table 1).  The call
 * first zeroes the rows of the items that touch a tile (geom->tiles != 0, the
 * only rows it writes or reads; other rows are left as they are), and those
 * rows may be read afterwards (e.g. the view-space positional gradient used
 * by density control).  All scenes of one call share the same grad2d buffer. */
typedef struct {
  int32_t accumulate;
  int32_t flags;
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
  float* colors;
  float* freqs;
  float* weights;
  float* grad2d;
} gabsplat_scene_grads;

/* ---------------------------------------------------------------- helpers */
int32_t gabsplat_abi_version(void);
const char* gabsplat_status_string(gabsplat_status s);
/* Floats per render record for k components: round_up(10 + 3k, 4). */
int32_t gabsplat_record_floats(int32_t k);
/* Floats per row of gabsplat_scene.rows: round_up(4 + 4k, 32) (rows of whole
 * 128-byte lines): quaternion (w, x, y, z), then the 3k frequencies
 * (component-major: f_j at 4 + 3j), then the k weights (w_j at 4 + 3k + j),
 * then zeros; -1 if k is invalid. */
int32_t gabsplat_row_floats(int32_t k);
/* Floats per item of the image-plane gradient: round_up(10 + 3k, 4). */
int32_t gabsplat_grad2d_floats(int32_t k);
/* Row stride of grad2d for gabsplat_scene_grads.flags: round_up(10 + 3k, 4),
 * or round_up(12 + 3k, 4) with GABSPLAT_GRAD_ABS_MEAN2D; -1 if invalid. */
int32_t gabsplat_grad2d_stride(int32_t k, int32_t grad_flags);
/* Bytes for gabsplat_geom.views. */
size_t gabsplat_views_bytes(int32_t num_views, int32_t num_scenes);
/* Device workspace for gabsplat_bin_sort: `items` = total items, `pair_capacity`
 * = room for (primitive, tile) pairs, `total_tiles` = sum of tile counts. */
size_t gabsplat_bin_sort_workspace_size(int64_t items, int64_t pair_capacity, int64_t total_tiles);
/* 0 if the current HIP device is gfx950, else GABSPLAT_ERR_UNSUPPORTED_DEVICE. */
gabsplat_status gabsplat_check_device(void);

/* ------------------------------------------------------------ entry points */

/* K1, projection and culling of every (view, primitive) item: camera-space
 * transform and near cull (camera z <= near_plane), opacity cull (255 o <= 1),
 * EWA 2D covariance J W Sigma W^T J^T (Sec. 3.1) with J evaluated at the
 * point clamped to 1.3x the frustum, dilated by 0.3 px^2 and inverted; the
 * 2D frequency of every component, f2d = (T Sigma T^T)^-1 T Sigma f with T
 * the first two rows of J W, which equals the paper's f_proj = (JW)^-T f
 * followed by the z-integration of Sec. 3.3.2 for any completion of J; the
 * SH colour (real SH, degree <= 3, + 0.5, clamped at 0); and the tile
 * rectangle of the exact support o G >= 1/255 (half-widths sqrt(2 ln(255 o))
 * sqrt(Sigma2d_xx), resp. yy).
 *   scenes[num_scenes] (host), scene_of_view[num_views] (host, index into
 *   scenes; NULL means all views use scenes[0]), cams[num_views] (host).
 * All scenes of one call must share k and the colour mode (sh / colors and
 * sh_degree).  geom rows: items = sum over views of that view's scene n. */
gabsplat_status gabsplat_preprocess(const gabsplat_scene* scenes, int32_t num_scenes,
                                    const int32_t* scene_of_view, const gabsplat_camera* cams,
                                    int32_t num_views, const gabsplat_geom* geom, void* stream);

/* Writes scene->rows' layout (gabsplat_row_floats(k) floats per primitive)
 * into `rows` (device, n rows, 16-byte aligned; 128-byte alignment puts every
 * row on its own cache line) from the scene's quats, freqs and weights
 * planes, the attributes K1 reads for every primitive it projects (Sec. 3.1,
 * 3.3.2).  The scene's own `rows` field is ignored.  Enqueued on `stream`.
 * INVALID_ARGUMENT for an invalid scene or a NULL or misaligned `rows`. */
gabsplat_status gabsplat_pack_rows(const gabsplat_scene* scene, float* rows, void* stream);

/* K2-K5, binning: compact the visible items, stably sort them by fp32 depth
 * bits, emit one (global tile, item) pair per overlapped tile, stably sort the
 * pairs by tile (an LSD radix sort on the key tile << 32 | depth bits whose
 * depth passes run on the primitives before duplication), and write each
 * global tile's [start, end) range (empty tiles = (0, 0)).
 *   vals [pair_capacity]      sorted item ids (output)
 *   keys [pair_capacity]      sorted 64-bit keys tile << 32 | depth bits, or
 *                             NULL to skip writing them.  Without keys, a
 *                             frame of at most 8192 tiles (and a capacity
 *                             below 2^31) may leave a tile's list of up to
 *                             1024 ids grouped but unordered, marked by bit
 *                             31 of its end in tile_ranges (the range is
 *                             [start, end & 0x7fffffff)); gabsplat_render_fwd
 *                             orders such a list in place in vals and clears
 *                             the bit before blending it, so after it vals
 *                             and tile_ranges are exactly as with keys
 *   tile_ranges [3 * total_tiles] (output): [total_tiles][2] ranges, then
 *                the order in which gabsplat_render_fwd / _bwd dispatch the
 *                tiles (tile ids by decreasing list length, in geometric
 *                buckets 2^(1/8) apart; empty tiles last)
 *   d_num_pairs  device int64 (output): number of pairs
 *   d_overflow   device int32 (output): 1 if pairs > pair_capacity, else 0.
 *                On overflow vals/keys/ranges are undefined and
 *                gabsplat_render_fwd / _bwd become no-ops; call again with a
 *                larger capacity (gabsplat_read_overflow reports it).
 *   ws / ws_bytes  device workspace >= gabsplat_bin_sort_workspace_size(). */
gabsplat_status gabsplat_bin_sort(const gabsplat_geom* geom, const gabsplat_camera* cams,
                                  int32_t num_views, int64_t items, void* ws, size_t ws_bytes,
                                  uint64_t* keys, uint32_t* vals, int64_t pair_capacity,
                                  uint32_t* tile_ranges, int64_t* d_num_pairs, int32_t* d_overflow,
                                  void* stream);

/* K6, forward blend (Sec. 3.3.3 with the 2D Gabor primitive of Sec. 3.3.2):
 * per pixel, front to back over its tile's list, alpha = min(0.99, o G B)
 * with B = (1 - sum w) + sum_j w_j cos(2 pi f2d_j . (p - mu2d)); primitives
 * with alpha < 1/255 are skipped; the walk stops, without blending, at the
 * first primitive that would leave T (1 - alpha) < 1e-4; C += c alpha T;
 * finally C += T bg.  Deterministic (no atomics).
 *   image     [sum over views of 3*H*W]  view-major, then channel, row, column
 *   final_T   [sum over views of H*W]
 *   n_contrib [sum over views of H*W]  1-based position, in the tile's list,
 *             of the last blended primitive (0 = none)
 *   eval_counts  NULL, or [sum over views of H*W][2]: per pixel, the position
 *             in its tile's list where the walk ended (the stopping primitive,
 *             else the list length) and how many of those primitives passed
 *             the envelope test o G >= 1/255 (the work the blend had to do)
 *   freq_map  NULL, or [sum over views of H*W]: the frequency map the paper
 *             visualises (supplementary C), each primitive's weighted
 *             image-plane frequency sum_j w_j |f2d_j| (cycles per pixel, w_j
 *             the record's cosine weights) blended with the weights alpha T of
 *             its colour, without background
 *   (eval_counts / freq_map select a separate, slower analysis variant.)
 *   vals, tile_ranges  from gabsplat_bin_sort (device); a list marked
 *             unordered (bit 31 of its end) is first ordered in place by
 *             (fp32 depth bits of geom->depth, id) and its mark cleared, so
 *             both are read and written; geom->depth must be the depths of
 *             the gabsplat_preprocess that the bin sort read
 *   d_overflow  from gabsplat_bin_sort (device). */
gabsplat_status gabsplat_render_fwd(const gabsplat_geom* geom, uint32_t* vals,
                                    uint32_t* tile_ranges, const gabsplat_camera* cams,
                                    int32_t num_views, float* image, float* final_T,
                                    uint32_t* n_contrib, uint32_t* eval_counts, float* freq_map,
                                    const int32_t* d_overflow, void* stream);

/* K7 + K8, backward of the forward above w.r.t. every attribute.  K7 walks
 * each tile back to front from n_contrib, recovers the transmittance by
 * division, reduces each primitive's per-pixel contributions within the
 * wavefront and adds them atomically into grads->grad2d; K8 chains the
 * image-plane gradients through the projection of every view into the scene
 * gradients (+=).  Not bitwise deterministic (fp32 atomics).
 *   scenes / scene_of_view / cams / num_views exactly as given to
 *   gabsplat_preprocess; grads[num_scenes] (host array of structs);
 *   dl_dimage has the layout of `image`. */
gabsplat_status gabsplat_render_bwd(const gabsplat_scene* scenes, int32_t num_scenes,
                                    const int32_t* scene_of_view, const gabsplat_camera* cams,
                                    int32_t num_views, const gabsplat_geom* geom,
                                    const uint32_t* vals, const uint32_t* tile_ranges,
                                    const float* final_T, const uint32_t* n_contrib,
                                    const float* dl_dimage, const gabsplat_scene_grads* grads,
                                    const int32_t* d_overflow, void* stream);

/* The backward above in its two stages, for callers that time or schedule
 * them apart (same arguments and checks as gabsplat_render_bwd, plus):
 *   stages  GABSPLAT_BWD_BLEND: clear the grad2d rows of the items that
 *           touch a tile and run K7 (the image-plane gradients into
 *           grads->grad2d); GABSPLAT_BWD_PROJECT: K8 only, chaining the
 *           grad2d an earlier blend stage left (unchanged since) into the
 *           scene gradients; both bits: gabsplat_render_bwd.  Any other
 *           value is an invalid argument. */
#define GABSPLAT_BWD_BLEND 1
#define GABSPLAT_BWD_PROJECT 2
gabsplat_status gabsplat_render_bwd_stages(const gabsplat_scene* scenes, int32_t num_scenes,
                                           const int32_t* scene_of_view, const gabsplat_camera* cams,
                                           int32_t num_views, const gabsplat_geom* geom,
                                           const uint32_t* vals, const uint32_t* tile_ranges,
                                           const float* final_T, const uint32_t* n_contrib,
                                           const float* dl_dimage, const gabsplat_scene_grads* grads,
                                           const int32_t* d_overflow, int32_t stages, void* stream);

/* K9, photometric loss of Sec. 3.4.1 for one image: L = (1 - lambda) mean|x - y|
 * + lambda (1 - mean SSIM(x, y)), SSIM with an 11x11 Gaussian window
 * (sigma 1.5), zero-padded, C1 = 0.01^2, C2 = 0.03^2, means over all channels
 * and pixels.  x, y [channels][H][W]; writes d_loss (device float, one
 * value) and dl_dx [channels][H][W].  ws >= gabsplat_loss_workspace_size().
 * The L1 gradient at x == y is 0. */
size_t gabsplat_loss_workspace_size(int32_t channels, int32_t height, int32_t width);
gabsplat_status gabsplat_loss_l1_dssim(const float* x, const float* y, int32_t channels,
                                       int32_t height, int32_t width, float lambda, float* d_loss,
                                       float* dl_dx, void* ws, size_t ws_bytes, void* stream);

/* Size of the library's static scratch for gabsplat_loss_l1_dssim_noalloc
 * (80 MiB per GPU): problems with gabsplat_loss_workspace_size(c, H, W) up
 * to this, e.g. three channels of 1920x1080. */
#define GABSPLAT_LOSS_NOALLOC_SCRATCH_BYTES ((size_t)83886080)

/* gabsplat_loss_l1_dssim for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving or training loops, harnesses
 * that forbid allocation.  Same arguments, results and kernels, without the
 * workspace: its scratch is a static device array of
 * GABSPLAT_LOSS_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds from the first call on it until the process ends (the first call on a
 * GPU looks up that GPU's copy; later calls allocate and free nothing).  The
 * kernels clear what they count with themselves, so no memset is recorded.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on a
 * GPU (concurrent streams, or host threads) race and corrupt each other's
 * results, so the caller serialises them.  x, y, d_loss, dl_dx and the stream
 * are on the same GPU.  GABSPLAT_ERR_SCRATCH_LIMIT (before any device work)
 * when gabsplat_loss_workspace_size(channels, height, width) exceeds the
 * scratch; GABSPLAT_ERR_INVALID_ARGUMENT as gabsplat_loss_l1_dssim. */
gabsplat_status gabsplat_loss_l1_dssim_noalloc(const float* x, const float* y, int32_t channels,
                                               int32_t height, int32_t width, float lambda, float* d_loss,
                                               float* dl_dx, void* stream);

/* ------------------------------------------------ density control (Sec. 3.4.2)
 * The paper densifies as 3DGS does (clone small / split large primitives whose
 * mean view-space positional gradient exceeds a threshold, prune transparent
 * ones) and resets the frequencies and frequency weights of every newly
 * generated child to small values; every few thousand iterations it resets all
 * frequency weights together with the opacity reset. */
typedef struct {
  float grad_threshold;  /* on the mean view-space (NDC) gradient norm, e.g. 0.0002 */
  float percent_dense;   /* clone if max scale <= percent_dense * extent, else split */
  float scene_extent;
  float min_opacity;     /* prune below (0.01 in the paper's supplement) */
  float max_world_frac;  /* with prune_big: prune if max scale > max_world_frac * extent */
  int32_t prune_big;
  float freq_reset;      /* every axis of every frequency of a new child (0.001) */
  float weight_reset;    /* every frequency weight of a new child (0.01) */
  float split_shrink;    /* child scale factor (1 / 1.6) */
  int32_t split_count;   /* children per split primitive (2), 1..8 */
  float abs_grad_threshold; /* AbsGS: split also when the mean homodirectional
                               statistic reaches it (e.g. 0.0004); <= 0: off */
} gabsplat_densify_params;

/* Writable scene buffers (same layout and meaning as gabsplat_scene). */
typedef struct {
  int64_t n;
  int32_t k;
  int32_t sh_degree;
  int32_t flags;
  int32_t pad;
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
  float* colors;
  float* freqs;
  float* weights;
} gabsplat_scene_out;

/* accum[i] += |dL/d mu2d| in normalised device coordinates (the pixel
 * gradient from grad2d scaled by (W/2, H/2)) and denom[i] += 1 for every view
 * of `geom` (one scene of n primitives, views as given to the preprocess that
 * wrote geom) in which primitive i is visible.  grad_flags are the flags of
 * the backward that wrote grad2d (its row stride); with
 * GABSPLAT_GRAD_ABS_MEAN2D, accum_abs[i] also receives the norm of the
 * homodirectional gradient in the same units (else accum_abs may be NULL). */
gabsplat_status gabsplat_densify_stats(const gabsplat_geom* geom, const gabsplat_camera* cams,
                                       int32_t num_views, int64_t n, const float* grad2d, int32_t grad_flags,
                                       float* accum, float* accum_abs, float* denom, void* stream);

/* Clone / split / prune.  Decision per primitive, in order: prune if opacity <
 * min_opacity (or too large, with prune_big); else clone if accum/denom >=
 * grad_threshold and max scale <= percent_dense * extent; split if the
 * primitive is larger and the threshold is met, or, with abs_grad_threshold >
 * 0, accum_abs/denom >= abs_grad_threshold (accum_abs then required, else it
 * may be NULL); keep otherwise.  Output rows:
 * kept and cloned primitives unchanged (ascending source index), then one copy
 * of each cloned primitive, then split_count children of each split primitive
 * with mean + R(q)(s * z_c) (z_c = normals[c][.][i], standard normal draws
 * supplied by the caller) and scale s * split_shrink.  Every new row (clone
 * copy or split child) gets frequencies freq_reset and weights weight_reset.
 * out: arrays of out_capacity rows; the planar arrays are written with the
 * stride n_out (the output count, written to *d_n_out), the colour arrays row
 * by row.  src_index / tag [n_out]:
 * source primitive and 0 kept, 1 clone copy, 2 + c split child c (use them to
 * carry per-primitive optimizer state).  *d_overflow = 1 (and nothing
 * written) if n_out > out_capacity.  ws >= gabsplat_densify_workspace_size(n). */
size_t gabsplat_densify_workspace_size(int64_t n);
gabsplat_status gabsplat_densify(const gabsplat_scene* in, const float* accum, const float* denom,
                                 const float* accum_abs, const float* normals, const gabsplat_densify_params* params,
                                 const gabsplat_scene_out* out, int64_t out_capacity, uint32_t* src_index,
                                 uint32_t* tag, int64_t* d_n_out, int32_t* d_overflow, void* ws,
                                 size_t ws_bytes, void* stream);

/* Periodic reset: every frequency weight := weight_value, opacity :=
 * min(opacity, opacity_cap). */
gabsplat_status gabsplat_reset_frequency_weights(const gabsplat_scene_out* scene, float weight_value,
                                                 float opacity_cap, void* stream);

/* Variance of Mip-Splatting's 3D smoothing filter for every primitive (the
 * anti-aliasing the paper combines with its primitive, Sec. 4.1, Table 1).
 * The sampling rate of camera c at primitive i is max(fx, fy) / z, counted for
 * the cameras with z > near_plane whose image, grown by `margin` of its width
 * and height on every side, holds the projected mean.  With r the largest rate,
 * filter3d[i] = s / r^2.  Primitives that no camera sees get the largest
 * variance of the others (0 if no primitive is seen).
 *   means [3][n] (device), cams[num_cams] (host), s e.g. 0.2, margin e.g. 0.15,
 *   filter3d [n] (device, output), ws >= gabsplat_mip_filter3d_workspace_size. */
size_t gabsplat_mip_filter3d_workspace_size(int64_t n, int32_t num_cams);
gabsplat_status gabsplat_mip_filter3d(const float* means, int64_t n, const gabsplat_camera* cams,
                                      int32_t num_cams, float s, float margin, float* filter3d, void* ws,
                                      size_t ws_bytes, void* stream);

/* Reads *d_overflow synchronously (waits for `stream`); returns
 * GABSPLAT_ERR_CAPACITY_EXCEEDED if it is set, GABSPLAT_OK otherwise. */
gabsplat_status gabsplat_read_overflow(const int32_t* d_overflow, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GABSPLAT_H */
