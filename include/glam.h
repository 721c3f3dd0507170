/* glam: MI355X (gfx950) kernels for the differentiable render of anchor-decoded
 * 3-D Gaussians, the per-iteration hot path of a Gaussian mapping backend
 * (GLAM-SLAM, Sec. III-A and III-D of the paper).
 *
 * One mapping iteration renders keyframe views and differentiates a photometric loss:
 *   glam_decode      anchor features -> Gaussians, view-conditioned MLPs (Eq. 2) with
 *                    one MLP set per spatial partition (Eq. 6)
 *   glam_project     3-D Gaussians -> projected 2-D Gaussians + footprint boxes
 *   glam_decode_project  the two above in one launch
 *   glam_bin_sort    (tile, depth) pairs, device radix sort, per-tile ranges
 *   glam_render_fwd  front-to-back alpha compositing per tile (Eq. 1)
 *   glam_loss        L1 + SSIM objective (Eq. 3) and its image gradient
 *   glam_render_bwd  reverse compositing, projection adjoint, decode adjoint
 *   glam_adam_step   the optimiser step of the mapping iteration (fused Adam)
 *   glam_sample_keyframes  which keyframes an iteration renders (host)
 *   glam_deform_anchors    loop-closure correction of the anchor grid (Eq. 7)
 *   glam_epipolar_triangulate  flow correspondences: epipolar filter, triangulation (Eq. 5)
 *   glam_voxelize    fused points -> unique voxels, those not yet anchors (Eq. 4)
 *   glam_insert_rows the growth's bookkeeping: new anchors inserted into per-anchor arrays
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers owned by the caller; the library never
 *    allocates, frees or keeps them.  Scratch memory comes from a caller workspace
 *    whose size glam_*_workspace_bytes() reports.
 *  - "[3][n]" is structure-of-arrays: three contiguous rows of n values.  Pointers
 *    must be 16-byte aligned.
 *  - Calls are asynchronous on the given stream and never synchronise, so a sequence
 *    of calls can be captured into a HIP graph.  They are reentrant; the library's only
 *    global state is glam_loss_noalloc's per-device scratch (see there).
 *  - Arguments are validated on the host before anything is launched; a rejected call
 *    returns GLAM_ERR_INVALID_ARG (or GLAM_ERR_WORKSPACE) and launches nothing.
 *  - Data-dependent overflow (more (tile, Gaussian) pairs than the caller's capacity)
 *    is detected on the device: the call sets the sticky word status[0] to
 *    GLAM_ERR_CAPACITY and writes the required pair count to status[2..3]; outputs of
 *    that call and of later calls reading them are then undefined (no memory outside
 *    the given buffers is touched).
 *  - No exception crosses the ABI and nothing is printed.
 *
 * View table.  Several keyframe views (possibly of different partitions and
 * resolutions) are processed by one call.  glam_views_build() derives, on the host,
 * one glam_view_info per view (offsets of its Gaussians, pixels and tiles in the
 * batched buffers); the caller copies that array verbatim to device memory and passes
 * both copies in a glam_views.  Offsets are view-major:
 *   view-Gaussians  [g_begin, g_begin + g_count) of every per-Gaussian array
 *   pixels          [pix_begin, pix_begin + W*H) of per-pixel arrays; images are
 *                   [3][H][W] planes starting at 3*pix_begin
 *   tiles           [tile_begin, tile_begin + tiles_x*tiles_y), row-major per view
 */
#ifndef GLAM_H
#define GLAM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLAM_OK = 0,
  GLAM_ERR_INVALID_ARG = 1,
  GLAM_ERR_WORKSPACE = 2,
  GLAM_ERR_CAPACITY = 3,
  GLAM_ERR_HIP = 4,
  GLAM_ERR_UNSUPPORTED = 5
} glam_status;

/* Human-readable name of a status (static storage). */
const char* glam_status_string(int32_t status);

/* Flags (bitwise or). */
enum {
  /* Gaussians are given directly (mean, log-scale, raw quaternion, opacity logit,
     colour) instead of being decoded from anchors; every view sees the same set. */
  GLAM_PLAIN = 1u << 0,
  /* Opacity activation sigmoid instead of the default tanh with non-positive values
     dropped (anchor mode); plain mode always uses sigmoid of the logit. */
  GLAM_OPACITY_SIGMOID = 1u << 1,
  /* Footprint of the 3-D Gaussian splatting lineage the paper builds on (Sec. II,
     Sec. III-A) instead of the default opacity-aware box: a square of radius
     r = ceil(3 sqrt(lambda_max)) pixels around the centre (lambda_max the larger
     eigenvalue of the dilated 2-D covariance), taken at tile granularity: a Gaussian is
     a candidate at every pixel of every tile that square's pixel centres reach.  It
     clips contributions with alpha >= 1/255 beyond 3 sigma whenever opacity exceeds
     255^-1 e^4.5 (about 0.353), and the image then depends on the tile edge.  Read by
     glam_project and glam_decode_project (the flag must then be passed to the backward
     calls too). */
  GLAM_FOOTPRINT_3SIGMA = 1u << 2,
  /* Backward only: reproducible gradients.  The per-Gaussian sums of the reverse
     compositing (the adjoint of Eq. 1) are formed without floating-point atomics: each
     (tile, Gaussian) pair and 8x8 quadrant stores its partial sums in a workspace, and
     a segmented reduction adds each Gaussian's partials in a fixed order (its tiles
     row-major, then quadrants).  Results are bit-identical from run to run and across
     persistent grid sizes (glam_tuning's blocks per CU); the tile edge, the long-tile
     threshold and the group widths choose the arithmetic path of each tile (where a
     long range is cut into chunks), so they must stay the same.
     Needs glam_bins.pair_begin from the
     glam_bin_sort call and glam_render_bwd_workspace_bytes with this flag. */
  GLAM_DETERMINISTIC_GRADS = 1u << 3,
  /* Backward only: also write the 2-D gradients d(u, v, A, B, C, opacity, r, g, b) of
     every view-Gaussian to glam_grads.d2d (stage-wise checks, inspection). */
  GLAM_RETURN_INTERMEDIATES = 1u << 4
};

/* Pinhole camera: world->camera rotation R (row-major) and translation t, OpenCV
   axes (x right, y down, z forward), focal lengths and principal point in pixels,
   image size, and the spatial partition (index of the MLP set, Eq. 6) whose anchors
   this view renders. */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t partition;
  int32_t reserved;
} glam_camera;

/* Per-view offsets into the batched buffers (filled by glam_views_build). */
typedef struct {
  glam_camera cam;
  int64_t g_begin, g_count;     /* view-Gaussians                                   */
  int64_t pix_begin;            /* pixels                                           */
  int32_t tile_begin;           /* tiles                                            */
  int32_t tiles_x, tiles_y;
  int32_t anchor_begin;         /* first anchor of the view's partition (anchor mode) */
  int32_t anchor_count;
  int32_t reserved;
} glam_view_info;

typedef struct {
  const glam_view_info* host;   /* [n] host memory                                 */
  const glam_view_info* dev;    /* [n] device copy of the same bytes               */
  int32_t n;
  int32_t tile_w, tile_h;       /* square tiles of 8, 16 or 32 pixels (binning
                                   granularity; compositing works on 8x8 quadrants) */
  int32_t reserved;
  int64_t n_gauss;              /* total view-Gaussians                            */
  int64_t n_pix;                /* total pixels                                    */
  int64_t n_tiles;              /* total tiles                                     */
} glam_views;

/* Fills info[n_views] and the totals of *views (everything except the host/dev
   pointers).  Anchor mode: part_begin[n_parts+1] (host) delimits each partition's
   anchors, each view gets anchor_count*K Gaussians.  Plain mode (part_begin NULL):
   every view gets plain_G Gaussians.  tile_w == tile_h in {8, 16, 32}, else
   GLAM_ERR_UNSUPPORTED.  Pure host function. */
glam_status glam_views_build(const glam_camera* cams, int32_t n_views,
                             const int32_t* part_begin, int32_t n_parts, int32_t K,
                             int64_t plain_G, int32_t tile_w, int32_t tile_h,
                             glam_view_info* info, glam_views* views);

/* Anchors (Sec. III-A, Scaffold-GS structure): position x_a, feature f_a (F values),
   one log-scale s_a and K offsets o_aj; the K Gaussians of anchor a sit at
   x_a + exp(s_a) o_aj.  Anchors are grouped contiguously by partition. */
typedef struct {
  const float* pos;        /* [3][A]                                                */
  const float* feat;       /* [A][F] row-major                                      */
  const float* log_scale;  /* [A]                                                   */
  const float* offs;       /* [3][A*K], Gaussian j of anchor a at a*K + j           */
  int32_t A, F, K;         /* built (F, K): (8, 10), (16, 4), (32, 10), (64, 10);
                              others: GLAM_ERR_UNSUPPORTED                          */
  int32_t hidden;          /* MLP hidden width, 32                                  */
} glam_anchors;

/* MLP sets, one per partition (Eq. 6): mlp[m][P] with P = glam_mlp_param_count(F, K,
   hidden), three two-layer ReLU MLPs in the order opacity (K outputs), colour (3K),
   covariance (7K: 3 scales then 4 quaternion values per Gaussian), each packed as
   W1[hidden][F+4], b1[hidden], W2[out][hidden], b2[out].  The MLP input is
   z = [f_a, d_ac, delta_ac] (Eq. 2): feature, unit view direction, distance. */
int32_t glam_mlp_param_count(int32_t F, int32_t K, int32_t hidden);

/* Gaussians, structure-of-arrays with row stride n.
   Anchor mode (decoded, per view-Gaussian): mean, scale, unit quaternion (w,x,y,z),
   opacity, colour.  Plain mode (shared by all views, n = G): mean, log-scale, raw
   quaternion, opacity logit, colour. */
typedef struct {
  float* mean;     /* [3][n] */
  float* scale;    /* [3][n] */
  float* quat;     /* [4][n] */
  float* opacity;  /* [n]    */
  float* rgb;      /* [3][n] */
  int64_t n;
} glam_gaussians;

/* Projected 2-D Gaussians, one per view-Gaussian (row stride views.n_gauss). */
typedef struct {
  float* uv;        /* [2][n] pixel-space centre                                    */
  float* conic;     /* [3][n] (A, B, C) of the inverse 2-D covariance               */
  float* depth;     /* [n]    camera-space z                                        */
  float* ext;       /* [2][n] footprint half extents, -1 when culled                */
  int32_t* ntiles;  /* [n]    tiles touched, 0 when culled                          */
  float* splat;     /* [n][12] packed render record (u, v, a, b, c, opacity, r, g, b,
                       pixel box x0|x1<<16 and y0|y1<<16 as bits, depth), where
                       (a, b, c) = -log2(e) (A/2, B, C/2): the splat's alpha at
                       offset (dx, dy) is opacity 2^(a dx^2 + b dx dy + c dy^2)      */
} glam_projected;

/* Words of the compositing work-queue buffer (two kernels x (16 counters on separate
   128-byte lines + a line holding the exit count and the long-tile counter)). */
#define GLAM_QUEUE_WORDS 1088

/* Schedule of the compositing over a binning (all fields 0 = the built-in default;
   the results never depend on the grid sizes, only the time does; the long-tile
   threshold and the group widths fix where a long range is cut into chunks, and so
   the FP32 rounding order there):
   long_log2         tiles whose range holds at least 2^long_log2 entries are listed
                     first in the work order and composited by whole workgroups
                     (default 10; 6..24)
   fwd_group_waves   waves per workgroup of the forward compositing grid: 4 (default),
                     8 or 16; a long tile's quadrant is split over that many waves
   fwd_blocks_per_cu persistent workgroups per CU of the forward compositing grid
                     (groups of 4: default and maximum 5; of 8: default and maximum 2;
                     of 16: 1)
   bwd_group_waves   the same for the backward compositing grid
   bwd_blocks_per_cu the same for the backward grid (groups of 4: default and maximum
                     6; of 8: 2; of 16: 1)
   non_persistent    1: glam_render_fwd and glam_composite_bwd / glam_render_bwd
                     launch no persistent grid and use no work queue: one workgroup of
                     four waves per four (tile, quadrant) items in tile order, each wave
                     walking its quadrant's whole range (long tiles too), as the
                     rasterisers of the 3DGS lineage launch one block per tile; the plain
                     form the batched step is measured against.  The widths, workgroup
                     counts and long-tile threshold then do not apply to those calls (the
                     threshold still orders the bins).  0: the persistent queue (default).
                     glam_render_fused_l1 always runs the persistent grid
   reserved          must be 0 */
typedef struct {
  int32_t long_log2;
  int32_t fwd_blocks_per_cu;
  int32_t bwd_blocks_per_cu;
  int32_t fwd_group_waves;
  int32_t bwd_group_waves;
  int32_t non_persistent;
  int32_t reserved[2];
} glam_tuning;

/* Sorted (tile, Gaussian) pairs, per-tile ranges and the compositing work order. */
typedef struct {
  uint64_t* keys;   /* [capacity] sorted keys: tile << depth_bits | depth key        */
  uint32_t* vals;   /* [capacity] sorted view-Gaussian indices                       */
  uint32_t* ranges; /* [n_tiles][2] [start, end) into keys/vals                      */
  int64_t capacity;
  int32_t* status;  /* [8] device: [0] sticky status, [1] pair count (low word),
                       [2..3] required capacity (int64), [4] depth key bits,
                       [5] tile key bits, [6] radix passes, [7] long tiles (range
                       of 2^tuning.long_log2 entries or more, listed first in order,
                       composited by whole workgroups); caller zeroes [0] once      */
  uint32_t* order;  /* [n_tiles] tiles by decreasing range length (power-of-two
                       classes), the order the compositing queue hands them out       */
  uint32_t* queue;  /* [GLAM_QUEUE_WORDS] device work-queue counters of the
                       compositing kernels; caller zeroes them once, every launch
                       leaves them zeroed                                             */
  glam_tuning tuning; /* host: the compositing schedule (rejected when out of range)  */
  uint32_t* pair_begin; /* [n_gauss] device, or NULL: glam_bin_sort then writes each
                           view-Gaussian's first pair before sorting (the exclusive
                           prefix sum of the tile counts; its pairs are that one and the
                           next ntiles - 1, its tiles row-major).  Required by
                           GLAM_DETERMINISTIC_GRADS                                      */
} glam_bins;

/* Workspace bytes glam_bin_sort needs for this view table and pair capacity. */
size_t glam_bin_sort_workspace_bytes(const glam_views* views, int64_t capacity);


/* --- forward -------------------------------------------------------------------- */

/* Eq. 2 + Eq. 6: for every view v, decode the anchors of partition cam.partition with
   MLP set mlp[partition] (mlp holds n_parts sets; a view whose partition is outside
   [0, n_parts) is rejected) into out (row stride views.n_gauss): mean = x_a + e^{s_a} o,
   scale = e^{s_a} sigmoid(y), quaternion y/|y|, opacity tanh(y) (or sigmoid), colour
   sigmoid(y).  FP32 MFMA for the MLPs. */
glam_status glam_decode(const glam_anchors* anchors, const float* mlp, int32_t n_parts,
                        const glam_views* views, uint32_t flags, glam_gaussians* out,
                        hipStream_t stream);

/* glam_decode followed by glam_project in one launch: each decoded Gaussian is projected
   from the registers that hold it (identical results to the two calls; saves re-reading
   the decoded Gaussians).  Same arguments and errors as glam_decode, plus the projection
   outputs proj (as glam_project). */
glam_status glam_decode_project(const glam_anchors* anchors, const float* mlp, int32_t n_parts,
                                const glam_views* views, uint32_t flags, glam_gaussians* out,
                                glam_projected* proj, hipStream_t stream);

/* Projection and footprint of every view-Gaussian: the step of the differentiable 3-D
   Gaussian rasteriser of Sec. III-A that maps each Gaussian onto the image plane, where
   Eq. 1 evaluates its alpha (EWA splatting, as in the 3DGS lineage the paper builds
   on).  Culls depth <= 0.2 and opacity
   <= 1/255; Jacobian x/z, y/z clamped to 1.15x the image (beyond a 0.15-image border);
   2-D covariance dilated by 0.3 px^2; footprint box: |x + 0.5 - u| <= ext_x with
   ext = sqrt(2 ln(255 opacity) Sigma2D_xx) (likewise y), outside of which the
   Gaussian's alpha is below 1/255. */
glam_status glam_project(const glam_gaussians* gauss, const glam_views* views, uint32_t flags,
                         glam_projected* out, hipStream_t stream);

/* The depth order Eq. 1 composites in (front to back, Sec. III-A), per tile of the
   lineage's tile-based rasteriser: tile binning and device LSD radix sort by (global
   tile, depth): pairs emitted per
   view-Gaussian in index order (row-major over its tiles), stable sort, so equal
   depths keep index order.  ranges of empty tiles are [0, 0).  Also writes order
   (longest ranges first) for the compositing work queue. */
glam_status glam_bin_sort(const glam_projected* proj, const glam_views* views, glam_bins* bins,
                          void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Eq. 1 per pixel centre (x+0.5, y+0.5), front to back over its tile's range:
   alpha = min(0.99, opacity exp(power)), skipped when alpha < 1/255, the walk stops
   before an entry that would take T below 1e-4.  A persistent grid pulls (tile,
   quadrant) items from bins->queue in bins->order.  Writes image [3][H][W] per view,
   final transmittance T_final and n_contrib (1 + range position of the last
   composited entry) per pixel.  bg: [3] device (background colour, may be NULL).
   n_eval (may be NULL): per pixel, the range entries visited up to and including the
   one that stopped the walk, or the whole range length if it never stopped (the
   Gaussian-pixel evaluation count of the definition, independent of any skipping). */
glam_status glam_render_fwd(const glam_projected* proj, const glam_bins* bins,
                            const glam_views* views, const float* bg, float* image,
                            float* T_final, int32_t* n_contrib, int32_t* n_eval,
                            hipStream_t stream);

/* Eq. 3 per view: L_v = mean |C - target| + w_ssim (1 - mean SSIM), SSIM over an 11x11
   box window with zero padding, C1 = 0.01^2, C2 = 0.03^2 (the paper leaves the weight
   and the window open; these are the readings of its anchor-based lineage).  image,
   target, dimage: [3][H][W] per view at 3 * pix_begin (device).  Writes dL/dimage of the
   step's loss, the sum of the views' losses (one sampled keyframe per iteration in the
   paper, Sec. IV-B; a batch of views here), loss[n_views] (device) and, if total is not
   NULL, total[0] = sum of loss[] in view order (device).  workspace:
   glam_loss_workspace_bytes. */
size_t glam_loss_workspace_bytes(const glam_views* views);
glam_status glam_loss(const glam_views* views, const float* image, const float* target,
                      float w_ssim, float* dimage, float* loss, float* total, void* workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): glam_loss without a workspace
   argument.  Its per-(32x32 tile, channel) partial sums live in a scratch array the
   library holds on each device for the life of the process, GLAM_LOSS_SCRATCH_BYTES
   bytes (glam_loss_workspace_bytes(views) <= that: up to about 1,490 views of 1226x370
   per call); larger view tables are rejected with GLAM_ERR_WORKSPACE before anything
   is launched.  Same arguments otherwise, same kernels and results as glam_loss.  The
   call allocates nothing.  The scratch's device address is resolved on the call's first
   use on a device (make one call there before capturing a graph if the capture mode
   forbids that query).  All calls on one device share its scratch: each call
   overwrites every partial sum it reads, so nothing needs clearing, but calls that
   overlap in time on one device (other streams, other host threads) race on it and
   must be serialised by the caller. */
#define GLAM_LOSS_SCRATCH_BYTES (16u << 20)
glam_status glam_loss_noalloc(const glam_views* views, const float* image, const float* target,
                              float w_ssim, float* dimage, float* loss, float* total,
                              hipStream_t stream);

/* --- backward ------------------------------------------------------------------- */

/* Gradients.  Intermediate buffers are required (the library allocates nothing):
   g2d [n_gauss][9], nine consecutive floats per view-Gaussian (so one wave adds all nine
   at once): the pixel sums of p dx, p dy, p dx^2, p dx dy, p dy^2 with p = dL/dpower
   and (dx, dy) = (u, v) - pixel centre, then d(opacity, r, g, b).  The gradients of the
   centre and conic follow as du = -(A m0 + B m1), dv = -(B m0 + C m1), dA = -m2/2,
   dB = -m3, dC = -m4/2 (power = -(A dx^2 + C dy^2)/2 - B dx dy);
   dgauss: d(mean, scale, quat, opacity, rgb) per view-Gaussian (anchor mode) or of
   the plain parameters (plain mode: d(mean, log-scale, raw quat, logit, rgb), n = G).
   Anchor mode outputs dfeat [A][F], doffs [3][A*K], dlog_scale [A], dmlp [M][P]. */
typedef struct {
  float* g2d;
  glam_gaussians dgauss;
  float* dfeat;
  float* doffs;
  float* dlog_scale;
  float* dmlp;
  float* d2d;  /* [9][n_gauss] (GLAM_RETURN_INTERMEDIATES, else unused and may be NULL):
                  d(u, v, A, B, C, opacity, r, g, b) per view-Gaussian, zero when culled */
} glam_grads;

/* Adjoint of Eq. 1 (the rasteriser of Sec. III-A is differentiated to minimise Eq. 3):
   reverse compositing from (T_final, n_contrib): T_i recovered by division by
   (1 - alpha_i), per-Gaussian gradients reduced across each wavefront before FP32
   atomics.  Overwrites g2d [n_gauss][9] (zeroes it first). */
glam_status glam_composite_bwd(const glam_projected* proj, const glam_bins* bins,
                               const glam_views* views, const float* bg, const float* T_final,
                               const int32_t* n_contrib, const float* dimage, float* g2d,
                               hipStream_t stream);

/* For a per-pixel loss (Eq. 3 with w_ssim = 0: L_v = mean |C - target| over the view's
   pixels and channels), the forward of Eq. 1, that loss and the adjoint of Eq. 1 in one
   pass over the tiles (Sec. III-A): each quadrant item is composited, its pixels take
   dL/dC = sign(C - target) / (3 W H) from their own values, and the item is walked back
   at once while its records are still cached, instead of glam_render_fwd, glam_loss and
   glam_composite_bwd (an SSIM term needs the whole image before any dL/dC).  Writes
   what those three write: image, T_final, n_contrib, dimage ([3][H][W] per view at
   3 * pix_begin, device), loss[n_views] (device), total[0] = sum of loss[] in view order
   if total is not NULL, and g2d [n_gauss][9] (zeroed first; FP32 atomics, as
   glam_composite_bwd).  target: [3][H][W] per view.  The grid is bins.tuning's backward
   schedule.  workspace: glam_render_fused_l1_workspace_bytes (one partial sum per 8x8
   quadrant item). */
size_t glam_render_fused_l1_workspace_bytes(const glam_views* views);
glam_status glam_render_fused_l1(const glam_projected* proj, const glam_bins* bins,
                                 const glam_views* views, const float* bg, const float* target,
                                 float* image, float* T_final, int32_t* n_contrib, float* dimage,
                                 float* loss, float* total, float* g2d, void* workspace,
                                 size_t workspace_bytes, hipStream_t stream);

/* Adjoint of the projection of Sec. III-A (see glam_project): g2d -> dgauss (anchor
   mode: per view-Gaussian; plain mode:
   summed over views into the plain parameter gradients).  Overwrites dgauss. */
glam_status glam_project_bwd(const glam_gaussians* gauss, const glam_projected* proj,
                             const glam_views* views, uint32_t flags, const float* g2d,
                             glam_gaussians* dgauss, hipStream_t stream);

/* Adjoint of Eq. 2 with Eq. 6's per-partition MLPs (Sec. III-A, III-D): dgauss ->
   dfeat, doffs, dlog_scale, dmlp, summed over the views of each partition.  Overwrites
   them.  workspace: glam_decode_bwd_workspace_bytes. */
size_t glam_decode_bwd_workspace_bytes(const glam_anchors* anchors, const glam_views* views,
                                       int32_t n_parts);
glam_status glam_decode_bwd(const glam_anchors* anchors, const float* mlp, int32_t n_parts,
                            const glam_views* views, uint32_t flags,
                            const glam_gaussians* dgauss, float* dfeat, float* doffs,
                            float* dlog_scale, float* dmlp, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* Workspace bytes of glam_render_bwd for these flags (0 when the arguments are invalid):
   the decode adjoint's (anchor mode; anchors and n_parts ignored in plain mode) and,
   with GLAM_DETERMINISTIC_GRADS, the per-(pair, quadrant) partials for a pair capacity
   of capacity (36 bytes per pair and 8x8 quadrant of a tile). */
size_t glam_render_bwd_workspace_bytes(const glam_anchors* anchors, const glam_views* views,
                                       int32_t n_parts, int64_t capacity, uint32_t flags);

/* The whole backward of a mapping iteration (the gradient of Eq. 3 with respect to
   the anchors and MLPs, Sec. III-A, III-B), the adjoint of Eq. 1 -> projection ->
   Eq. 2 / Eq. 6 for the
   image gradient dimage (the loss gradient of glam_loss, or any other): composite
   adjoint (g2d), projection adjoint (dgauss), then in anchor mode the decode adjoint
   (dfeat, doffs, dlog_scale, dmlp), each overwritten.  flags: those of the forward calls
   (GLAM_PLAIN, GLAM_OPACITY_SIGMOID, GLAM_FOOTPRINT_3SIGMA) plus
   GLAM_DETERMINISTIC_GRADS (needs bins->pair_begin as written by the glam_bin_sort that
   produced bins) and GLAM_RETURN_INTERMEDIATES (needs grads->d2d).  workspace:
   glam_render_bwd_workspace_bytes(anchors, views, n_parts, bins->capacity, flags)
   bytes (may be NULL when that is 0).  GLAM_ERR_UNSUPPORTED when the reproducible
   partials would need more than 2^32 slots. */
glam_status glam_render_bwd(const glam_projected* proj, const glam_bins* bins,
                            const glam_views* views, const float* bg, const float* T_final,
                            const int32_t* n_contrib, const float* dimage,
                            const glam_gaussians* gauss, const glam_anchors* anchors,
                            const float* mlp, int32_t n_parts, uint32_t flags,
                            glam_grads* grads, void* workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* --- optimiser step ------------------------------------------------------------- */

/* One parameter group of the Adam update: param, grad, m and v are [n] device arrays
   (16-byte aligned; the caller zeroes m and v before step 1).  The learning rate is
   periodic in the element index: element i takes lr[k] for the segment k of (i mod
   period) in [seg_end[k-1], seg_end[k]) (seg_end[-1] = 0; 1 <= n_seg <= 4, seg_end
   increasing, seg_end[n_seg-1] == period).  A plain array is period = n, one segment;
   the packed MLP sets of all partitions are period = the parameters of one set, one
   segment per MLP. */
typedef struct {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t n;
  int32_t period;
  int32_t n_seg;
  int32_t seg_end[4];
  float lr[4];
} glam_adam_group;

#define GLAM_ADAM_MAX_GROUPS 16

/* The mapping iteration's optimiser step (the update that follows the backward; the
   Gaussian optimisation of Sec. III-B minimises Eq. 3, with Adam as in the 3DGS and
   Scaffold-GS lineage): Adam (Kingma & Ba) over all groups in one launch, step t >= 1 (bias corrections
   1 - beta^t), per element
     m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
     param -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
   1 <= n_groups <= GLAM_ADAM_MAX_GROUPS; 0 <= beta1, beta2 < 1; eps > 0; learning
   rates finite and >= 0; otherwise GLAM_ERR_INVALID_ARG before any launch. */
glam_status glam_adam_step(const glam_adam_group* groups, int32_t n_groups, int32_t step,
                           float beta1, float beta2, float eps, hipStream_t stream);

/* Keyframe sampler of a mapping iteration (Sec. IV-B: the k most recent keyframes with
   probability p, the older ones otherwise): count keyframe indices drawn from n_keyframes
   (0 = oldest): with probability p_recent uniformly among the k_recent most recent,
   otherwise uniformly among the older ones (all keyframes are recent when n_keyframes
   <= k_recent).  Draws come from Philox4x32-10 (Salmon et al., SC 2011) keyed by seed,
   at counters counter, counter + 1, ... (one counter per draw: the first word decides
   recent or old, the second picks the keyframe), so a draw is reproducible from
   (seed, counter).  out: [count] host.  Pure host function. */
glam_status glam_sample_keyframes(int32_t n_keyframes, int32_t k_recent, float p_recent,
                                  int32_t count, uint64_t seed, uint64_t counter, int32_t* out);

/* --- loop closure ----------------------------------------------------------------- */

/* One keyframe's loop-closure correction: its pose before (a camera whose intrinsics and
   image size also define the keyframe's view frustum) and its corrected world->camera
   pose. */
typedef struct {
  glam_camera before;
  float R_new[9];
  float t_new[3];
} glam_keyframe_fix;

/* Eq. 7 (loop closures, Sec. III-E): each corrected keyframe i moves the anchors of its
   view frustum by
   dT_i = T_new,i^-1 T_old,i (T = world->camera), so they keep their coordinates in the
   keyframe's camera frame.  An anchor lies in the frustum when its depth in the old
   camera frame is in [near, far] and it projects inside the image; an anchor in several
   frusta follows the keyframe whose old camera centre is nearest (ties: the lower
   index).  Positions move as x <- R_d x + t_d and the anchor's K offsets rotate with it,
   o <- R_d o; anchors outside every frustum stay.  pos [3][A] and offs [3][A*K] device,
   updated in place; fixes [n_fix] device; owner [A] device (may be NULL) receives the
   keyframe applied or -1.  0 < near < far. */
glam_status glam_deform_anchors(float* pos, float* offs, int32_t A, int32_t K,
                                const glam_keyframe_fix* fixes, int32_t n_fix, float near,
                                float far, int32_t* owner, hipStream_t stream);

/* --- flow densification ------------------------------------------------------------ */

/* Eq. 5 (flow densification, Sec. III-C): filters N correspondences x1 <-> x2 between
   two keyframes with known cameras by
   the epipolar residual |x2^T F x1| < tau (x homogeneous pixel coordinates [u, v, 1]) and
   triangulates the retained ones.  F = [e2]x P2 P1^+ with P = K [R | t], e2 = P2 C1 (C1
   the first camera's centre) and P1^+ the pseudo-inverse of P1, scaled to unit Frobenius
   norm with the sign that makes its largest-magnitude entry positive (tau is in those
   units); computed on the host in double precision.  Retained pairs are triangulated by
   linear least squares with the known poses (the four DLT rows in normalised image
   coordinates, X = (X, Y, Z, 1)), in double precision on the GPU.  x1, x2 [2][N] device
   (u row, then v row); residual [N], keep [N] (1 retained, 0 not, or when the
   triangulation is singular), X [3][N] world points (NaN where keep is 0) device. */
glam_status glam_epipolar_triangulate(const glam_camera* cam1, const glam_camera* cam2,
                                      const float* x1, const float* x2, int64_t n, float tau,
                                      float* residual, int32_t* keep, float* X,
                                      hipStream_t stream);

/* --- anchor voxelisation and growth -------------------------------------------------- */

/* Bytes of workspace glam_voxelize needs for n_points points (0 when n_points is out of
   range). */
size_t glam_voxelize_workspace_bytes(int64_t n_points);

/* Eq. 4 (Sec. III-B): the fused point cloud (tracked points and triangulated flow points)
   snapped to the voxel grid of size eps, keeping unique voxels, and of those the ones
   not already anchors (the incremental growth of the anchor set).  Per point and axis
   k = round(p / eps), the FP32 quotient rounded to the nearest integer with ties to
   even; k must lie in [-2^20, 2^20) on every axis, otherwise (or for a NaN coordinate,
   as in a rejected triangulation) the point is dropped and counted.  A voxel's key packs
   (k_x + 2^20, k_y + 2^20, k_z + 2^20) into bits 62..42, 41..21, 20..0, so key order is
   lexicographic (x, y, z) order; its centre is k * eps (FP32 product).
     points [3][n_points] device
     existing [n_existing] device: keys of the current anchors, strictly ascending
     new_keys [capacity], new_centres [3][capacity] device: the voxels of the points
       whose keys are absent from existing, ascending by key (centres row by row with
       row stride capacity)
     merged [n_existing + capacity] device, or NULL: the ascending union of existing and
       the new keys (the key set after growth), in its first n_existing + min(count,
       capacity) entries
     counts [2] int64 device: the number of new voxels (which may exceed capacity: then
       only the first capacity are written and merged lacks the rest), and the number of
       dropped points
   n_points <= 2^31 (else GLAM_ERR_UNSUPPORTED); eps > 0 and finite.  Workspace:
   glam_voxelize_workspace_bytes(n_points).  If existing is not strictly ascending the
   outputs are unspecified, but no memory outside the given buffers is touched. */
glam_status glam_voxelize(const float* points, int64_t n_points, float eps,
                          const uint64_t* existing, int64_t n_existing, uint64_t* new_keys,
                          float* new_centres, int64_t capacity, uint64_t* merged,
                          int64_t* counts, void* workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* The bookkeeping of anchor growth (Sec. III-B, Eq. 4): anchors are stored grouped by
   partition (Eq. 6), so the anchors a keyframe adds are inserted at the end of its
   partition's range in every per-anchor array (and in the optimiser's moments), and the
   later partitions' ranges shift by n_new.  Copies rows rows of n_old * width floats
   from src to dst rows of (n_old + n_new) * width floats, inserting n_new * width floats
   at float at * width of each row (0 <= at <= n_old): taken from ins (rows rows of
   n_new * width floats starting ins_stride >= n_new * width floats apart, device, may be
   NULL: the centres glam_voxelize writes have ins_stride = its capacity) or, without
   ins, all equal to fill.  The
   layouts of the library's anchors are of this form: pos and offs [3][...] (rows 3,
   width 1 and K), feat [A][F] and log_scale [A] (rows 1, width F and 1).  src, dst
   device, 16-byte aligned, not overlapping; rows <= 65535.  The caller updates its
   partition offsets. */
glam_status glam_insert_rows(const float* src, float* dst, int32_t rows, int64_t n_old,
                             int32_t width, int64_t at, int64_t n_new, const float* ins,
                             int64_t ins_stride, float fill, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
