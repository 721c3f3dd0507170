/* FP64 CPU oracle of the anchor-decoded Gaussian-splatting render.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's CPU
 * baseline may load this library.  It shares no code, header, table or helper with
 * the HIP path; the two meet only through the seeded inputs of the synth module.
 *
 * Every stage is the plain definition written out in double precision, slow and
 * loop-based, following the paper:
 *   decode      view-conditioned anchor MLPs, Eq. 2 (Sec. III-A) with one MLP set per
 *               spatial partition, Eq. 6 (Sec. III-D)
 *   project     the projected 2-D Gaussian of each 3-D Gaussian (Sec. III-A), by the
 *               EWA / 3DGS construction the paper builds on
 *   bin + sort  tile lists ordered by depth (the tile-based rasteriser of Sec. II/III-A)
 *   render      front-to-back alpha compositing, Eq. 1 (Sec. III-A)
 *   loss        L1 + SSIM objective, Eq. 3 (Sec. III-A)
 *   backward    analytic gradients of all of the above
 * Constants the paper leaves open (clamps, thresholds, footprint rule, activations,
 * loss weights) are the readings listed at each function.
 *
 * Arrays are structure-of-arrays: "[3][G]" means three contiguous rows of G values.
 */
#ifndef GLAM_ORACLE_H
#define GLAM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pinhole camera: world->camera rotation R (row-major) and translation t,
   OpenCV axes (x right, y down, z forward), intrinsics, image size. */
typedef struct {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t W, H;
} orc_cam;

enum { ORC_OPACITY_TANH = 0, ORC_OPACITY_SIGMOID = 1 };

/* Ambiguity flag bits of a pixel (decisions that FP32 and FP64 may take apart). */
enum {
  ORC_AMB_ALPHA = 1,  /* some alpha within 1e-6 of the 1/255 skip threshold       */
  ORC_AMB_T = 2,      /* some transmittance within 1e-8 of the 1e-4 stop threshold */
  ORC_AMB_DEPTH = 4,  /* two candidates with a relative depth gap below 1e-6       */
  ORC_AMB_CLAMP = 8   /* some alpha within 1e-6 of the 0.99 clamp (gradient kink)  */
};

int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Widths of the ambiguity windows of the ORC_AMB_* flags (defaults 1e-6, 1e-8, 1e-6,
   1e-6): |alpha - 1/255| < alpha, |T' - 1e-4| < T, relative depth gap < depth,
   |raw alpha - 0.99| < clamp.  Bookkeeping for parity tests; values are unaffected. */
void orc_set_margins(double alpha, double T, double depth, double clamp);

/* Magnitude mode (0 off, the default): orc_render_bwd then accumulates, per element,
   the sum of the magnitudes of the terms the element is a sum of (every factor by its
   absolute value), the scale of the element's rounding error in finite precision. */
void orc_set_magnitude_mode(int on);

/* Number of packed parameters of one partition's MLP set. */
int orc_mlp_param_count(int F, int K, int hidden);

/* Decode the anchors of one partition for one camera (Eq. 2, Eq. 6).
   pos[3][A], feat[A][F], log_scale[A], offs[3][A*K], mlp packed as
   (opacity, colour, covariance) x (W1[hidden][F+4], b1, W2[out][hidden], b2).
   Outputs activated Gaussians [.][A*K]: mean[3], scale[3], unit quat[4] (w,x,y,z),
   opacity, rgb[3].  Gaussian a*K+j belongs to anchor a. */
void orc_decode(int A, int F, int K, int hidden, const double* pos, const double* feat,
                const double* log_scale, const double* offs, const double* mlp,
                const orc_cam* cam, int opacity_mode, double* mean, double* scale,
                double* quat, double* opacity, double* rgb);

/* orc_decode with its discrete decisions exposed: relu_out[A][3][hidden] (may be NULL)
   receives, per anchor, MLP (opacity, colour, covariance) and hidden unit, whether the
   ReLU passed (1) or not (0); relu_in (may be NULL) imposes those decisions instead of
   taking them (the MLP then stays the same linear map near the point where they were
   taken: finite-difference checks). */
void orc_decode_ex(int A, int F, int K, int hidden, const double* pos, const double* feat,
                   const double* log_scale, const double* offs, const double* mlp,
                   const orc_cam* cam, int opacity_mode, double* mean, double* scale,
                   double* quat, double* opacity, double* rgb, const uint8_t* relu_in,
                   uint8_t* relu_out);

/* Adjoint of orc_decode.  Accumulates (+=) into dfeat[A][F], doffs[3][A*K],
   dlog_scale[A] and dmlp[P] from gradients of the decoded Gaussians. */
void orc_decode_bwd(int A, int F, int K, int hidden, const double* pos, const double* feat,
                    const double* log_scale, const double* offs, const double* mlp,
                    const orc_cam* cam, int opacity_mode, const double* dmean,
                    const double* dscale, const double* dquat, const double* dopacity,
                    const double* drgb, double* dfeat, double* doffs, double* dlog_scale,
                    double* dmlp);

/* Plain (anchor-free) parameters -> activated Gaussians: scale = exp(log_scale),
   q = q_raw / sqrt(|q_raw|^2 + 1e-24), opacity = sigmoid(logit). */
void orc_plain_activate(int G, const double* log_scale, const double* quat_raw,
                        const double* logit, double* scale, double* quat, double* opacity);
/* Its adjoint (overwrites the outputs). */
void orc_plain_activate_bwd(int G, const double* log_scale, const double* quat_raw,
                            const double* logit, const double* dscale, const double* dquat,
                            const double* dopacity, double* dlog_scale, double* dquat_raw,
                            double* dlogit);

/* Projection and footprint of G activated Gaussians for one camera.
   Outputs uv[2][G], conic[3][G] (A, B, C of the inverse 2-D covariance), cov2d[3][G]
   (a, b, c), depth[G] (camera z), ext[2][G] (half extents of the footprint box, -1 if
   culled), prect[4][G] (inclusive pixel box x0, x1, y0, y1; x0 > x1 if culled) and
   ntiles[G] (tiles of tile_w x tile_h touched, 0 if culled). */
void orc_project(int G, const double* mean, const double* scale, const double* quat,
                 const double* opacity, const orc_cam* cam, int tile_w, int tile_h,
                 double* uv, double* conic, double* cov2d, double* depth, double* ext,
                 int32_t* prect, int32_t* ntiles);

/* orc_project with the Jacobian clamp decision exposed and a choice of footprint:
   clamp_out[G][2] (may be NULL) receives per Gaussian and axis 0 (free), 1 (clamped at
   the low limit) or 2 (high limit); clamp_in (may be NULL) imposes those decisions.
   footprint 0: the opacity-aware box (orc_project).  footprint 1: the square of the
   3-D Gaussian splatting lineage, ext = r = ceil(3 sqrt(lambda_max)) on both axes
   (lambda_max the larger eigenvalue of the dilated 2-D covariance), the pixel centres
   within r of the centre selecting tiles of tile_w x tile_h, and prect widened to
   those tiles (clipped to the image): the Gaussian is a candidate at every pixel of
   every tile it is binned to, so the image depends on the tile size. */
void orc_project_ex(int G, const double* mean, const double* scale, const double* quat,
                    const double* opacity, const orc_cam* cam, int tile_w, int tile_h,
                    double* uv, double* conic, double* cov2d, double* depth, double* ext,
                    int32_t* prect, int32_t* ntiles, const int8_t* clamp_in, int8_t* clamp_out,
                    int footprint);

/* Adjoint of orc_project for the differentiable outputs (uv, conic) plus the
   pass-through opacity and colour.  g2d[9][G] = d(u, v, A, B, C, opacity, r, g, b).
   Overwrites dmean[3][G], dscale[3][G], dquat[4][G], dopacity[G], drgb[3][G]. */
void orc_project_bwd(int G, const double* mean, const double* scale, const double* quat,
                     const double* opacity, const orc_cam* cam, const int32_t* ntiles,
                     const double* g2d, double* dmean, double* dscale, double* dquat,
                     double* dopacity, double* drgb);

/* Footprint box from single-precision centre and half extents, evaluated with the
   same IEEE single operations a GPU uses (stage-wise check of tile assignment).
   ext < 0 marks a culled Gaussian. */
void orc_rect_f32(int G, const float* u, const float* v, const float* ex, const float* ey,
                  int W, int H, int tile_w, int tile_h, int32_t* prect, int32_t* ntiles);

/* Tile binning and depth sort over several views.  Gaussian g of view k lies in
   [gbegin[k], gbegin[k+1]); view k's tiles are numbered from tile_base[k], row-major
   over tiles_x[k] x tiles_y[k].  Pairs (global tile, depth bits) are emitted per
   Gaussian in increasing index and, within a Gaussian, row-major over its tiles, then
   stably sorted by (tile, depth), so equal depths keep increasing index.  Fills
   tile[P], vals[P] (P = sum of the Gaussians' tile counts) and ranges[T][2]
   ([start, end), zero when empty). */
void orc_bin_sort(int n_views, const int64_t* gbegin, const int32_t* tiles_x,
                  const int32_t* tiles_y, const int64_t* tile_base, int tile_w, int tile_h,
                  const int32_t* prect, const double* depth, int64_t G, int64_t T_total,
                  int32_t* tile, int32_t* vals, int64_t* ranges);

/* Forward compositing of one view over its tile lists (Eq. 1).  Per-Gaussian arrays
   are view-local: uv[2][G], conic[3][G], opacity[G], rgb[3][G], prect[4][G], depth[G].
   vals hold view-local Gaussian indices; ranges[T][2] index into vals.
   Outputs image[3][H][W], T_final[H*W], n_contrib[H*W] (1 + position in the tile
   list of the last composited Gaussian), n_eval[H*W] (entries visited up to and
   including the stopping one), amb[H*W] (ORC_AMB_* bits). */
void orc_render_fwd(int G, const double* uv, const double* conic, const double* opacity,
                    const double* rgb, const int32_t* prect, const double* depth,
                    const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                    int tile_h, const double* bg, double* image, double* T_final,
                    int32_t* n_contrib, int32_t* n_eval, uint8_t* amb);

/* Backward compositing of one view: gradients of a loss with image gradient
   dimage[3][H][W] with respect to g2d[9][G] = (u, v, A, B, C, opacity, r, g, b).
   Uses the forward transmittances it stores itself (no division).  Overwrites g2d. */
void orc_render_bwd(int G, const double* uv, const double* conic, const double* opacity,
                    const double* rgb, const int32_t* prect, const double* depth,
                    const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                    int tile_h, const double* bg, const double* dimage, double* g2d);

/* The composited list of every pixel of one view (same arguments as orc_render_fwd):
   the view-local Gaussians that took part, front to back, and whether each one's alpha
   was clamped at 0.99.  Returns a handle and the total number of entries; the caller
   allocates offsets[H*W+1], ids[total] and clamped[total] and passes them with the
   handle to orc_render_lists_take, which fills them (pixel p's list is
   [offsets[p], offsets[p+1])) and releases the handle.  Together with the decode and
   projection decisions these are every discrete decision of the forward pass
   (candidate set, depth order, skips, stop, clamps). */
void* orc_render_lists(int G, const double* uv, const double* conic, const double* opacity,
                       const double* rgb, const int32_t* prect, const double* depth,
                       const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                       int tile_h, int64_t* total);
void orc_render_lists_take(void* handle, int64_t* offsets, int32_t* ids, uint8_t* clamped);

/* Eq. 1 over given composited lists (from orc_render_lists), the decisions held fixed:
   per pixel C = sum_i c_i a_i prod_{j<i}(1 - a_j) + bg prod_i (1 - a_i) with
   a_i = opacity_i exp(power_i), or 0.99 where clamped[i].  The function of the
   parameters that the analytic adjoint differentiates (finite-difference checks). */
void orc_render_frozen(int G, const double* uv, const double* conic, const double* opacity,
                       const double* rgb, int W, int H, const double* bg,
                       const int64_t* offsets, const int32_t* ids, const uint8_t* clamped,
                       double* image, double* T_final);

/* Brute-force compositing without tiles: every Gaussian whose footprint box holds
   the pixel, ordered by (depth, index).  Same outputs as orc_render_fwd except that
   n_contrib counts positions in the pixel's own list. */
void orc_render_brute(int G, const double* uv, const double* conic, const double* opacity,
                      const double* rgb, const int32_t* prect, const double* depth, int W,
                      int H, const double* bg, double* image, double* T_final,
                      int32_t* n_contrib, uint8_t* amb);

/* Direct-formula backward of the brute-force compositing, O(n^2) per pixel:
   d C / d alpha_i = c_i prod_{j<i}(1 - a_j) - sum_{k>i} c_k a_k prod_{j<k, j!=i}(1 - a_j)
   evaluated term by term (tiny scenes only).  Overwrites g2d[9][G]. */
void orc_render_brute_bwd(int G, const double* uv, const double* conic,
                          const double* opacity, const double* rgb, const int32_t* prect,
                          const double* depth, int W, int H, const double* bg,
                          const double* dimage, double* g2d);

/* Photometric loss of one view, Eq. 3: L = mean|C - T| + w_ssim * (1 - mean SSIM),
   SSIM with an 11x11 box window, zero padding, constants 0.01^2 and 0.03^2.
   Writes the per-pixel loss terms loss_px[H*W] (summing to L), the SSIM map
   ssim[3][H][W] and dimage[3][H][W] = dL/dC.  Returns L. */
double orc_loss(int W, int H, const double* image, const double* target, double w_ssim,
                double* loss_px, double* ssim, double* dimage);

/* orc_loss with the sign of each L1 term given (l1_sign[3][H][W] of -1, 0, 1; NULL: the
   sign of C - T): the L1 term becomes sign * (C - T).  Finite-difference checks. */
double orc_loss_signed(int W, int H, const double* image, const double* target, double w_ssim,
                       const double* l1_sign, double* loss_px, double* ssim, double* dimage);

#ifdef __cplusplus
}
#endif
#endif
