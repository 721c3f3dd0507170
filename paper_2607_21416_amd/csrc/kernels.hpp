// Host-side launchers of the glam kernels (each in its own .hip file).
#pragma once

#include <hip/hip_runtime.h>

#include "glam.h"

namespace glam {

// Tile edges the binning and compositing support (square tiles, multiples of the 8x8
// compositing quadrant).
inline bool tile_edge_supported(int e) { return e == 8 || e == 16 || e == 32; }
inline int tile_log2(int e) { return e == 8 ? 3 : (e == 16 ? 4 : 5); }

// Compositing schedule defaults and limits (glam_tuning).
// Workgroups of 4 waves: up to 5 (forward) and 6 (backward) per CU; of 8 waves: up to
// 2 per CU; of 16: one.
constexpr int kDefaultLongLog2 = 10;
constexpr int kMaxFwdBlocksPerCU = 5, kMaxBwdBlocksPerCU = 6;
inline bool group_ok(int waves, int blocks, int max4) {
  if (waves == 0 || waves == 4) return blocks >= 0 && blocks <= max4;
  if (waves == 8 || waves == 16) return blocks >= 0 && blocks * waves <= 16;
  return false;
}
inline bool tuning_ok(const glam_tuning& t) {
  return (t.long_log2 == 0 || (t.long_log2 >= 6 && t.long_log2 <= 24)) &&
         group_ok(t.fwd_group_waves, t.fwd_blocks_per_cu, kMaxFwdBlocksPerCU) &&
         group_ok(t.bwd_group_waves, t.bwd_blocks_per_cu, kMaxBwdBlocksPerCU) &&
         (t.non_persistent == 0 || t.non_persistent == 1) && t.reserved[0] == 0 && t.reserved[1] == 0;
}

// Compute units of the current device (256 if the runtime cannot say).
int cu_count();

glam_status launch_project(const glam_gaussians& g, const glam_views& v, bool plain, bool sigma3,
                           const glam_projected& out, hipStream_t s);
glam_status launch_project_bwd(const glam_gaussians& g, const glam_projected& proj, const glam_views& v,
                               bool plain, const float* g2d, const glam_gaussians& dg, float* d2d, hipStream_t s);

size_t bin_sort_workspace(const glam_views& v, long long capacity);
glam_status launch_bin_sort(const glam_projected& proj, const glam_views& v, const glam_bins& bins,
                            void* ws, size_t ws_bytes, hipStream_t s);

glam_status launch_render_fwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                              const float* bg, float* image, float* T_final, int32_t* n_contrib,
                              int32_t* n_eval, hipStream_t s);
// det_part (may be null): the reproducible backward's partial buffer of
// det_partial_bytes, in place of floating-point atomics.
size_t det_partial_bytes(const glam_views& v, long long capacity);
bool det_supported(const glam_views& v, long long capacity);
glam_status launch_composite_bwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                                 const float* bg, const float* T_final, const int32_t* n_contrib,
                                 const float* dimage, float* g2d, float* det_part, hipStream_t s);

// The forward, the L1 term of the loss and the compositing adjoint in one pass (a
// per-pixel loss); its workspace holds one partial sum per quadrant item (and, with no
// Gaussians, the loss kernel's partial sums).
size_t fused_l1_workspace(const glam_views& v);
glam_status launch_fused_l1(const glam_projected& proj, const glam_bins& bins, const glam_views& v, const float* bg,
                            const float* target, float* image, float* T_final, int32_t* n_contrib, float* dimage,
                            float* loss, float* total, float* g2d, void* ws, hipStream_t s);

// The views' L1 losses from per-(tile, quadrant) sums of |C - target| (the fused pass's):
// l1_part[(tile << ql) | quadrant].
glam_status launch_l1_reduce(const glam_views& v, int ql, const float* l1_part, float* loss, float* total,
                             hipStream_t s);

size_t loss_workspace(const glam_views& v);
glam_status launch_loss(const glam_views& v, const float* image, const float* target, float w_ssim,
                        float* dimage, float* loss, float* total, void* ws, hipStream_t s);
glam_status launch_loss_noalloc(const glam_views& v, const float* image, const float* target, float w_ssim,
                                float* dimage, float* loss, float* total, hipStream_t s);

glam_status launch_decode(const glam_anchors& a, const float* mlp, const glam_views& v, bool sigmoid_opacity,
                          bool sigma3, const glam_gaussians& out, const glam_projected* proj, hipStream_t s);
size_t decode_bwd_workspace(const glam_anchors& a, const glam_views& v, int n_parts);
glam_status launch_decode_bwd(const glam_anchors& a, const float* mlp, int n_parts, const glam_views& v,
                              bool sigmoid_opacity, const glam_gaussians& dg, float* dfeat, float* doffs,
                              float* dlog_scale, float* dmlp, void* ws, hipStream_t s);

bool adam_groups_ok(const glam_adam_group* groups, int n_groups);
glam_status launch_adam(const glam_adam_group* groups, int n_groups, int step, float beta1, float beta2, float eps,
                        hipStream_t s);
void sample_keyframes(int n, int k_recent, float p_recent, int count, uint64_t seed, uint64_t counter,
                      int32_t* out);

glam_status launch_deform(float* pos, float* offs, int A, int K, const glam_keyframe_fix* fixes, int n_fix,
                          float near, float far, int32_t* owner, hipStream_t s);

bool fundamental_from_cameras(const glam_camera& c1, const glam_camera& c2, double F[9]);
glam_status launch_epipolar(const glam_camera& c1, const glam_camera& c2, const float* x1, const float* x2,
                            long long n, float tau, float* residual, int32_t* keep, float* X, hipStream_t s);

constexpr long long kVoxelMaxPoints = 1ll << 31;
size_t voxelize_workspace(long long n);
glam_status launch_voxelize(const float* points, long long n, float eps, const uint64_t* existing,
                            long long n_existing, uint64_t* new_keys, float* new_pos, long long capacity,
                            uint64_t* merged, int64_t* counts, void* ws, hipStream_t s);
glam_status launch_insert_rows(const float* src, float* dst, int rows, long long n_old, int width, long long at,
                               long long n_new, const float* ins, long long ins_stride, float fill, hipStream_t s);

}  // namespace glam
