// C ABI of the glam library: host-side validation, view table construction, and the
// launch sequence of every entry point.  Nothing here allocates device memory or
// synchronises; every launch goes to the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "glam.h"
#include "kernels.hpp"

namespace glam {
bool decode_supported(int F, int K);
}

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool ok_ptr(const void* p) { return p != nullptr && aligned16(p); }

// The host table is consistent with the totals (what the workspace queries read).
bool views_host_ok(const glam_views* v) {
  if (!v || !v->host || v->n <= 0) return false;
  if (v->tile_w != v->tile_h || !glam::tile_edge_supported(v->tile_w)) return false;
  if (v->n_gauss < 0 || v->n_pix <= 0 || v->n_tiles <= 0) return false;
  // totals must agree with the host table
  long long g = 0, p = 0, t = 0;
  for (int i = 0; i < v->n; ++i) {
    const glam_view_info& vi = v->host[i];
    if (vi.g_begin != g || vi.pix_begin != p || vi.tile_begin != t) return false;
    if (vi.cam.width <= 0 || vi.cam.height <= 0 || vi.cam.width > 32767 || vi.cam.height > 32767) return false;
    g += vi.g_count;
    p += (long long)vi.cam.width * vi.cam.height;
    t += (long long)vi.tiles_x * vi.tiles_y;
  }
  return g == v->n_gauss && p == v->n_pix && t == v->n_tiles && t < (1ll << 31) && g < (1ll << 32);
}

bool views_ok(const glam_views* v) { return views_host_ok(v) && v->dev != nullptr; }

bool gauss_ok(const glam_gaussians* g, bool need) {
  if (!g) return false;
  if (!need) return true;
  return ok_ptr(g->mean) && ok_ptr(g->scale) && ok_ptr(g->quat) && ok_ptr(g->opacity) && ok_ptr(g->rgb) && g->n > 0;
}

bool anchors_ok(const glam_anchors* a) {
  return a && ok_ptr(a->pos) && ok_ptr(a->feat) && ok_ptr(a->log_scale) && ok_ptr(a->offs) && a->A > 0 &&
         a->hidden == 32 && a->K > 0 && a->K <= 16 && (a->F == 8 || a->F == 16 || a->F == 32 || a->F == 64);
}

bool anchor_views_ok(const glam_anchors* a, const glam_views* v) {
  // every view's partition range lies inside the anchors and carries anchor_count*K
  // Gaussians; a partition's views form one contiguous run
  for (int i = 0; i < v->n; ++i) {
    const glam_view_info& vi = v->host[i];
    if (vi.anchor_begin < 0 || vi.anchor_count < 0 || (long long)vi.anchor_begin + vi.anchor_count > a->A) return false;
    if (vi.g_count != (long long)vi.anchor_count * a->K) return false;
    if (vi.cam.partition < 0) return false;
    for (int j = 0; j < i; ++j)
      if (v->host[j].cam.partition == vi.cam.partition && v->host[i - 1].cam.partition != vi.cam.partition)
        return false;
  }
  return true;
}

bool proj_ok(const glam_projected* p) {
  return p && ok_ptr(p->uv) && ok_ptr(p->conic) && ok_ptr(p->depth) && ok_ptr(p->ext) && ok_ptr(p->ntiles) &&
         ok_ptr(p->splat);
}

bool bins_ok(const glam_bins* b) {
  return b && ok_ptr(b->keys) && ok_ptr(b->vals) && ok_ptr(b->ranges) && ok_ptr(b->status) && ok_ptr(b->order) &&
         ok_ptr(b->queue) && b->capacity > 0 && b->capacity < (1ll << 32) && glam::tuning_ok(b->tuning) &&
         (b->pair_begin == nullptr || aligned16(b->pair_begin));
}

// Flags each entry point understands (anything else is rejected).
constexpr uint32_t kForwardFlags = GLAM_PLAIN | GLAM_OPACITY_SIGMOID | GLAM_FOOTPRINT_3SIGMA;
constexpr uint32_t kBackwardFlags = kForwardFlags | GLAM_DETERMINISTIC_GRADS | GLAM_RETURN_INTERMEDIATES;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int max_partition(const glam_views* v) {
  int m = -1;
  for (int i = 0; i < v->n; ++i) m = v->host[i].cam.partition > m ? v->host[i].cam.partition : m;
  return m;
}

}  // namespace

extern "C" {

const char* glam_status_string(int32_t s) {
  switch (s) {
    case GLAM_OK: return "ok";
    case GLAM_ERR_INVALID_ARG: return "invalid argument";
    case GLAM_ERR_WORKSPACE: return "workspace too small";
    case GLAM_ERR_CAPACITY: return "pair capacity exceeded";
    case GLAM_ERR_HIP: return "HIP launch error";
    case GLAM_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int32_t glam_mlp_param_count(int32_t F, int32_t K, int32_t hidden) {
  if (F <= 0 || K <= 0 || hidden <= 0) return -1;
  const int n_in = F + 4;
  return 3 * (hidden * n_in + hidden) + (K + 3 * K + 7 * K) * (hidden + 1);
}

glam_status glam_views_build(const glam_camera* cams, int32_t n_views, const int32_t* part_begin, int32_t n_parts,
                             int32_t K, int64_t plain_G, int32_t tile_w, int32_t tile_h, glam_view_info* info,
                             glam_views* views) {
  if (!cams || !info || !views || n_views <= 0) return GLAM_ERR_INVALID_ARG;
  if (tile_w != tile_h || !glam::tile_edge_supported(tile_w)) return GLAM_ERR_UNSUPPORTED;
  if (part_begin && (n_parts <= 0 || K <= 0)) return GLAM_ERR_INVALID_ARG;
  if (!part_begin && plain_G <= 0) return GLAM_ERR_INVALID_ARG;
  long long g = 0, p = 0, t = 0;
  for (int i = 0; i < n_views; ++i) {
    const glam_camera& c = cams[i];
    if (c.width <= 0 || c.height <= 0 || c.width > 32767 || c.height > 32767) return GLAM_ERR_INVALID_ARG;
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return GLAM_ERR_INVALID_ARG;
    glam_view_info& vi = info[i];
    std::memset(&vi, 0, sizeof(vi));
    vi.cam = c;
    vi.tiles_x = (c.width + tile_w - 1) / tile_w;
    vi.tiles_y = (c.height + tile_h - 1) / tile_h;
    vi.g_begin = g;
    vi.pix_begin = p;
    vi.tile_begin = (int32_t)t;
    if (part_begin) {
      if (c.partition < 0 || c.partition >= n_parts) return GLAM_ERR_INVALID_ARG;
      vi.anchor_begin = part_begin[c.partition];
      vi.anchor_count = part_begin[c.partition + 1] - part_begin[c.partition];
      if (vi.anchor_count < 0) return GLAM_ERR_INVALID_ARG;
      vi.g_count = (long long)vi.anchor_count * K;
    } else {
      vi.g_count = plain_G;
    }
    g += vi.g_count;
    p += (long long)c.width * c.height;
    t += (long long)vi.tiles_x * vi.tiles_y;
  }
  if (t >= (1ll << 31) || g >= (1ll << 32)) return GLAM_ERR_UNSUPPORTED;
  views->n = n_views;
  views->tile_w = tile_w;
  views->tile_h = tile_h;
  views->n_gauss = g;
  views->n_pix = p;
  views->n_tiles = t;
  return GLAM_OK;
}

size_t glam_bin_sort_workspace_bytes(const glam_views* views, int64_t capacity) {
  if (!views_host_ok(views) || capacity <= 0) return 0;
  return glam::bin_sort_workspace(*views, capacity);
}

glam_status glam_decode(const glam_anchors* anchors, const float* mlp, int32_t n_parts, const glam_views* views,
                        uint32_t flags, glam_gaussians* out, hipStream_t stream) {
  if (!anchors_ok(anchors) || !ok_ptr(mlp) || !views_ok(views) || !gauss_ok(out, true) || n_parts <= 0)
    return GLAM_ERR_INVALID_ARG;
  if ((flags & GLAM_PLAIN) || (flags & ~kForwardFlags)) return GLAM_ERR_INVALID_ARG;
  if (!anchor_views_ok(anchors, views) || out->n != views->n_gauss || max_partition(views) >= n_parts)
    return GLAM_ERR_INVALID_ARG;
  if (!glam::decode_supported(anchors->F, anchors->K)) return GLAM_ERR_UNSUPPORTED;
  return glam::launch_decode(*anchors, mlp, *views, (flags & GLAM_OPACITY_SIGMOID) != 0,
                             (flags & GLAM_FOOTPRINT_3SIGMA) != 0, *out, nullptr, stream);
}

glam_status glam_decode_project(const glam_anchors* anchors, const float* mlp, int32_t n_parts,
                                const glam_views* views, uint32_t flags, glam_gaussians* out,
                                glam_projected* proj, hipStream_t stream) {
  if (!anchors_ok(anchors) || !ok_ptr(mlp) || !views_ok(views) || !gauss_ok(out, true) || n_parts <= 0 ||
      !proj_ok(proj))
    return GLAM_ERR_INVALID_ARG;
  if ((flags & GLAM_PLAIN) || (flags & ~kForwardFlags)) return GLAM_ERR_INVALID_ARG;
  if (!anchor_views_ok(anchors, views) || out->n != views->n_gauss || max_partition(views) >= n_parts)
    return GLAM_ERR_INVALID_ARG;
  if (!glam::decode_supported(anchors->F, anchors->K)) return GLAM_ERR_UNSUPPORTED;
  return glam::launch_decode(*anchors, mlp, *views, (flags & GLAM_OPACITY_SIGMOID) != 0,
                             (flags & GLAM_FOOTPRINT_3SIGMA) != 0, *out, proj, stream);
}

glam_status glam_project(const glam_gaussians* gauss, const glam_views* views, uint32_t flags, glam_projected* out,
                         hipStream_t stream) {
  if (!views_ok(views) || !gauss_ok(gauss, true) || !proj_ok(out) || (flags & ~kForwardFlags))
    return GLAM_ERR_INVALID_ARG;
  const bool plain = (flags & GLAM_PLAIN) != 0;
  if (plain) {
    for (int i = 0; i < views->n; ++i)
      if (views->host[i].g_count != gauss->n) return GLAM_ERR_INVALID_ARG;
  } else if (gauss->n != views->n_gauss) {
    return GLAM_ERR_INVALID_ARG;
  }
  return glam::launch_project(*gauss, *views, plain, (flags & GLAM_FOOTPRINT_3SIGMA) != 0, *out, stream);
}

glam_status glam_bin_sort(const glam_projected* proj, const glam_views* views, glam_bins* bins, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  if (!proj_ok(proj) || !views_ok(views) || !bins_ok(bins) || !ok_ptr(workspace)) return GLAM_ERR_INVALID_ARG;
  if (workspace_bytes < glam::bin_sort_workspace(*views, bins->capacity)) return GLAM_ERR_WORKSPACE;
  return glam::launch_bin_sort(*proj, *views, *bins, workspace, workspace_bytes, stream);
}

glam_status glam_render_fwd(const glam_projected* proj, const glam_bins* bins, const glam_views* views,
                            const float* bg, float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval,
                            hipStream_t stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !views_ok(views) || !ok_ptr(image) || !ok_ptr(T_final) ||
      !ok_ptr(n_contrib) || (bg && !aligned16(bg)) || (n_eval && !aligned16(n_eval)))
    return GLAM_ERR_INVALID_ARG;
  return glam::launch_render_fwd(*proj, *bins, *views, bg, image, T_final, n_contrib, n_eval, stream);
}

size_t glam_loss_workspace_bytes(const glam_views* views) {
  if (!views_host_ok(views)) return 0;
  return glam::loss_workspace(*views);
}

glam_status glam_loss(const glam_views* views, const float* image, const float* target, float w_ssim, float* dimage,
                      float* loss, float* total, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!views_ok(views) || !ok_ptr(image) || !ok_ptr(target) || !ok_ptr(dimage) || !ok_ptr(loss) ||
      !ok_ptr(workspace) || !(w_ssim >= 0.f) || (total && !aligned16(total)))
    return GLAM_ERR_INVALID_ARG;
  if (workspace_bytes < glam::loss_workspace(*views)) return GLAM_ERR_WORKSPACE;
  return glam::launch_loss(*views, image, target, w_ssim, dimage, loss, total, workspace, stream);
}

glam_status glam_loss_noalloc(const glam_views* views, const float* image, const float* target, float w_ssim,
                              float* dimage, float* loss, float* total, hipStream_t stream) {
  if (!views_ok(views) || !ok_ptr(image) || !ok_ptr(target) || !ok_ptr(dimage) || !ok_ptr(loss) ||
      !(w_ssim >= 0.f) || (total && !aligned16(total)))
    return GLAM_ERR_INVALID_ARG;
  if (glam::loss_workspace(*views) > GLAM_LOSS_SCRATCH_BYTES) return GLAM_ERR_WORKSPACE;
  return glam::launch_loss_noalloc(*views, image, target, w_ssim, dimage, loss, total, stream);
}

glam_status glam_composite_bwd(const glam_projected* proj, const glam_bins* bins, const glam_views* views,
                               const float* bg, const float* T_final, const int32_t* n_contrib, const float* dimage,
                               float* g2d, hipStream_t stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !views_ok(views) || !ok_ptr(T_final) || !ok_ptr(n_contrib) ||
      !ok_ptr(dimage) || !ok_ptr(g2d) || (bg && !aligned16(bg)))
    return GLAM_ERR_INVALID_ARG;
  return glam::launch_composite_bwd(*proj, *bins, *views, bg, T_final, n_contrib, dimage, g2d, nullptr, stream);
}

size_t glam_render_fused_l1_workspace_bytes(const glam_views* views) {
  if (!views_host_ok(views)) return 0;
  const size_t a = glam::fused_l1_workspace(*views), b = glam::loss_workspace(*views);
  return a > b ? a : b;
}

glam_status glam_render_fused_l1(const glam_projected* proj, const glam_bins* bins, const glam_views* views,
                                 const float* bg, const float* target, float* image, float* T_final,
                                 int32_t* n_contrib, float* dimage, float* loss, float* total, float* g2d,
                                 void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !views_ok(views) || !ok_ptr(target) || !ok_ptr(image) ||
      !ok_ptr(T_final) || !ok_ptr(n_contrib) || !ok_ptr(dimage) || !ok_ptr(loss) || !ok_ptr(g2d) ||
      !ok_ptr(workspace) || (bg && !aligned16(bg)) || (total && !aligned16(total)))
    return GLAM_ERR_INVALID_ARG;
  if (workspace_bytes < glam_render_fused_l1_workspace_bytes(views)) return GLAM_ERR_WORKSPACE;
  return glam::launch_fused_l1(*proj, *bins, *views, bg, target, image, T_final, n_contrib, dimage, loss, total, g2d,
                               workspace, stream);
}

glam_status glam_project_bwd(const glam_gaussians* gauss, const glam_projected* proj, const glam_views* views,
                             uint32_t flags, const float* g2d, glam_gaussians* dgauss, hipStream_t stream) {
  if (!gauss_ok(gauss, true) || !proj_ok(proj) || !views_ok(views) || !ok_ptr(g2d) || !gauss_ok(dgauss, true) ||
      (flags & ~kBackwardFlags))
    return GLAM_ERR_INVALID_ARG;
  const bool plain = (flags & GLAM_PLAIN) != 0;
  if (plain) {
    if (dgauss->n != gauss->n) return GLAM_ERR_INVALID_ARG;
    for (int i = 0; i < views->n; ++i)
      if (views->host[i].g_count != gauss->n) return GLAM_ERR_INVALID_ARG;
  } else if (gauss->n != views->n_gauss || dgauss->n != views->n_gauss) {
    return GLAM_ERR_INVALID_ARG;
  }
  return glam::launch_project_bwd(*gauss, *proj, *views, plain, g2d, *dgauss, nullptr, stream);
}

size_t glam_decode_bwd_workspace_bytes(const glam_anchors* anchors, const glam_views* views, int32_t n_parts) {
  if (!anchors || !views_host_ok(views) || n_parts <= 0) return 0;
  return glam::decode_bwd_workspace(*anchors, *views, n_parts);
}

glam_status glam_decode_bwd(const glam_anchors* anchors, const float* mlp, int32_t n_parts, const glam_views* views,
                            uint32_t flags, const glam_gaussians* dgauss, float* dfeat, float* doffs,
                            float* dlog_scale, float* dmlp, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
  if (!anchors_ok(anchors) || !ok_ptr(mlp) || !views_ok(views) || !gauss_ok(dgauss, true) || !ok_ptr(dfeat) ||
      !ok_ptr(doffs) || !ok_ptr(dlog_scale) || !ok_ptr(dmlp) || !ok_ptr(workspace) || n_parts <= 0)
    return GLAM_ERR_INVALID_ARG;
  if ((flags & GLAM_PLAIN) || (flags & ~kBackwardFlags)) return GLAM_ERR_INVALID_ARG;
  if (!anchor_views_ok(anchors, views) || dgauss->n != views->n_gauss || max_partition(views) >= n_parts)
    return GLAM_ERR_INVALID_ARG;
  if (!glam::decode_supported(anchors->F, anchors->K)) return GLAM_ERR_UNSUPPORTED;
  if (workspace_bytes < glam::decode_bwd_workspace(*anchors, *views, n_parts)) return GLAM_ERR_WORKSPACE;
  return glam::launch_decode_bwd(*anchors, mlp, n_parts, *views, (flags & GLAM_OPACITY_SIGMOID) != 0, *dgauss, dfeat,
                                 doffs, dlog_scale, dmlp, workspace, stream);
}

size_t glam_render_bwd_workspace_bytes(const glam_anchors* anchors, const glam_views* views, int32_t n_parts,
                                       int64_t capacity, uint32_t flags) {
  if (!views_host_ok(views) || (flags & ~kBackwardFlags)) return 0;
  size_t n = 0;
  if (!(flags & GLAM_PLAIN)) {
    if (!anchors || n_parts <= 0) return 0;
    n = align256(glam::decode_bwd_workspace(*anchors, *views, n_parts));
  }
  if (flags & GLAM_DETERMINISTIC_GRADS) {
    if (capacity <= 0) return 0;
    n += align256(glam::det_partial_bytes(*views, capacity));
  }
  return n;
}

glam_status glam_render_bwd(const glam_projected* proj, const glam_bins* bins, const glam_views* views,
                            const float* bg, const float* T_final, const int32_t* n_contrib, const float* dimage,
                            const glam_gaussians* gauss, const glam_anchors* anchors, const float* mlp,
                            int32_t n_parts, uint32_t flags, glam_grads* grads, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
  if (!grads || (flags & ~kBackwardFlags)) return GLAM_ERR_INVALID_ARG;
  const bool plain = (flags & GLAM_PLAIN) != 0;
  const bool det = (flags & GLAM_DETERMINISTIC_GRADS) != 0;
  const bool inter = (flags & GLAM_RETURN_INTERMEDIATES) != 0;
  // validate everything before the first launch
  if (!proj_ok(proj) || !bins_ok(bins) || !views_ok(views) || !ok_ptr(T_final) || !ok_ptr(n_contrib) ||
      !ok_ptr(dimage) || !ok_ptr(grads->g2d) || !gauss_ok(gauss, true) || !gauss_ok(&grads->dgauss, true) ||
      (bg && !aligned16(bg)) || (inter && !ok_ptr(grads->d2d)) || (det && !bins->pair_begin))
    return GLAM_ERR_INVALID_ARG;
  if (plain) {
    if (grads->dgauss.n != gauss->n) return GLAM_ERR_INVALID_ARG;
    for (int i = 0; i < views->n; ++i)
      if (views->host[i].g_count != gauss->n) return GLAM_ERR_INVALID_ARG;
  } else {
    if (!anchors_ok(anchors) || !ok_ptr(mlp) || !ok_ptr(grads->dfeat) || !ok_ptr(grads->doffs) ||
        !ok_ptr(grads->dlog_scale) || !ok_ptr(grads->dmlp) || !ok_ptr(workspace) || n_parts <= 0)
      return GLAM_ERR_INVALID_ARG;
    if (!anchor_views_ok(anchors, views) || max_partition(views) >= n_parts || gauss->n != views->n_gauss ||
        grads->dgauss.n != views->n_gauss)
      return GLAM_ERR_INVALID_ARG;
    if (!glam::decode_supported(anchors->F, anchors->K)) return GLAM_ERR_UNSUPPORTED;
  }
  if (det && !glam::det_supported(*views, bins->capacity)) return GLAM_ERR_UNSUPPORTED;
  if (det && !ok_ptr(workspace)) return GLAM_ERR_INVALID_ARG;
  if (workspace_bytes < glam_render_bwd_workspace_bytes(anchors, views, n_parts, bins->capacity, flags))
    return GLAM_ERR_WORKSPACE;
  // workspace: the decode adjoint's part (anchor mode), then the reproducible partials
  char* ws = static_cast<char*>(workspace);
  const size_t dec_bytes = plain ? 0 : align256(glam::decode_bwd_workspace(*anchors, *views, n_parts));
  float* det_part = det ? reinterpret_cast<float*>(ws + dec_bytes) : nullptr;
  glam_status s = glam::launch_composite_bwd(*proj, *bins, *views, bg, T_final, n_contrib, dimage, grads->g2d,
                                             det_part, stream);
  if (s != GLAM_OK) return s;
  s = glam::launch_project_bwd(*gauss, *proj, *views, plain, grads->g2d, grads->dgauss, inter ? grads->d2d : nullptr,
                               stream);
  if (s != GLAM_OK || plain) return s;
  return glam::launch_decode_bwd(*anchors, mlp, n_parts, *views, (flags & GLAM_OPACITY_SIGMOID) != 0, grads->dgauss,
                                 grads->dfeat, grads->doffs, grads->dlog_scale, grads->dmlp, workspace, stream);
}

glam_status glam_adam_step(const glam_adam_group* groups, int32_t n_groups, int32_t step, float beta1, float beta2,
                           float eps, hipStream_t stream) {
  if (!glam::adam_groups_ok(groups, n_groups) || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return GLAM_ERR_INVALID_ARG;
  return glam::launch_adam(groups, n_groups, step, beta1, beta2, eps, stream);
}

glam_status glam_sample_keyframes(int32_t n_keyframes, int32_t k_recent, float p_recent, int32_t count,
                                  uint64_t seed, uint64_t counter, int32_t* out) {
  if (n_keyframes <= 0 || k_recent <= 0 || count < 0 || (count > 0 && !out) || !(p_recent >= 0.f && p_recent <= 1.f))
    return GLAM_ERR_INVALID_ARG;
  glam::sample_keyframes(n_keyframes, k_recent, p_recent, count, seed, counter, out);
  return GLAM_OK;
}

glam_status glam_deform_anchors(float* pos, float* offs, int32_t A, int32_t K, const glam_keyframe_fix* fixes,
                                int32_t n_fix, float near, float far, int32_t* owner, hipStream_t stream) {
  if (A < 0 || K < 0 || n_fix < 0 || !(near > 0.f) || !(far > near) || (owner && !aligned16(owner)))
    return GLAM_ERR_INVALID_ARG;
  if (A > 0 && (!ok_ptr(pos) || (K > 0 && !ok_ptr(offs)) || (n_fix > 0 && !ok_ptr(fixes))))
    return GLAM_ERR_INVALID_ARG;
  return glam::launch_deform(pos, offs, A, K, fixes, n_fix, near, far, owner, stream);
}

glam_status glam_epipolar_triangulate(const glam_camera* cam1, const glam_camera* cam2, const float* x1,
                                      const float* x2, int64_t n, float tau, float* residual, int32_t* keep,
                                      float* X, hipStream_t stream) {
  if (!cam1 || !cam2 || n < 0 || !(tau >= 0.f) || !(cam1->fx > 0.f) || !(cam1->fy > 0.f) || !(cam2->fx > 0.f) ||
      !(cam2->fy > 0.f))
    return GLAM_ERR_INVALID_ARG;
  if (n > 0 && (!ok_ptr(x1) || !ok_ptr(x2) || !ok_ptr(residual) || !ok_ptr(keep) || !ok_ptr(X)))
    return GLAM_ERR_INVALID_ARG;
  return glam::launch_epipolar(*cam1, *cam2, x1, x2, n, tau, residual, keep, X, stream);
}

size_t glam_voxelize_workspace_bytes(int64_t n_points) {
  return n_points < 0 || n_points > glam::kVoxelMaxPoints ? 0 : glam::voxelize_workspace(n_points);
}

glam_status glam_voxelize(const float* points, int64_t n_points, float eps, const uint64_t* existing,
                          int64_t n_existing, uint64_t* new_keys, float* new_centres, int64_t capacity,
                          uint64_t* merged, int64_t* counts, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
  if (n_points < 0 || n_existing < 0 || capacity < 0 || !(eps > 0.f) || !std::isfinite(eps) || !ok_ptr(counts))
    return GLAM_ERR_INVALID_ARG;
  if (n_points > glam::kVoxelMaxPoints) return GLAM_ERR_UNSUPPORTED;
  if ((n_points > 0 && !ok_ptr(points)) || (n_existing > 0 && !ok_ptr(existing)) ||
      (capacity > 0 && (!ok_ptr(new_keys) || !ok_ptr(new_centres))) || (merged && !aligned16(merged)))
    return GLAM_ERR_INVALID_ARG;
  if (!workspace || !aligned16(workspace)) return GLAM_ERR_WORKSPACE;
  if (workspace_bytes < glam::voxelize_workspace(n_points)) return GLAM_ERR_WORKSPACE;
  return glam::launch_voxelize(points, n_points, eps, existing, n_existing, new_keys, new_centres, capacity, merged,
                               counts, workspace, stream);
}

glam_status glam_insert_rows(const float* src, float* dst, int32_t rows, int64_t n_old, int32_t width, int64_t at,
                             int64_t n_new, const float* ins, int64_t ins_stride, float fill, hipStream_t stream) {
  if (rows < 0 || rows > 65535 || n_old < 0 || width < 0 || n_new < 0 || at < 0 || at > n_old)
    return GLAM_ERR_INVALID_ARG;
  if (ins && ins_stride < n_new * (long long)width) return GLAM_ERR_INVALID_ARG;
  const long long len_old = n_old * (long long)width, len_new = (n_old + n_new) * (long long)width;
  if (len_new >= (1ll << 31)) return GLAM_ERR_UNSUPPORTED;
  if (rows > 0 && len_new > 0) {
    if (!ok_ptr(dst) || (len_old > 0 && !ok_ptr(src)) || (ins && !aligned16(ins))) return GLAM_ERR_INVALID_ARG;
    // src and dst must not overlap (the copy is not ordered)
    const char *s0 = reinterpret_cast<const char*>(src), *d0 = reinterpret_cast<const char*>(dst);
    const size_t sb = 4ull * rows * len_old, db = 4ull * rows * len_new;
    if (len_old > 0 && s0 < d0 + db && d0 < s0 + sb) return GLAM_ERR_INVALID_ARG;
  }
  return glam::launch_insert_rows(src, dst, rows, n_old, width, at, n_new, ins, ins_stride, fill, stream);
}

}  // extern "C"

