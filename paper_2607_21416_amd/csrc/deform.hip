// Loop-closure deformation of the anchor grid (Eq. 7): every corrected keyframe moves
// the anchors of its old view frustum rigidly with its pose correction, so that they
// keep their coordinates in its camera frame; an anchor seen by several corrected
// keyframes follows the nearest of them.
//
// One thread per anchor walks the corrections (the table is read by every thread of a
// wave at the same address, so its loads are broadcast), keeps the nearest keyframe
// whose frustum holds the anchor, then applies that keyframe's rigid correction to the
// position and rotates the anchor's offsets.  Bound by the corrections walked per
// anchor (a few dozen FMAs each); positions and offsets are read and written once.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

__global__ void __launch_bounds__(256) deform_kernel(float* pos, float* offs, int A, int K,
                                                     const glam_keyframe_fix* fixes, int n_fix, float near,
                                                     float far, int32_t* owner) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A) return;
  const float x[3] = {pos[a], pos[(size_t)A + a], pos[2 * (size_t)A + a]};
  int best = -1;
  float best_d2 = 0.f;
  for (int i = 0; i < n_fix; ++i) {
    const glam_camera& c = fixes[i].before;
    float y[3];
    for (int r = 0; r < 3; ++r) y[r] = fmaf(c.R[3 * r], x[0], fmaf(c.R[3 * r + 1], x[1], fmaf(c.R[3 * r + 2], x[2], c.t[r])));
    if (!(y[2] >= near && y[2] <= far)) continue;
    const float u = fmaf(c.fx, y[0] / y[2], c.cx), v = fmaf(c.fy, y[1] / y[2], c.cy);
    if (!(u >= 0.f && u < (float)c.width && v >= 0.f && v < (float)c.height)) continue;
    // distance to the old camera centre = length of the camera-frame coordinates
    const float d2 = fmaf(y[0], y[0], fmaf(y[1], y[1], y[2] * y[2]));
    if (best < 0 || d2 < best_d2) {
      best = i;
      best_d2 = d2;
    }
  }
  if (owner) owner[a] = best;
  if (best < 0) return;
  // dT = T_new^-1 T_old: R_d = R_new^T R_old, t_d = R_new^T (t_old - t_new)
  const glam_keyframe_fix& f = fixes[best];
  float Rd[9], td[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      Rd[3 * r + c] = fmaf(f.R_new[r], f.before.R[c], fmaf(f.R_new[3 + r], f.before.R[3 + c], f.R_new[6 + r] * f.before.R[6 + c]));
    td[r] = fmaf(f.R_new[r], f.before.t[0] - f.t_new[0],
                 fmaf(f.R_new[3 + r], f.before.t[1] - f.t_new[1], f.R_new[6 + r] * (f.before.t[2] - f.t_new[2])));
  }
  for (int r = 0; r < 3; ++r)
    pos[(size_t)r * A + a] = fmaf(Rd[3 * r], x[0], fmaf(Rd[3 * r + 1], x[1], fmaf(Rd[3 * r + 2], x[2], td[r])));
  const size_t AK = (size_t)A * K;
  for (int j = 0; j < K; ++j) {
    const size_t o = (size_t)a * K + j;
    const float ov[3] = {offs[o], offs[AK + o], offs[2 * AK + o]};
    for (int r = 0; r < 3; ++r) offs[r * AK + o] = fmaf(Rd[3 * r], ov[0], fmaf(Rd[3 * r + 1], ov[1], Rd[3 * r + 2] * ov[2]));
  }
}

}  // namespace

glam_status launch_deform(float* pos, float* offs, int A, int K, const glam_keyframe_fix* fixes, int n_fix,
                          float near, float far, int32_t* owner, hipStream_t s) {
  if (A == 0) return GLAM_OK;
  hipLaunchKernelGGL(deform_kernel, dim3((unsigned)((A + 255) / 256)), dim3(256), 0, s, pos, offs, A, K, fixes,
                     n_fix, near, far, owner);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
