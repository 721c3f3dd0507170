// The forward projection of one 3-D Gaussian to its 2-D splat (shared by the projection
// kernel and the decode kernel's fused output stage, so both compute identical bits).
#pragma once

#include "common.hpp"

namespace glam {

// Everything the projection computes for one Gaussian, kept for the adjoint.
struct ProjState {
  float t[3];
  float xt, yt;
  bool clamp_x, clamp_y;
  float J00, J02, J11, J12;
  float Rq[9];
  float Sig[6];   // xx, xy, xz, yy, yz, zz
  float M[6];     // J R_cam, 2x3
  float a, b, c;  // dilated 2-D covariance
  float inv_det;
  float conic[3];
  float u, v;
};

__device__ __forceinline__ void quat_rot(const float q[4], float R[9]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// a . b + c, as accurate as if computed in twice the working precision and rounded once:
// the compensated dot product (Dot2, Ogita, Rump and Oishi, "Accurate sum and dot
// product", SIAM J. Sci. Comput. 26(6), 2005) carries the exact error of every product
// (by an FMA) and of every sum (by the two-sum identity) and adds them at the end.  A
// camera-frame coordinate is the small difference of world-frame terms: kilometres along
// a path, the plain FP32 evaluation loses about five digits of it; this one loses none.
__device__ __forceinline__ float dot3_add(float a0, float a1, float a2, float b0, float b1, float b2, float c) {
#pragma clang fp contract(off)
  const float a[3] = {a0, a1, a2}, b[3] = {b0, b1, b2};
  float s = c, e = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float p = a[k] * b[k];
    const float pe = fmaf(a[k], b[k], -p);  // a b = p + pe exactly
    const float x = s + p;
    const float z = x - s;
    const float se = (s - (x - z)) + (p - z);  // s + p = x + se exactly
    s = x;
    e += pe + se;
  }
  return s + e;
}

// Returns false when the Gaussian is behind the near plane (nothing else is valid then).
__device__ __forceinline__ bool project_state(const glam_camera& cam, const float mu[3],
                                              const float s[3], const float q[4], ProjState& p) {
  const float* R = cam.R;
  for (int i = 0; i < 3; ++i) p.t[i] = dot3_add(R[3 * i], R[3 * i + 1], R[3 * i + 2], mu[0], mu[1], mu[2], cam.t[i]);
  const float tx = p.t[0], ty = p.t[1], tz = p.t[2];
  if (!(tz > kZNear)) return false;
  const float W = (float)cam.width, H = (float)cam.height;
  const float lxl = (-cam.cx - 0.15f * W) / cam.fx, lxh = (1.15f * W - cam.cx) / cam.fx;
  const float lyl = (-cam.cy - 0.15f * H) / cam.fy, lyh = (1.15f * H - cam.cy) / cam.fy;
  const float iz = 1.0f / tz;
  const float rx = tx * iz, ry = ty * iz;
  p.clamp_x = rx < lxl || rx > lxh;
  p.clamp_y = ry < lyl || ry > lyh;
  p.xt = fminf(fmaxf(rx, lxl), lxh) * tz;
  p.yt = fminf(fmaxf(ry, lyl), lyh) * tz;
  p.J00 = cam.fx * iz;
  p.J11 = cam.fy * iz;
  p.J02 = -cam.fx * p.xt * iz * iz;
  p.J12 = -cam.fy * p.yt * iz * iz;
  quat_rot(q, p.Rq);
  const float s0 = s[0] * s[0], s1 = s[1] * s[1], s2 = s[2] * s[2];
  const float* Q = p.Rq;
  p.Sig[0] = Q[0] * Q[0] * s0 + Q[1] * Q[1] * s1 + Q[2] * Q[2] * s2;
  p.Sig[1] = Q[0] * Q[3] * s0 + Q[1] * Q[4] * s1 + Q[2] * Q[5] * s2;
  p.Sig[2] = Q[0] * Q[6] * s0 + Q[1] * Q[7] * s1 + Q[2] * Q[8] * s2;
  p.Sig[3] = Q[3] * Q[3] * s0 + Q[4] * Q[4] * s1 + Q[5] * Q[5] * s2;
  p.Sig[4] = Q[3] * Q[6] * s0 + Q[4] * Q[7] * s1 + Q[5] * Q[8] * s2;
  p.Sig[5] = Q[6] * Q[6] * s0 + Q[7] * Q[7] * s1 + Q[8] * Q[8] * s2;
  // M = J R_cam
  for (int j = 0; j < 3; ++j) {
    p.M[j] = p.J00 * R[j] + p.J02 * R[6 + j];
    p.M[3 + j] = p.J11 * R[3 + j] + p.J12 * R[6 + j];
  }
  // T = M Sigma, Sigma2D = T M^T
  const float S[9] = {p.Sig[0], p.Sig[1], p.Sig[2], p.Sig[1], p.Sig[3], p.Sig[4], p.Sig[2], p.Sig[4], p.Sig[5]};
  float T0[3], T1[3];
  for (int j = 0; j < 3; ++j) {
    T0[j] = p.M[0] * S[j] + p.M[1] * S[3 + j] + p.M[2] * S[6 + j];
    T1[j] = p.M[3] * S[j] + p.M[4] * S[3 + j] + p.M[5] * S[6 + j];
  }
  p.a = T0[0] * p.M[0] + T0[1] * p.M[1] + T0[2] * p.M[2] + kDilation;
  p.b = T0[0] * p.M[3] + T0[1] * p.M[4] + T0[2] * p.M[5];
  p.c = T1[0] * p.M[3] + T1[1] * p.M[4] + T1[2] * p.M[5] + kDilation;
  const float det = p.a * p.c - p.b * p.b;
  p.inv_det = 1.0f / det;
  p.conic[0] = p.c * p.inv_det;
  p.conic[1] = -p.b * p.inv_det;
  p.conic[2] = p.a * p.inv_det;
  p.u = fmaf(cam.fx, tx * iz, cam.cx);
  p.v = fmaf(cam.fy, ty * iz, cam.cy);
  return true;
}

// Writes view-Gaussian i's projection: centre, depth, conic, footprint extents, tile
// count for tiles of edge 2^tl, and the packed render record.  Culls depth <= 0.2 and
// opacity <= 1/255.  Default footprint: the box holds every pixel whose alpha can reach
// 1/255.  sigma3 (the 3-D Gaussian splatting lineage's footprint): the pixel centres
// within r = ceil(3 sqrt(lambda_max)) of the centre on each axis select the tiles, and
// the record's box is widened to those tiles' pixels, so the Gaussian is a candidate at
// every pixel of its tiles; ext then holds r on both axes.
__device__ __forceinline__ void project_one(const glam_camera& cam, const float mu[3], const float s[3],
                                            const float q[4], float op, const float rgb[3], long long i,
                                            long long n, int tl, bool sigma3, const glam_projected& out) {
  ProjState p;
  bool vis = project_state(cam, mu, s, q, p);
  float ex = -1.f, ey = -1.f;
  int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
  if (vis && 255.f * op > 1.f) {
    if (sigma3) {
      // larger eigenvalue of [[a, b], [b, c]]
      const float hd = 0.5f * (p.a - p.c);
      const float lmax = 0.5f * (p.a + p.c) + sqrtf(hd * hd + p.b * p.b);
      ex = ey = ceilf(3.f * sqrtf(lmax));
    } else {
      const float kappa = 2.f * logf(255.f * op);
      ex = sqrtf(kappa * p.a);
      ey = sqrtf(kappa * p.c);
    }
    // pixel x is inside when |x + 0.5 - u| <= ex; each bound is two IEEE single adds
    const float lx = fmaxf(ceilf(p.u - (ex + 0.5f)), 0.f);
    const float hx = fminf(floorf(p.u + (ex - 0.5f)), (float)(cam.width - 1));
    const float ly = fmaxf(ceilf(p.v - (ey + 0.5f)), 0.f);
    const float hy = fminf(floorf(p.v + (ey - 0.5f)), (float)(cam.height - 1));
    if (lx <= hx && ly <= hy) {
      x0 = (int)lx; x1 = (int)hx; y0 = (int)ly; y1 = (int)hy;
    } else {
      vis = false;
    }
  } else {
    vis = false;
  }
  out.uv[i] = p.u;
  out.uv[n + i] = p.v;
  out.depth[i] = p.t[2];
  if (!vis) { ex = -1.f; ey = -1.f; }
  out.ext[i] = ex;
  out.ext[n + i] = ey;
  if (vis) {
    out.conic[i] = p.conic[0];
    out.conic[n + i] = p.conic[1];
    out.conic[2 * n + i] = p.conic[2];
  } else {
    out.conic[i] = 0.f; out.conic[n + i] = 0.f; out.conic[2 * n + i] = 0.f;
  }
  // tiles of edge 2^tl touched by the pixel box
  out.ntiles[i] = vis ? ((x1 >> tl) - (x0 >> tl) + 1) * ((y1 >> tl) - (y0 >> tl) + 1) : 0;
  float4* rec = reinterpret_cast<float4*>(out.splat + i * kSplatWords);
  if (vis) {
    if (sigma3) {  // every pixel of the touched tiles
      x0 = (x0 >> tl) << tl;
      y0 = (y0 >> tl) << tl;
      x1 = min((((x1 >> tl) + 1) << tl) - 1, cam.width - 1);
      y1 = min((((y1 >> tl) + 1) << tl) - 1, cam.height - 1);
    }
    const uint32_t bx = (uint32_t)x0 | ((uint32_t)x1 << 16);
    const uint32_t by = (uint32_t)y0 | ((uint32_t)y1 << 16);
    // the conic as a base-2 exponent: -log2(e) (A/2, B, C/2)
    constexpr float kLog2e = 1.4426950408889634f;
    rec[0] = make_float4(p.u, p.v, -0.5f * kLog2e * p.conic[0], -kLog2e * p.conic[1]);
    rec[1] = make_float4(-0.5f * kLog2e * p.conic[2], op, rgb[0], rgb[1]);
    rec[2] = make_float4(rgb[2], __uint_as_float(bx), __uint_as_float(by), p.t[2]);
  }
}

}  // namespace glam
