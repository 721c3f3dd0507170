// Projection of 3-D Gaussians to 2-D splats with an opacity-aware footprint box, and
// its adjoint.  One thread per view-Gaussian, structure-of-arrays loads and stores
// (consecutive lanes touch consecutive addresses of every row).
#include "common.hpp"
#include "kernels.hpp"
#include "projection.hpp"

namespace glam {

// Gathers one Gaussian's activated parameters.  Plain mode applies the activations
// (scale = exp(log-scale), q = q / sqrt(|q|^2 + 1e-24), opacity = sigmoid(logit)).
struct GaussIn {
  float mu[3], s[3], q[4], op, rgb[3];
};

__device__ __forceinline__ void load_gauss(const glam_gaussians& g, long long i, bool plain,
                                           GaussIn& o) {
  const long long n = g.n;
  for (int k = 0; k < 3; ++k) o.mu[k] = g.mean[k * n + i];
  for (int k = 0; k < 3; ++k) o.s[k] = g.scale[k * n + i];
  for (int k = 0; k < 4; ++k) o.q[k] = g.quat[k * n + i];
  o.op = g.opacity[i];
  for (int k = 0; k < 3; ++k) o.rgb[k] = g.rgb[k * n + i];
  if (plain) {
    for (int k = 0; k < 3; ++k) o.s[k] = expf(o.s[k]);
    const float inv = rsqrtf(o.q[0] * o.q[0] + o.q[1] * o.q[1] + o.q[2] * o.q[2] + o.q[3] * o.q[3] + 1e-24f);
    for (int k = 0; k < 4; ++k) o.q[k] *= inv;
    o.op = sigmoid(o.op);
  }
}

__global__ void __launch_bounds__(256) project_kernel(glam_gaussians gauss, const glam_view_info* views,
                                                      int n_views, long long n_total, int plain, int tl,
                                                      int sigma3, glam_projected out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_total) return;
  const int vi = find_view(views, n_views, i, [](const glam_view_info& v) { return v.g_begin; });
  const glam_view_info& vw = views[vi];
  const glam_camera cam = vw.cam;
  const long long src = plain ? i - vw.g_begin : i;
  GaussIn g;
  load_gauss(gauss, src, plain != 0, g);
  project_one(cam, g.mu, g.s, g.q, g.op, g.rgb, i, n_total, tl, sigma3 != 0, out);
}

// Adjoint of the projection for one view-Gaussian.  g2d[n][9] holds, summed over the
// pixels, the moments m = (p dx, p dy, p dx^2, p dx dy, p dy^2) of p = dL/dpower with
// (dx, dy) = (u, v) - pixel centre, then d(opacity, r, g, b).  Since
// power = -(A dx^2 + C dy^2)/2 - B dx dy, the centre and conic gradients are
// du = -(A m0 + B m1), dv = -(B m0 + C m1), dA = -m2/2, dB = -m3, dC = -m4/2.
// Writes d(mean, scale, quat) of the activated parameters into d*.
__device__ __forceinline__ void project_adjoint(const glam_camera& cam, const GaussIn& g,
                                                const ProjState& p, const float* gi,
                                                float dmu[3], float ds[3], float dq[4]) {
  const float cA = p.conic[0], cB = p.conic[1], cC = p.conic[2];
  const float du = -(cA * gi[0] + cB * gi[1]), dv = -(cB * gi[0] + cC * gi[1]);
  const float dA = -0.5f * gi[2], dB = -gi[3], dC = -0.5f * gi[4];
  const float a = p.a, b = p.b, c = p.c, id2 = p.inv_det * p.inv_det;
  const float da = (dA * (-c * c) + dB * (b * c) + dC * (-b * b)) * id2;
  const float db = (dA * (2.f * b * c) - dB * (a * c + b * b) + dC * (2.f * a * b)) * id2;
  const float dc = (dA * (-b * b) + dB * (a * b) + dC * (-a * a)) * id2;
  const float G00 = da, G01 = 0.5f * db, G11 = dc;
  const float* M = p.M;
  // dSigma = M^T G M (symmetric 3x3)
  float GM0[3], GM1[3];  // rows of G M
  for (int j = 0; j < 3; ++j) {
    GM0[j] = G00 * M[j] + G01 * M[3 + j];
    GM1[j] = G01 * M[j] + G11 * M[3 + j];
  }
  float dS[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) dS[3 * i + j] = M[i] * GM0[j] + M[3 + i] * GM1[j];
  // dM = 2 G M Sigma
  const float S[9] = {p.Sig[0], p.Sig[1], p.Sig[2], p.Sig[1], p.Sig[3], p.Sig[4], p.Sig[2], p.Sig[4], p.Sig[5]};
  float dM[6];
  for (int j = 0; j < 3; ++j) {
    dM[j] = 2.f * (GM0[0] * S[j] + GM0[1] * S[3 + j] + GM0[2] * S[6 + j]);
    dM[3 + j] = 2.f * (GM1[0] * S[j] + GM1[1] * S[3 + j] + GM1[2] * S[6 + j]);
  }
  const float* R = cam.R;
  // M = J R  ->  dJ = dM R^T (only the nonzero entries of J matter)
  const float dJ00 = dM[0] * R[0] + dM[1] * R[1] + dM[2] * R[2];
  const float dJ02 = dM[0] * R[6] + dM[1] * R[7] + dM[2] * R[8];
  const float dJ11 = dM[3] * R[3] + dM[4] * R[4] + dM[5] * R[5];
  const float dJ12 = dM[3] * R[6] + dM[4] * R[7] + dM[5] * R[8];
  const float tx = p.t[0], ty = p.t[1], tz = p.t[2];
  const float iz = 1.f / tz, iz2 = iz * iz, iz3 = iz2 * iz;
  const float fx = cam.fx, fy = cam.fy;
  float dt0 = du * fx * iz;
  float dt1 = dv * fy * iz;
  float dt2 = -(du * fx * tx + dv * fy * ty) * iz2;
  dt2 += -(dJ00 * fx + dJ11 * fy) * iz2;
  dt2 += 2.f * (dJ02 * fx * p.xt + dJ12 * fy * p.yt) * iz3;
  const float gx = dJ02 * (-fx * iz2), gy = dJ12 * (-fy * iz2);
  if (!p.clamp_x) dt0 += gx; else dt2 += gx * (p.xt * iz);
  if (!p.clamp_y) dt1 += gy; else dt2 += gy * (p.yt * iz);
  for (int k = 0; k < 3; ++k) dmu[k] = R[k] * dt0 + R[3 + k] * dt1 + R[6 + k] * dt2;
  // Sigma = N N^T, N = Rq diag(s): dN = 2 dS N
  const float* Q = p.Rq;
  float dRq[9];
  for (int k = 0; k < 3; ++k) {
    float acc = 0.f;
    for (int i = 0; i < 3; ++i) {
      const float dN = 2.f * (dS[3 * i + 0] * Q[0 + k] * g.s[k] + dS[3 * i + 1] * Q[3 + k] * g.s[k] +
                              dS[3 * i + 2] * Q[6 + k] * g.s[k]);
      acc += dN * Q[3 * i + k];
      dRq[3 * i + k] = dN * g.s[k];
    }
    ds[k] = acc;
  }
  const float w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
  const float* d = dRq;
  dq[0] = 2.f * (-z * d[1] + y * d[2] + z * d[3] - x * d[5] - y * d[6] + x * d[7]);
  dq[1] = 2.f * (y * d[1] + z * d[2] + y * d[3] - 2.f * x * d[4] - w * d[5] + z * d[6] + w * d[7] - 2.f * x * d[8]);
  dq[2] = 2.f * (-2.f * y * d[0] + x * d[1] + w * d[2] + x * d[3] + z * d[5] - w * d[6] + z * d[7] - 2.f * y * d[8]);
  dq[3] = 2.f * (-2.f * z * d[0] - w * d[1] + x * d[2] + w * d[3] - 2.f * z * d[4] + y * d[5] + x * d[6] + y * d[7]);
}

// Anchor mode: one thread per view-Gaussian.
// The 2-D gradients d(u, v, A, B, C, opacity, r, g, b) of view-Gaussian i, [9][n], from
// its moments and conic (zero where culled: no moments, zero conic).
__device__ __forceinline__ void write_d2d(const glam_projected& proj, long long i, long long n, const float gi[9],
                                          float* d2d) {
  const float cA = proj.conic[i], cB = proj.conic[n + i], cC = proj.conic[2 * n + i];
  d2d[i] = -(cA * gi[0] + cB * gi[1]);
  d2d[n + i] = -(cB * gi[0] + cC * gi[1]);
  d2d[2 * n + i] = -0.5f * gi[2];
  d2d[3 * n + i] = -gi[3];
  d2d[4 * n + i] = -0.5f * gi[4];
  for (int k = 5; k < 9; ++k) d2d[k * n + i] = gi[k];
}

__global__ void __launch_bounds__(256) project_bwd_kernel(glam_gaussians gauss, const glam_projected proj,
                                                          const glam_view_info* views, int n_views,
                                                          long long n_total, const float* g2d,
                                                          glam_gaussians dg, float* d2d) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_total) return;
  const long long n = n_total;
  float gi[9];
  for (int k = 0; k < 9; ++k) gi[k] = g2d[i * 9 + k];
  if (d2d) write_d2d(proj, i, n, gi, d2d);
  float dmu[3] = {0.f, 0.f, 0.f}, ds[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f};
  if (proj.ntiles[i] > 0) {
    const int vi = find_view(views, n_views, i, [](const glam_view_info& v) { return v.g_begin; });
    const glam_camera cam = views[vi].cam;
    GaussIn g;
    load_gauss(gauss, i, false, g);
    ProjState p;
    project_state(cam, g.mu, g.s, g.q, p);
    project_adjoint(cam, g, p, gi, dmu, ds, dq);
  }
  for (int k = 0; k < 3; ++k) dg.mean[k * n + i] = dmu[k];
  for (int k = 0; k < 3; ++k) dg.scale[k * n + i] = ds[k];
  for (int k = 0; k < 4; ++k) dg.quat[k * n + i] = dq[k];
  dg.opacity[i] = gi[5];
  for (int k = 0; k < 3; ++k) dg.rgb[k * n + i] = gi[6 + k];
}

// Plain mode: one thread per Gaussian, summing its views in order, then the adjoint of
// the activations (exp, quaternion normalisation, sigmoid).
__global__ void __launch_bounds__(256) project_bwd_plain_kernel(glam_gaussians gauss, const glam_projected proj,
                                                                const glam_view_info* views, int n_views,
                                                                long long G, long long n_total,
                                                                const float* g2d, glam_gaussians dg,
                                                                float* d2d) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  GaussIn gin;
  load_gauss(gauss, g, true, gin);
  float dmu[3] = {0.f, 0.f, 0.f}, ds[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f};
  float dop = 0.f, drgb[3] = {0.f, 0.f, 0.f};
  for (int v = 0; v < n_views; ++v) {
    const long long i = views[v].g_begin + g;
    float gi[9];
    for (int k = 0; k < 9; ++k) gi[k] = g2d[i * 9 + k];
    if (d2d) write_d2d(proj, i, n_total, gi, d2d);
    dop += gi[5];
    for (int k = 0; k < 3; ++k) drgb[k] += gi[6 + k];
    if (proj.ntiles[i] == 0) continue;
    ProjState p;
    project_state(views[v].cam, gin.mu, gin.s, gin.q, p);
    float a[3], b[3], c[4];
    project_adjoint(views[v].cam, gin, p, gi, a, b, c);
    for (int k = 0; k < 3; ++k) { dmu[k] += a[k]; ds[k] += b[k]; }
    for (int k = 0; k < 4; ++k) dq[k] += c[k];
  }
  const long long n = G;
  // log-scale: d/dl exp(l) = exp(l)
  for (int k = 0; k < 3; ++k) dg.scale[k * n + g] = ds[k] * gin.s[k];
  // raw quaternion: (dq - q (q . dq)) / norm
  const float qr[4] = {gauss.quat[g], gauss.quat[n + g], gauss.quat[2 * n + g], gauss.quat[3 * n + g]};
  const float nrm = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3] + 1e-24f);
  const float qd = gin.q[0] * dq[0] + gin.q[1] * dq[1] + gin.q[2] * dq[2] + gin.q[3] * dq[3];
  for (int k = 0; k < 4; ++k) dg.quat[k * n + g] = (dq[k] - gin.q[k] * qd) / nrm;
  for (int k = 0; k < 3; ++k) dg.mean[k * n + g] = dmu[k];
  dg.opacity[g] = dop * gin.op * (1.f - gin.op);
  for (int k = 0; k < 3; ++k) dg.rgb[k * n + g] = drgb[k];
}

glam_status launch_project(const glam_gaussians& g, const glam_views& v, bool plain, bool sigma3,
                           const glam_projected& out, hipStream_t s) {
  const long long n = v.n_gauss;
  if (n == 0) return GLAM_OK;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(256), 0, s, g, v.dev, v.n, n, plain ? 1 : 0,
                     tile_log2(v.tile_w), sigma3 ? 1 : 0, out);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

glam_status launch_project_bwd(const glam_gaussians& g, const glam_projected& proj, const glam_views& v,
                               bool plain, const float* g2d, const glam_gaussians& dg, float* d2d, hipStream_t s) {
  if (plain) {
    const long long G = g.n;
    if (G == 0) return GLAM_OK;
    hipLaunchKernelGGL(project_bwd_plain_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, g, proj,
                       v.dev, v.n, G, (long long)v.n_gauss, g2d, dg, d2d);
  } else {
    const long long n = v.n_gauss;
    if (n == 0) return GLAM_OK;
    hipLaunchKernelGGL(project_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, proj, v.dev,
                       v.n, n, g2d, dg, d2d);
  }
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
