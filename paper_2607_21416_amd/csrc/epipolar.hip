// Flow densification (Eq. 5): the epipolar filter of two-view correspondences and the
// triangulation of the retained ones with the known keyframe poses.
//
// The fundamental matrix follows the paper's construction from the two projection
// matrices, F = [e2]x P2 P1^+ with e2 = P2 C1, once per call on the host in double
// precision (a 3x4 pseudo-inverse, P1^T (P1 P1^T)^-1).  Per correspondence, one thread
// evaluates the algebraic residual and, for a retained pair, solves the 3x3 normal
// equations of the linear triangulation (rows u p3 - p1, v p3 - p2 of each normalised
// projection [R | t]) by Cramer's rule, both in FP64 (the chip's vector FP64 rate is half
// its FP32 rate; the work is a few hundred operations per pair, and the normal matrix of
// a short baseline is ill-conditioned in FP32).
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

struct EpiParams {
  double F[9];
  double P1[12], P2[12];  // [R | t] of each view (normalised image coordinates)
  double ifx1, ify1, cx1, cy1, ifx2, ify2, cx2, cy2;
  double tau;
};

__global__ void __launch_bounds__(256) epipolar_kernel(EpiParams e, const float* x1, const float* x2, long long n,
                                                       float* residual, int32_t* keep, float* X) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u1 = x1[i], v1 = x1[n + i], u2 = x2[i], v2 = x2[n + i];
  // x2^T F x1
  const double f0 = e.F[0] * u1 + e.F[1] * v1 + e.F[2];
  const double f1 = e.F[3] * u1 + e.F[4] * v1 + e.F[5];
  const double f2 = e.F[6] * u1 + e.F[7] * v1 + e.F[8];
  const double r = fabs(u2 * f0 + v2 * f1 + f2);
  residual[i] = (float)r;
  int ok = r < e.tau;
  double pt[3] = {NAN, NAN, NAN};
  if (ok) {
    // normalised coordinates and the four rows a_k . (X, Y, Z, 1) = 0
    const double a1 = (u1 - e.cx1) * e.ifx1, b1 = (v1 - e.cy1) * e.ify1;
    const double a2 = (u2 - e.cx2) * e.ifx2, b2 = (v2 - e.cy2) * e.ify2;
    double rows[4][4];
    for (int c = 0; c < 4; ++c) {
      rows[0][c] = a1 * e.P1[8 + c] - e.P1[c];
      rows[1][c] = b1 * e.P1[8 + c] - e.P1[4 + c];
      rows[2][c] = a2 * e.P2[8 + c] - e.P2[c];
      rows[3][c] = b2 * e.P2[8 + c] - e.P2[4 + c];
    }
    // normal equations M X = rhs, M = A3^T A3, rhs = -A3^T a4
    double M[3][3], rhs[3];
    for (int p = 0; p < 3; ++p) {
      rhs[p] = 0.0;
      for (int q = 0; q < 3; ++q) M[p][q] = 0.0;
      for (int k = 0; k < 4; ++k) {
        rhs[p] -= rows[k][p] * rows[k][3];
        for (int q = 0; q < 3; ++q) M[p][q] += rows[k][p] * rows[k][q];
      }
    }
    const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1], c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2],
                 c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    const double tr = M[0][0] + M[1][1] + M[2][2];
    if (fabs(det) > 1e-12 * tr * tr * tr) {
      const double inv = 1.0 / det;
      const double c10 = M[0][2] * M[2][1] - M[0][1] * M[2][2], c11 = M[0][0] * M[2][2] - M[0][2] * M[2][0],
                   c12 = M[0][1] * M[2][0] - M[0][0] * M[2][1];
      const double c20 = M[0][1] * M[1][2] - M[0][2] * M[1][1], c21 = M[0][2] * M[1][0] - M[0][0] * M[1][2],
                   c22 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
      // X = M^-1 rhs with M^-1 = adj(M) / det (M symmetric)
      pt[0] = (c00 * rhs[0] + c10 * rhs[1] + c20 * rhs[2]) * inv;
      pt[1] = (c01 * rhs[0] + c11 * rhs[1] + c21 * rhs[2]) * inv;
      pt[2] = (c02 * rhs[0] + c12 * rhs[1] + c22 * rhs[2]) * inv;
    } else {
      ok = 0;
    }
  }
  keep[i] = ok;
  for (int k = 0; k < 3; ++k) X[k * n + i] = (float)pt[k];
}

// P = K [R | t] as a 3x4 row-major matrix.
void projection(const glam_camera& c, double P[12]) {
  const double K[9] = {c.fx, 0.0, c.cx, 0.0, c.fy, c.cy, 0.0, 0.0, 1.0};
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 4; ++k) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += K[3 * r + m] * (k < 3 ? (double)c.R[3 * m + k] : (double)c.t[m]);
      P[4 * r + k] = acc;
    }
}

bool invert3(const double A[9], double out[9]) {
  const double c0 = A[4] * A[8] - A[5] * A[7], c1 = A[5] * A[6] - A[3] * A[8], c2 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c0 + A[1] * c1 + A[2] * c2;
  if (!(std::fabs(det) > 0.0)) return false;
  const double inv = 1.0 / det;
  out[0] = c0 * inv;
  out[1] = (A[2] * A[7] - A[1] * A[8]) * inv;
  out[2] = (A[1] * A[5] - A[2] * A[4]) * inv;
  out[3] = c1 * inv;
  out[4] = (A[0] * A[8] - A[2] * A[6]) * inv;
  out[5] = (A[2] * A[3] - A[0] * A[5]) * inv;
  out[6] = c2 * inv;
  out[7] = (A[1] * A[6] - A[0] * A[7]) * inv;
  out[8] = (A[0] * A[4] - A[1] * A[3]) * inv;
  return true;
}

}  // namespace

// F = [e2]x P2 P1^+, unit Frobenius norm, largest-magnitude entry positive.
bool fundamental_from_cameras(const glam_camera& c1, const glam_camera& c2, double F[9]) {
  double P1[12], P2[12];
  projection(c1, P1);
  projection(c2, P2);
  // camera centre C1 = -R1^T t1 (homogeneous, w = 1)
  double C1[4] = {0.0, 0.0, 0.0, 1.0};
  for (int k = 0; k < 3; ++k)
    C1[k] = -((double)c1.R[k] * c1.t[0] + (double)c1.R[3 + k] * c1.t[1] + (double)c1.R[6 + k] * c1.t[2]);
  double e2[3];
  for (int r = 0; r < 3; ++r) e2[r] = P2[4 * r] * C1[0] + P2[4 * r + 1] * C1[1] + P2[4 * r + 2] * C1[2] + P2[4 * r + 3];
  // P1^+ = P1^T (P1 P1^T)^-1 (4x3)
  double G[9], Gi[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += P1[4 * r + k] * P1[4 * c + k];
      G[3 * r + c] = acc;
    }
  if (!invert3(G, Gi)) return false;
  double Pp[12];  // 4x3
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int r = 0; r < 3; ++r) acc += P1[4 * r + k] * Gi[3 * r + c];
      Pp[3 * k + c] = acc;
    }
  double M[9];  // P2 P1^+ (3x3)
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += P2[4 * r + k] * Pp[3 * k + c];
      M[3 * r + c] = acc;
    }
  const double S[9] = {0.0, -e2[2], e2[1], e2[2], 0.0, -e2[0], -e2[1], e2[0], 0.0};
  double norm = 0.0, big = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += S[3 * r + k] * M[3 * k + c];
      F[3 * r + c] = acc;
      norm += acc * acc;
      if (std::fabs(acc) > std::fabs(big)) big = acc;
    }
  if (!(norm > 0.0)) return false;
  const double s = (big < 0.0 ? -1.0 : 1.0) / std::sqrt(norm);
  for (int k = 0; k < 9; ++k) F[k] *= s;
  return true;
}

glam_status launch_epipolar(const glam_camera& c1, const glam_camera& c2, const float* x1, const float* x2,
                            long long n, float tau, float* residual, int32_t* keep, float* X, hipStream_t s) {
  EpiParams e{};
  if (!fundamental_from_cameras(c1, c2, e.F)) return GLAM_ERR_INVALID_ARG;
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) {
      e.P1[4 * r + k] = c1.R[3 * r + k];
      e.P2[4 * r + k] = c2.R[3 * r + k];
    }
    e.P1[4 * r + 3] = c1.t[r];
    e.P2[4 * r + 3] = c2.t[r];
  }
  e.ifx1 = 1.0 / c1.fx;
  e.ify1 = 1.0 / c1.fy;
  e.cx1 = c1.cx;
  e.cy1 = c1.cy;
  e.ifx2 = 1.0 / c2.fx;
  e.ify2 = 1.0 / c2.fy;
  e.cx2 = c2.cx;
  e.cy2 = c2.cy;
  e.tau = tau;
  if (n == 0) return GLAM_OK;
  hipLaunchKernelGGL(epipolar_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, e, x1, x2, n, residual,
                     keep, X);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
