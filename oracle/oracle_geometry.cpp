// FP64 oracle, geometry half: anchor decode, plain activation, projection and their
// adjoints.  Test infrastructure only (see oracle.h).  Plain loops, no blocking or
// fusion beyond what the definitions state.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "oracle.h"

namespace {

double sigmoid(double x) { return 1.0 / (1.0 + std::exp(-x)); }

// Quaternion normalisation with a zero-norm guard: q / sqrt(|q|^2 + 1e-24).
const double kQuatEps = 1e-24;

// Offsets of one MLP inside a partition's packed parameter vector.
struct MlpView {
  int w1, b1, w2, b2, out;
};

MlpView mlp_view(int F, int K, int hidden, int which) {
  const int n_in = F + 4;
  const int outs[3] = {K, 3 * K, 7 * K};
  int off = 0;
  for (int l = 0; l < which; ++l) off += hidden * n_in + hidden + outs[l] * hidden + outs[l];
  MlpView v;
  v.w1 = off;
  v.b1 = v.w1 + hidden * n_in;
  v.w2 = v.b1 + hidden;
  v.b2 = v.w2 + outs[which] * hidden;
  v.out = outs[which];
  return v;
}

// Camera centre x_c = -R^T t.
void camera_centre(const orc_cam* c, double xc[3]) {
  for (int i = 0; i < 3; ++i)
    xc[i] = -(c->R[0 * 3 + i] * c->t[0] + c->R[1 * 3 + i] * c->t[1] + c->R[2 * 3 + i] * c->t[2]);
}

// MLP input of anchor a, Eq. 2: z = [f_a, d_ac, delta_ac] with delta_ac = |x_a - x_c|
// and d_ac = (x_a - x_c) / delta_ac.
void mlp_input(int A, int F, const double* pos, const double* feat, int a, const double xc[3],
               std::vector<double>& z) {
  z.assign(F + 4, 0.0);
  for (int k = 0; k < F; ++k) z[k] = feat[(size_t)a * F + k];
  double diff[3];
  for (int i = 0; i < 3; ++i) diff[i] = pos[(size_t)i * A + a] - xc[i];
  const double delta = std::sqrt(diff[0] * diff[0] + diff[1] * diff[1] + diff[2] * diff[2]);
  for (int i = 0; i < 3; ++i) z[F + i] = diff[i] / delta;
  z[F + 3] = delta;
}

// Two-layer ReLU MLP: pre = W1 z + b1, h = max(pre, 0), y = W2 h + b2.
// relu_in (may be null) holds the ReLU decisions fixed (unit i passes when relu_in[i]);
// relu_out (may be null) receives the decisions taken.
void mlp_forward(const double* p, const MlpView& v, int hidden, int n_in,
                 const std::vector<double>& z, std::vector<double>& pre, std::vector<double>& h,
                 std::vector<double>& y, const uint8_t* relu_in = nullptr,
                 uint8_t* relu_out = nullptr) {
  pre.assign(hidden, 0.0);
  h.assign(hidden, 0.0);
  y.assign(v.out, 0.0);
  for (int i = 0; i < hidden; ++i) {
    double s = p[v.b1 + i];
    for (int k = 0; k < n_in; ++k) s += p[v.w1 + i * n_in + k] * z[k];
    pre[i] = s;
    const bool on = relu_in ? relu_in[i] != 0 : s > 0.0;
    h[i] = on ? s : 0.0;
    if (relu_out) relu_out[i] = on ? 1 : 0;
  }
  for (int o = 0; o < v.out; ++o) {
    double s = p[v.b2 + o];
    for (int i = 0; i < hidden; ++i) s += p[v.w2 + o * hidden + i] * h[i];
    y[o] = s;
  }
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Adjoint of quat_to_rot: dL/dq from dL/dR.
void quat_to_rot_bwd(const double q[4], const double dR[9], double dq[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  // partial derivatives of each entry written out
  dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] +
               w * dR[7] - 2 * x * dR[8]);
  dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
               z * dR[7] - 2 * y * dR[8]);
  dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] +
               x * dR[6] + y * dR[7]);
}

// Everything the projection of one Gaussian computes, kept for the adjoint.
struct Proj {
  bool visible;
  double t[3];
  double xt, yt;          // clamped x/z, y/z (times z) used in the Jacobian
  bool clamp_x, clamp_y;  // whether the clamp was active
  double limx_lo, limx_hi, limy_lo, limy_hi;
  double J[6];            // 2x3
  double Rq[9];           // rotation of the Gaussian
  double Sigma[9];        // 3-D covariance
  double M[6];            // J * R_cam (2x3)
  double a, b, c;         // 2-D covariance (dilated)
  double det;
  double conic[3];
  double u, v;
  double ex, ey;
  int x0, x1, y0, y1;
};

const double kZNear = 0.2;     // cull depth
const double kDilation = 0.3;  // added to the 2-D covariance diagonal, pixels^2
const double kAlphaMin = 1.0 / 255.0;

// Projection of one Gaussian (Sec. III-A's projected 2-D Gaussian, built as in the
// EWA splatting the 3DGS lineage uses).
// clamp_in (may be null): the Jacobian clamp decision held fixed per axis, 0 free,
// 1 at the low limit, 2 at the high limit (finite-difference checks only).
// footprint: 0 the opacity-aware box (alpha >= 1/255 can only occur inside it); 1 the
// 3-D Gaussian splatting lineage's square of radius ceil(3 sqrt(lambda_max)), widened to
// whole tiles of tile_w x tile_h pixels.
void project_one(const orc_cam* cam, const double mu[3], const double s[3], const double q[4],
                 double opacity, Proj& p, const int8_t* clamp_in = nullptr, int footprint = 0,
                 int tile_w = 16, int tile_h = 16) {
  p.visible = false;
  p.x0 = 0; p.x1 = -1; p.y0 = 0; p.y1 = -1;
  p.ex = p.ey = -1.0;
  const double* R = cam->R;
  for (int i = 0; i < 3; ++i)
    p.t[i] = R[i * 3 + 0] * mu[0] + R[i * 3 + 1] * mu[1] + R[i * 3 + 2] * mu[2] + cam->t[i];
  const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
  // fill everything that does not need tz > 0 so that the adjoint never reads junk
  p.u = p.v = 0.0;
  if (!(tz > kZNear)) return;
  const double W = cam->W, H = cam->H;
  // Jacobian clamp: x/z kept within [(-cx - 0.15 W)/fx, (1.15 W - cx)/fx], likewise y.
  p.limx_lo = (-cam->cx - 0.15 * W) / cam->fx;
  p.limx_hi = (1.15 * W - cam->cx) / cam->fx;
  p.limy_lo = (-cam->cy - 0.15 * H) / cam->fy;
  p.limy_hi = (1.15 * H - cam->cy) / cam->fy;
  const double rx = tx / tz, ry = ty / tz;
  p.clamp_x = rx < p.limx_lo || rx > p.limx_hi;
  p.clamp_y = ry < p.limy_lo || ry > p.limy_hi;
  p.xt = std::min(std::max(rx, p.limx_lo), p.limx_hi) * tz;
  p.yt = std::min(std::max(ry, p.limy_lo), p.limy_hi) * tz;
  if (clamp_in) {
    p.clamp_x = clamp_in[0] != 0;
    p.clamp_y = clamp_in[1] != 0;
    p.xt = (clamp_in[0] == 1 ? p.limx_lo : clamp_in[0] == 2 ? p.limx_hi : rx) * tz;
    p.yt = (clamp_in[1] == 1 ? p.limy_lo : clamp_in[1] == 2 ? p.limy_hi : ry) * tz;
  }
  p.J[0] = cam->fx / tz; p.J[1] = 0.0; p.J[2] = -cam->fx * p.xt / (tz * tz);
  p.J[3] = 0.0; p.J[4] = cam->fy / tz; p.J[5] = -cam->fy * p.yt / (tz * tz);
  quat_to_rot(q, p.Rq);
  // Sigma = Rq diag(s^2) Rq^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += p.Rq[i * 3 + k] * s[k] * s[k] * p.Rq[j * 3 + k];
      p.Sigma[i * 3 + j] = acc;
    }
  // M = J R_cam
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += p.J[i * 3 + k] * R[k * 3 + j];
      p.M[i * 3 + j] = acc;
    }
  // Sigma2D = M Sigma M^T + dilation I
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += p.M[i * 3 + k] * p.Sigma[k * 3 + l] * p.M[j * 3 + l];
      S2[i * 2 + j] = acc;
    }
  p.a = S2[0] + kDilation;
  p.b = 0.5 * (S2[1] + S2[2]);
  p.c = S2[3] + kDilation;
  p.det = p.a * p.c - p.b * p.b;
  p.conic[0] = p.c / p.det;
  p.conic[1] = -p.b / p.det;
  p.conic[2] = p.a / p.det;
  p.u = cam->fx * tx / tz + cam->cx;
  p.v = cam->fy * ty / tz + cam->cy;
  // Opacity-aware footprint: outside |dx| <= sqrt(2 ln(255 alpha) a) (likewise y) the
  // Gaussian's alpha is below the 1/255 skip threshold, so the box is conservative.
  if (!(255.0 * opacity > 1.0)) return;
  if (footprint == 1) {
    // three standard deviations along the 2-D covariance's major axis, rounded up
    const double lmax = 0.5 * (p.a + p.c) + std::sqrt(0.25 * (p.a - p.c) * (p.a - p.c) + p.b * p.b);
    p.ex = p.ey = std::ceil(3.0 * std::sqrt(lmax));
  } else {
    const double kappa = 2.0 * std::log(255.0 * opacity);
    p.ex = std::sqrt(kappa * p.a);
    p.ey = std::sqrt(kappa * p.c);
  }
  // pixel x holds its centre at x + 0.5: include x when |x + 0.5 - u| <= ex
  double lx = std::ceil(p.u - p.ex - 0.5), hx = std::floor(p.u + p.ex - 0.5);
  double ly = std::ceil(p.v - p.ey - 0.5), hy = std::floor(p.v + p.ey - 0.5);
  lx = std::max(lx, 0.0); hx = std::min(hx, W - 1.0);
  ly = std::max(ly, 0.0); hy = std::min(hy, H - 1.0);
  if (lx > hx || ly > hy) { p.ex = p.ey = -1.0; return; }
  p.x0 = (int)lx; p.x1 = (int)hx; p.y0 = (int)ly; p.y1 = (int)hy;
  if (footprint == 1) {
    // a candidate at every pixel of the tiles the square reaches
    p.x0 = (p.x0 / tile_w) * tile_w;
    p.y0 = (p.y0 / tile_h) * tile_h;
    p.x1 = std::min((p.x1 / tile_w + 1) * tile_w - 1, cam->W - 1);
    p.y1 = std::min((p.y1 / tile_h + 1) * tile_h - 1, cam->H - 1);
  }
  p.visible = true;
}

}  // namespace

extern "C" {

int orc_mlp_param_count(int F, int K, int hidden) {
  MlpView v = mlp_view(F, K, hidden, 2);
  return v.b2 + v.out;
}

void orc_decode_ex(int A, int F, int K, int hidden, const double* pos, const double* feat,
                   const double* log_scale, const double* offs, const double* mlp,
                   const orc_cam* cam, int opacity_mode, double* mean, double* scale,
                   double* quat, double* opacity, double* rgb, const uint8_t* relu_in,
                   uint8_t* relu_out);

void orc_decode(int A, int F, int K, int hidden, const double* pos, const double* feat,
                const double* log_scale, const double* offs, const double* mlp,
                const orc_cam* cam, int opacity_mode, double* mean, double* scale,
                double* quat, double* opacity, double* rgb) {
  orc_decode_ex(A, F, K, hidden, pos, feat, log_scale, offs, mlp, cam, opacity_mode, mean, scale,
                quat, opacity, rgb, nullptr, nullptr);
}

void orc_decode_ex(int A, int F, int K, int hidden, const double* pos, const double* feat,
                   const double* log_scale, const double* offs, const double* mlp,
                   const orc_cam* cam, int opacity_mode, double* mean, double* scale,
                   double* quat, double* opacity, double* rgb, const uint8_t* relu_in,
                   uint8_t* relu_out) {
  const int n_in = F + 4;
  const size_t GK = (size_t)A * K;
  double xc[3];
  camera_centre(cam, xc);
  MlpView mv[3];
  for (int l = 0; l < 3; ++l) mv[l] = mlp_view(F, K, hidden, l);
  std::vector<double> z, pre, h, y[3];
  for (int a = 0; a < A; ++a) {
    mlp_input(A, F, pos, feat, a, xc, z);
    for (int l = 0; l < 3; ++l) {
      const size_t o = ((size_t)a * 3 + l) * hidden;
      mlp_forward(mlp, mv[l], hidden, n_in, z, pre, h, y[l], relu_in ? relu_in + o : nullptr,
                  relu_out ? relu_out + o : nullptr);
    }
    const double es = std::exp(log_scale[a]);
    for (int j = 0; j < K; ++j) {
      const size_t g = (size_t)a * K + j;
      // opacity: tanh (a non-positive value drops the Gaussian) or sigmoid
      opacity[g] = opacity_mode == ORC_OPACITY_TANH ? std::tanh(y[0][j]) : sigmoid(y[0][j]);
      for (int c = 0; c < 3; ++c) rgb[c * GK + g] = sigmoid(y[1][3 * j + c]);
      for (int k = 0; k < 3; ++k) scale[k * GK + g] = es * sigmoid(y[2][7 * j + k]);
      double qq = kQuatEps;
      for (int k = 0; k < 4; ++k) qq += y[2][7 * j + 3 + k] * y[2][7 * j + 3 + k];
      const double n = std::sqrt(qq);
      for (int k = 0; k < 4; ++k) quat[k * GK + g] = y[2][7 * j + 3 + k] / n;
      for (int i = 0; i < 3; ++i) mean[i * GK + g] = pos[(size_t)i * A + a] + es * offs[i * GK + g];
    }
  }
}

void orc_decode_bwd(int A, int F, int K, int hidden, const double* pos, const double* feat,
                    const double* log_scale, const double* offs, const double* mlp,
                    const orc_cam* cam, int opacity_mode, const double* dmean,
                    const double* dscale, const double* dquat, const double* dopacity,
                    const double* drgb, double* dfeat, double* doffs, double* dlog_scale,
                    double* dmlp) {
  const int n_in = F + 4;
  const size_t GK = (size_t)A * K;
  double xc[3];
  camera_centre(cam, xc);
  MlpView mv[3];
  for (int l = 0; l < 3; ++l) mv[l] = mlp_view(F, K, hidden, l);
  std::vector<double> z, pre[3], h[3], y[3], dy[3];
  for (int a = 0; a < A; ++a) {
    mlp_input(A, F, pos, feat, a, xc, z);
    for (int l = 0; l < 3; ++l) mlp_forward(mlp, mv[l], hidden, n_in, z, pre[l], h[l], y[l]);
    for (int l = 0; l < 3; ++l) dy[l].assign(mv[l].out, 0.0);
    const double es = std::exp(log_scale[a]);
    double ds = 0.0;
    for (int j = 0; j < K; ++j) {
      const size_t g = (size_t)a * K + j;
      // opacity
      if (opacity_mode == ORC_OPACITY_TANH) {
        const double al = std::tanh(y[0][j]);
        if (al > 0.0) dy[0][j] = dopacity[g] * (1.0 - al * al);
      } else {
        const double al = sigmoid(y[0][j]);
        dy[0][j] = dopacity[g] * al * (1.0 - al);
      }
      // colour
      for (int c = 0; c < 3; ++c) {
        const double col = sigmoid(y[1][3 * j + c]);
        dy[1][3 * j + c] = drgb[c * GK + g] * col * (1.0 - col);
      }
      // scale = e^s sigmoid(y)
      for (int k = 0; k < 3; ++k) {
        const double sg = sigmoid(y[2][7 * j + k]);
        dy[2][7 * j + k] = dscale[k * GK + g] * es * sg * (1.0 - sg);
        ds += dscale[k * GK + g] * es * sg;
      }
      // quaternion normalisation
      double qq = kQuatEps;
      for (int k = 0; k < 4; ++k) qq += y[2][7 * j + 3 + k] * y[2][7 * j + 3 + k];
      const double n = std::sqrt(qq);
      double qdq = 0.0;
      for (int k = 0; k < 4; ++k) qdq += (y[2][7 * j + 3 + k] / n) * dquat[k * GK + g];
      for (int k = 0; k < 4; ++k)
        dy[2][7 * j + 3 + k] = (dquat[k * GK + g] - (y[2][7 * j + 3 + k] / n) * qdq) / n;
      // mean = x_a + e^s o
      for (int i = 0; i < 3; ++i) {
        doffs[i * GK + g] += es * dmean[i * GK + g];
        ds += es * offs[i * GK + g] * dmean[i * GK + g];
      }
    }
    dlog_scale[a] += ds;
    // MLP adjoints
    std::vector<double> dz(n_in, 0.0);
    for (int l = 0; l < 3; ++l) {
      const MlpView& v = mv[l];
      std::vector<double> dh(hidden, 0.0);
      for (int o = 0; o < v.out; ++o) {
        dmlp[v.b2 + o] += dy[l][o];
        for (int i = 0; i < hidden; ++i) {
          dmlp[v.w2 + o * hidden + i] += dy[l][o] * h[l][i];
          dh[i] += mlp[v.w2 + o * hidden + i] * dy[l][o];
        }
      }
      for (int i = 0; i < hidden; ++i) {
        const double dp = pre[l][i] > 0.0 ? dh[i] : 0.0;  // ReLU'(0) = 0
        dmlp[v.b1 + i] += dp;
        for (int k = 0; k < n_in; ++k) {
          dmlp[v.w1 + i * n_in + k] += dp * z[k];
          dz[k] += mlp[v.w1 + i * n_in + k] * dp;
        }
      }
    }
    for (int k = 0; k < F; ++k) dfeat[(size_t)a * F + k] += dz[k];
  }
}

void orc_plain_activate(int G, const double* log_scale, const double* quat_raw,
                        const double* logit, double* scale, double* quat, double* opacity) {
  for (int g = 0; g < G; ++g) {
    for (int k = 0; k < 3; ++k) scale[(size_t)k * G + g] = std::exp(log_scale[(size_t)k * G + g]);
    double qq = kQuatEps;
    for (int k = 0; k < 4; ++k) qq += quat_raw[(size_t)k * G + g] * quat_raw[(size_t)k * G + g];
    const double n = std::sqrt(qq);
    for (int k = 0; k < 4; ++k) quat[(size_t)k * G + g] = quat_raw[(size_t)k * G + g] / n;
    opacity[g] = sigmoid(logit[g]);
  }
}

void orc_plain_activate_bwd(int G, const double* log_scale, const double* quat_raw,
                            const double* logit, const double* dscale, const double* dquat,
                            const double* dopacity, double* dlog_scale, double* dquat_raw,
                            double* dlogit) {
  for (int g = 0; g < G; ++g) {
    for (int k = 0; k < 3; ++k)
      dlog_scale[(size_t)k * G + g] =
          dscale[(size_t)k * G + g] * std::exp(log_scale[(size_t)k * G + g]);
    double qq = kQuatEps;
    for (int k = 0; k < 4; ++k) qq += quat_raw[(size_t)k * G + g] * quat_raw[(size_t)k * G + g];
    const double n = std::sqrt(qq);
    double qdq = 0.0;
    for (int k = 0; k < 4; ++k) qdq += (quat_raw[(size_t)k * G + g] / n) * dquat[(size_t)k * G + g];
    for (int k = 0; k < 4; ++k)
      dquat_raw[(size_t)k * G + g] =
          (dquat[(size_t)k * G + g] - (quat_raw[(size_t)k * G + g] / n) * qdq) / n;
    const double al = sigmoid(logit[g]);
    dlogit[g] = dopacity[g] * al * (1.0 - al);
  }
}

void orc_project_ex(int G, const double* mean, const double* scale, const double* quat,
                    const double* opacity, const orc_cam* cam, int tile_w, int tile_h,
                    double* uv, double* conic, double* cov2d, double* depth, double* ext,
                    int32_t* prect, int32_t* ntiles, const int8_t* clamp_in, int8_t* clamp_out,
                    int footprint);

void orc_project(int G, const double* mean, const double* scale, const double* quat,
                 const double* opacity, const orc_cam* cam, int tile_w, int tile_h,
                 double* uv, double* conic, double* cov2d, double* depth, double* ext,
                 int32_t* prect, int32_t* ntiles) {
  orc_project_ex(G, mean, scale, quat, opacity, cam, tile_w, tile_h, uv, conic, cov2d, depth, ext,
                 prect, ntiles, nullptr, nullptr, 0);
}

void orc_project_ex(int G, const double* mean, const double* scale, const double* quat,
                    const double* opacity, const orc_cam* cam, int tile_w, int tile_h,
                    double* uv, double* conic, double* cov2d, double* depth, double* ext,
                    int32_t* prect, int32_t* ntiles, const int8_t* clamp_in, int8_t* clamp_out,
                    int footprint) {
  for (int g = 0; g < G; ++g) {
    double mu[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) { mu[k] = mean[(size_t)k * G + g]; s[k] = scale[(size_t)k * G + g]; }
    for (int k = 0; k < 4; ++k) q[k] = quat[(size_t)k * G + g];
    Proj p;
    project_one(cam, mu, s, q, opacity[g], p, clamp_in ? clamp_in + 2 * (size_t)g : nullptr, footprint,
                tile_w, tile_h);
    if (clamp_out) {
      // which limit, if any, the Jacobian clamp took on each axis
      int8_t cx = 0, cy = 0;
      if (p.t[2] > kZNear) {
        const double rx = p.t[0] / p.t[2], ry = p.t[1] / p.t[2];
        cx = rx < p.limx_lo ? 1 : rx > p.limx_hi ? 2 : 0;
        cy = ry < p.limy_lo ? 1 : ry > p.limy_hi ? 2 : 0;
        if (clamp_in) { cx = clamp_in[2 * (size_t)g]; cy = clamp_in[2 * (size_t)g + 1]; }
      }
      clamp_out[2 * (size_t)g] = cx;
      clamp_out[2 * (size_t)g + 1] = cy;
    }
    uv[g] = p.u; uv[(size_t)G + g] = p.v;
    depth[g] = p.t[2];
    if (p.t[2] > kZNear) {
      conic[g] = p.conic[0]; conic[(size_t)G + g] = p.conic[1]; conic[2 * (size_t)G + g] = p.conic[2];
      cov2d[g] = p.a; cov2d[(size_t)G + g] = p.b; cov2d[2 * (size_t)G + g] = p.c;
    } else {
      for (int k = 0; k < 3; ++k) { conic[k * (size_t)G + g] = 0.0; cov2d[k * (size_t)G + g] = 0.0; }
    }
    ext[g] = p.ex; ext[(size_t)G + g] = p.ey;
    prect[g] = p.x0; prect[(size_t)G + g] = p.x1;
    prect[2 * (size_t)G + g] = p.y0; prect[3 * (size_t)G + g] = p.y1;
    ntiles[g] = p.visible ? (p.x1 / tile_w - p.x0 / tile_w + 1) * (p.y1 / tile_h - p.y0 / tile_h + 1) : 0;
  }
}

void orc_project_bwd(int G, const double* mean, const double* scale, const double* quat,
                     const double* opacity, const orc_cam* cam, const int32_t* ntiles,
                     const double* g2d, double* dmean, double* dscale, double* dquat,
                     double* dopacity, double* drgb) {
  const double* R = cam->R;
  for (int g = 0; g < G; ++g) {
    for (int k = 0; k < 3; ++k) { dmean[k * (size_t)G + g] = 0.0; dscale[k * (size_t)G + g] = 0.0; }
    for (int k = 0; k < 4; ++k) dquat[k * (size_t)G + g] = 0.0;
    dopacity[g] = g2d[5 * (size_t)G + g];
    for (int c = 0; c < 3; ++c) drgb[c * (size_t)G + g] = g2d[(6 + c) * (size_t)G + g];
    if (ntiles[g] == 0) continue;
    double mu[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) { mu[k] = mean[(size_t)k * G + g]; s[k] = scale[(size_t)k * G + g]; }
    for (int k = 0; k < 4; ++k) q[k] = quat[(size_t)k * G + g];
    Proj p;
    project_one(cam, mu, s, q, opacity[g], p);
    const double du = g2d[g], dv = g2d[(size_t)G + g];
    const double dA = g2d[2 * (size_t)G + g], dB = g2d[3 * (size_t)G + g], dC = g2d[4 * (size_t)G + g];
    // conic = (c, -b, a) / det
    const double a = p.a, b = p.b, c = p.c, det = p.det, d2 = det * det;
    const double da = dA * (-c * c / d2) + dB * (b * c / d2) + dC * (-b * b / d2);
    const double db = dA * (2 * b * c / d2) + dB * (-(a * c + b * b) / d2) + dC * (2 * a * b / d2);
    const double dc = dA * (-b * b / d2) + dB * (a * b / d2) + dC * (-a * a / d2);
    // symmetric gradient of Sigma2D (b appears in both off-diagonal entries)
    const double G2[4] = {da, 0.5 * db, 0.5 * db, dc};
    // dL/dSigma = M^T G2 M
    double dSig[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 2; ++k)
          for (int l = 0; l < 2; ++l) acc += p.M[k * 3 + i] * G2[k * 2 + l] * p.M[l * 3 + j];
        dSig[i * 3 + j] = acc;
      }
    // dL/dM = 2 G2 M Sigma
    double dM[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 2; ++k)
          for (int l = 0; l < 3; ++l) acc += 2.0 * G2[i * 2 + k] * p.M[k * 3 + l] * p.Sigma[l * 3 + j];
        dM[i * 3 + j] = acc;
      }
    // M = J R_cam  ->  dL/dJ = dM R_cam^T
    double dJ[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += dM[i * 3 + k] * R[j * 3 + k];
        dJ[i * 3 + j] = acc;
      }
    const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
    const double fx = cam->fx, fy = cam->fy;
    double dt[3] = {0.0, 0.0, 0.0};
    // mean2d
    dt[0] += du * fx / tz;
    dt[1] += dv * fy / tz;
    dt[2] += -du * fx * tx / (tz * tz) - dv * fy * ty / (tz * tz);
    // J00 = fx/tz, J11 = fy/tz
    dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[4] * (-fy / (tz * tz));
    // J02 = -fx xt / tz^2 with xt = clamp(tx/tz) tz
    dt[2] += dJ[2] * (2.0 * fx * p.xt / (tz * tz * tz));
    dt[2] += dJ[5] * (2.0 * fy * p.yt / (tz * tz * tz));
    const double dJ02_dxt = -fx / (tz * tz), dJ12_dyt = -fy / (tz * tz);
    if (!p.clamp_x) dt[0] += dJ[2] * dJ02_dxt;
    else dt[2] += dJ[2] * dJ02_dxt * (p.xt / tz);  // xt = L tz, dxt/dtz = L
    if (!p.clamp_y) dt[1] += dJ[5] * dJ12_dyt;
    else dt[2] += dJ[5] * dJ12_dyt * (p.yt / tz);
    // t = R mu + t_cw
    for (int k = 0; k < 3; ++k)
      dmean[k * (size_t)G + g] = R[0 * 3 + k] * dt[0] + R[1 * 3 + k] * dt[1] + R[2 * 3 + k] * dt[2];
    // Sigma = N N^T with N = Rq diag(s): dN = 2 dSig N (dSig symmetric)
    double N[9], dN[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) N[i * 3 + k] = p.Rq[i * 3 + k] * s[k];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int l = 0; l < 3; ++l) acc += (dSig[i * 3 + l] + dSig[l * 3 + i]) * N[l * 3 + k];
        dN[i * 3 + k] = acc;
      }
    double dRq[9];
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int i = 0; i < 3; ++i) acc += dN[i * 3 + k] * p.Rq[i * 3 + k];
      dscale[k * (size_t)G + g] = acc;
      for (int i = 0; i < 3; ++i) dRq[i * 3 + k] = dN[i * 3 + k] * s[k];
    }
    double dq[4];
    quat_to_rot_bwd(q, dRq, dq);
    for (int k = 0; k < 4; ++k) dquat[k * (size_t)G + g] = dq[k];
  }
}

void orc_rect_f32(int G, const float* u, const float* v, const float* ex, const float* ey,
                  int W, int H, int tile_w, int tile_h, int32_t* prect, int32_t* ntiles) {
  for (int g = 0; g < G; ++g) {
    prect[g] = 0; prect[(size_t)G + g] = -1; prect[2 * (size_t)G + g] = 0; prect[3 * (size_t)G + g] = -1;
    ntiles[g] = 0;
    if (!(ex[g] >= 0.0f) || !(ey[g] >= 0.0f)) continue;
    // volatile keeps every operation a separately rounded IEEE single op
    volatile float hx = ex[g] + 0.5f;
    volatile float lo_x = u[g] - hx;
    volatile float gx = ex[g] - 0.5f;
    volatile float hi_x = u[g] + gx;
    volatile float hy = ey[g] + 0.5f;
    volatile float lo_y = v[g] - hy;
    volatile float gy = ey[g] - 0.5f;
    volatile float hi_y = v[g] + gy;
    float lx = std::max(std::ceil((float)lo_x), 0.0f), hx2 = std::min(std::floor((float)hi_x), (float)(W - 1));
    float ly = std::max(std::ceil((float)lo_y), 0.0f), hy2 = std::min(std::floor((float)hi_y), (float)(H - 1));
    if (lx > hx2 || ly > hy2) continue;
    const int x0 = (int)lx, x1 = (int)hx2, y0 = (int)ly, y1 = (int)hy2;
    prect[g] = x0; prect[(size_t)G + g] = x1; prect[2 * (size_t)G + g] = y0; prect[3 * (size_t)G + g] = y1;
    ntiles[g] = (x1 / tile_w - x0 / tile_w + 1) * (y1 / tile_h - y0 / tile_h + 1);
  }
}

}  // extern "C"
