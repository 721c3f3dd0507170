// Photometric loss of Eq. 3 per view: L = mean |C - target| + w (1 - mean SSIM), SSIM
// with an 11x11 box window and zero padding, and dL/dC.
//
// Two stencil passes over 16x16 tiles, each staging a 26x26 halo in LDS and summing
// the window separably (rows, then columns):
//   A: window means of x, y, x^2, y^2, xy -> SSIM map value and its partials with
//      respect to mean(x), E[x^2], E[xy] (three maps per channel), per-tile sums;
//   B: window sums of those partials (the adjoint of the window mean is the same
//      box) combined with the L1 sign into dL/dC.
// A last kernel reduces the per-tile sums of each view in double precision.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kR = 5, kWin = 2 * kR + 1, kHalo = kTile + 2 * kR;  // 26
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct LossGeom {
  int view, W, H, x0, y0;
  long long pix_begin, tile_local;
};

__device__ __forceinline__ LossGeom loss_geom(const glam_view_info* views, int n_views, int tile) {
  LossGeom g;
  g.view = find_view(views, n_views, tile, [](const glam_view_info& v) { return (long long)v.tile_begin; });
  const glam_view_info& vw = views[g.view];
  const int lt = tile - vw.tile_begin;
  g.W = vw.cam.width;
  g.H = vw.cam.height;
  g.x0 = (lt % vw.tiles_x) * kTile;
  g.y0 = (lt / vw.tiles_x) * kTile;
  g.pix_begin = vw.pix_begin;
  g.tile_local = lt;
  return g;
}

// Loads a 26x26 halo of one plane (zero outside the image) into s.
__device__ __forceinline__ void load_halo(const float* plane, const LossGeom& g, float (*s)[kHalo]) {
  for (int k = threadIdx.x; k < kHalo * kHalo; k += 256) {
    const int hy = k / kHalo, hx = k % kHalo;
    const int x = g.x0 - kR + hx, y = g.y0 - kR + hy;
    s[hy][hx] = (x >= 0 && x < g.W && y >= 0 && y < g.H) ? plane[(long long)y * g.W + x] : 0.f;
  }
}

__global__ void __launch_bounds__(256) ssim_fwd_kernel(const glam_view_info* views, int n_views, const float* image,
                                                       const float* target, float w_ssim, float* maps,
                                                       long long n_pix, float* partial) {
  __shared__ float s_x[kHalo][kHalo], s_y[kHalo][kHalo];
  __shared__ float s_h[5][kHalo][kTile];
  __shared__ float s_red[2][256];
  const LossGeom g = loss_geom(views, n_views, blockIdx.x);
  const int t = threadIdx.x, lx = t & 15, ly = t >> 4;
  const int x = g.x0 + lx, y = g.y0 + ly;
  const bool inside = x < g.W && y < g.H;
  const long long HW = (long long)g.W * g.H;
  const long long p = (long long)y * g.W + x;
  float l1 = 0.f, ssum = 0.f;
  for (int c = 0; c < 3; ++c) {
    const float* xp = image + 3 * g.pix_begin + c * HW;
    const float* yp = target + 3 * g.pix_begin + c * HW;
    if (inside) l1 += fabsf(xp[p] - yp[p]);
    if (w_ssim == 0.f) continue;
    __syncthreads();
    load_halo(xp, g, s_x);
    load_halo(yp, g, s_y);
    __syncthreads();
    for (int k = t; k < kHalo * kTile; k += 256) {
      const int hy = k / kTile, cx = k % kTile;
      float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
      for (int o = 0; o < kWin; ++o) {
        const float u = s_x[hy][cx + o], v = s_y[hy][cx + o];
        a += u; b += v; aa += u * u; bb += v * v; ab += u * v;
      }
      s_h[0][hy][cx] = a; s_h[1][hy][cx] = b; s_h[2][hy][cx] = aa; s_h[3][hy][cx] = bb; s_h[4][hy][cx] = ab;
    }
    __syncthreads();
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int o = 0; o < kWin; ++o)
      for (int q = 0; q < 5; ++q) m[q] += s_h[q][ly + o][lx];
    if (inside) {
      const float inv = 1.f / 121.f;
      const float mx = m[0] * inv, my = m[1] * inv;
      const float vx = m[2] * inv - mx * mx, vy = m[3] * inv - my * my, cxy = m[4] * inv - mx * my;
      const float n1 = 2.f * mx * my + kC1, n2 = 2.f * cxy + kC2;
      const float d1 = mx * mx + my * my + kC1, d2 = vx + vy + kC2;
      const float id = 1.f / (d1 * d2);
      const float sv = n1 * n2 * id;
      ssum += sv;
      float* mp = maps + (long long)c * 3 * n_pix + g.pix_begin;
      mp[p] = (2.f * my * n2 - 2.f * my * n1) * id - sv * (2.f * mx * d2 - 2.f * mx * d1) * id;
      mp[n_pix + p] = -sv / d2;
      mp[2 * n_pix + p] = 2.f * n1 * id;
    }
  }
  s_red[0][t] = l1;
  s_red[1][t] = ssum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) { s_red[0][t] += s_red[0][t + off]; s_red[1][t] += s_red[1][t + off]; }
    __syncthreads();
  }
  if (t == 0) { partial[2 * blockIdx.x] = s_red[0][0]; partial[2 * blockIdx.x + 1] = s_red[1][0]; }
}

__global__ void __launch_bounds__(256) ssim_bwd_kernel(const glam_view_info* views, int n_views, const float* image,
                                                       const float* target, float w_ssim, const float* maps,
                                                       long long n_pix, float* dimage) {
  __shared__ float s_m[3][kHalo][kHalo];
  __shared__ float s_h[3][kHalo][kTile];
  const LossGeom g = loss_geom(views, n_views, blockIdx.x);
  const int t = threadIdx.x, lx = t & 15, ly = t >> 4;
  const int x = g.x0 + lx, y = g.y0 + ly;
  const bool inside = x < g.W && y < g.H;
  const long long HW = (long long)g.W * g.H;
  const long long p = (long long)y * g.W + x;
  const float inv_n = 1.f / (3.f * (float)HW);
  for (int c = 0; c < 3; ++c) {
    const float* xp = image + 3 * g.pix_begin + c * HW;
    const float* yp = target + 3 * g.pix_begin + c * HW;
    float grad = 0.f;
    float xv = 0.f, yv = 0.f;
    if (inside) {
      xv = xp[p]; yv = yp[p];
      const float d = xv - yv;
      grad = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * inv_n;
    }
    if (w_ssim != 0.f) {
      __syncthreads();
      const float* mp = maps + (long long)c * 3 * n_pix + g.pix_begin;
      for (int q = 0; q < 3; ++q) load_halo(mp + q * n_pix, g, s_m[q]);
      __syncthreads();
      for (int k = t; k < kHalo * kTile; k += 256) {
        const int hy = k / kTile, cx = k % kTile;
        float a = 0.f, b = 0.f, cc = 0.f;
        for (int o = 0; o < kWin; ++o) { a += s_m[0][hy][cx + o]; b += s_m[1][hy][cx + o]; cc += s_m[2][hy][cx + o]; }
        s_h[0][hy][cx] = a; s_h[1][hy][cx] = b; s_h[2][hy][cx] = cc;
      }
      __syncthreads();
      float a = 0.f, b = 0.f, cc = 0.f;
      for (int o = 0; o < kWin; ++o) { a += s_h[0][ly + o][lx]; b += s_h[1][ly + o][lx]; cc += s_h[2][ly + o][lx]; }
      grad -= w_ssim * inv_n * (1.f / 121.f) * (a + 2.f * xv * b + yv * cc);
    }
    if (inside) dimage[3 * g.pix_begin + c * HW + p] = grad;
  }
}

__global__ void __launch_bounds__(256) loss_reduce_kernel(const glam_view_info* views, const float* partial,
                                                          float w_ssim, float* loss) {
  __shared__ double s_a[256], s_b[256];
  const glam_view_info& vw = views[blockIdx.x];
  const int n = vw.tiles_x * vw.tiles_y;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    a += partial[2 * (vw.tile_begin + k)];
    b += partial[2 * (vw.tile_begin + k) + 1];
  }
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) { s_a[threadIdx.x] += s_a[threadIdx.x + off]; s_b[threadIdx.x] += s_b[threadIdx.x + off]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnt = 3.0 * (double)vw.cam.width * (double)vw.cam.height;
    double L = s_a[0] / cnt;
    if (w_ssim != 0.f) L += (double)w_ssim * (1.0 - s_b[0] / cnt);
    loss[blockIdx.x] = (float)L;
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t loss_workspace(const glam_views& v) {
  return align256(4ull * 9 * (size_t)v.n_pix) + align256(8ull * (size_t)v.n_tiles);
}

glam_status launch_loss(const glam_views& v, const float* image, const float* target, float w_ssim,
                        float* dimage, float* loss, void* ws, hipStream_t s) {
  if (v.n_tiles == 0) return GLAM_OK;
  float* maps = static_cast<float*>(ws);
  float* partial = reinterpret_cast<float*>(static_cast<char*>(ws) + align256(4ull * 9 * (size_t)v.n_pix));
  hipLaunchKernelGGL(ssim_fwd_kernel, dim3((unsigned)v.n_tiles), dim3(256), 0, s, v.dev, v.n, image, target, w_ssim,
                     maps, (long long)v.n_pix, partial);
  hipLaunchKernelGGL(ssim_bwd_kernel, dim3((unsigned)v.n_tiles), dim3(256), 0, s, v.dev, v.n, image, target, w_ssim,
                     maps, (long long)v.n_pix, dimage);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(v.n), dim3(256), 0, s, v.dev, partial, w_ssim, loss);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
