// Photometric loss of Eq. 3 per view: L = mean |C - target| + w (1 - mean SSIM), SSIM
// with an 11x11 box window and zero padding, and dL/dC.
//
// One fused kernel per (32x32 output tile, channel).  With q ranging over the window
// centres that touch the tile (a 42x42 region) and the inputs those windows read (a
// 52x52 region, zero outside the image), the workgroup
//   1. stages x = image and y = target of the 52x52 region in LDS,
//   2. sums x, y, x^2, y^2, xy along rows (11 wide) for the 42 window columns,
//   3. sums those down columns (11 tall) to the window statistics at every q, and
//      writes SSIM(q) and its partials with respect to mean(x), E[x^2] and E[xy]
//      (zero where q is outside the image) to LDS,
//   4-5. box-sums the partials over the window around every output pixel (the adjoint
//      of the window mean is the same box) and combines them with the L1 sign into
//      dL/dC, written once.
// Row and column sums slide along short register-held runs (add the entering term,
// subtract the leaving one).  Per-(tile, channel) sums of |x - y| and SSIM go to a
// small workspace; a last kernel reduces each view's sums in double precision (one
// workgroup for all views when they are few, which also adds up the step's total).
// Nothing but the image, the target and dL/dC touches HBM.  The per-view L1 losses of the
// fused forward + loss + adjoint pass are reduced here too, from its per-item sums.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

// The scratch of glam_loss_noalloc (the per-(tile, channel) partial sums that
// glam_loss keeps in its caller's workspace): one array per device, for the life of
// the process.  Host code never passes the array's name to a kernel (on the host it is
// only a stand-in); it passes the device address hipGetSymbolAddress resolves, once
// per device, with that device current.
static __device__ __align__(256) unsigned char scratch[GLAM_LOSS_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The current device's scratch address (resolved on its first use).
glam_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GLAM_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return GLAM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GLAM_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GLAM_OK;
}

constexpr int kR = 5, kWin = 2 * kR + 1;
constexpr int kT = 32;               // output tile edge
constexpr int kQ = kT + 2 * kR;      // 42: window centres touching the tile
constexpr int kI = kT + 4 * kR;      // 52: inputs those windows read
constexpr int kIS = kI + 1, kQS = kQ + 1, kTS = kT + 1;  // padded LDS row strides
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;
// 512 threads per workgroup: the LDS plan allows two workgroups per CU, so eight waves
// per workgroup keep four per SIMD resident
constexpr int kThreads = 512;
constexpr int kRun4 = 4;                  // step 4: runs of 4 output columns
constexpr int kRun5 = kT * kT / kThreads;  // step 5: rows per run (16 runs of 2 per column)
static_assert((kThreads / kT) * kRun5 == kT && kRun5 >= 1, "step 5 covers the tile");

// LDS plan (floats): region A holds the staged inputs, later the partial maps;
// region B holds the row sums of the statistics, later the row sums of the partials.
constexpr int kA = 2 * kI * kIS;     // 5512 >= 3 * kQ * kQS = 5418
constexpr int kB = 5 * kI * kQS;     // 11180 >= 3 * kQ * kTS = 4158
static_assert(3 * kQ * kQS <= kA && 3 * kQ * kTS <= kB, "LDS aliasing");

__device__ __forceinline__ float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__global__ void __launch_bounds__(kThreads) loss_kernel(const glam_view_info* views, int max_t32, const float* image,
                                                   const float* target, float w_ssim, float* dimage,
                                                   float* partial) {
  __shared__ float sA[kA];
  __shared__ float sB[kB];
  __shared__ float s_red[2][kThreads / 64];
  const glam_view_info vw = views[blockIdx.y];
  const int W = vw.cam.width, H = vw.cam.height;
  const int tx_n = (W + kT - 1) / kT, ty_n = (H + kT - 1) / kT;
  const int t32 = blockIdx.x;
  if (t32 >= tx_n * ty_n) return;
  const int c = blockIdx.z;
  const int x0 = (t32 % tx_n) * kT, y0 = (t32 / tx_n) * kT;
  const long long HW = (long long)W * H;
  const float* xp = image + 3 * vw.pix_begin + c * HW;
  const float* yp = target + 3 * vw.pix_begin + c * HW;
  const int t = threadIdx.x;
  float ssum = 0.f;
  // partials of the window around output pixel (io, jo) are summed in step 5
  float* sP = sA;                    // [3][kQ][kQS]
  float* sHP = sB;                   // [3][kQ][kTS]
  if (w_ssim != 0.f) {
    // 1. inputs of the 52x52 region
    float* sx = sA;
    float* sy = sA + kI * kIS;
    // all loads in flight before the first LDS store; element k = t + kThreads n is
    // (row, column) (k / kI, k % kI), stepped from n to n + 1 without a division, and
    // every lane loads (pixel 0 where the element is outside the image, then zero)
    constexpr int kLoads = (kI * kI + kThreads - 1) / kThreads;
    constexpr int kStepR = kThreads / kI, kStepJ = kThreads % kI;
    float vx[kLoads], vy[kLoads];
    int rr[kLoads], cc[kLoads];
    {
      int r = t / kI, j = t % kI;
#pragma unroll
      for (int n = 0; n < kLoads; ++n) {
        rr[n] = r;
        cc[n] = j;
        const int gx = x0 - 2 * kR + j, gy = y0 - 2 * kR + r;
        const bool in = r < kI && (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
        const unsigned o = in ? (unsigned)(gy * W + gx) : 0u;  // < W H < 2^30 (edges below 2^15)
        const float a = xp[o], b = yp[o];
        vx[n] = in ? a : 0.f;
        vy[n] = in ? b : 0.f;
        j += kStepJ;
        r += kStepR;
        if (j >= kI) { j -= kI; ++r; }
      }
    }
#pragma unroll
    for (int n = 0; n < kLoads; ++n) {
      if (rr[n] < kI) {
        sx[rr[n] * kIS + cc[n]] = vx[n];
        sy[rr[n] * kIS + cc[n]] = vy[n];
      }
    }
    __syncthreads();
    // 2. row sums: 52 rows x 42 window columns, runs of 7 columns
    float* sH = sB;                  // [5][kI][kQS]
    for (int task = t; task < kI * 6; task += kThreads) {
      const int r = task % kI, j0 = (task / kI) * 7;
      const float* rx = sx + r * kIS + j0;
      const float* ry = sy + r * kIS + j0;
      float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
      for (int o = 0; o < kWin; ++o) {
        const float u = rx[o], v = ry[o];
        a += u; b += v; aa += u * u; bb += v * v; ab += u * v;
      }
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const int idx = r * kQS + j0 + m;
        sH[idx] = a; sH[kI * kQS + idx] = b; sH[2 * kI * kQS + idx] = aa;
        sH[3 * kI * kQS + idx] = bb; sH[4 * kI * kQS + idx] = ab;
        if (m < 6) {
          const float ui = rx[m + kWin], vi = ry[m + kWin], uo = rx[m], vo = ry[m];
          a += ui - uo; b += vi - vo; aa += ui * ui - uo * uo; bb += vi * vi - vo * vo; ab += ui * vi - uo * vo;
        }
      }
    }
    __syncthreads();
    // 3. column sums -> window statistics, SSIM and its partials at 42x42 centres,
    //    runs of 7 rows
    float sp0[7], sp1[7], sp2[7];
    int jj = 0, i0 = 0;
    const bool has3 = t < kQ * 6;
    if (has3) {
      jj = t % kQ;
      i0 = (t / kQ) * 7;
      float m5[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int o = 0; o < kWin; ++o) acc += sH[q * kI * kQS + (i0 + o) * kQS + jj];
        m5[q] = acc;
      }
      const int gx = x0 - kR + jj;
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const int i = i0 + m, gy = y0 - kR + i;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const float inv = 1.f / 121.f;
        const float mx = m5[0] * inv, my = m5[1] * inv;
        const float vx = m5[2] * inv - mx * mx, vy = m5[3] * inv - my * my, cxy = m5[4] * inv - mx * my;
        const float n1 = 2.f * mx * my + kC1, n2 = 2.f * cxy + kC2;
        const float d1 = mx * mx + my * my + kC1, d2 = vx + vy + kC2;
        // hardware reciprocals (1 ulp): d1, d2 >= C1, C2 > 0
        const float rd2 = __builtin_amdgcn_rcpf(d2);
        const float id = __builtin_amdgcn_rcpf(d1) * rd2;
        const float sv = n1 * n2 * id;
        const bool own = i >= kR && i < kR + kT && jj >= kR && jj < kR + kT;
        if (in && own) ssum += sv;
        sp0[m] = in ? (2.f * my * n2 - 2.f * my * n1) * id - sv * (2.f * mx * d2 - 2.f * mx * d1) * id : 0.f;
        sp1[m] = in ? -sv * rd2 : 0.f;
        sp2[m] = in ? 2.f * n1 * id : 0.f;
        if (m < 6) {
#pragma unroll
          for (int q = 0; q < 5; ++q)
            m5[q] += sH[q * kI * kQS + (i + kWin) * kQS + jj] - sH[q * kI * kQS + i * kQS + jj];
        }
      }
    }
    __syncthreads();  // region A (inputs) is dead: the partial maps take its place
    if (has3) {
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const int idx = (i0 + m) * kQS + jj;
        sP[idx] = sp0[m]; sP[kQ * kQS + idx] = sp1[m]; sP[2 * kQ * kQS + idx] = sp2[m];
      }
    }
    __syncthreads();
    // 4. row sums of the partials: 42 rows x 32 output columns, runs of 4
    for (int task = t; task < kQ * (kT / kRun4); task += kThreads) {
      const int i = task % kQ, j0 = (task / kQ) * kRun4;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const float* row = sP + p * kQ * kQS + i * kQS + j0;
        float acc = 0.f;
#pragma unroll
        for (int o = 0; o < kWin; ++o) acc += row[o];
#pragma unroll
        for (int m = 0; m < kRun4; ++m) {
          sHP[p * kQ * kTS + i * kTS + j0 + m] = acc;
          if (m < kRun4 - 1) acc += row[m + kWin] - row[m];
        }
      }
    }
    __syncthreads();
  }
  // 5. column sums of the partials and dL/dC: 32 output columns x runs of 2 rows
  const long long n_all = 3 * HW;
  const float inv_n = 1.f / (float)n_all;
  const int jo = t % kT, io0 = (t / kT) * kRun5;
  float pa = 0.f, pb = 0.f, pc = 0.f;
  if (w_ssim != 0.f) {
#pragma unroll
    for (int o = 0; o < kWin; ++o) {
      pa += sHP[(io0 + o) * kTS + jo];
      pb += sHP[kQ * kTS + (io0 + o) * kTS + jo];
      pc += sHP[2 * kQ * kTS + (io0 + o) * kTS + jo];
    }
  }
  float l1 = 0.f;
  const int gx = x0 + jo;
  float xs[kRun5], ys[kRun5];
#pragma unroll
  for (int m = 0; m < kRun5; ++m) {
    const int gy = y0 + io0 + m;
    const bool in = gx < W && gy < H;
    const long long o = in ? (long long)gy * W + gx : 0;
    xs[m] = in ? xp[o] : 0.f;
    ys[m] = in ? yp[o] : 0.f;
  }
#pragma unroll
  for (int m = 0; m < kRun5; ++m) {
    const int io = io0 + m, gy = y0 + io;
    if (gx < W && gy < H) {
      const long long o = (long long)gy * W + gx;
      const float xv = xs[m], yv = ys[m];
      const float d = xv - yv;
      l1 += fabsf(d);
      float g = sgn(d) * inv_n;
      if (w_ssim != 0.f) g -= w_ssim * inv_n * (1.f / 121.f) * (pa + 2.f * xv * pb + yv * pc);
      dimage[3 * vw.pix_begin + c * HW + o] = g;
    }
    if (w_ssim != 0.f && m < kRun5 - 1) {
      pa += sHP[(io + kWin) * kTS + jo] - sHP[io * kTS + jo];
      pb += sHP[kQ * kTS + (io + kWin) * kTS + jo] - sHP[kQ * kTS + io * kTS + jo];
      pc += sHP[2 * kQ * kTS + (io + kWin) * kTS + jo] - sHP[2 * kQ * kTS + io * kTS + jo];
    }
  }
  // per-(tile, channel) sums
  l1 = wave_sum(l1);
  ssum = wave_sum(ssum);
  if ((t & 63) == 0) { s_red[0][t >> 6] = l1; s_red[1][t >> 6] = ssum; }
  __syncthreads();
  if (t == 0) {
    float a = 0.f, b = 0.f;
    for (int w = 0; w < kThreads / 64; ++w) { a += s_red[0][w]; b += s_red[1][w]; }
    float* pp = partial + 2 * (((long long)blockIdx.y * max_t32 + t32) * 3 + c);
    pp[0] = a;
    pp[1] = b;
  }
}

// Sums of a and b over a workgroup of 256 threads, in double precision and a fixed
// order: each wave's lanes by a butterfly, then the four waves in order.  Every thread
// calls it and gets both sums.  s: 8 doubles of LDS, free again when it returns.
__device__ __forceinline__ void block_sum256(double& a, double& b, double* s) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    s[threadIdx.x >> 6] = a;
    s[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = ((s[0] + s[1]) + s[2]) + s[3];
  b = ((s[4] + s[5]) + s[6]) + s[7];
  __syncthreads();
}

// View v's loss from its per-(tile, channel) sums, by the workgroup (thread t adds the
// sums t, t + 256, ...).  Every thread calls it.
__device__ void reduce_view(const glam_view_info& vw, int v, int max_t32, const float* partial, float w_ssim,
                            float* loss, double* s) {
  const int n = 3 * ((vw.cam.width + kT - 1) / kT) * ((vw.cam.height + kT - 1) / kT);
  const float* pv = partial + 2 * 3 * (long long)v * max_t32;
  double a = 0.0, b = 0.0;
#pragma unroll 4
  for (int k = threadIdx.x; k < n; k += 256) {
    a += pv[2 * k];
    b += pv[2 * k + 1];
  }
  block_sum256(a, b, s);
  if (threadIdx.x == 0) {
    const double cnt = 3.0 * (double)vw.cam.width * (double)vw.cam.height;
    double L = a / cnt;
    if (w_ssim != 0.f) L += (double)w_ssim * (1.0 - b / cnt);
    loss[v] = (float)L;
  }
}

// One workgroup per view.
__global__ void __launch_bounds__(256) loss_reduce_kernel(const glam_view_info* views, int max_t32,
                                                          const float* partial, float w_ssim, float* loss) {
  __shared__ double s[8];
  reduce_view(views[blockIdx.x], blockIdx.x, max_t32, partial, w_ssim, loss, s);
}

// A few views: one workgroup reduces them in view order and then adds their losses
// (the step's total), in one launch.
constexpr int kOneBlockViews = 64;
__global__ void __launch_bounds__(256) loss_reduce_total_kernel(const glam_view_info* views, int n_views,
                                                                int max_t32, const float* partial, float w_ssim,
                                                                float* loss, float* total) {
  __shared__ double s[8];
  for (int v = 0; v < n_views; ++v) reduce_view(views[v], v, max_t32, partial, w_ssim, loss, s);
  if (threadIdx.x == 0 && total) {
    double acc = 0.0;
    for (int v = 0; v < n_views; ++v) acc += (double)loss[v];
    *total = (float)acc;
  }
}

// The step's loss: the views' losses added in view order (double precision).
__global__ void loss_total_kernel(const float* loss, int n, float* total) {
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int v = 0; v < n; ++v) acc += (double)loss[v];
  *total = (float)acc;
}

// View v's L1 loss from the fused pass's per-item sums, by the workgroup (thread t adds
// the sums t, t + 256, ...); one workgroup per view, or one for all views (which then
// also adds up the total) when they are few.  Every thread calls it.
__device__ void l1_reduce_view(const glam_view_info& vw, int v, int ql, const float* l1_part, float* loss, double* s) {
  const long long i0 = vw.tile_begin << ql;
  const long long n = (long long)(vw.tiles_x * vw.tiles_y) << ql;
  double a = 0.0;
#pragma unroll 4
  for (long long k = threadIdx.x; k < n; k += 256) a += l1_part[i0 + k];
  double unused = 0.0;
  block_sum256(a, unused, s);
  if (threadIdx.x == 0) loss[v] = (float)(a / (3.0 * (double)vw.cam.width * (double)vw.cam.height));
}

__global__ void __launch_bounds__(256) l1_reduce_kernel(const glam_view_info* views, int n_views, int ql,
                                                        const float* l1_part, float* loss, float* total, int one) {
  __shared__ double s[8];
  if (one) {
    for (int v = 0; v < n_views; ++v) l1_reduce_view(views[v], v, ql, l1_part, loss, s);
    if (threadIdx.x == 0 && total) {
      double acc = 0.0;
      for (int v = 0; v < n_views; ++v) acc += (double)loss[v];
      *total = (float)acc;
    }
  } else {
    l1_reduce_view(views[blockIdx.x], blockIdx.x, ql, l1_part, loss, s);
  }
}

int max_tiles32(const glam_views& v) {
  int mx = 0;
  for (int i = 0; i < v.n; ++i) {
    const glam_camera& c = v.host[i].cam;
    const int n = ((c.width + kT - 1) / kT) * ((c.height + kT - 1) / kT);
    mx = n > mx ? n : mx;
  }
  return mx;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t loss_workspace(const glam_views& v) { return align256(8ull * 3 * (size_t)max_tiles32(v) * (size_t)v.n); }

glam_status launch_l1_reduce(const glam_views& v, int ql, const float* l1_part, float* loss, float* total,
                             hipStream_t s) {
  if (v.n <= kOneBlockViews) {
    hipLaunchKernelGGL(l1_reduce_kernel, dim3(1), dim3(256), 0, s, v.dev, v.n, ql, l1_part, loss, total, 1);
  } else {
    hipLaunchKernelGGL(l1_reduce_kernel, dim3(v.n), dim3(256), 0, s, v.dev, v.n, ql, l1_part, loss, total, 0);
    if (total) hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(64), 0, s, loss, v.n, total);
  }
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

glam_status launch_loss_noalloc(const glam_views& v, const float* image, const float* target, float w_ssim,
                                float* dimage, float* loss, float* total, hipStream_t s) {
  if (loss_workspace(v) > GLAM_LOSS_SCRATCH_BYTES) return GLAM_ERR_WORKSPACE;
  void* ws = nullptr;
  const glam_status st = scratch_address(&ws);
  if (st != GLAM_OK) return st;
  return launch_loss(v, image, target, w_ssim, dimage, loss, total, ws, s);
}

glam_status launch_loss(const glam_views& v, const float* image, const float* target, float w_ssim,
                        float* dimage, float* loss, float* total, void* ws, hipStream_t s) {
  if (v.n_tiles == 0 || v.n == 0) return GLAM_OK;
  const int mt = max_tiles32(v);
  float* partial = static_cast<float*>(ws);
  hipLaunchKernelGGL(loss_kernel, dim3((unsigned)mt, (unsigned)v.n, 3), dim3(kThreads), 0, s, v.dev, mt, image, target,
                     w_ssim, dimage, partial);
  if (v.n <= kOneBlockViews) {
    hipLaunchKernelGGL(loss_reduce_total_kernel, dim3(1), dim3(256), 0, s, v.dev, v.n, mt, partial, w_ssim, loss,
                       total);
  } else {
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(v.n), dim3(256), 0, s, v.dev, mt, partial, w_ssim, loss);
    if (total) hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(64), 0, s, loss, v.n, total);
  }
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
