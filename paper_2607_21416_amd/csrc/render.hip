// Front-to-back alpha compositing (Eq. 1) per 16x16 tile and its reverse-order adjoint.
//
// One workgroup of 256 lanes (four wave64) per tile; each wave owns an 8x8 quadrant so
// that its lanes see nearly the same Gaussians.  The tile's sorted range is walked in
// batches of 256 records gathered from HBM into LDS (one 48-byte record per lane).
// Before evaluating a batch, each wave builds a 64-bit ballot mask per quarter of the
// batch of the records whose footprint box meets its quadrant and visits only those
// (in order).  A wave whose lanes have all terminated stops evaluating; the workgroup
// leaves when all 256 lanes have (block-wide count at each batch boundary).
//
// The backward pass walks the same ranges from each pixel's last contributor down,
// recovering T_i = T_{i+1} / (1 - alpha_i) from the stored final transmittance.  Per
// Gaussian, the nine gradient terms are summed across the wave (DPP row reductions)
// and added to HBM by nine lanes with one atomic instruction.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kBatch = 256;

// alpha of one record at pixel centre (px, py), shared by both passes so that their
// skip and stop decisions are bit-identical.
__device__ __forceinline__ float splat_alpha(const float4& r0, const float4& r1, float px, float py,
                                             float& dx, float& dy, float& ep, float& raw) {
  dx = r0.x - px;
  dy = r0.y - py;
  const float q = fmaf(r0.z * dx, dx, (r1.x * dy) * dy);
  const float power = fmaf(-0.5f, q, -((r0.w * dx) * dy));
  ep = __expf(power);
  raw = r1.y * ep;
  return fminf(kAlphaMax, raw);
}

struct TileGeom {
  int view;
  int x, y;            // this lane's pixel
  bool inside;
  int qx0, qx1, qy0, qy1;  // this wave's quadrant, clipped; empty if qx0 > qx1
  long long pix;       // pixel index in the batched per-pixel arrays
  int W, H;
  long long pix_begin;
};

__device__ __forceinline__ TileGeom tile_geom(const glam_view_info* views, int n_views, int tile) {
  TileGeom g;
  g.view = find_view(views, n_views, tile, [](const glam_view_info& v) { return (long long)v.tile_begin; });
  const glam_view_info& vw = views[g.view];
  const int lt = tile - vw.tile_begin;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qx = tx * kTile + (w & 1) * 8, qy = ty * kTile + (w >> 1) * 8;
  g.W = vw.cam.width;
  g.H = vw.cam.height;
  g.x = qx + (lane & 7);
  g.y = qy + (lane >> 3);
  g.inside = g.x < g.W && g.y < g.H;
  g.qx0 = qx; g.qy0 = qy;
  g.qx1 = min(qx + 7, g.W - 1);
  g.qy1 = min(qy + 7, g.H - 1);
  g.pix_begin = vw.pix_begin;
  g.pix = vw.pix_begin + (long long)g.y * g.W + g.x;
  return g;
}

__device__ __forceinline__ bool box_meets(float bxf, float byf, const TileGeom& g) {
  const uint32_t bx = __float_as_uint(bxf), by = __float_as_uint(byf);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16);
  const int y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  return x0 <= g.qx1 && x1 >= g.qx0 && y0 <= g.qy1 && y1 >= g.qy0;
}

// Per-lane component index of the values reduce9 leaves in lanes 16r + k (k < 3), or -1:
// the same swaps applied to the value tags (the swap instructions move whole rows, so
// each lane's two swap outputs always belong to one component).
struct Reduce9Map {
  int comp;
};

__device__ __forceinline__ uint32_t swap32_first(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_permlane32_swap(a, b, false, false)[0];
}
__device__ __forceinline__ uint32_t swap16_first(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_permlane16_swap(a, b, false, false)[0];
}

__device__ __forceinline__ float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float row_sum(float v) {
  v += dpp<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  return v;
}

__device__ __forceinline__ Reduce9Map reduce9_map() {
  const uint32_t none = 0xffffffffu;
  const uint32_t w0 = swap32_first(0, 1), w1 = swap32_first(2, 3), w2 = swap32_first(4, 5), w3 = swap32_first(6, 7),
                 w4 = swap32_first(8, none);
  const uint32_t x0 = swap16_first(w0, w1), x1 = swap16_first(w2, w3), x2 = swap16_first(w4, none);
  const int k = threadIdx.x & 15;
  Reduce9Map m;
  m.comp = k == 0 ? (int)x0 : (k == 1 ? (int)x1 : (k == 2 ? (int)x2 : -1));
  return m;
}

// Sum of nine per-lane values over the wave, scattered so that nine lanes hold one
// total each (reduce-scatter): two cross-half swaps halve the values per lane, then
// each 16-lane row is reduced with DPP.  The caller's wave must be fully active.
__device__ __forceinline__ float reduce9(const float v[9], const Reduce9Map& m) {
  const float w0 = swap32_sum(v[0], v[1]), w1 = swap32_sum(v[2], v[3]), w2 = swap32_sum(v[4], v[5]),
              w3 = swap32_sum(v[6], v[7]), w4 = swap32_sum(v[8], 0.f);
  const float x0 = row_sum(swap16_sum(w0, w1)), x1 = row_sum(swap16_sum(w2, w3)), x2 = row_sum(swap16_sum(w4, 0.f));
  const int k = threadIdx.x & 15;
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}

__global__ void __launch_bounds__(256) render_fwd_kernel(const float* __restrict__ splat,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges,
                                                         const glam_view_info* views, int n_views,
                                                         const float* bg, float* image, float* T_final,
                                                         int32_t* n_contrib, int32_t* n_eval, uint32_t capacity,
                                                         uint32_t n_gauss) {
  __shared__ float4 s_r0[kBatch], s_r1[kBatch];
  __shared__ float s_b[kBatch];
  __shared__ uint2 s_box[kBatch];
  const int tile = blockIdx.x;
  const TileGeom tg = tile_geom(views, n_views, tile);
  const int t = threadIdx.x, lane = t & 63;
  const uint32_t e = min(ranges[2 * tile + 1], capacity);
  const uint32_t s = min(ranges[2 * tile], e);
  const float px = tg.x + 0.5f, py = tg.y + 0.5f;
  const bool quad_live = tg.qx0 <= tg.qx1 && tg.qy0 <= tg.qy1;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = 0, stop = (int)(e - s);
  bool done = !tg.inside;
  for (uint32_t b0 = s; b0 < e; b0 += kBatch) {
    if (__syncthreads_count(done) == kBatch) break;
    const uint32_t j = b0 + t;
    if (j < e) {
      const uint32_t gid = min(vals[j], n_gauss - 1);
      const float4* r = reinterpret_cast<const float4*>(splat + (size_t)gid * kSplatWords);
      s_r0[t] = r[0];
      s_r1[t] = r[1];
      const float4 r2 = r[2];
      s_b[t] = r2.x;
      s_box[t] = make_uint2(__float_as_uint(r2.y), __float_as_uint(r2.z));
    }
    __syncthreads();
    const int nb = (int)min((uint32_t)kBatch, e - b0);
    const int base = (int)(b0 - s) + 1;
    if (quad_live && __ballot(!done) != 0) {
      bool wave_done = false;
      for (int k = 0; k < 4 && !wave_done; ++k) {
        const int idx = 64 * k + lane;
        const bool hit = idx < nb && box_meets(__uint_as_float(s_box[idx].x), __uint_as_float(s_box[idx].y), tg);
        uint64_t m = __ballot(hit);
        while (m) {
          const int i = 64 * k + (int)__builtin_ctzll(m);
          m &= m - 1;
          const float4 r0 = s_r0[i], r1 = s_r1[i];
          const float cb = s_b[i];
          float dx, dy, ep, raw;
          const float alpha = splat_alpha(r0, r1, px, py, dx, dy, ep, raw);
          const float Tn = T * (1.f - alpha);
          const bool ok = !done && alpha >= kAlphaMin;
          const bool halt = ok && Tn < kTMin;
          const bool take = ok && !(Tn < kTMin);
          const float wgt = take ? alpha * T : 0.f;
          C0 = fmaf(r1.z, wgt, C0);
          C1 = fmaf(r1.w, wgt, C1);
          C2 = fmaf(cb, wgt, C2);
          T = take ? Tn : T;
          last = take ? base + i : last;
          stop = halt ? base + i : stop;
          done = done || halt;
          if (__ballot(!done) == 0) {
            wave_done = true;
            break;
          }
        }
      }
    }
    __syncthreads();
  }
  if (tg.inside) {
    const long long HW = (long long)tg.W * tg.H;
    const long long p = (long long)tg.y * tg.W + tg.x;
    float* img = image + 3 * tg.pix_begin;
    const float b0 = bg ? bg[0] : 0.f, b1 = bg ? bg[1] : 0.f, b2 = bg ? bg[2] : 0.f;
    img[p] = fmaf(T, b0, C0);
    img[HW + p] = fmaf(T, b1, C1);
    img[2 * HW + p] = fmaf(T, b2, C2);
    T_final[tg.pix] = T;
    n_contrib[tg.pix] = last;
    if (n_eval) n_eval[tg.pix] = stop;
  }
}

__global__ void __launch_bounds__(256) composite_bwd_kernel(const float* __restrict__ splat,
                                                            const uint32_t* __restrict__ vals,
                                                            const uint32_t* __restrict__ ranges,
                                                            const glam_view_info* views, int n_views,
                                                            const float* bg, const float* T_final,
                                                            const int32_t* n_contrib, const float* dimage,
                                                            float* g2d, uint32_t capacity, uint32_t n_gauss) {
  __shared__ float4 s_r0[kBatch], s_r1[kBatch];
  __shared__ float s_b[kBatch];
  __shared__ uint2 s_box[kBatch];
  __shared__ uint32_t s_gid[kBatch];
  __shared__ int s_max;
  const int tile = blockIdx.x;
  const TileGeom tg = tile_geom(views, n_views, tile);
  const int t = threadIdx.x, lane = t & 63;
  const uint32_t e = min(ranges[2 * tile + 1], capacity);
  const uint32_t s = min(ranges[2 * tile], e);
  const float px = tg.x + 0.5f, py = tg.y + 0.5f;
  const bool quad_live = tg.qx0 <= tg.qx1 && tg.qy0 <= tg.qy1;
  const Reduce9Map rmap = reduce9_map();
  float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  float B0 = bg ? bg[0] : 0.f, B1 = bg ? bg[1] : 0.f, B2 = bg ? bg[2] : 0.f;
  int last = 0;
  if (tg.inside) {
    const long long HW = (long long)tg.W * tg.H;
    const long long p = (long long)tg.y * tg.W + tg.x;
    const float* di = dimage + 3 * tg.pix_begin;
    T = T_final[tg.pix];
    last = min(n_contrib[tg.pix], (int32_t)(e - s));
    g0 = di[p]; g1 = di[HW + p]; g2 = di[2 * HW + p];
  }
  if (t == 0) s_max = 0;
  __syncthreads();
  atomicMax(&s_max, last);
  __syncthreads();
  const int maxlast = s_max;
  for (int hi = maxlast; hi > 0; hi -= kBatch) {
    const int lo = max(0, hi - kBatch);
    const int nb = hi - lo;
    if (t < nb) {
      const uint32_t gid = min(vals[s + lo + t], n_gauss - 1);
      const float4* r = reinterpret_cast<const float4*>(splat + (size_t)gid * kSplatWords);
      s_r0[t] = r[0];
      s_r1[t] = r[1];
      const float4 r2 = r[2];
      s_b[t] = r2.x;
      s_box[t] = make_uint2(__float_as_uint(r2.y), __float_as_uint(r2.z));
      s_gid[t] = gid;
    }
    __syncthreads();
    if (quad_live && __ballot(last > lo) != 0) {
      for (int k = 3; k >= 0; --k) {
        const int idx = 64 * k + lane;
        const bool hit = idx < nb && box_meets(__uint_as_float(s_box[idx].x), __uint_as_float(s_box[idx].y), tg);
        uint64_t m = __ballot(hit);
        while (m) {
          const int bit = 63 - __clzll((unsigned long long)m);
          m &= ~(1ull << bit);
          const int i = 64 * k + bit;
          const float4 r0 = s_r0[i], r1 = s_r1[i];
          const float cb = s_b[i];
          float dx, dy, ep, raw;
          const float alpha = splat_alpha(r0, r1, px, py, dx, dy, ep, raw);
          const bool contrib = lo + i < last && alpha >= kAlphaMin;
          if (__ballot(contrib) == 0) continue;
          // T in front of this Gaussian: T_i = T_{i+1} / (1 - alpha_i)
          T = contrib ? T * __builtin_amdgcn_rcpf(1.f - alpha) : T;
          const float wgt = contrib ? alpha * T : 0.f;
          const float dal = contrib ? T * (g0 * (r1.z - B0) + g1 * (r1.w - B1) + g2 * (cb - B2)) : 0.f;
          const float aB = contrib ? alpha : 0.f;
          B0 = fmaf(aB, r1.z - B0, B0);
          B1 = fmaf(aB, r1.w - B1, B1);
          B2 = fmaf(aB, cb - B2, B2);
          const bool free_alpha = raw <= kAlphaMax;  // alpha not clamped: it depends on its inputs
          const float dop = free_alpha ? dal * ep : 0.f;
          const float dp = free_alpha ? dal * alpha : 0.f;
          float v[9];
          v[0] = -dp * (r0.z * dx + r0.w * dy);
          v[1] = -dp * (r0.w * dx + r1.x * dy);
          v[2] = -0.5f * dp * dx * dx;
          v[3] = -dp * dx * dy;
          v[4] = -0.5f * dp * dy * dy;
          v[5] = dop;
          v[6] = g0 * wgt;
          v[7] = g1 * wgt;
          v[8] = g2 * wgt;
          const float tot = reduce9(v, rmap);
          if (rmap.comp >= 0) atomicAdd(&g2d[(size_t)s_gid[i] * 9 + rmap.comp], tot);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void background_kernel(const glam_view_info* views, int n_views, long long n_pix, const float* bg,
                                  float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pix) return;
  const int vi = find_view(views, n_views, i, [](const glam_view_info& v) { return v.pix_begin; });
  const glam_view_info& vw = views[vi];
  const long long HW = (long long)vw.cam.width * vw.cam.height, p = i - vw.pix_begin;
  for (int c = 0; c < 3; ++c) image[3 * vw.pix_begin + c * HW + p] = bg ? bg[c] : 0.f;
  T_final[i] = 1.f;
  n_contrib[i] = 0;
  if (n_eval) n_eval[i] = 0;
}

__global__ void zero_kernel(float* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

glam_status launch_background(const glam_views& v, const float* bg, float* image, float* T_final,
                              int32_t* n_contrib, int32_t* n_eval, hipStream_t s) {
  hipLaunchKernelGGL(background_kernel, dim3((unsigned)((v.n_pix + 255) / 256)), dim3(256), 0, s, v.dev, v.n,
                     (long long)v.n_pix, bg, image, T_final, n_contrib, n_eval);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace

glam_status launch_render_fwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                              const float* bg, float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval,
                              hipStream_t s) {
  if (v.n_tiles == 0 || v.n_gauss == 0) {
    // nothing to composite: background everywhere
    return launch_background(v, bg, image, T_final, n_contrib, n_eval, s);
  }
  hipLaunchKernelGGL(render_fwd_kernel, dim3((unsigned)v.n_tiles), dim3(256), 0, s, proj.splat, bins.vals,
                     bins.ranges, v.dev, v.n, bg, image, T_final, n_contrib, n_eval, (uint32_t)bins.capacity,
                     (uint32_t)v.n_gauss);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

glam_status launch_composite_bwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                                 const float* bg, const float* T_final, const int32_t* n_contrib,
                                 const float* dimage, float* g2d, hipStream_t s) {
  const long long n = 9 * v.n_gauss;
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g2d, n);
  if (v.n_tiles > 0 && v.n_gauss > 0)
    hipLaunchKernelGGL(composite_bwd_kernel, dim3((unsigned)v.n_tiles), dim3(256), 0, s, proj.splat, bins.vals,
                       bins.ranges, v.dev, v.n, bg, T_final, n_contrib, dimage, g2d, (uint32_t)bins.capacity,
                       (uint32_t)v.n_gauss);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
