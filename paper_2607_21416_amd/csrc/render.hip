// Front-to-back alpha compositing (Eq. 1) and its reverse-order adjoint.
//
// Work decomposition.  Gaussians are binned to 16x16 tiles; each tile is split into
// four 8x8 quadrants, and one wave64 composites one quadrant (one pixel per lane).
// The (tile, quadrant) items are pulled from a device work queue by a persistent grid
// (a few workgroups per CU, their four waves fully independent: no workgroup barrier
// anywhere), in longest-range-first order, so that the few very long tiles near the
// horizon start first and the short ones fill in behind them.  The queue counter
// resets itself when the last wave of a launch leaves.
//
// Per item, a wave walks its tile's depth-sorted range in batches of 64: lane l
// gathers the 48-byte record of entry b0+l from HBM (the next batch is prefetched into
// registers while the current one is composited), tests its footprint box against
// the quadrant, and the hits are compacted into a wave-private LDS buffer (ballot +
// lane-mask prefix count).  The wave then walks the hits in order; all lanes read the
// same record (LDS broadcast) and composite their own pixel.  The wave leaves as soon
// as all 64 of its pixels have stopped.
//
// The backward walks the same ranges from the wave's last contributor down,
// recovering T_i = T_{i+1} / (1 - alpha_i) from the stored final transmittance.  Per
// Gaussian, the nine gradient terms of the wave's pixels are summed with a
// reduce-scatter (two gfx950 lane-swap stages, then DPP within 16-lane rows) and nine
// lanes add the totals to HBM with one atomic instruction.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kWaves = 4;        // waves per workgroup (independent)
constexpr int kIlp = 4;          // hits whose alphas a wave evaluates side by side
constexpr int kBlocksPerCU = 8;  // persistent workgroups per CU

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

struct Item {
  int x, y;                // this lane's pixel
  bool inside;
  int qx0, qx1, qy0, qy1;  // the wave's quadrant, clipped to the image (empty if qx0 > qx1)
  int W, H;
  long long pix_begin;
  long long pix;           // this lane's pixel in the batched per-pixel arrays
};

__device__ __forceinline__ Item make_item(const glam_view_info* views, int n_views, int tile, int quad, int lane) {
  Item it;
  const int v = find_view(views, n_views, tile, [](const glam_view_info& w) { return (long long)w.tile_begin; });
  const glam_view_info& vw = views[v];
  const int lt = tile - vw.tile_begin;
  const int qx = (lt % vw.tiles_x) * kTile + (quad & 1) * 8, qy = (lt / vw.tiles_x) * kTile + (quad >> 1) * 8;
  it.W = vw.cam.width;
  it.H = vw.cam.height;
  it.x = qx + (lane & 7);
  it.y = qy + (lane >> 3);
  it.inside = it.x < it.W && it.y < it.H;
  it.qx0 = qx;
  it.qy0 = qy;
  it.qx1 = min(qx + 7, it.W - 1);
  it.qy1 = min(qy + 7, it.H - 1);
  it.pix_begin = vw.pix_begin;
  it.pix = vw.pix_begin + (long long)it.y * it.W + it.x;
  return it;
}

__device__ __forceinline__ bool box_meets(float bxf, float byf, const Item& it) {
  const uint32_t bx = __float_as_uint(bxf), by = __float_as_uint(byf);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16);
  const int y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  return x0 <= it.qx1 && x1 >= it.qx0 && y0 <= it.qy1 && y1 >= it.qy0;
}

// Work queue.  Device-scope atomics are served at the memory side, so one counter would
// serialise every grab; the longest-first tile list is dealt round-robin over kQueues
// counters (one 128-byte line each), and workgroup b pulls from counter b % kQueues.
// Workgroups are dealt to the 8 XCDs round-robin, so all workgroups of one counter sit
// on one XCD; the four quadrant items of a tile are consecutive grabs of one counter, so
// the tile's records are fetched into that XCD's L2 once and read there four times.
// An item is 4 * (tile rank) + quadrant.
// Words [0, kQueues*32) of a queue region hold the counters, word kQueues*32 the exit
// count.  The last wave to leave resets all of them for the next launch.
constexpr int kQueues = 16;
constexpr int kQueueWords = kQueues * 32 + 32;
static_assert(2 * kQueueWords == GLAM_QUEUE_WORDS, "queue layout");

__device__ __forceinline__ uint32_t next_item(uint32_t* q, int lane) {
  const uint32_t nq = min((uint32_t)kQueues, gridDim.x);  // every counter in use has workgroups
  const uint32_t qi = blockIdx.x % nq;
  uint32_t v = 0;
  if (lane == 0) v = atomicAdd(&q[32 * qi], 1u);
  v = __builtin_amdgcn_readfirstlane(v);
  return ((v >> 2) * nq + qi) * 4u + (v & 3u);
}

__device__ __forceinline__ void leave_queue(uint32_t* q, uint32_t total_waves, int lane) {
  if (lane == 0) {
    const uint32_t n = atomicAdd(&q[32 * kQueues], 1u);
    if (n == total_waves - 1) {
      for (int i = 0; i < kQueues; ++i) atomicExch(&q[32 * i], 0u);
      atomicExch(&q[32 * kQueues], 0u);
    }
  }
}

// The few longest items (horizon tiles, thousands of entries) bound the kernel's end:
// their waves get a higher issue priority on their SIMD, the short items fill in around
// them.
constexpr uint32_t kLongRange = 1024;
__device__ __forceinline__ void long_item_priority(uint32_t len) {
  if (len >= kLongRange) __builtin_amdgcn_s_setprio(2);
  else __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// Gathered record of one range entry.
struct Rec {
  float4 r0, r1, r2;
};

__device__ __forceinline__ Rec load_rec(const float* splat, uint32_t gid) {
  const float4* r = reinterpret_cast<const float4*>(splat + (size_t)gid * kSplatWords);
  Rec o;
  o.r0 = r[0];
  o.r1 = r[1];
  o.r2 = r[2];
  return o;
}

// Wave-private compacted batch: (u, v, A, B), (C, opacity, r, g), (b, entry offset or
// Gaussian index as bits).
struct WaveLds {
  float4 r0[64];
  float4 r1[64];
  float2 bx[64];
};

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBlocksPerCU))) render_fwd_kernel(const float* __restrict__ splat,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ order, uint32_t* queue,
                                                         const glam_view_info* views, int n_views, int n_tiles,
                                                         const float* bg, float* image, float* T_final,
                                                         int32_t* n_contrib, int32_t* n_eval, uint32_t capacity,
                                                         uint32_t n_gauss) {
  __shared__ WaveLds lds[kWaves];
  const int lane = threadIdx.x & 63;
  WaveLds& L = lds[threadIdx.x >> 6];
  const uint32_t n_items = 4u * (uint32_t)n_tiles;
  const float b0c = bg ? bg[0] : 0.f, b1c = bg ? bg[1] : 0.f, b2c = bg ? bg[2] : 0.f;
  for (uint32_t item = next_item(queue, lane); item < n_items; item = next_item(queue, lane)) {
    const int tile = (int)min(order[item >> 2], (uint32_t)n_tiles - 1);
    const Item it = make_item(views, n_views, tile, (int)(item & 3u), lane);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    long_item_priority(e - s);
    const float px = it.x + 0.5f, py = it.y + 0.5f;
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int last = 0, stop = (int)(e - s);
    bool done = !it.inside;
    const bool live = it.qx0 <= it.qx1 && it.qy0 <= it.qy1;
    // prefetch the first batch
    Rec nxt;
    if (live && s + lane < e) nxt = load_rec(splat, min(vals[s + lane], n_gauss - 1));
    for (uint32_t b0 = s; live && b0 < e; b0 += 64) {
      const Rec cur = nxt;
      const bool valid = b0 + lane < e;
      if (b0 + 64 + lane < e) nxt = load_rec(splat, min(vals[b0 + 64 + lane], n_gauss - 1));
      const bool hit = valid && box_meets(cur.r2.y, cur.r2.z, it);
      const uint64_t hm = __ballot(hit);
      if (hit) {
        const int pos = __popcll(hm & lanemask_lt(lane));
        L.r0[pos] = cur.r0;
        L.r1[pos] = cur.r1;
        L.bx[pos] = make_float2(cur.r2.x, __int_as_float(lane));
      }
      __builtin_amdgcn_wave_barrier();
      const int nhit = __popcll(hm);
      const int base = (int)(b0 - s) + 1;
      bool wave_done = false;
      // One hit, in order: the skip and stop rules of Eq. 1 on this lane's pixel.
      auto apply = [&](float alpha, const float4& r1, const float2& bx) {
        const float Tn = T * (1.f - alpha);
        const bool ok = !done && alpha >= kAlphaMin;
        const bool halt = ok && Tn < kTMin;
        const bool take = ok && !(Tn < kTMin);
        const float wgt = take ? alpha * T : 0.f;
        C0 = fmaf(r1.z, wgt, C0);
        C1 = fmaf(r1.w, wgt, C1);
        C2 = fmaf(bx.x, wgt, C2);
        T = take ? Tn : T;
        const int entry = base + __float_as_int(bx.y);
        last = take ? entry : last;
        stop = halt ? entry : stop;
        done = done || halt;
      };
      // groups of kIlp hits: their alphas are independent and computed side by side,
      // only the transmittance updates run in sequence
      int i = 0;
      for (; i + kIlp <= nhit; i += kIlp) {
        float4 r0[kIlp], r1[kIlp];
        float2 bx[kIlp];
        float alpha[kIlp];
#pragma unroll
        for (int k = 0; k < kIlp; ++k) {
          r0[k] = L.r0[i + k];
          r1[k] = L.r1[i + k];
          bx[k] = L.bx[i + k];
        }
#pragma unroll
        for (int k = 0; k < kIlp; ++k) {
          float dx, dy, ep, raw;
          alpha[k] = splat_alpha(r0[k], r1[k], px, py, dx, dy, ep, raw);
        }
#pragma unroll
        for (int k = 0; k < kIlp; ++k) apply(alpha[k], r1[k], bx[k]);
        if (__ballot(!done) == 0) {
          wave_done = true;
          break;
        }
      }
      for (; !wave_done && i < nhit; ++i) {
        const float4 r0 = L.r0[i], r1 = L.r1[i];
        const float2 bx = L.bx[i];
        float dx, dy, ep, raw;
        apply(splat_alpha(r0, r1, px, py, dx, dy, ep, raw), r1, bx);
        if (__ballot(!done) == 0) wave_done = true;
      }
      __builtin_amdgcn_wave_barrier();
      if (wave_done) break;
    }
    if (it.inside) {
      const long long HW = (long long)it.W * it.H;
      const long long p = (long long)it.y * it.W + it.x;
      float* img = image + 3 * it.pix_begin;
      img[p] = fmaf(T, b0c, C0);
      img[HW + p] = fmaf(T, b1c, C1);
      img[2 * HW + p] = fmaf(T, b2c, C2);
      T_final[it.pix] = T;
      n_contrib[it.pix] = last;
      if (n_eval) n_eval[it.pix] = stop;
    }
  }
  leave_queue(queue, gridDim.x * kWaves, lane);
}

// ---------------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------------

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

// Component of the total that reduce9 leaves in this lane (lanes 16r + k, k < 3), or -1:
// the swaps applied to the value tags.  Each swap moves whole rows or half-waves, so a
// lane's two swap outputs always belong to one component, whatever half goes where.
__device__ __forceinline__ int reduce9_comp() {
  const uint32_t none = 0xffffffffu;
  const uint32_t w0 = swap32_first(0, 1), w1 = swap32_first(2, 3), w2 = swap32_first(4, 5), w3 = swap32_first(6, 7),
                 w4 = swap32_first(8, none);
  const uint32_t x0 = swap16_first(w0, w1), x1 = swap16_first(w2, w3), x2 = swap16_first(w4, none);
  const int k = threadIdx.x & 15;
  return k == 0 ? (int)x0 : (k == 1 ? (int)x1 : (k == 2 ? (int)x2 : -1));
}

// Sum of nine per-lane values over the wave, scattered so that nine lanes hold one total
// each (reduce-scatter).  The wave must be fully active.
__device__ __forceinline__ float reduce9(const float v[9]) {
  const float w0 = swap32_sum(v[0], v[1]), w1 = swap32_sum(v[2], v[3]), w2 = swap32_sum(v[4], v[5]),
              w3 = swap32_sum(v[6], v[7]), w4 = swap32_sum(v[8], 0.f);
  const float x0 = row_sum(swap16_sum(w0, w1)), x1 = row_sum(swap16_sum(w2, w3)), x2 = row_sum(swap16_sum(w4, 0.f));
  const int k = threadIdx.x & 15;
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}

__device__ __forceinline__ int wave_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}

__global__ void __launch_bounds__(256) composite_bwd_kernel(const float* __restrict__ splat,
                                                            const uint32_t* __restrict__ vals,
                                                            const uint32_t* __restrict__ ranges,
                                                            const uint32_t* __restrict__ order, uint32_t* queue,
                                                            const glam_view_info* views, int n_views, int n_tiles,
                                                            const float* bg, const float* T_final,
                                                            const int32_t* n_contrib, const float* dimage,
                                                            float* g2d, uint32_t capacity, uint32_t n_gauss) {
  __shared__ WaveLds lds[kWaves];
  const int lane = threadIdx.x & 63;
  WaveLds& L = lds[threadIdx.x >> 6];
  const int comp = reduce9_comp();
  const uint32_t n_items = 4u * (uint32_t)n_tiles;
  for (uint32_t item = next_item(queue + kQueueWords, lane); item < n_items;
       item = next_item(queue + kQueueWords, lane)) {
    const int tile = (int)min(order[item >> 2], (uint32_t)n_tiles - 1);
    const Item it = make_item(views, n_views, tile, (int)(item & 3u), lane);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    long_item_priority(e - s);
    const float px = it.x + 0.5f, py = it.y + 0.5f;
    float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    float B0 = bg ? bg[0] : 0.f, B1 = bg ? bg[1] : 0.f, B2 = bg ? bg[2] : 0.f;
    int last = 0;
    if (it.inside) {
      const long long HW = (long long)it.W * it.H;
      const long long p = (long long)it.y * it.W + it.x;
      const float* di = dimage + 3 * it.pix_begin;
      T = T_final[it.pix];
      last = min(n_contrib[it.pix], (int32_t)(e - s));
      g0 = di[p];
      g1 = di[HW + p];
      g2 = di[2 * HW + p];
    }
    const bool live = it.qx0 <= it.qx1 && it.qy0 <= it.qy1;
    const int top = live ? wave_max(last) : 0;
    // batches of 64 entries from the top down; the next lower batch is prefetched
    Rec nxt;
    uint32_t ngid = 0;
    if (top > 0) {
      const int lo = max(0, top - 64);
      if (lo + lane < top) {
        ngid = min(vals[s + lo + lane], n_gauss - 1);
        nxt = load_rec(splat, ngid);
      }
    }
    for (int hi = top; hi > 0; hi -= 64) {
      const int lo = max(0, hi - 64);
      const Rec cur = nxt;
      const uint32_t cgid = ngid;
      const bool valid = lo + lane < hi;
      if (lo > 0) {
        const int lo2 = max(0, lo - 64);
        if (lo2 + lane < lo) {
          ngid = min(vals[s + lo2 + lane], n_gauss - 1);
          nxt = load_rec(splat, ngid);
        }
      }
      const bool hit = valid && box_meets(cur.r2.y, cur.r2.z, it);
      const uint64_t hm = __ballot(hit);
      if (hit) {
        const int pos = __popcll(hm & lanemask_lt(lane));
        L.r0[pos] = cur.r0;
        L.r1[pos] = cur.r1;
        L.bx[pos] = make_float2(cur.r2.x, __uint_as_float(cgid));
      }
      __builtin_amdgcn_wave_barrier();
      const int nhit = __popcll(hm);
      // hits in reverse order; the entry offset of hit i is the position of the i-th
      // set bit of the ballot mask
      uint64_t rem = hm;
      for (int i = nhit - 1; i >= 0; --i) {
        const int bit = 63 - __clzll((unsigned long long)rem);
        rem &= ~(1ull << bit);
        const float4 r0 = L.r0[i], r1 = L.r1[i];
        const float2 bx = L.bx[i];
        float dx, dy, ep, raw;
        const float alpha = splat_alpha(r0, r1, px, py, dx, dy, ep, raw);
        const bool contrib = lo + bit < last && alpha >= kAlphaMin;
        if (__ballot(contrib) == 0) continue;
        // T in front of this Gaussian: T_i = T_{i+1} / (1 - alpha_i)
        T = contrib ? T * __builtin_amdgcn_rcpf(1.f - alpha) : T;
        const float wgt = contrib ? alpha * T : 0.f;
        const float cb = bx.x;
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
        const float tot = reduce9(v);
        if (comp >= 0) atomicAdd(&g2d[(size_t)__float_as_uint(bx.y) * 9 + comp], tot);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  leave_queue(queue + kQueueWords, gridDim.x * kWaves, lane);
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

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus;
}

// Persistent grid: a fixed number of workgroups per CU, never more than the items need.
unsigned persistent_blocks(long long n_items, int waves_per_block, int blocks_per_cu) {
  const long long want = (long long)cu_count() * blocks_per_cu;
  const long long need = (n_items + waves_per_block - 1) / waves_per_block;
  return (unsigned)(need < want ? (need > 0 ? need : 1) : want);
}

glam_status launch_render_fwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                              const float* bg, float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval,
                              hipStream_t s) {
  if (v.n_tiles == 0 || v.n_gauss == 0) {
    // nothing to composite: background everywhere
    return launch_background(v, bg, image, T_final, n_contrib, n_eval, s);
  }
  hipLaunchKernelGGL(render_fwd_kernel, dim3(persistent_blocks(4 * v.n_tiles, kWaves, kBlocksPerCU)),
                     dim3(64 * kWaves), 0, s, proj.splat, bins.vals, bins.ranges, bins.order, bins.queue, v.dev, v.n,
                     (int)v.n_tiles, bg, image, T_final, n_contrib, n_eval, (uint32_t)bins.capacity,
                     (uint32_t)v.n_gauss);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

glam_status launch_composite_bwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                                 const float* bg, const float* T_final, const int32_t* n_contrib,
                                 const float* dimage, float* g2d, hipStream_t s) {
  const long long n = 9 * v.n_gauss;
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g2d, n);
  if (v.n_tiles > 0 && v.n_gauss > 0)
    hipLaunchKernelGGL(composite_bwd_kernel, dim3(persistent_blocks(4 * v.n_tiles, kWaves, kBlocksPerCU)),
                       dim3(64 * kWaves), 0, s, proj.splat, bins.vals, bins.ranges, bins.order, bins.queue, v.dev,
                       v.n, (int)v.n_tiles, bg, T_final, n_contrib, dimage, g2d, (uint32_t)bins.capacity,
                       (uint32_t)v.n_gauss);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
