// Front-to-back alpha compositing (Eq. 1) and its reverse-order adjoint.
//
// Work decomposition.  Gaussians are binned to square tiles (8, 16 or 32 pixels, 16 by
// default); each tile is split into 8x8 quadrants, and one wave64 composites one
// quadrant (one pixel per lane).  The (tile, quadrant) items are pulled from a device
// work queue by a persistent grid (a few workgroups per CU), in longest-range-first
// order.
//
// Per item, a wave walks its tile's depth-sorted range in batches of 64: lane l
// gathers the 48-byte record of entry b0+l from HBM (the next batch is prefetched into
// registers while the current one is composited), tests its footprint box against
// the quadrant, and the hits are compacted into a wave-private LDS buffer (ballot +
// lane-mask prefix count).  The wave then walks the hits in order; all lanes read the
// same record (LDS broadcast) and composite their own pixel.  The wave leaves as soon
// as all 64 of its pixels have stopped.
//
// Long tiles.  A few tiles near the horizon hold thousands of entries whose pixels
// never saturate; walked by one wave they would set the kernel's length.  Their
// quadrants are taken first, each by a whole workgroup (4, 8 or 16 waves, a schedule
// choice): the range is cut into the fewest rounds of at most 64 entries per wave, and
// each round into equal chunks, one per wave.  Compositing over a chunk is an affine map of
// the state in front of it -- the colour grows by T times the chunk's own colour L
// and T is scaled by the chunk's own transmittance P, both computed from T = 1 -- so
// each wave first composites its chunk locally (no stop rule), the waves exchange
// (L, P) through LDS, and every wave then knows the transmittance in front of its
// chunk.  The one chunk in which a pixel's transmittance falls below the stop
// threshold (the product crosses it there and nowhere else, since it only decreases)
// is composited again exactly, entry by entry, from that transmittance.
//
// The backward walks the same ranges from the wave's last contributor down,
// recovering T_i = T_{i+1} / (1 - alpha_i) from the stored final transmittance and
// carrying the colour behind, B <- B + alpha_i (c_i - B).  Per Gaussian, the nine
// accumulated terms (the opacity and colour gradients, and five moments of dL/dpower
// from which the projection adjoint forms the centre and conic gradients) of the
// wave's pixels are summed with a reduce-scatter (two gfx950
// lane-swap stages, then DPP within 16-lane rows) and nine lanes add the totals to HBM
// with one atomic instruction.  For long tiles the workgroup takes rounds of chunks
// from the back: each wave composites its chunk locally, and the state behind
// a chunk follows from the chunks behind it in the round (T divided by their P, B
// mapped through their affine maps B -> L + P B).  The longest tile's critical path is
// its length over the workgroup's width, which is why wide workgroups pay on single
// views, whose few horizon tiles would otherwise outlast the rest of the grid.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kIlp = 4;          // hits whose alphas a wave evaluates side by side
// Waves per SIMD the kernels are compiled for (the register budget): with workgroups
// of four waves, the most workgroups per CU the schedule may ask for; wider workgroups
// are compiled for four waves per SIMD (one workgroup of 16 or two of 8 per CU).
constexpr int kFwdWavesPerEU = kMaxFwdBlocksPerCU;
constexpr int kBwdWavesPerEU = kMaxBwdBlocksPerCU;
constexpr int kWideWavesPerEU = 4;
constexpr int kChunk = 64;       // entries per wave and round of a long tile, at most

// Rounds of a long range of n entries walked by kW waves: the fewest rounds of at most
// kChunk entries per wave, each cut into kW equal chunks (the last ones may be short or
// empty).
struct Rounds {
  int span;  // entries per round (the last round may hold fewer)
  int ch;    // entries per wave and round
};
template <int kW>
__device__ __forceinline__ Rounds long_rounds(int n) {
  const int rounds = max(1, (n + kW * kChunk - 1) / (kW * kChunk));
  const int span = (n + rounds - 1) / rounds;
  return Rounds{span, (span + kW - 1) / kW};
}

// alpha of one record at pixel centre (px, py), shared by both passes so that their
// skip and stop decisions are bit-identical.  The record holds the conic as a base-2
// exponent, (a, b, c) = -log2(e) (A/2, B, C/2): with (dx, dy) = centre - pixel,
// alpha = min(0.99, opacity 2^(a dx^2 + b dx dy + c dy^2)); ep = 2^(...) = e^power.
__device__ __forceinline__ float splat_alpha(const float4& r0, const float4& r1, float px, float py,
                                             float& dx, float& dy, float& ep, float& raw) {
  dx = r0.x - px;
  dy = r0.y - py;
  const float e2 = fmaf(dx, fmaf(r0.z, dx, r0.w * dy), (r1.x * dy) * dy);
  ep = __builtin_amdgcn_exp2f(e2);
  raw = r1.y * ep;
  return fminf(kAlphaMax, raw);
}

__device__ __forceinline__ float splat_alpha(const float4& r0, const float4& r1, float px, float py) {
  float dx, dy, ep, raw;
  return splat_alpha(r0, r1, px, py, dx, dy, ep, raw);
}

struct Item {
  int x, y;                // this lane's pixel
  bool inside;
  bool live;               // the quadrant has pixels in the image
  int qx0, qx1, qy0, qy1;  // the wave's quadrant, clipped to the image
  int W, H;
  long long pix_begin;
  long long pix;           // this lane's pixel in the batched per-pixel arrays
};

// Item of quadrant `quad` of `tile` (tiles of edge 2^tl hold 2^(tl-3) x 2^(tl-3) quadrants).
__device__ __forceinline__ Item make_item(const glam_view_info* views, int n_views, int tile, int quad, int lane,
                                          int tl) {
  Item it;
  const int v = find_view(views, n_views, tile, [](const glam_view_info& w) { return (long long)w.tile_begin; });
  const glam_view_info& vw = views[v];
  const int lt = tile - vw.tile_begin;
  const int qpr = tl - 3;  // log2 of the quadrants per tile row
  const int qx = ((lt % vw.tiles_x) << tl) + (quad & ((1 << qpr) - 1)) * 8;
  const int qy = ((lt / vw.tiles_x) << tl) + (quad >> qpr) * 8;
  it.W = vw.cam.width;
  it.H = vw.cam.height;
  it.x = qx + (lane & 7);
  it.y = qy + (lane >> 3);
  it.inside = it.x < it.W && it.y < it.H;
  it.qx0 = qx;
  it.qy0 = qy;
  it.qx1 = min(qx + 7, it.W - 1);
  it.qy1 = min(qy + 7, it.H - 1);
  it.live = it.qx0 <= it.qx1 && it.qy0 <= it.qy1;
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

// Whether the Gaussian's alpha can reach 1/255 at any pixel centre of the quadrant: the
// largest value over the centres' rectangle of the record's exponent
// Q = a dx^2 + b dx dy + c dy^2 (a negative definite form) against -log2(255 opacity).
// The form peaks (Q = 0) at the centre, so over the rectangle it is 0 when the centre is
// inside, else its largest value lies on an edge, where it is the clamped
// one-dimensional maximum.  The test runs per batch entry (one entry per lane) and keeps
// a margin, so it only drops entries whose alpha is below the threshold at every pixel
// of the quadrant: the box test passes whole footprint boxes, the ellipse inside
// can miss the quadrant.
__device__ __forceinline__ float edge_max(float a, float b, float c, float f, float lo, float hi) {
  // Q along an edge where one offset is fixed at f and the other, d, runs over [lo, hi]:
  // a f^2 + d (c d + b f), largest at d = -b f / (2 c)
  const float d = __builtin_amdgcn_fmed3f(-0.5f * b * f * __builtin_amdgcn_rcpf(c), lo, hi);
  return fmaf(a * f, f, d * fmaf(c, d, b * f));
}

__device__ __forceinline__ bool ellipse_meets(const float4& r0, const float4& r1, const Item& it) {
  const float u = r0.x, v = r0.y, a = r0.z, b = r0.w, c = r1.x;
  // offsets of the rectangle's edges from the centre
  const float lx = it.qx0 + 0.5f - u, hx = it.qx1 + 0.5f - u;
  const float ly = it.qy0 + 0.5f - v, hy = it.qy1 + 0.5f - v;
  const bool inside = lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f;
  const float q = fmaxf(fmaxf(edge_max(a, b, c, lx, ly, hy), edge_max(a, b, c, hx, ly, hy)),
                        fmaxf(edge_max(c, b, a, ly, lx, hx), edge_max(c, b, a, hy, lx, hx)));
  // opacity 2^Q >= 1/255, with a margin of 0.0073 in Q
  const float lim = -__log2f(255.f * r1.y) - 0.0073f;
  return inside || q >= lim;
}

// Work queue.  Device-scope atomics are served at the memory side, so one counter would
// serialise every grab; the longest-first tile list (after the long tiles) is dealt
// round-robin over kQueues counters (one 128-byte line each), and workgroup b pulls
// from counter b % kQueues.  Workgroups are dealt to the 8 XCDs round-robin, so all
// workgroups of one counter sit on one XCD; the quadrant items of a tile (2^ql of them:
// 1, 4 or 16 for tiles of edge 8, 16 or 32) are consecutive grabs of one counter, so the
// tile's records are fetched into that XCD's L2 once and read there 2^ql times.  An
// item is 2^ql * (tile rank) + quadrant.
// Words [0, kQueues*32) of a queue region hold the counters, word kQueues*32 the exit
// count and word kQueues*32 + 1 the counter of the long-tile items (taken by whole
// workgroups).  The last wave to leave resets all of them for the next launch.
constexpr int kQueues = 16;
constexpr int kQueueWords = kQueues * 32 + 32;
constexpr int kExitWord = kQueues * 32, kLongWord = kQueues * 32 + 1;
static_assert(2 * kQueueWords == GLAM_QUEUE_WORDS, "queue layout");

__device__ __forceinline__ uint32_t next_item(uint32_t* q, int lane, int ql) {
  const uint32_t nq = min((uint32_t)kQueues, gridDim.x);  // every counter in use has workgroups
  const uint32_t qi = blockIdx.x % nq;
  uint32_t v = 0;
  if (lane == 0) v = atomicAdd(&q[32 * qi], 1u);
  v = __builtin_amdgcn_readfirstlane(v);
  return (((v >> ql) * nq + qi) << ql) | (v & ((1u << ql) - 1u));
}

// Next long-tile item for the whole workgroup (every thread must call it).
__device__ __forceinline__ uint32_t next_long_item(uint32_t* q, uint32_t* s_item) {
  if (threadIdx.x == 0) *s_item = atomicAdd(&q[kLongWord], 1u);
  __syncthreads();
  const uint32_t v = *s_item;
  __syncthreads();
  return v;
}

__device__ __forceinline__ void leave_queue(uint32_t* q, uint32_t total_waves, int lane) {
  if (lane == 0) {
    const uint32_t n = atomicAdd(&q[kExitWord], 1u);
    if (n == total_waves - 1) {
      for (int i = 0; i < kQueues; ++i) atomicExch(&q[32 * i], 0u);
      atomicExch(&q[kLongWord], 0u);
      atomicExch(&q[kExitWord], 0u);
    }
  }
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

// Wave-private compacted batch: (u, v, a, b), (c, opacity, r, g), (b, tag as bits); the
// hits are followed by kIlp null records (opacity 0, so alpha 0), so that groups of kIlp
// hits need no tail.
struct WaveLds {
  float4 r0[64 + kIlp];
  float4 r1[64 + kIlp];
  float2 bx[64 + kIlp];
};

// Exchange of a forward long-tile round: per wave and lane, its chunk's local
// transmittance P, then (T after, weighted colour) and (last, stop entry, state).
template <int kW>
struct FwdRound {
  float p[kW][64];
  float4 a[kW][64];
  float4 b[kW][64];
};

// Exchange of a backward long-tile round, double-buffered (one barrier per round): per
// wave and lane, the chunk's local (P, L0, L1, L2).
template <int kW>
struct BwdRound {
  float4 a[2][kW][64];
};

// Gathers the records of entries [c0, c1) (absolute positions in vals, at most 64),
// one entry per lane, into registers; lanes past the end keep their old values.
__device__ __forceinline__ void fetch_batch(const float* splat, const uint32_t* vals, uint32_t c0, uint32_t c1,
                                            uint32_t n_gauss, int lane, Rec& rec, uint32_t& gid) {
  if (c0 + lane < c1) {
    gid = min(vals[c0 + lane], n_gauss - 1);
    rec = load_rec(splat, gid);
  }
}

// Compacts the hits among one gathered batch into L in entry order (bx.y takes `tag`),
// pads them with null records and returns the hit mask: bit l is the batch's entry l.
__device__ __forceinline__ uint64_t compact_hits(const Rec& cur, bool valid, float tag, const Item& it, WaveLds& L,
                                                 int lane) {
  const bool hit = valid && box_meets(cur.r2.y, cur.r2.z, it) && ellipse_meets(cur.r0, cur.r1, it);
  const uint64_t hm = __ballot(hit);
  if (hit) {
    const int pos = __popcll(hm & lanemask_lt(lane));
    L.r0[pos] = cur.r0;
    L.r1[pos] = cur.r1;
    L.bx[pos] = make_float2(cur.r2.x, tag);
  }
  if (lane < kIlp) {
    const int pos = __popcll(hm) + lane;
    L.r0[pos] = make_float4(0.f, 0.f, 0.f, 0.f);
    L.r1[pos] = make_float4(0.f, 0.f, 0.f, 0.f);
    L.bx[pos] = make_float2(0.f, 0.f);
  }
  __builtin_amdgcn_wave_barrier();
  return hm;
}

// Walks entries [c0, c1) (absolute positions in vals) front to back in batches of 64
// with a register prefetch of the next batch; the hits of each batch are compacted into
// L (tag: the entry's number, first_tag for entry c0) and on_batch(nhit) is called; it
// returns true to end the walk.
template <class OnBatch>
__device__ __forceinline__ void walk_front(const float* splat, const uint32_t* vals, uint32_t c0, uint32_t c1,
                                           int first_tag, uint32_t n_gauss, const Item& it, WaveLds& L, int lane,
                                           OnBatch on_batch) {
  if (!it.live || c0 >= c1) return;
  Rec nxt;
  uint32_t gid;
  fetch_batch(splat, vals, c0, c1, n_gauss, lane, nxt, gid);
  for (uint32_t b0 = c0; b0 < c1; b0 += 64) {
    const Rec cur = nxt;
    const bool valid = b0 + lane < c1;
    if (b0 + 64 < c1) fetch_batch(splat, vals, b0 + 64, c1, n_gauss, lane, nxt, gid);
    const int tag = first_tag + (int)(b0 - c0) + lane;
    const uint64_t hm = compact_hits(cur, valid, __int_as_float(tag), it, L, lane);
    const bool end = on_batch(__popcll(hm));
    __builtin_amdgcn_wave_barrier();
    if (end) break;
  }
}

// ---------------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------------

// Per-pixel compositing state; entries are numbered 1.. within the tile range.
struct FwdState {
  float T, C0, C1, C2;
  int last;  // entry of the last composited Gaussian (0: none)
  int stop;  // entry that stopped the walk, or the range length
  bool done;
};

// One hit, in order: the skip and stop rules of Eq. 1 on this lane's pixel (kStop: also
// record the entry that stops the walk).
template <bool kStop>
__device__ __forceinline__ void fwd_apply(FwdState& st, float alpha, const float4& r1, const float2& bx) {
  const float Tn = fmaf(-alpha, st.T, st.T);
  const bool ok = !st.done && alpha >= kAlphaMin;
  const bool halt = ok && Tn < kTMin;
  const bool take = ok && !halt;
  const float wgt = (take ? alpha : 0.f) * st.T;
  st.C0 = fmaf(r1.z, wgt, st.C0);
  st.C1 = fmaf(r1.w, wgt, st.C1);
  st.C2 = fmaf(bx.x, wgt, st.C2);
  st.T = take ? Tn : st.T;
  st.last = take ? __float_as_int(bx.y) : st.last;
  if (kStop) st.stop = halt ? __float_as_int(bx.y) : st.stop;
  st.done = st.done || halt;
}

// The exact walk of Eq. 1 over the nhit compacted hits in L (tags: entry numbers).
// Groups of kIlp hits evaluate their alphas side by side; only the updates run in
// sequence.  Returns true once every pixel has stopped.
template <bool kStop>
__device__ __forceinline__ bool fwd_exact_hits(const WaveLds& L, int nhit, float px, float py, FwdState& st) {
  for (int i = 0; i < nhit; i += kIlp) {
    float4 r1[kIlp];
    float2 bx[kIlp];
    float alpha[kIlp];
#pragma unroll
    for (int k = 0; k < kIlp; ++k) {
      r1[k] = L.r1[i + k];
      bx[k] = L.bx[i + k];
      alpha[k] = splat_alpha(L.r0[i + k], r1[k], px, py);
    }
#pragma unroll
    for (int k = 0; k < kIlp; ++k) fwd_apply<kStop>(st, alpha[k], r1[k], bx[k]);
    if (__ballot(!st.done) == 0) return true;
  }
  return false;
}

// The exact walk of Eq. 1 over entries [c0, c1) of the range starting at s.
template <bool kStop>
__device__ void fwd_exact(const float* splat, const uint32_t* vals, uint32_t s, uint32_t c0, uint32_t c1,
                          uint32_t n_gauss, const Item& it, WaveLds& L, int lane, float px, float py, FwdState& st) {
  if (__ballot(!st.done) == 0) return;
  walk_front(splat, vals, c0, c1, (int)(c0 - s) + 1, n_gauss, it, L, lane,
             [&](int nhit) { return fwd_exact_hits<kStop>(L, nhit, px, py, st); });
}

// Local compositing of the nhit compacted hits in L (tags: entry numbers) from T = 1
// without the stop rule (pixels with `dead` set take no part): the chunk's own colour
// L, transmittance P and last composited entry.
__device__ __forceinline__ void fwd_local_hits(const WaveLds& L, int nhit, float px, float py, bool dead, float& P,
                                               float& L0, float& L1, float& L2, int& last) {
  P = 1.f;
  L0 = L1 = L2 = 0.f;
  last = 0;
  for (int i = 0; i < nhit; i += kIlp) {
    float4 r1[kIlp];
    float2 bx[kIlp];
    float alpha[kIlp];
#pragma unroll
    for (int k = 0; k < kIlp; ++k) {
      r1[k] = L.r1[i + k];
      bx[k] = L.bx[i + k];
      alpha[k] = splat_alpha(L.r0[i + k], r1[k], px, py);
    }
#pragma unroll
    for (int k = 0; k < kIlp; ++k) {
      const bool take = !dead && alpha[k] >= kAlphaMin;
      const float wgt = (take ? alpha[k] : 0.f) * P;
      L0 = fmaf(r1[k].z, wgt, L0);
      L1 = fmaf(r1[k].w, wgt, L1);
      L2 = fmaf(bx[k].x, wgt, L2);
      P = take ? fmaf(-alpha[k], P, P) : P;
      last = take ? __float_as_int(bx[k].y) : last;
    }
  }
}

__device__ __forceinline__ void fwd_write(const Item& it, const FwdState& st, const float* bgc, float* image,
                                          float* T_final, int32_t* n_contrib, int32_t* n_eval) {
  if (!it.inside) return;
  const long long HW = (long long)it.W * it.H;
  const long long p = (long long)it.y * it.W + it.x;
  float* img = image + 3 * it.pix_begin;
  img[p] = fmaf(st.T, bgc[0], st.C0);
  img[HW + p] = fmaf(st.T, bgc[1], st.C1);
  img[2 * HW + p] = fmaf(st.T, bgc[2], st.C2);
  T_final[it.pix] = st.T;
  n_contrib[it.pix] = st.last;
  if (n_eval) n_eval[it.pix] = st.stop;
}

// A long tile's quadrant, composited by the whole workgroup in rounds of kW chunks.
// A chunk is one gathered batch: its hits stay in L for the exact pass, and the next
// round's records are fetched while the current round is composited.
static_assert(kChunk == 64, "a long-tile chunk is one gathered batch");
// Returns the pixel's final state (the same in every wave).
template <bool kStop, int kW>
__device__ FwdState fwd_long(const float* splat, const uint32_t* vals, uint32_t s, uint32_t e, uint32_t n_gauss,
                         const Item& it, WaveLds& L, FwdRound<kW>& R, int w, int lane, const float* bgc,
                         float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval) {
  const float px = it.x + 0.5f, py = it.y + 0.5f;
  const int n = (int)(e - s);
  const Rounds rd = long_rounds<kW>(n);
  FwdState st{1.f, 0.f, 0.f, 0.f, 0, n, !it.inside};
  Rec nxt;
  uint32_t gid;
  {
    const int c0 = min(rd.span, w * rd.ch);
    fetch_batch(splat, vals, s + c0, s + min(c0 + rd.ch, rd.span), n_gauss, lane, nxt, gid);
  }
  for (int r0 = 0; r0 < n; r0 += rd.span) {
    const int r1 = min(n, r0 + rd.span);
    const int c0 = min(r1, r0 + w * rd.ch), c1 = min(r1, c0 + rd.ch);
    const Rec cur = nxt;
    if (r1 < n) {
      const int q1 = min(n, r1 + rd.span);
      const int n0 = min(q1, r1 + w * rd.ch);
      fetch_batch(splat, vals, s + n0, s + min(q1, n0 + rd.ch), n_gauss, lane, nxt, gid);
    }
    // 1. this wave's chunk, locally (st.done is the same in every wave)
    const int tag = c0 + 1 + lane;  // entry number
    const uint64_t hm = __ballot(!st.done) ? compact_hits(cur, c0 + lane < c1, __int_as_float(tag), it, L, lane) : 0ull;
    const int nhit = __popcll(hm);
    float P, L0, L1, L2;
    int llast;
    fwd_local_hits(L, nhit, px, py, st.done, P, L0, L1, L2, llast);
    R.p[w][lane] = P;
    __syncthreads();
    // 2. transmittance in front of the chunk; the chunk where the pixel stops is redone
    //    exactly from it
    float Tin = st.T;
    bool before = st.done;
    for (int j = 0; j < w; ++j) {
      const float Pj = R.p[j][lane];
      if (!before) {
        if (Tin * Pj < kTMin) before = true;
        else Tin *= Pj;
      }
    }
    const bool here = !before && Tin * P < kTMin;
    FwdState ex{Tin, 0.f, 0.f, 0.f, 0, n, !here};
    if (__ballot(here)) fwd_exact_hits<kStop>(L, nhit, px, py, ex);
    const int state = before ? 0 : (here ? 2 : 1);
    R.a[w][lane] = here ? make_float4(ex.T, ex.C0, ex.C1, ex.C2) : make_float4(Tin * P, Tin * L0, Tin * L1, Tin * L2);
    R.b[w][lane] = make_float4(__int_as_float(here ? ex.last : llast), __int_as_float(here ? ex.stop : n),
                               __int_as_float(state), 0.f);
    __syncthreads();
    // 3. every wave merges the round's chunks in order (identically).  The next round
    //    writes p only after this barrier, and a and b only after its first one, which
    //    every wave reaches after this merge.
    for (int j = 0; j < kW; ++j) {
      const float4 bj = R.b[j][lane];
      const int sj = __float_as_int(bj.z);
      if (sj == 0) continue;
      const float4 aj = R.a[j][lane];
      st.T = aj.x;
      st.C0 += aj.y;
      st.C1 += aj.z;
      st.C2 += aj.w;
      const int lj = __float_as_int(bj.x);
      st.last = lj > 0 ? lj : st.last;
      if (sj == 2) {
        st.stop = __float_as_int(bj.y);
        st.done = true;
      }
    }
    if (__ballot(!st.done) == 0) break;  // the same decision in every wave
  }
  if (w == 0) fwd_write(it, st, bgc, image, T_final, n_contrib, n_eval);
  return st;
}

// kCount: also record per pixel the entry that stopped the walk (n_eval).
template <bool kCount, int kW>
__global__ void __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(kW == 4 ? kFwdWavesPerEU
                                                                                      : kWideWavesPerEU)))
render_fwd_kernel(const float* __restrict__ splat, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, const int32_t* status,
                  uint32_t* queue, const glam_view_info* views, int n_views, int n_tiles, int tl,
                  const float* bg, float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval,
                  uint32_t capacity, uint32_t n_gauss, int direct) {
  __shared__ WaveLds lds[kW];
  __shared__ FwdRound<kW> round;
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  WaveLds& L = lds[w];
  const float bgc[3] = {bg ? bg[0] : 0.f, bg ? bg[1] : 0.f, bg ? bg[2] : 0.f};
  const uint32_t n_long = min((uint32_t)status[7], (uint32_t)n_tiles);
  const int ql = 2 * (tl - 3);  // log2 of the quadrants per tile
  if (direct) {  // no queue: wave w of workgroup b takes item kW b + w in tile order, whole range
    const uint32_t item = blockIdx.x * kW + w;
    if (item < ((uint32_t)n_tiles << ql)) {
      const int tile = (int)(item >> ql);
      const Item it = make_item(views, n_views, tile, (int)(item & ((1u << ql) - 1u)), lane, tl);
      const uint32_t e = min(ranges[2 * tile + 1], capacity);
      const uint32_t s = min(ranges[2 * tile], e);
      FwdState st{1.f, 0.f, 0.f, 0.f, 0, (int)(e - s), !it.inside};
      fwd_exact<kCount>(splat, vals, s, s, e, n_gauss, it, L, lane, it.x + 0.5f, it.y + 0.5f, st);
      fwd_write(it, st, bgc, image, T_final, n_contrib, n_eval);
    }
    return;
  }
  // long tiles first, one quadrant per workgroup
  __builtin_amdgcn_s_setprio(2);
  for (uint32_t li = next_long_item(queue, &s_item); li < (n_long << ql); li = next_long_item(queue, &s_item)) {
    const int tile = (int)min(order[li >> ql], (uint32_t)n_tiles - 1);
    const Item it = make_item(views, n_views, tile, (int)(li & ((1u << ql) - 1u)), lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    fwd_long<kCount, kW>(splat, vals, s, e, n_gauss, it, L, round, w, lane, bgc, image, T_final, n_contrib, n_eval);
  }
  __builtin_amdgcn_s_setprio(0);
  // the other tiles, one quadrant per wave
  const uint32_t n_items = ((uint32_t)n_tiles - n_long) << ql;
  for (uint32_t item = next_item(queue, lane, ql); item < n_items; item = next_item(queue, lane, ql)) {
    const int tile = (int)min(order[n_long + (item >> ql)], (uint32_t)n_tiles - 1);
    const Item it = make_item(views, n_views, tile, (int)(item & ((1u << ql) - 1u)), lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    FwdState st{1.f, 0.f, 0.f, 0.f, 0, (int)(e - s), !it.inside};
    fwd_exact<kCount>(splat, vals, s, s, e, n_gauss, it, L, lane, it.x + 0.5f, it.y + 0.5f, st);
    fwd_write(it, st, bgc, image, T_final, n_contrib, n_eval);
  }
  leave_queue(queue, gridDim.x * kW, lane);
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
// Per-Gaussian reduction of the nine gradient terms, split in two.  Per hit, two
// lane-swap stages fold the nine per-lane values to partial sums over four lanes: each
// of x0 and x1 then holds four components, one per 16-lane row, and x2 the ninth in
// its first row.  Those 144 words go to a wave-private LDS slot with the Gaussian's
// index.  Every kFlush hits one flush sums each (hit, component) row of 16 words in its
// own lane and issues all their atomics with one instruction: the per-hit DPP folding
// and its wait states are replaced by one LDS store per register.
constexpr int kFlush = 4;         // hits staged per flush (9 kFlush lanes flush)
// x0, x1 and x2 (64 lanes each; only x2's first row is read), padded by four words so
// that the flush's 16-byte reads of the kFlush slots spread over all 64 banks (three
// passes per read instead of twelve)
constexpr int kStageWords = 196;
struct GradStage {
  float v[kFlush][kStageWords];
  uint32_t gid[kFlush];
};
static_assert(9 * kFlush <= 64, "one flush lane per (hit, component)");

// Offset in a slot of the row holding component lane % 9 after the swap stages: the
// stages are applied to component tags (the swaps move whole rows or half-waves, so a
// row holds one component), and the row whose tag matches is looked up.
__device__ __forceinline__ int stage_offset(int lane) {
  const uint32_t none = 0xffffffffu, c = (uint32_t)(lane % 9);
  const uint32_t x0 = swap16_first(swap32_first(0, 1), swap32_first(2, 3));
  const uint32_t x1 = swap16_first(swap32_first(4, 5), swap32_first(6, 7));
  const uint32_t x2 = swap16_first(swap32_first(8, none), none);
  int off = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if ((uint32_t)__builtin_amdgcn_readlane((int)x0, 16 * r) == c) off = 16 * r;
    if ((uint32_t)__builtin_amdgcn_readlane((int)x1, 16 * r) == c) off = 64 + 16 * r;
  }
  if ((uint32_t)__builtin_amdgcn_readlane((int)x2, 0) == c) off = 128;
  return off;
}

// Sums the n staged hits (lane 9 h + c: component c of hit h) and adds them to the
// Gaussian's nine words with one atomic instruction, or (kDet) stores them to the
// hit's own partial slot, whose index the hit carries in place of the Gaussian's.  The
// wave must be fully active.
template <bool kDet>
__device__ __forceinline__ void stage_flush(GradStage& G, int n, int off, int lane, float* g2d) {
  __builtin_amdgcn_wave_barrier();
  const int h = lane / 9, c = lane - 9 * (lane / 9);
  if (h < n) {
    const float4* p = reinterpret_cast<const float4*>(&G.v[h][off]);
    const float4 a = p[0], b = p[1], d = p[2], e = p[3];
    const float sum = (((a.x + a.y) + (a.z + a.w)) + ((b.x + b.y) + (b.z + b.w))) +
                      (((d.x + d.y) + (d.z + d.w)) + ((e.x + e.y) + (e.z + e.w)));
    if (kDet)
      g2d[(size_t)G.gid[h] * 9 + c] = sum;
    else
      atomicAdd(&g2d[(size_t)G.gid[h] * 9 + c], sum);
  }
  __builtin_amdgcn_wave_barrier();
}

// Stages one hit's nine per-lane values (a fully active wave); flushes when full.
template <bool kDet>
__device__ __forceinline__ void stage_hit(const float v[9], uint32_t gid, GradStage& G, int& nst, int off, int lane,
                                          float* g2d) {
  const float w0 = swap32_sum(v[0], v[1]), w1 = swap32_sum(v[2], v[3]), w2 = swap32_sum(v[4], v[5]),
              w3 = swap32_sum(v[6], v[7]), w4 = swap32_sum(v[8], 0.f);
  const float x0 = swap16_sum(w0, w1), x1 = swap16_sum(w2, w3), x2 = swap16_sum(w4, 0.f);
  float* sl = G.v[nst];
  sl[lane] = x0;
  sl[64 + lane] = x1;
  sl[128 + lane] = x2;
  G.gid[nst] = gid;  // the same value from every lane
  if (++nst == kFlush) {
    stage_flush<kDet>(G, kFlush, off, lane, g2d);
    nst = 0;
  }
}

// The partial slot of one (range entry, quadrant) of the reproducible backward: the
// entry's Gaussian gid took its pairs at [pair_begin[gid], pair_begin[gid] + ntiles),
// one per tile of its box, row-major; this item's tile (tx, ty) picks one, and the
// quadrant's index within the tile (2^ql of them) the slot within the pair.
__device__ __forceinline__ uint32_t det_slot(const Rec& r, uint32_t gid, const uint32_t* pair_begin, int tx, int ty,
                                             int tl, int ql, int quad) {
  const uint32_t bx = __float_as_uint(r.r2.y), by = __float_as_uint(r.r2.z);
  const int tx0 = (int)(bx & 0xffffu) >> tl, tx1 = (int)(bx >> 16) >> tl, ty0 = (int)(by & 0xffffu) >> tl;
  const uint32_t pair = pair_begin[gid] + (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
  return (pair << ql) | (uint32_t)quad;
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

// Per-pixel state of the backward walk: transmittance in front of the current entry,
// colour behind it, dL/dC and the pixel's last composited entry.
struct BwdState {
  float T, B0, B1, B2;
  float g0, g1, g2;
  int last;
};

// The hits of one batch (mask hm over the batch's entries, the first at range offset
// lo; compacted into L with the Gaussian's index as tag) in reverse order: per hit
// T_i = T_{i+1} / (1 - alpha_i), the nine gradient terms, one reduction and one atomic
// per Gaussian, then the colour behind.
template <bool kDet>
__device__ __forceinline__ void bwd_hits(const WaveLds& L, uint64_t hm, int lo, float px, float py, int lane,
                                         GradStage& G, int& nst, int off, BwdState& st, float* g2d) {
  const int nhit = __popcll(hm);
  // the entry offset of hit i is the position of the i-th set bit of the mask
  uint64_t rem = hm;
  for (int i = nhit - 1; i >= 0; --i) {
    const int bit = 63 - __clzll((unsigned long long)rem);
    rem &= ~(1ull << bit);
    const float4 r0 = L.r0[i], r1 = L.r1[i];
    const float2 bx = L.bx[i];
    float dx, dy, ep, raw;
    const float alpha = splat_alpha(r0, r1, px, py, dx, dy, ep, raw);
    const bool contrib = lo + bit < st.last && alpha >= kAlphaMin;
    if (__ballot(contrib) == 0) continue;
    // T in front of this Gaussian: T_i = T_{i+1} / (1 - alpha_i)
    const float Tc = st.T * __builtin_amdgcn_rcpf(1.f - alpha);
    st.T = contrib ? Tc : st.T;
    const float aB = contrib ? alpha : 0.f;
    const float wgt = aB * st.T;  // alpha_i T_i, 0 off the contributors
    const float d0 = r1.z - st.B0, d1 = r1.w - st.B1, d2 = bx.x - st.B2;
    const float dal = st.T * fmaf(st.g0, d0, fmaf(st.g1, d1, st.g2 * d2));
    st.B0 = fmaf(aB, d0, st.B0);
    st.B1 = fmaf(aB, d1, st.B1);
    st.B2 = fmaf(aB, d2, st.B2);
    // dL/dalpha where alpha is not clamped (there it depends on its inputs)
    const float df = contrib && raw <= kAlphaMax ? dal : 0.f;
    const float dp = df * alpha;
    float v[9];
    // moments of dL/dpower; the projection adjoint applies the conic
    v[0] = dp * dx;
    v[1] = dp * dy;
    v[2] = v[0] * dx;
    v[3] = v[0] * dy;
    v[4] = v[1] * dy;
    v[5] = df * ep;
    v[6] = st.g0 * wgt;
    v[7] = st.g1 * wgt;
    v[8] = st.g2 * wgt;
    stage_hit<kDet>(v, __float_as_uint(bx.y), G, nst, off, lane, g2d);
  }
}

// What the reproducible backward needs to name a hit's partial slot (see det_slot).
struct DetCtx {
  const uint32_t* pair_begin;
  int tx, ty, tl, ql, quad;
};

// The compaction tag of a gathered entry: its Gaussian, or (kDet) its partial slot.
template <bool kDet>
__device__ __forceinline__ float hit_tag(const Rec& r, uint32_t gid, const DetCtx& dc, bool valid) {
  if (!kDet) return __uint_as_float(gid);
  return __uint_as_float(valid ? det_slot(r, gid, dc.pair_begin, dc.tx, dc.ty, dc.tl, dc.ql, dc.quad) : 0u);
}

// The reverse walk over range offsets [lo_end, hi) (from hi - 1 down), relative to the
// range start s, in batches of 64 with a register prefetch of the next batch.
template <bool kDet>
__device__ void bwd_walk(const float* splat, const uint32_t* vals, uint32_t s, int lo_end, int hi, uint32_t n_gauss,
                         const Item& it, WaveLds& L, int lane, GradStage& G, int& nst, int off, BwdState& st,
                         float* g2d, const DetCtx& dc) {
  if (!it.live || hi <= lo_end) return;
  const float px = it.x + 0.5f, py = it.y + 0.5f;
  Rec nxt;
  uint32_t ngid = 0;
  fetch_batch(splat, vals, s + max(lo_end, hi - 64), s + hi, n_gauss, lane, nxt, ngid);
  for (int bh = hi; bh > lo_end; bh -= 64) {
    const int lo = max(lo_end, bh - 64);
    const Rec cur = nxt;
    const uint32_t cgid = ngid;
    if (lo > lo_end) fetch_batch(splat, vals, s + max(lo_end, lo - 64), s + lo, n_gauss, lane, nxt, ngid);
    const bool valid = lo + lane < bh;
    const uint64_t hm = compact_hits(cur, valid, hit_tag<kDet>(cur, cgid, dc, valid), it, L, lane);
    bwd_hits<kDet>(L, hm, lo, px, py, lane, G, nst, off, st, g2d);
    __builtin_amdgcn_wave_barrier();
  }
}

// Local front-to-back compositing of one batch's hits (mask hm, the first entry at
// range offset lo, compacted in L) over the pixel's composited entries (offset < last,
// alpha >= 1/255): the batch's own colour L and transmittance P.
__device__ __forceinline__ void bwd_local_hits(const WaveLds& L, uint64_t hm, int lo, int last, float px, float py,
                                               float& P, float& L0, float& L1, float& L2) {
  P = 1.f;
  L0 = L1 = L2 = 0.f;
  const int nhit = __popcll(hm);
  uint64_t rem = hm;
  for (int i = 0; i < nhit; i += kIlp) {
    float4 r1[kIlp];
    float2 bx[kIlp];
    float alpha[kIlp];
    int off[kIlp];
#pragma unroll
    for (int k = 0; k < kIlp; ++k) {
      r1[k] = L.r1[i + k];
      bx[k] = L.bx[i + k];
      alpha[k] = splat_alpha(L.r0[i + k], r1[k], px, py);  // 0 on the null records
      off[k] = rem ? __builtin_ctzll(rem) : 0;  // offset of hit i + k (unused past the last hit)
      rem &= rem - 1;
    }
#pragma unroll
    for (int k = 0; k < kIlp; ++k) {
      const bool take = lo + off[k] < last && alpha[k] >= kAlphaMin;
      const float wgt = (take ? alpha[k] : 0.f) * P;
      L0 = fmaf(r1[k].z, wgt, L0);
      L1 = fmaf(r1[k].w, wgt, L1);
      L2 = fmaf(bx[k].x, wgt, L2);
      P = take ? fmaf(-alpha[k], P, P) : P;
    }
  }
}

__device__ __forceinline__ BwdState bwd_begin(const Item& it, uint32_t n, const float* bgc, const float* T_final,
                                              const int32_t* n_contrib, const float* dimage) {
  BwdState st{1.f, bgc[0], bgc[1], bgc[2], 0.f, 0.f, 0.f, 0};
  if (it.inside) {
    const long long HW = (long long)it.W * it.H;
    const long long p = (long long)it.y * it.W + it.x;
    const float* di = dimage + 3 * it.pix_begin;
    st.T = T_final[it.pix];
    st.last = min(n_contrib[it.pix], (int32_t)n);
    st.g0 = di[p];
    st.g1 = di[HW + p];
    st.g2 = di[2 * HW + p];
  }
  return st;
}

// A long tile's quadrant, by the whole workgroup in rounds of kW chunks from the back.
// A chunk is one gathered batch, compacted once for both passes; the next round's
// records are fetched while the current round is walked.
template <bool kDet, int kW>
__device__ void bwd_long(const float* splat, const uint32_t* vals, uint32_t s, uint32_t n_gauss, const Item& it,
                         WaveLds& L, BwdRound<kW>& R, int w, int lane, GradStage& G, int& nst, int off, BwdState st,
                         float* g2d, const DetCtx& dc) {
  const float px = it.x + 0.5f, py = it.y + 0.5f;
  const int top = it.live ? wave_max(st.last) : 0;  // the same in every wave
  const Rounds rd = long_rounds<kW>(top);
  Rec nxt;
  uint32_t ngid = 0;
  {
    const int lo = max(0, top - rd.span), c1 = max(lo, top - w * rd.ch);
    fetch_batch(splat, vals, s + max(lo, c1 - rd.ch), s + c1, n_gauss, lane, nxt, ngid);
  }
  int buf = 0;
  for (int hi = top; hi > 0; hi -= rd.span, buf ^= 1) {
    const int lo = max(0, hi - rd.span);
    const int c1 = max(lo, hi - w * rd.ch), c0 = max(lo, c1 - rd.ch);
    const Rec cur = nxt;
    const uint32_t cgid = ngid;
    if (lo > 0) {
      const int nlo = max(0, lo - rd.span), n1 = max(nlo, lo - w * rd.ch);
      fetch_batch(splat, vals, s + max(nlo, n1 - rd.ch), s + n1, n_gauss, lane, nxt, ngid);
    }
    const bool valid = c0 + lane < c1;
    const uint64_t hm = compact_hits(cur, valid, hit_tag<kDet>(cur, cgid, dc, valid), it, L, lane);
    float P, L0, L1, L2;
    bwd_local_hits(L, hm, c0, st.last, px, py, P, L0, L1, L2);
    R.a[buf][w][lane] = make_float4(P, L0, L1, L2);
    // One barrier per round: the buffer written here is next written two rounds on,
    // after the next round's barrier, which every wave reaches after reading this one.
    __syncthreads();
    // state behind this wave's chunk, from the chunks behind it in the round
    BwdState cs = st;
    for (int j = 0; j < w; ++j) {
      const float4 pj = R.a[buf][j][lane];
      cs.T = cs.T / pj.x;
      cs.B0 = fmaf(pj.x, cs.B0, pj.y);
      cs.B1 = fmaf(pj.x, cs.B1, pj.z);
      cs.B2 = fmaf(pj.x, cs.B2, pj.w);
    }
    bwd_hits<kDet>(L, hm, c0, px, py, lane, G, nst, off, cs, g2d);
    // state in front of the round (identical in every wave)
    for (int j = 0; j < kW; ++j) {
      const float4 pj = R.a[buf][j][lane];
      st.T = st.T / pj.x;
      st.B0 = fmaf(pj.x, st.B0, pj.y);
      st.B1 = fmaf(pj.x, st.B1, pj.z);
      st.B2 = fmaf(pj.x, st.B2, pj.w);
    }
  }
  // the workgroup's next item rewrites the exchange buffers only after the barrier in
  // next_long_item, which every wave reaches after its last read here
}

// kDet: g2d is the partial buffer of the reproducible backward ([pairs << ql][9], zeroed
// by the caller), each (range entry, quadrant) hit storing its own nine sums there.
template <bool kDet, int kW>
__global__ void __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(kW == 4 ? kBwdWavesPerEU
                                                                                      : kWideWavesPerEU)))
composite_bwd_kernel(
    const float* __restrict__ splat, const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ order, const int32_t* status, uint32_t* queue, const glam_view_info* views,
    int n_views, int n_tiles, int tl, const float* bg, const float* T_final, const int32_t* n_contrib,
    const float* dimage, float* g2d, uint32_t capacity, uint32_t n_gauss, const uint32_t* pair_begin, int direct) {
  __shared__ WaveLds lds[kW];
  __shared__ BwdRound<kW> round;
  __shared__ GradStage stage[kW];
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  WaveLds& L = lds[w];
  GradStage& G = stage[w];
  const int off = stage_offset(lane);
  int nst = 0;  // staged hits of this wave (uniform)
  const float bgc[3] = {bg ? bg[0] : 0.f, bg ? bg[1] : 0.f, bg ? bg[2] : 0.f};
  const uint32_t n_long = min((uint32_t)status[7], (uint32_t)n_tiles);
  uint32_t* q = queue + kQueueWords;
  const int ql = 2 * (tl - 3);  // log2 of the quadrants per tile
  if (direct) {  // no queue: wave w of workgroup b takes item kW b + w in tile order, whole range
    const uint32_t item = blockIdx.x * kW + w;
    if (item < ((uint32_t)n_tiles << ql)) {
      const int tile = (int)(item >> ql);
      const int quad = (int)(item & ((1u << ql) - 1u));
      const Item it = make_item(views, n_views, tile, quad, lane, tl);
      const uint32_t e = min(ranges[2 * tile + 1], capacity);
      const uint32_t s = min(ranges[2 * tile], e);
      BwdState st = bwd_begin(it, e - s, bgc, T_final, n_contrib, dimage);
      const int top = it.live ? wave_max(st.last) : 0;
      const DetCtx dc{pair_begin, it.qx0 >> tl, it.qy0 >> tl, tl, ql, quad};
      bwd_walk<kDet>(splat, vals, s, 0, top, n_gauss, it, L, lane, G, nst, off, st, g2d, dc);
    }
    stage_flush<kDet>(G, nst, off, lane, g2d);
    return;
  }
  __builtin_amdgcn_s_setprio(2);
  for (uint32_t li = next_long_item(q, &s_item); li < (n_long << ql); li = next_long_item(q, &s_item)) {
    const int tile = (int)min(order[li >> ql], (uint32_t)n_tiles - 1);
    const int quad = (int)(li & ((1u << ql) - 1u));
    const Item it = make_item(views, n_views, tile, quad, lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    const DetCtx dc{pair_begin, it.qx0 >> tl, it.qy0 >> tl, tl, ql, quad};
    bwd_long<kDet, kW>(splat, vals, s, n_gauss, it, L, round, w, lane, G, nst, off,
                   bwd_begin(it, e - s, bgc, T_final, n_contrib, dimage), g2d, dc);
  }
  __builtin_amdgcn_s_setprio(0);
  const uint32_t n_items = ((uint32_t)n_tiles - n_long) << ql;
  for (uint32_t item = next_item(q, lane, ql); item < n_items; item = next_item(q, lane, ql)) {
    const int tile = (int)min(order[n_long + (item >> ql)], (uint32_t)n_tiles - 1);
    const int quad = (int)(item & ((1u << ql) - 1u));
    const Item it = make_item(views, n_views, tile, quad, lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    BwdState st = bwd_begin(it, e - s, bgc, T_final, n_contrib, dimage);
    const int top = it.live ? wave_max(st.last) : 0;
    const DetCtx dc{pair_begin, it.qx0 >> tl, it.qy0 >> tl, tl, ql, quad};
    bwd_walk<kDet>(splat, vals, s, 0, top, n_gauss, it, L, lane, G, nst, off, st, g2d, dc);
  }
  stage_flush<kDet>(G, nst, off, lane, g2d);
  leave_queue(q, gridDim.x * kW, lane);
}

// ---------------------------------------------------------------------------------
// forward, L1 loss and adjoint in one pass (a per-pixel loss)
// ---------------------------------------------------------------------------------

__device__ __forceinline__ float l1_sign(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// The L1 term of Eq. 3 at this lane's pixel, from its composited state: |C - target|
// summed over the channels (returned), dL/dC = sign(C - target) / (3 W H) into dimage
// (when given) and the adjoint's starting state (T_final, background, dL/dC, last
// composited entry), as the loss kernel and the backward's set-up would give them.
__device__ __forceinline__ float l1_start(const Item& it, const FwdState& st, const float* bgc, const float* target,
                                          float* dimage, BwdState& b) {
  b = BwdState{st.T, bgc[0], bgc[1], bgc[2], 0.f, 0.f, 0.f, st.last};
  if (!it.inside) return 0.f;
  const long long HW = (long long)it.W * it.H;
  const long long p = (long long)it.y * it.W + it.x;
  const float* tg = target + 3 * it.pix_begin;
  const float inv_n = 1.f / (float)(3 * HW);
  const float d0 = fmaf(st.T, bgc[0], st.C0) - tg[p];
  const float d1 = fmaf(st.T, bgc[1], st.C1) - tg[HW + p];
  const float d2 = fmaf(st.T, bgc[2], st.C2) - tg[2 * HW + p];
  b.g0 = l1_sign(d0) * inv_n;
  b.g1 = l1_sign(d1) * inv_n;
  b.g2 = l1_sign(d2) * inv_n;
  if (dimage) {
    float* di = dimage + 3 * it.pix_begin;
    di[p] = b.g0;
    di[HW + p] = b.g1;
    di[2 * HW + p] = b.g2;
  }
  return fabsf(d0) + fabsf(d1) + fabsf(d2);
}

// Exchange buffers of a long item: the forward's, then (after a barrier) the backward's.
template <int kW>
union FusedRound {
  FwdRound<kW> f;
  BwdRound<kW> b;
};

// Per quadrant item: the forward of Eq. 1 (as render_fwd_kernel), the pixels' L1 terms
// and dL/dC, then at once the reverse walk of the adjoint (as composite_bwd_kernel) over
// the records the forward has just gathered.  l1_part[(tile << ql) | quadrant] takes the
// item's sum of |C - target|.
template <int kW>
__global__ void __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(kW == 4 ? kBwdWavesPerEU
                                                                                      : kWideWavesPerEU)))
fused_l1_kernel(const float* __restrict__ splat, const uint32_t* __restrict__ vals,
                const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, const int32_t* status,
                uint32_t* queue, const glam_view_info* views, int n_views, int n_tiles, int tl, const float* bg,
                const float* target, float* image, float* T_final, int32_t* n_contrib, float* dimage, float* g2d,
                float* l1_part, uint32_t capacity, uint32_t n_gauss) {
  __shared__ WaveLds lds[kW];
  __shared__ FusedRound<kW> round;
  __shared__ GradStage stage[kW];
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  WaveLds& L = lds[w];
  GradStage& G = stage[w];
  const int off = stage_offset(lane);
  int nst = 0;
  const float bgc[3] = {bg ? bg[0] : 0.f, bg ? bg[1] : 0.f, bg ? bg[2] : 0.f};
  const uint32_t n_long = min((uint32_t)status[7], (uint32_t)n_tiles);
  const int ql = 2 * (tl - 3);
  const DetCtx dc{nullptr, 0, 0, tl, ql, 0};  // floating-point atomics: no partial slots
  __builtin_amdgcn_s_setprio(2);
  for (uint32_t li = next_long_item(queue, &s_item); li < (n_long << ql); li = next_long_item(queue, &s_item)) {
    const int tile = (int)min(order[li >> ql], (uint32_t)n_tiles - 1);
    const int quad = (int)(li & ((1u << ql) - 1u));
    const Item it = make_item(views, n_views, tile, quad, lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    const FwdState fs =
        fwd_long<false, kW>(splat, vals, s, e, n_gauss, it, L, round.f, w, lane, bgc, image, T_final, n_contrib,
                            nullptr);
    BwdState bs;
    const float l1 = wave_sum(l1_start(it, fs, bgc, target, w == 0 ? dimage : nullptr, bs));
    if (w == 0 && lane == 0) l1_part[((size_t)tile << ql) | (size_t)quad] = l1;
    __syncthreads();  // every wave has read the forward's exchange: the backward's may overwrite it
    bwd_long<false, kW>(splat, vals, s, n_gauss, it, L, round.b, w, lane, G, nst, off, bs, g2d, dc);
  }
  __builtin_amdgcn_s_setprio(0);
  const uint32_t n_items = ((uint32_t)n_tiles - n_long) << ql;
  for (uint32_t item = next_item(queue, lane, ql); item < n_items; item = next_item(queue, lane, ql)) {
    const int tile = (int)min(order[n_long + (item >> ql)], (uint32_t)n_tiles - 1);
    const int quad = (int)(item & ((1u << ql) - 1u));
    const Item it = make_item(views, n_views, tile, quad, lane, tl);
    const uint32_t e = min(ranges[2 * tile + 1], capacity);
    const uint32_t s = min(ranges[2 * tile], e);
    FwdState st{1.f, 0.f, 0.f, 0.f, 0, (int)(e - s), !it.inside};
    fwd_exact<false>(splat, vals, s, s, e, n_gauss, it, L, lane, it.x + 0.5f, it.y + 0.5f, st);
    fwd_write(it, st, bgc, image, T_final, n_contrib, nullptr);
    BwdState bs;
    const float l1 = wave_sum(l1_start(it, st, bgc, target, dimage, bs));
    if (lane == 0) l1_part[((size_t)tile << ql) | (size_t)quad] = l1;
    const int top = it.live ? wave_max(bs.last) : 0;
    bwd_walk<false>(splat, vals, s, 0, top, n_gauss, it, L, lane, G, nst, off, bs, g2d, dc);
  }
  stage_flush<false>(G, nst, off, lane, g2d);
  leave_queue(queue, gridDim.x * kW, lane);
}

// The reproducible backward's segmented reduction: view-Gaussian g's nine sums are its
// partials [pair_begin[g] << ql, (pair_begin[g] + ntiles[g]) << ql) added in that order
// (tiles row-major, then quadrants).
__global__ void __launch_bounds__(256) det_reduce_kernel(const float* __restrict__ part,
                                                         const uint32_t* __restrict__ pair_begin,
                                                         const int32_t* __restrict__ ntiles, long long n_gauss,
                                                         int ql, uint32_t capacity, float* g2d) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_gauss) return;
  float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int nt = ntiles[g];
  if (nt > 0) {
    const uint32_t b = pair_begin[g];
    const uint32_t e = min(b + (uint32_t)nt, capacity);
    for (size_t k = (size_t)b << ql; k < ((size_t)max(b, e) << ql); ++k) {
      const float* p = part + k * 9;
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] += p[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) g2d[g * 9 + c] = acc[c];
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

// Zero fill with 16-byte stores (the head up to 16-byte alignment and the tail scalar).
__global__ void __launch_bounds__(256) zero_kernel(float* p, long long n) {
  const long long head = min(n, (long long)((16 - ((uintptr_t)p & 15)) & 15) / 4);
  const long long n4 = (n - head) / 4;
  float4* q = reinterpret_cast<float4*>(p + head);
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long i = i0; i < n4; i += stride) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i0 < head) p[i0] = 0.f;
  const long long t = head + 4 * n4 + i0;
  if (t < n) p[t] = 0.f;
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

// The compiled (waves per workgroup, workgroups per CU) of a schedule: group 0 is the
// default four; blocks 0 is the default for the group (the compiled occupancy).
template <int kW, bool kFwd>
constexpr int default_blocks() {
  return kW == 4 ? (kFwd ? kFwdWavesPerEU : kBwdWavesPerEU) : 4 * kWideWavesPerEU / kW;
}

glam_status launch_render_fwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                              const float* bg, float* image, float* T_final, int32_t* n_contrib, int32_t* n_eval,
                              hipStream_t s) {
  if (v.n_tiles == 0 || v.n_gauss == 0) {
    // nothing to composite: background everywhere
    return launch_background(v, bg, image, T_final, n_contrib, n_eval, s);
  }
  const int tl = tile_log2(v.tile_w), ql = 2 * (tl - 3);
  if (((unsigned long long)v.n_tiles << ql) >= (1ull << 32)) return GLAM_ERR_UNSUPPORTED;
  const bool direct = bins.tuning.non_persistent != 0;
  const int gw = direct ? 4 : (bins.tuning.fwd_group_waves > 0 ? bins.tuning.fwd_group_waves : 4);
  const long long items = v.n_tiles << ql;
  auto launch = [&](auto kernel, int kw, int dflt) {
    const int bpc = bins.tuning.fwd_blocks_per_cu > 0 ? bins.tuning.fwd_blocks_per_cu : dflt;
    const unsigned grid = direct ? (unsigned)((items + kw - 1) / kw) : persistent_blocks(items, kw, bpc);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64 * kw), 0, s, proj.splat, bins.vals, bins.ranges, bins.order,
                       bins.status, bins.queue, v.dev, v.n, (int)v.n_tiles, tl, bg, image, T_final, n_contrib, n_eval,
                       (uint32_t)bins.capacity, (uint32_t)v.n_gauss, direct ? 1 : 0);
  };
  if (gw == 16)
    launch(n_eval ? render_fwd_kernel<true, 16> : render_fwd_kernel<false, 16>, 16, default_blocks<16, true>());
  else if (gw == 8)
    launch(n_eval ? render_fwd_kernel<true, 8> : render_fwd_kernel<false, 8>, 8, default_blocks<8, true>());
  else
    launch(n_eval ? render_fwd_kernel<true, 4> : render_fwd_kernel<false, 4>, 4, default_blocks<4, true>());
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

size_t det_partial_bytes(const glam_views& v, long long capacity) {
  const int ql = 2 * (tile_log2(v.tile_w) - 3);
  return (size_t)capacity * ((size_t)1 << ql) * 9 * sizeof(float);
}

bool det_supported(const glam_views& v, long long capacity) {
  const int ql = 2 * (tile_log2(v.tile_w) - 3);
  return ((unsigned long long)capacity << ql) < (1ull << 32);
}

glam_status launch_composite_bwd(const glam_projected& proj, const glam_bins& bins, const glam_views& v,
                                 const float* bg, const float* T_final, const int32_t* n_contrib,
                                 const float* dimage, float* g2d, float* det_part, hipStream_t s) {
  const int tl = tile_log2(v.tile_w), ql = 2 * (tl - 3);
  if (((unsigned long long)v.n_tiles << ql) >= (1ull << 32)) return GLAM_ERR_UNSUPPORTED;
  const bool det = det_part != nullptr;
  if (det && !det_supported(v, bins.capacity)) return GLAM_ERR_UNSUPPORTED;
  // the atomics add into g2d; the reproducible path stores into its zeroed partials
  float* acc = det ? det_part : g2d;
  const long long n = det ? (long long)(det_partial_bytes(v, bins.capacity) / sizeof(float)) : 9 * v.n_gauss;
  if (n > 0)
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)min((n / 4 + 255) / 256 + 1, 8LL * cu_count())), dim3(256), 0, s,
                       acc, n);
  const bool direct = bins.tuning.non_persistent != 0;
  const int gw = direct ? 4 : (bins.tuning.bwd_group_waves > 0 ? bins.tuning.bwd_group_waves : 4);
  const long long items = v.n_tiles << ql;
  auto launch = [&](auto kernel, int kw, int dflt) {
    const int bpc = bins.tuning.bwd_blocks_per_cu > 0 ? bins.tuning.bwd_blocks_per_cu : dflt;
    const unsigned grid = direct ? (unsigned)((items + kw - 1) / kw) : persistent_blocks(items, kw, bpc);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64 * kw), 0, s, proj.splat, bins.vals, bins.ranges, bins.order,
                       bins.status, bins.queue, v.dev, v.n, (int)v.n_tiles, tl, bg, T_final, n_contrib, dimage, acc,
                       (uint32_t)bins.capacity, (uint32_t)v.n_gauss, bins.pair_begin, direct ? 1 : 0);
  };
  if (v.n_tiles > 0 && v.n_gauss > 0) {
    if (gw == 16)
      launch(det ? composite_bwd_kernel<true, 16> : composite_bwd_kernel<false, 16>, 16, default_blocks<16, false>());
    else if (gw == 8)
      launch(det ? composite_bwd_kernel<true, 8> : composite_bwd_kernel<false, 8>, 8, default_blocks<8, false>());
    else
      launch(det ? composite_bwd_kernel<true, 4> : composite_bwd_kernel<false, 4>, 4, default_blocks<4, false>());
  }
  if (det && v.n_gauss > 0)
    hipLaunchKernelGGL(det_reduce_kernel, dim3((unsigned)((v.n_gauss + 255) / 256)), dim3(256), 0, s, det_part,
                       bins.pair_begin, proj.ntiles, (long long)v.n_gauss, ql, (uint32_t)bins.capacity, g2d);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

size_t fused_l1_workspace(const glam_views& v) {
  const int ql = 2 * (tile_log2(v.tile_w) - 3);
  return (size_t)((long long)v.n_tiles << ql) * sizeof(float);
}

glam_status launch_fused_l1(const glam_projected& proj, const glam_bins& bins, const glam_views& v, const float* bg,
                            const float* target, float* image, float* T_final, int32_t* n_contrib, float* dimage,
                            float* loss, float* total, float* g2d, void* ws, hipStream_t s) {
  const int tl = tile_log2(v.tile_w), ql = 2 * (tl - 3);
  if (((unsigned long long)v.n_tiles << ql) >= (1ull << 32)) return GLAM_ERR_UNSUPPORTED;
  float* l1_part = static_cast<float*>(ws);
  const long long n = 9 * v.n_gauss;
  if (n > 0)
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)min((n / 4 + 255) / 256 + 1, 8LL * cu_count())), dim3(256), 0, s,
                       g2d, n);
  if (v.n_gauss == 0) {
    // nothing to composite or differentiate: the background image and its L1 term
    glam_status st = launch_background(v, bg, image, T_final, n_contrib, nullptr, s);
    if (st != GLAM_OK) return st;
    return launch_loss(v, image, target, 0.f, dimage, loss, total, ws, s);
  }
  const int gw = bins.tuning.bwd_group_waves > 0 ? bins.tuning.bwd_group_waves : 4;
  const long long items = v.n_tiles << ql;
  auto launch = [&](auto kernel, int kw, int dflt) {
    const int bpc = bins.tuning.bwd_blocks_per_cu > 0 ? bins.tuning.bwd_blocks_per_cu : dflt;
    hipLaunchKernelGGL(kernel, dim3(persistent_blocks(items, kw, bpc)), dim3(64 * kw), 0, s, proj.splat, bins.vals,
                       bins.ranges, bins.order, bins.status, bins.queue, v.dev, v.n, (int)v.n_tiles, tl, bg, target,
                       image, T_final, n_contrib, dimage, g2d, l1_part, (uint32_t)bins.capacity, (uint32_t)v.n_gauss);
  };
  if (gw == 16)
    launch(fused_l1_kernel<16>, 16, default_blocks<16, false>());
  else if (gw == 8)
    launch(fused_l1_kernel<8>, 8, default_blocks<8, false>());
  else
    launch(fused_l1_kernel<4>, 4, default_blocks<4, false>());
  if (hipGetLastError() != hipSuccess) return GLAM_ERR_HIP;
  return launch_l1_reduce(v, ql, l1_part, loss, total, s);
}

}  // namespace glam
