// Tile binning and depth sort.
//
//  1. scan_reduce      per 1024 view-Gaussians: sum of tile counts, max depth bits
//  2. scan_plan        one block: exclusive scan of the block sums, pair count P,
//                      capacity check, lossless key width (tile bits + depth bits) and
//                      the number of 8-bit radix passes
//  3. duplicate        per view-Gaussian: its pairs, key = tile << dbits | depth key,
//                      value = view-Gaussian index, in index order (row-major tiles)
//  4. radix passes     LSD, reduce-then-scan (no inter-block waiting), two launches
//                      per pass: upsweep digit histogram per block, also added into
//                      per-group totals (groups of 32 blocks); downsweep: each block's
//                      digit offsets from the group totals and the counts of the
//                      blocks before it in its group, then the scatter with a stable
//                      in-block rank from wave ballots
//  5. ranges           [start, end) of every tile (cleared by the plan kernel)
//  6. order            the compositing work order, longest ranges first (one workgroup
//                      when the tiles are few)
//
// Every kernel reads P and the key layout from the device-side plan, so the whole
// sequence runs without a host round trip (and can be captured in a graph).  Passes
// beyond the plan's count exit at once.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kScanThreads = 256, kScanItems = 4, kScanBlock = kScanThreads * kScanItems;
// Radix sort blocks of kSortThreads x items keys: 1024 keys (4 per thread) for up to
// 2^20 pairs of capacity, where 2048-key blocks would leave most CUs with one block or
// none and each block's ranking chain sets the pass time; 2048 keys above, where the
// blocks fill the chip either way and fewer of them mean less counting and scanning.
constexpr int kSortThreads = 256;
constexpr long long kSmallSortCapacity = 1ll << 20;
int sort_items(long long capacity) { return capacity <= kSmallSortCapacity ? 4 : 8; }
constexpr int kRadixBits = 8, kRadix = 1 << kRadixBits;
constexpr int kMaxSortBlocks = 4096;
constexpr int kMaxPasses = 8;            // tile bits (at most 33) + depth bits (at most 31)
constexpr int kGroup = 32;               // radix blocks per group total
constexpr uint32_t kDepthBase = 0x3E4CCCCDu;  // bit pattern of 0.2f: every visible depth is above it

struct Plan {
  uint32_t P;          // pair count (clamped to capacity)
  uint32_t dbits;      // depth key bits
  uint32_t npasses;    // radix passes
  uint32_t tbits;      // tile key bits
  uint32_t tiles_per_block;
  uint32_t n_sort_tiles;
  uint32_t active_blocks;  // workgroups of a radix pass that have tiles
  uint32_t pad[9];
};

constexpr int kLptBuckets = 32;

struct Layout {
  size_t partial_sum, partial_max, plan, keys_alt, vals_alt, count, gsum, lpt, total;
  int n_scan_blocks, n_sort_blocks, sort_items, n_groups;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout(long long n_gauss, long long capacity) {
  Layout L;
  L.n_scan_blocks = (int)((n_gauss + kScanBlock - 1) / kScanBlock);
  if (L.n_scan_blocks < 1) L.n_scan_blocks = 1;
  L.sort_items = sort_items(capacity);
  const long long sort_tile = (long long)kSortThreads * L.sort_items;
  long long tiles = (capacity + sort_tile - 1) / sort_tile;
  L.n_sort_blocks = (int)(tiles < 1 ? 1 : (tiles > kMaxSortBlocks ? kMaxSortBlocks : tiles));
  L.n_groups = (L.n_sort_blocks + kGroup - 1) / kGroup;
  size_t o = 0;
  L.partial_sum = o; o = align256(o + 4ull * L.n_scan_blocks);
  L.partial_max = o; o = align256(o + 4ull * L.n_scan_blocks);
  L.plan = o; o = align256(o + sizeof(Plan));
  L.keys_alt = o; o = align256(o + 8ull * (size_t)capacity);
  L.vals_alt = o; o = align256(o + 4ull * (size_t)capacity);
  L.count = o; o = align256(o + 4ull * kRadix * L.n_sort_blocks);
  L.gsum = o; o = align256(o + 4ull * kRadix * L.n_groups * kMaxPasses);
  L.lpt = o; o = align256(o + 4ull * 2 * kLptBuckets);
  L.total = o;
  return L;
}

int bit_length(uint64_t x) {
  int b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

__device__ __forceinline__ int dbit_length(uint32_t x) { return x ? 32 - __clz(x) : 0; }

// Inclusive scan of one value per thread over a workgroup of 256 threads: each wave scans
// its 64 lanes with shuffles, then adds the totals of the waves before it (one barrier).
// s_wave: 4 words of LDS; every thread calls it.
__device__ __forceinline__ uint32_t block_scan256(uint32_t v, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(v, o);
    v += lane >= o ? u : 0u;
  }
  if (lane == 63) s_wave[w] = v;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) before += k < w ? s_wave[k] : 0u;
  return v + before;
}

__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const int32_t* ntiles, const float* depth,
                                                                   long long n, uint32_t* psum, uint32_t* pmax) {
  __shared__ uint32_t s_sum, s_max;
  if (threadIdx.x == 0) { s_sum = 0; s_max = 0; }
  __syncthreads();
  const long long base = (long long)blockIdx.x * kScanBlock;
  uint32_t sum = 0, mx = 0;
  int32_t nt[kScanItems];
  uint32_t db[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {  // all loads in flight first
    const long long g = base + (long long)i * kScanThreads + threadIdx.x;
    nt[i] = g < n ? ntiles[g] : 0;
    db[i] = g < n ? __float_as_uint(depth[g]) : 0u;
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    sum += (uint32_t)nt[i];
    if (nt[i] > 0) mx = max(mx, db[i]);
  }
  atomicAdd(&s_sum, sum);
  atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x == 0) { psum[blockIdx.x] = s_sum; pmax[blockIdx.x] = s_max; }
}

// One block of 1024 threads: exclusive scan of the block sums in place, and the plan.
// Also clears the tile ranges and the longest-first counters for this call.
__global__ void __launch_bounds__(1024) scan_plan_kernel(uint32_t* psum, const uint32_t* pmax, int nb,
                                                         long long capacity, long long n_tiles, int n_sort_blocks,
                                                         int sort_tile, Plan* plan, int32_t* status,
                                                         uint32_t* ranges, uint32_t* lpt) {
  __shared__ unsigned long long s_part[1024];
  __shared__ uint32_t s_max[1024];
  const int t = threadIdx.x;
  for (long long i = t; i < 2 * n_tiles; i += 1024) ranges[i] = 0u;
  if (t < 2 * kLptBuckets) lpt[t] = 0u;
  const int per = (nb + 1023) / 1024;
  const int lo = min(nb, t * per), hi = min(nb, lo + per);
  unsigned long long local = 0;
  uint32_t mx = 0;
  for (int i = lo; i < hi; ++i) { local += psum[i]; mx = max(mx, pmax[i]); }
  s_part[t] = local;
  s_max[t] = mx;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    unsigned long long v = t >= off ? s_part[t - off] : 0ull;
    uint32_t m = t >= off ? s_max[t - off] : 0u;
    __syncthreads();
    s_part[t] += v;
    s_max[t] = max(s_max[t], m);
    __syncthreads();
  }
  unsigned long long run = s_part[t] - local;  // exclusive prefix of this thread's segment
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = psum[i];
    psum[i] = (uint32_t)run;
    run += v;
  }
  if (t == 1023) {
    const unsigned long long P = s_part[1023];
    const uint32_t maxbits = s_max[1023];
    Plan pl;
    for (int k = 0; k < 9; ++k) pl.pad[k] = 0;
    long long Pc = (long long)P;
    if (Pc > capacity) {
      status[0] = GLAM_ERR_CAPACITY;
      Pc = capacity;
    }
    status[1] = (int32_t)(uint32_t)Pc;
    status[2] = (int32_t)(uint32_t)(P & 0xffffffffull);
    status[3] = (int32_t)(uint32_t)(P >> 32);
    pl.P = (uint32_t)Pc;
    pl.dbits = (P > 0 && maxbits > kDepthBase) ? (uint32_t)dbit_length(maxbits - kDepthBase) : 1u;
    pl.tbits = n_tiles > 1 ? (uint32_t)(64 - __clzll((unsigned long long)(n_tiles - 1))) : 0u;
    pl.npasses = Pc > 0 ? (pl.dbits + pl.tbits + kRadixBits - 1) / kRadixBits : 0u;
    pl.n_sort_tiles = (uint32_t)((Pc + sort_tile - 1) / sort_tile);
    pl.tiles_per_block = (pl.n_sort_tiles + n_sort_blocks - 1) / n_sort_blocks;
    pl.active_blocks = pl.tiles_per_block ? (pl.n_sort_tiles + pl.tiles_per_block - 1) / pl.tiles_per_block : 0u;
    status[4] = (int32_t)pl.dbits;
    status[5] = (int32_t)pl.tbits;
    status[6] = (int32_t)pl.npasses;
    *plan = pl;
  }
}

// Pairs of every view-Gaussian.  A workgroup takes the pairs of 1024 consecutive
// view-Gaussians: it stages their tile boxes in LDS with the exclusive prefix of their
// pair counts (the first-level scan redone in LDS), then each thread emits pairs
// k = t, t + 256, ... of the workgroup's range, finding its Gaussian by binary search
// in the prefix, so every pair costs the same and the stores are coalesced.  Also
// clears the radix passes' group totals (gsum, gsum_words words).
__global__ void __launch_bounds__(kScanThreads) duplicate_kernel(const int32_t* ntiles, const float* splat,
                                                                 long long n, const glam_view_info* views,
                                                                 int n_views, int tl, const uint32_t* psum,
                                                                 const Plan* plan, uint64_t* keys_out,
                                                                 uint32_t* vals_out, uint64_t* keys_alt,
                                                                 uint32_t* vals_alt, uint32_t* pair_begin,
                                                                 uint32_t* gsum, int gsum_words) {
  for (int i = blockIdx.x * kScanThreads + threadIdx.x; i < gsum_words; i += gridDim.x * kScanThreads) gsum[i] = 0u;
  __shared__ uint32_t s_pre[kScanBlock];   // count, then exclusive prefix within the workgroup
  __shared__ uint32_t s_tile[kScanBlock];  // global tile of the box's top-left corner
  __shared__ uint32_t s_dim[kScanBlock];   // box width in tiles | view tiles_x << 16
  __shared__ uint32_t s_dkey[kScanBlock];  // depth key
  __shared__ uint32_t s_scan[kScanThreads];
  __shared__ int s_view0;
  const Plan pl = *plan;
  const int t = threadIdx.x;
  const long long base = (long long)blockIdx.x * kScanBlock;
  const uint32_t gbase = psum[blockIdx.x];  // this block's first pair (the plan kernel's prefix)
  if (t == 0) s_view0 = find_view(views, n_views, base, [](const glam_view_info& v) { return v.g_begin; });
  // tile counts and boxes side by side (a box is only used where its count is positive)
  int32_t cnt[kScanItems];
  float4 rec[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const long long g = base + i * kScanThreads + t;
    cnt[i] = g < n ? ntiles[g] : 0;
    rec[i] = g < n ? reinterpret_cast<const float4*>(splat + g * kSplatWords)[2] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  const int v0 = s_view0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int j = i * kScanThreads + t;
    const long long g = base + j;
    uint32_t tile0 = 0, dim = 0, dkey = 0;
    if (cnt[i] > 0) {
      int vi = v0;
      while (vi + 1 < n_views && views[vi + 1].g_begin <= g) ++vi;
      const glam_view_info& vw = views[vi];
      const uint32_t bx = __float_as_uint(rec[i].y), by = __float_as_uint(rec[i].z);
      const int tx0 = (int)(bx & 0xffffu) >> tl, tx1 = (int)(bx >> 16) >> tl;  // tiles of edge 2^tl
      const int ty0 = (int)(by & 0xffffu) >> tl;
      tile0 = (uint32_t)(vw.tile_begin + (long long)ty0 * vw.tiles_x + tx0);
      dim = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)vw.tiles_x << 16);
      dkey = __float_as_uint(rec[i].w) - kDepthBase;
    }
    s_pre[j] = (uint32_t)cnt[i];
    s_tile[j] = tile0;
    s_dim[j] = dim;
    s_dkey[j] = dkey;
  }
  __syncthreads();
  // exclusive prefix: thread t scans entries [8t, 8t + 8), then the 256 thread sums
  uint32_t local[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) { local[i] = sum; sum += s_pre[t * kScanItems + i]; }
  const uint32_t incl = block_scan256(sum, s_scan);
  if (t == kScanThreads - 1) s_scan[4] = incl;
  __syncthreads();
  const uint32_t before = incl - sum;
  const uint32_t total = s_scan[4];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s_pre[t * kScanItems + i] = before + local[i];
  __syncthreads();
  if (pair_begin) {  // each view-Gaussian's first pair, in the same order as the emission below
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const long long g = base + i * kScanThreads + t;
      if (g < n) pair_begin[g] = gbase + s_pre[i * kScanThreads + t];
    }
  }
  uint64_t* kout = (pl.npasses & 1u) ? keys_alt : keys_out;
  uint32_t* vout = (pl.npasses & 1u) ? vals_alt : vals_out;
  for (uint32_t k = t; k < total; k += kScanThreads) {
    // last entry whose prefix is <= k (zero-count entries share the next one's prefix)
    int lo = 0, hi = kScanBlock - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const uint32_t r = k - s_pre[lo];
    const uint32_t dim = s_dim[lo];
    const uint32_t w = dim & 0xffffu, tx = dim >> 16;
    const uint32_t ty = r / w;
    const uint64_t tile = (uint64_t)(s_tile[lo] + ty * tx + (r - ty * w));
    const uint32_t off = gbase + k;
    if (off < pl.P) {
      kout[off] = (tile << pl.dbits) | (uint64_t)s_dkey[lo];
      vout[off] = (uint32_t)(base + lo);
    }
  }
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lanes of this wave holding the same digit (among `valid` lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Digit counts of this block's keys: count[block][digit], and added into the group
// totals gsum[pass][block / kGroup][digit].
template <int kSortItems>
__global__ void __launch_bounds__(kSortThreads) radix_upsweep_kernel(const Plan* plan, int pass, int n_groups,
                                                                     const uint64_t* keys_out,
                                                                     const uint64_t* keys_alt, uint32_t* count,
                                                                     uint32_t* gsum) {
  const Plan pl = *plan;
  if ((uint32_t)pass >= pl.npasses || blockIdx.x >= pl.active_blocks) return;
  __shared__ uint32_t s_cnt[kRadix];
  s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t* src = ((pass & 1) == 0) == ((pl.npasses & 1u) == 0) ? keys_out : keys_alt;
  constexpr int kSortTile = kSortThreads * kSortItems;
  const int shift = pass * kRadixBits;
  const uint32_t t0 = blockIdx.x * pl.tiles_per_block;
  const uint32_t t1 = min(pl.n_sort_tiles, t0 + pl.tiles_per_block);
  for (uint32_t tile = t0; tile < t1; ++tile) {
    const uint32_t start = tile * kSortTile;
    uint32_t d[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {  // all loads in flight first
      const uint32_t idx = start + i * kSortThreads + threadIdx.x;
      d[i] = idx < pl.P ? (uint32_t)(src[idx] >> shift) & (kRadix - 1) : 0u;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const bool valid = start + i * kSortThreads + threadIdx.x < pl.P;
      const uint64_t peers = match_digit(d[i], valid);
      if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&s_cnt[d[i]], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  const uint32_t c = s_cnt[threadIdx.x];
  count[(size_t)blockIdx.x * kRadix + threadIdx.x] = c;
  if (c) atomicAdd(&gsum[((size_t)pass * n_groups + blockIdx.x / kGroup) * kRadix + threadIdx.x], c);
}

template <int kSortItems>
__global__ void __launch_bounds__(kSortThreads) radix_downsweep_kernel(const Plan* plan, int pass, int n_groups,
                                                                       const uint32_t* count, const uint32_t* gsum,
                                                                       uint64_t* keys_out, uint32_t* vals_out,
                                                                       uint64_t* keys_alt, uint32_t* vals_alt) {
  const Plan pl = *plan;
  if ((uint32_t)pass >= pl.npasses || blockIdx.x >= pl.active_blocks) return;
  constexpr int kSortTile = kSortThreads * kSortItems;
  // the per-(item round, wave, digit) counts, and once ranked the tile's keys and values
  // in digit order
  __shared__ __align__(16) uint32_t s_lds[kSortItems * (kSortThreads / 64) * kRadix];
  static_assert(kSortTile * (sizeof(uint64_t) + sizeof(uint32_t)) <= sizeof(s_lds), "staging fits");
  auto& s_cnt = *reinterpret_cast<uint32_t(*)[kSortItems][kSortThreads / 64][kRadix]>(s_lds);
  uint64_t* s_key = reinterpret_cast<uint64_t*>(s_lds);
  uint32_t* s_val = s_lds + 2 * kSortTile;
  __shared__ uint32_t s_run[kRadix];
  __shared__ uint32_t s_scan[kRadix];
  __shared__ uint32_t s_lbase[kRadix];
  const bool src_is_out = ((pass & 1) == 0) == ((pl.npasses & 1u) == 0);
  const uint64_t* ksrc = src_is_out ? keys_out : keys_alt;
  const uint32_t* vsrc = src_is_out ? vals_out : vals_alt;
  uint64_t* kdst = src_is_out ? keys_alt : keys_out;
  uint32_t* vdst = src_is_out ? vals_alt : vals_out;
  const int shift = pass * kRadixBits;
  const int t = threadIdx.x, w = t >> 6;
  // where digit t of this block goes: the keys of smaller digits (exclusive scan of the
  // digit totals), then digit t's keys in the groups before this block's and in the
  // blocks before it in its group; every load in flight before the first sum
  const int grp = (int)blockIdx.x / kGroup, b0 = grp * kGroup;
  const int ng = (int)((pl.active_blocks + kGroup - 1) / kGroup);
  const uint32_t* gs = gsum + (size_t)pass * n_groups * kRadix + t;
  uint32_t tot = 0, before = 0;
  {
    uint32_t vg[kGroup], vb[kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      vg[k] = k < ng ? gs[(size_t)k * kRadix] : 0u;
      vb[k] = b0 + k < (int)blockIdx.x ? count[(size_t)(b0 + k) * kRadix + t] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      tot += vg[k];
      before += (k < grp ? vg[k] : 0u) + vb[k];
    }
  }
  for (int g0 = kGroup; g0 < ng; g0 += kGroup) {  // more than kGroup groups
    uint32_t vg[kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k) vg[k] = g0 + k < ng ? gs[(size_t)(g0 + k) * kRadix] : 0u;
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      tot += vg[k];
      before += g0 + k < grp ? vg[k] : 0u;
    }
  }
  s_run[t] = block_scan256(tot, s_scan) - tot + before;
  __syncthreads();
  const uint32_t t0 = blockIdx.x * pl.tiles_per_block;
  const uint32_t t1 = min(pl.n_sort_tiles, t0 + pl.tiles_per_block);
  uint32_t* cnt = s_lds;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    for (int k = t; k < kSortItems * (kSortThreads / 64) * kRadix; k += kSortThreads) cnt[k] = 0;
    __syncthreads();
    const uint32_t start = tile * kSortTile;
    uint64_t key[kSortItems];
    uint32_t val[kSortItems], rank[kSortItems], dig[kSortItems];
    bool valid[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {  // all loads in flight first
      const uint32_t idx = start + i * kSortThreads + t;
      valid[i] = idx < pl.P;
      key[i] = valid[i] ? ksrc[idx] : 0ull;
      val[i] = valid[i] ? vsrc[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      dig[i] = (uint32_t)(key[i] >> shift) & (kRadix - 1);
      const uint64_t peers = match_digit(dig[i], valid[i]);
      rank[i] = (uint32_t)__popcll(peers & lanemask_lt());
      if (valid[i] && rank[i] == 0) s_cnt[i][w][dig[i]] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit (thread t = digit t): exclusive prefix over (item round, wave); the 32
    // counts are read before any is rewritten
    constexpr int kSlots = kSortItems * (kSortThreads / 64);
    uint32_t c[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) c[k] = s_cnt[k / (kSortThreads / 64)][k % (kSortThreads / 64)][t];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      s_cnt[k / (kSortThreads / 64)][k % (kSortThreads / 64)][t] = run;
      run += c[k];
    }
    // first place of digit t in the tile's own digit order
    const uint32_t lbase = block_scan256(run, s_scan + 4 * (1 + (tile & 1))) - run;
    s_lbase[t] = lbase;
    uint32_t lpos[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) lpos[i] = s_cnt[i][w][dig[i]] + rank[i];
    __syncthreads();
    // the tile in digit order in LDS (over the counts, which are no longer needed), then
    // written out by consecutive threads so that each digit's run is stored contiguously
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      if (!valid[i]) continue;
      const uint32_t lp = s_lbase[dig[i]] + lpos[i];
      s_key[lp] = key[i];
      s_val[lp] = val[i];
    }
    __syncthreads();
    const uint32_t n_here = min((uint32_t)kSortTile, pl.P - min(pl.P, start));
    for (uint32_t j = t; j < n_here; j += kSortThreads) {
      const uint64_t k = s_key[j];
      const uint32_t d = (uint32_t)(k >> shift) & (kRadix - 1);
      const uint32_t pos = s_run[d] + (j - s_lbase[d]);
      if (pos < pl.P) {  // always true for consistent counts; keeps any fault impossible
        kdst[pos] = k;
        vdst[pos] = s_val[j];
      }
    }
    __syncthreads();
    s_run[t] += run;
    __syncthreads();
  }
}

// Work order of the compositing queue: tiles by power-of-two class of their range
// length, longest first (empty tiles last).  Counting sort over 32 classes; the order
// inside a class is arbitrary (it only schedules work).
__device__ __forceinline__ int lpt_bucket(const uint32_t* ranges, long long t) {
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  const int bits = len ? 32 - __clz(len) : 0;  // bit length
  return min(kLptBuckets - 1, 32 - bits);
}

__global__ void __launch_bounds__(256) lpt_count_kernel(const uint32_t* ranges, long long n_tiles, uint32_t* lpt) {
  __shared__ uint32_t h[kLptBuckets];
  if (threadIdx.x < kLptBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_tiles) atomicAdd(&h[lpt_bucket(ranges, t)], 1u);
  __syncthreads();
  if (threadIdx.x < kLptBuckets && h[threadIdx.x]) atomicAdd(&lpt[threadIdx.x], h[threadIdx.x]);
}

// Also records in status[7] the number of long tiles (range length at least
// 2^long_log2), which are exactly the first classes of the order.
__global__ void __launch_bounds__(256) lpt_scatter_kernel(const uint32_t* ranges, long long n_tiles, uint32_t* lpt,
                                                          int long_log2, uint32_t* order, int32_t* status) {
  __shared__ uint32_t base[kLptBuckets], h[kLptBuckets], blk[kLptBuckets];
  if (threadIdx.x < kLptBuckets) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kLptBuckets; ++b) {
      base[b] = run;
      run += lpt[b];
      if (b == kLptBuckets - 1 - long_log2 && blockIdx.x == 0) status[7] = (int32_t)run;
    }
  }
  __syncthreads();
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  uint32_t local = 0;
  if (t < n_tiles) {
    b = lpt_bucket(ranges, t);
    local = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kLptBuckets) blk[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&lpt[kLptBuckets + threadIdx.x], h[threadIdx.x]) : 0u;
  __syncthreads();
  if (t < n_tiles) {
    const uint32_t pos = base[b] + blk[b] + local;
    if (pos < (uint64_t)n_tiles) order[pos] = (uint32_t)t;
  }
}

// Up to kLptOneBlock tiles: the whole work order in one workgroup (class counts and
// slots in LDS), in one launch.
constexpr int kLptOneBlock = 16384;
__global__ void __launch_bounds__(1024) lpt_one_block_kernel(const uint32_t* ranges, long long n_tiles, int long_log2,
                                                             uint32_t* order, int32_t* status) {
  __shared__ uint32_t h[kLptBuckets], base[kLptBuckets];
  if (threadIdx.x < kLptBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  for (long long t = threadIdx.x; t < n_tiles; t += 1024) atomicAdd(&h[lpt_bucket(ranges, t)], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kLptBuckets; ++b) {
      base[b] = run;
      run += h[b];
      if (b == kLptBuckets - 1 - long_log2) status[7] = (int32_t)run;
    }
  }
  __syncthreads();
  for (long long t = threadIdx.x; t < n_tiles; t += 1024) {
    const uint32_t pos = atomicAdd(&base[lpt_bucket(ranges, t)], 1u);
    if (pos < (uint64_t)n_tiles) order[pos] = (uint32_t)t;
  }
}

__global__ void ranges_mark_kernel(const Plan* plan, const uint64_t* keys, uint32_t* ranges, long long n_tiles) {
  const Plan pl = *plan;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pl.P) return;
  const uint64_t tile = keys[i] >> pl.dbits;
  if (tile >= (uint64_t)n_tiles) return;
  if (i == 0 || (keys[i - 1] >> pl.dbits) != tile) ranges[2 * tile] = i;
  if (i + 1 == pl.P || (keys[i + 1] >> pl.dbits) != tile) ranges[2 * tile + 1] = i + 1;
}

}  // namespace

size_t bin_sort_workspace(const glam_views& v, long long capacity) {
  return layout(v.n_gauss, capacity).total;
}

glam_status launch_bin_sort(const glam_projected& proj, const glam_views& v, const glam_bins& bins, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  const Layout L = layout(v.n_gauss, bins.capacity);
  if (ws_bytes < L.total) return GLAM_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  uint32_t* psum = reinterpret_cast<uint32_t*>(w + L.partial_sum);
  uint32_t* pmax = reinterpret_cast<uint32_t*>(w + L.partial_max);
  Plan* plan = reinterpret_cast<Plan*>(w + L.plan);
  uint64_t* keys_alt = reinterpret_cast<uint64_t*>(w + L.keys_alt);
  uint32_t* vals_alt = reinterpret_cast<uint32_t*>(w + L.vals_alt);
  uint32_t* count = reinterpret_cast<uint32_t*>(w + L.count);
  uint32_t* gsum = reinterpret_cast<uint32_t*>(w + L.gsum);
  const long long n = v.n_gauss;
  // host bound on the passes: tile bits are known, depth keys take at most 31 bits
  const int tbits = v.n_tiles > 1 ? bit_length((uint64_t)(v.n_tiles - 1)) : 0;
  const int max_passes = (tbits + 31 + kRadixBits - 1) / kRadixBits;
  if (max_passes > kMaxPasses) return GLAM_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(L.n_scan_blocks), dim3(kScanThreads), 0, s, proj.ntiles, proj.depth,
                     n, psum, pmax);
  uint32_t* lpt = reinterpret_cast<uint32_t*>(w + L.lpt);
  hipLaunchKernelGGL(scan_plan_kernel, dim3(1), dim3(1024), 0, s, psum, pmax, L.n_scan_blocks,
                     (long long)bins.capacity, (long long)v.n_tiles, L.n_sort_blocks, kSortThreads * L.sort_items,
                     plan, bins.status, bins.ranges, lpt);
  hipLaunchKernelGGL(duplicate_kernel, dim3(L.n_scan_blocks), dim3(kScanThreads), 0, s, proj.ntiles, proj.splat,
                     n, v.dev, v.n, tile_log2(v.tile_w), psum, plan, bins.keys, bins.vals, keys_alt, vals_alt,
                     bins.pair_begin, gsum, max_passes * L.n_groups * kRadix);
  for (int p = 0; p < max_passes; ++p) {
    if (L.sort_items == 4)
      hipLaunchKernelGGL(radix_upsweep_kernel<4>, dim3(L.n_sort_blocks), dim3(kSortThreads), 0, s, plan, p,
                         L.n_groups, bins.keys, keys_alt, count, gsum);
    else
      hipLaunchKernelGGL(radix_upsweep_kernel<8>, dim3(L.n_sort_blocks), dim3(kSortThreads), 0, s, plan, p,
                         L.n_groups, bins.keys, keys_alt, count, gsum);
    if (L.sort_items == 4)
      hipLaunchKernelGGL(radix_downsweep_kernel<4>, dim3(L.n_sort_blocks), dim3(kSortThreads), 0, s, plan, p,
                         L.n_groups, count, gsum, bins.keys, bins.vals, keys_alt, vals_alt);
    else
      hipLaunchKernelGGL(radix_downsweep_kernel<8>, dim3(L.n_sort_blocks), dim3(kSortThreads), 0, s, plan, p,
                         L.n_groups, count, gsum, bins.keys, bins.vals, keys_alt, vals_alt);
  }
  if (bins.capacity > 0)
    hipLaunchKernelGGL(ranges_mark_kernel, dim3((unsigned)((bins.capacity + 255) / 256)), dim3(256), 0, s, plan,
                       bins.keys, bins.ranges, (long long)v.n_tiles);
  const int long_log2 = bins.tuning.long_log2 > 0 ? bins.tuning.long_log2 : kDefaultLongLog2;
  if (v.n_tiles <= kLptOneBlock) {
    hipLaunchKernelGGL(lpt_one_block_kernel, dim3(1), dim3(1024), 0, s, bins.ranges, (long long)v.n_tiles, long_log2,
                       bins.order, bins.status);
  } else {
    const unsigned tb = (unsigned)((v.n_tiles + 255) / 256);
    hipLaunchKernelGGL(lpt_count_kernel, dim3(tb), dim3(256), 0, s, bins.ranges, (long long)v.n_tiles, lpt);
    hipLaunchKernelGGL(lpt_scatter_kernel, dim3(tb), dim3(256), 0, s, bins.ranges, (long long)v.n_tiles, lpt,
                       long_log2, bins.order, bins.status);
  }
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
