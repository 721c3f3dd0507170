// Anchor voxelisation and growth (Eq. 4): a point cloud snapped to the voxel grid, the
// unique voxels it occupies, and those not yet in the anchor set.
//
//  1. quantise   per point: k = round(p / eps) per axis in FP32 (nearest, ties to even),
//                packed into a 63-bit key; a dropped point (out of the key range, or NaN)
//                leaves the all-ones key.  Each workgroup reduces the range of its valid
//                keys and its dropped count into a partial record (no global atomics:
//                same-address atomics from every wave serialise in L2)
//  2. plan       one workgroup reduces the partials: the per-axis key ranges give a
//                compact key (each axis offset by its minimum and given just the bits of
//                its range, in x, y, z order, so it sorts like the full key) and with it
//                the number of 8-bit radix passes; dropped slots are then read as the
//                smallest valid key, a duplicate the unique step removes
//  3. sort       LSD radix on the compact digits (reduce-then-scan: per-workgroup digit
//                counts, one workgroup per digit scanning over the workgroups, a stable
//                scatter ranked by wave ballots); passes beyond the planned count exit
//                at once
//  4. select     a key is new when it differs from its predecessor and a binary search
//                does not find it among the existing (sorted) keys; a scan of the flags
//                places it, with its voxel centre; optionally the sorted union of the
//                existing and the new keys is written (a merge by binary searches)
// Everything runs without a host round trip.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kVThreads = 256, kVItems = 4, kVTile = kVThreads * kVItems;
constexpr int kVStage = 2048;  // existing keys a flag workgroup searches in LDS
constexpr int kVRadix = 256;
constexpr int kVMaxPasses = 8;
constexpr int kPlanThreads = 1024;
constexpr int kKeyBits = 21;
constexpr long long kKeyOff = 1ll << (kKeyBits - 1);
constexpr unsigned long long kFieldMask = (1ull << kKeyBits) - 1;
constexpr unsigned long long kDroppedKey = ~0ull;  // valid keys are below 2^63

// Range of one quantise workgroup's valid keys, and its dropped points.
struct VoxPartial {
  unsigned long long kmin;  // smallest valid key, all ones if none
  int lo[3], hi[3];         // per-axis range of the biased fields; lo > hi if none
  unsigned dropped;
  unsigned pad;
};

// Plan of one call (in the workspace), written by the plan kernel.
struct VoxState {
  unsigned long long fill;    // read in place of a dropped point's key
  unsigned long long n_sort;  // entries to sort: all slots if any point is valid, else 0
  unsigned long long dropped;
  int lo[3];                  // per-axis minimum of the biased fields
  int shift_y, shift_x;       // compact key: (x - lo) << shift_x | (y - lo) << shift_y | (z - lo)
  int npasses;
};

// The FP32 quotient p / eps is taken as the double quotient rounded to float: with 53 >=
// 2 * 24 + 2 bits the double rounding is innocuous, so it is the correctly rounded FP32
// quotient whatever the compiler's FP32 division mode.
__device__ __forceinline__ bool quantise(float p, float eps, int& field) {
  const float q = rintf((float)((double)p / (double)eps));  // nearest, ties to even
  if (!(q >= (float)-kKeyOff && q < (float)kKeyOff)) return false;
  field = (int)q + (int)kKeyOff;
  return true;
}

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
#pragma unroll
  for (int o = 32; o; o >>= 1) v = op(v, (T)__shfl_xor(v, o));
  return v;
}

struct MinOp {
  template <class T>
  __device__ T operator()(T a, T b) const { return a < b ? a : b; }
};
struct MaxOp {
  template <class T>
  __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};

__device__ __forceinline__ void combine(VoxPartial& a, const VoxPartial& b) {
  a.kmin = min(a.kmin, b.kmin);
  for (int c = 0; c < 3; ++c) {
    a.lo[c] = min(a.lo[c], b.lo[c]);
    a.hi[c] = max(a.hi[c], b.hi[c]);
  }
  a.dropped += b.dropped;
}

__device__ __forceinline__ VoxPartial wave_partial(VoxPartial p) {
  p.kmin = wave_reduce(p.kmin, MinOp{});
  for (int c = 0; c < 3; ++c) {
    p.lo[c] = wave_reduce(p.lo[c], MinOp{});
    p.hi[c] = wave_reduce(p.hi[c], MaxOp{});
  }
  p.dropped = wave_reduce(p.dropped, [](unsigned a, unsigned b) { return a + b; });
  return p;
}

__device__ __forceinline__ VoxPartial empty_partial() {
  VoxPartial p;
  p.kmin = ~0ull;
  for (int c = 0; c < 3; ++c) {
    p.lo[c] = INT_MAX;
    p.hi[c] = INT_MIN;
  }
  p.dropped = 0;
  p.pad = 0;
  return p;
}

// One thread per point: its key (or the dropped marker) in input order, and one partial
// record per workgroup.
__global__ void __launch_bounds__(kVThreads) vox_quantise_kernel(const float* pts, long long n, float eps,
                                                                 unsigned long long* keys, VoxPartial* part) {
  const long long i = (long long)blockIdx.x * kVThreads + threadIdx.x;
  VoxPartial p = empty_partial();
  if (i < n) {
    int f[3];
    const bool ok = quantise(pts[i], eps, f[0]) && quantise(pts[n + i], eps, f[1]) &&
                    quantise(pts[2 * n + i], eps, f[2]);
    unsigned long long key = kDroppedKey;
    if (ok) {
      key = ((unsigned long long)f[0] << (2 * kKeyBits)) | ((unsigned long long)f[1] << kKeyBits) |
            (unsigned long long)f[2];
      p.kmin = key;
      for (int c = 0; c < 3; ++c) p.lo[c] = p.hi[c] = f[c];
    } else {
      p.dropped = 1;
    }
    keys[i] = key;
  }
  p = wave_partial(p);
  __shared__ VoxPartial s[kVThreads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x == 0) {
    VoxPartial r = s[0];
    for (int w = 1; w < kVThreads / 64; ++w) combine(r, s[w]);
    part[blockIdx.x] = r;
  }
}

__device__ __forceinline__ int bit_width(int v) { return v > 0 ? 32 - __clz(v) : 0; }

__global__ void __launch_bounds__(kPlanThreads) vox_plan_kernel(const VoxPartial* part, int n_part, long long n,
                                                                VoxState* st) {
  VoxPartial p = empty_partial();
  for (int j = threadIdx.x; j < n_part; j += kPlanThreads) combine(p, part[j]);
  p = wave_partial(p);
  __shared__ VoxPartial s[kPlanThreads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x != 0) return;
  VoxPartial r = s[0];
  for (int w = 1; w < kPlanThreads / 64; ++w) combine(r, s[w]);
  VoxState o;
  const bool any = r.kmin != ~0ull;
  o.fill = r.kmin;
  o.n_sort = any ? (unsigned long long)n : 0ull;
  o.dropped = r.dropped;
  int width[3];
  for (int c = 0; c < 3; ++c) {
    o.lo[c] = any ? r.lo[c] : 0;
    width[c] = any ? bit_width(r.hi[c] - r.lo[c]) : 0;
  }
  o.shift_y = width[2];
  o.shift_x = width[1] + width[2];
  const int bits = any && n > 1 ? width[0] + width[1] + width[2] : 0;
  o.npasses = (bits + 7) / 8;
  *st = o;
}

__device__ __forceinline__ unsigned long long load_key(const unsigned long long* k, unsigned long long i,
                                                       unsigned long long fill) {
  const unsigned long long v = k[i];
  return v == kDroppedKey ? fill : v;
}

// Compact key: the same order as the full key over the keys of this call.
__device__ __forceinline__ unsigned long long compact(unsigned long long key, const VoxState& p) {
  const unsigned long long fx = key >> (2 * kKeyBits), fy = (key >> kKeyBits) & kFieldMask, fz = key & kFieldMask;
  return ((fx - (unsigned)p.lo[0]) << p.shift_x) | ((fy - (unsigned)p.lo[1]) << p.shift_y) | (fz - (unsigned)p.lo[2]);
}

__device__ __forceinline__ unsigned digit(unsigned long long key, const VoxState& p, int pass) {
  return (unsigned)(compact(key, p) >> (8 * pass)) & 255u;
}

// Lanes of this wave holding the same 8-bit digit (among `valid` lanes).
__device__ __forceinline__ unsigned long long same_digit(unsigned d, bool valid) {
  unsigned long long peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const unsigned long long m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Per-workgroup digit counts of pass `pass` (counts[digit * n_blocks + block]).
__global__ void __launch_bounds__(kVThreads) vox_count_kernel(const VoxState* st, int pass, int n_blocks,
                                                              const unsigned long long* a, const unsigned long long* b,
                                                              unsigned* counts) {
  const VoxState p = *st;
  if (pass >= p.npasses) return;
  const unsigned long long n = p.n_sort;
  const unsigned long long* src = (pass & 1) ? b : a;
  __shared__ unsigned s[kVRadix];
  s[threadIdx.x] = 0;
  const unsigned long long base = (unsigned long long)blockIdx.x * kVTile;
  unsigned d[kVItems];
  bool valid[kVItems];
#pragma unroll
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long idx = base + (unsigned long long)i * kVThreads + threadIdx.x;
    valid[i] = idx < n;
    d[i] = valid[i] ? digit(load_key(src, idx, p.fill), p, pass) : 0u;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long peers = same_digit(d[i], valid[i]);
    if (valid[i] && (peers & lanes_below(lane)) == 0) atomicAdd(&s[d[i]], (unsigned)__popcll(peers));
  }
  __syncthreads();
  counts[(size_t)threadIdx.x * n_blocks + blockIdx.x] = s[threadIdx.x];
}

// Inclusive scan across a 256-thread workgroup (s: 256 words of LDS); total receives the
// workgroup's sum.
__device__ __forceinline__ unsigned block_scan_256(unsigned v, unsigned* s, unsigned& total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
#pragma unroll
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned u = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += u;
    __syncthreads();
  }
  const unsigned r = s[t];
  total = s[255];
  __syncthreads();
  return r;
}

// Exclusive scan of one digit's per-workgroup counts over the workgroups (one workgroup
// per digit, in place), and the digit's total.
__global__ void __launch_bounds__(256) vox_scan_kernel(const VoxState* st, int pass, int n_blocks, unsigned* counts,
                                                       unsigned* totals) {
  if (pass >= st->npasses) return;
  __shared__ unsigned s[256];
  unsigned* row = counts + (size_t)blockIdx.x * n_blocks;
  unsigned carry = 0;
  for (int b0 = 0; b0 < n_blocks; b0 += 256) {
    const int b = b0 + (int)threadIdx.x;
    const unsigned v = b < n_blocks ? row[b] : 0u;
    unsigned chunk;
    const unsigned inc = block_scan_256(v, s, chunk);
    if (b < n_blocks) row[b] = carry + inc - v;
    carry += chunk;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of pass `pass`: rank within the workgroup by (item round, wave, lane).
// Writes the keys with dropped slots already replaced.
__global__ void __launch_bounds__(kVThreads) vox_scatter_kernel(const VoxState* st, int pass, int n_blocks,
                                                                unsigned long long* a, unsigned long long* b,
                                                                const unsigned* offsets, const unsigned* totals) {
  const VoxState p = *st;
  if (pass >= p.npasses) return;
  const unsigned long long n = p.n_sort;
  const unsigned long long* src = (pass & 1) ? b : a;
  unsigned long long* dst = (pass & 1) ? a : b;
  __shared__ __align__(16) unsigned s_cnt[kVItems][kVThreads / 64][kVRadix];
  static_assert(kVTile * sizeof(unsigned long long) <= sizeof(s_cnt), "staging fits");
  __shared__ unsigned s_base[kVRadix];
  __shared__ unsigned s_lbase[kVRadix];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const unsigned long long base = (unsigned long long)blockIdx.x * kVTile;
  unsigned long long key[kVItems];
  bool valid[kVItems];
#pragma unroll
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long idx = base + (unsigned long long)i * kVThreads + t;
    valid[i] = idx < n;
    key[i] = valid[i] ? load_key(src, idx, p.fill) : 0ull;
  }
  for (int k = t; k < kVItems * (kVThreads / 64) * kVRadix; k += kVThreads) (&s_cnt[0][0][0])[k] = 0;
  // first place of digit t in this workgroup: keys of smaller digits, then of digit t in
  // earlier workgroups
  {
    const unsigned tot = totals[t];
    unsigned all;
    const unsigned inc = block_scan_256(tot, s_base, all);
    s_base[t] = inc - tot + offsets[(size_t)t * n_blocks + blockIdx.x];
  }
  unsigned dig[kVItems], rank[kVItems];
#pragma unroll
  for (int i = 0; i < kVItems; ++i) {
    dig[i] = digit(key[i], p, pass);
    const unsigned long long peers = same_digit(dig[i], valid[i]);
    rank[i] = (unsigned)__popcll(peers & lanes_below(lane));
    if (valid[i] && rank[i] == 0) s_cnt[i][w][dig[i]] = (unsigned)__popcll(peers);
  }
  __syncthreads();
  // per digit (thread t = digit t): exclusive prefix over (item round, wave)
  unsigned run = 0;
  for (int i = 0; i < kVItems; ++i)
    for (int ww = 0; ww < kVThreads / 64; ++ww) {
      const unsigned c = s_cnt[i][ww][t];
      s_cnt[i][ww][t] = run;
      run += c;
    }
  // first place of digit t in the tile's own digit order
  unsigned all;
  const unsigned lbase = block_scan_256(run, s_lbase, all) - run;
  s_lbase[t] = lbase;
  unsigned lpos[kVItems];
#pragma unroll
  for (int i = 0; i < kVItems; ++i) lpos[i] = s_cnt[i][w][dig[i]] + rank[i];
  __syncthreads();
  // the tile in digit order in LDS (over the counts), written out by consecutive
  // threads so that each digit's run is stored contiguously
  unsigned long long* s_key = reinterpret_cast<unsigned long long*>(&s_cnt[0][0][0]);
#pragma unroll
  for (int i = 0; i < kVItems; ++i)
    if (valid[i]) s_key[s_lbase[dig[i]] + lpos[i]] = key[i];
  __syncthreads();
  const unsigned n_here = (unsigned)min((unsigned long long)kVTile, n - min(n, base));
  for (unsigned j = t; j < n_here; j += kVThreads) {
    const unsigned long long k = s_key[j];
    const unsigned d = digit(k, p, pass);
    const unsigned long long pos = (unsigned long long)s_base[d] + (j - s_lbase[d]);
    if (pos < n) dst[pos] = k;
  }
}

__device__ __forceinline__ long long count_below(const uint64_t* a, long long n, uint64_t key) {
  long long lo = 0, hi = n;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// New-key flags (first of a run of equal keys, absent from the existing keys), their sum
// per tile of kVTile sorted keys, and for each new key the number of existing keys below
// it (its offset in the grown set).  A tile's keys can only match existing keys between
// its first and last key: that range is found once per tile and searched in LDS when it
// fits there.
__global__ void __launch_bounds__(kVThreads) vox_flag_kernel(const VoxState* st, const unsigned long long* a,
                                                             const unsigned long long* b, const uint64_t* existing,
                                                             long long n_existing, unsigned* flags, unsigned* below,
                                                             unsigned* block_sums) {
  const VoxState p = *st;
  const unsigned long long n = p.n_sort;
  const unsigned long long* k = (p.npasses & 1) ? b : a;  // where the last pass wrote
  const unsigned long long base = (unsigned long long)blockIdx.x * kVTile;
  __shared__ uint64_t s_ex[kVStage];
  __shared__ long long s_rng[2];
  __shared__ unsigned s_sum[kVThreads / 64];
  const int t = threadIdx.x;
  const bool any = base < n;
  if (any && n_existing > 0 && (t == 0 || t == 64)) {
    const unsigned long long last = min(base + kVTile, n) - 1;
    // [first existing >= first key, first existing > last key)
    s_rng[t == 0 ? 0 : 1] = t == 0 ? count_below(existing, n_existing, load_key(k, base, p.fill))
                                   : count_below(existing, n_existing, load_key(k, last, p.fill) + 1);
  }
  __syncthreads();
  const long long lo = any && n_existing > 0 ? s_rng[0] : 0, hi = any && n_existing > 0 ? s_rng[1] : 0;
  const long long m = hi - lo;
  const bool staged = m <= kVStage;
  if (staged)
    for (long long j = t; j < m; j += kVThreads) s_ex[j] = existing[lo + j];
  __syncthreads();
  unsigned acc = 0;
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long idx = base + (unsigned long long)i * kVThreads + t;
    if (idx >= n) continue;
    const unsigned long long key = load_key(k, idx, p.fill);
    bool f = idx == 0 || load_key(k, idx - 1, p.fill) != key;
    long long j = lo;
    if (f && m > 0) {
      if (staged) {
        long long l = 0, h = m;
        while (l < h) {
          const long long mid = (l + h) >> 1;
          if (s_ex[mid] < key) l = mid + 1; else h = mid;
        }
        f = !(l < m && s_ex[l] == key);
        j = lo + l;
      } else {
        j = lo + count_below(existing + lo, m, key);
        f = !(j < hi && existing[j] == key);
      }
    }
    flags[idx] = f ? 1u : 0u;
    below[idx] = (unsigned)j;
    acc += f ? 1u : 0u;
  }
  acc = wave_reduce(acc, [](unsigned x, unsigned y) { return x + y; });
  if ((t & 63) == 0) s_sum[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    unsigned r = 0;
    for (int w = 0; w < kVThreads / 64; ++w) r += s_sum[w];
    block_sums[blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(1024) vox_block_scan_kernel(unsigned* block_sums, int n_blocks,
                                                              unsigned long long* total) {
  __shared__ unsigned s[1024];
  const int per = (n_blocks + 1023) / 1024;
  const int lo = min(n_blocks, (int)threadIdx.x * per), hi = min(n_blocks, lo + per);
  unsigned local = 0;
  for (int i = lo; i < hi; ++i) local += block_sums[i];
  s[threadIdx.x] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned run = s[threadIdx.x] - local;
  for (int i = lo; i < hi; ++i) {
    const unsigned v = block_sums[i];
    block_sums[i] = run;
    run += v;
  }
  if (threadIdx.x == 1023) *total = s[1023];
}

// Places the flagged keys (their order is the sorted order), their voxel centres and
// their entries of the grown set; workgroup 0 also reports the counts.
__global__ void __launch_bounds__(kVThreads) vox_place_kernel(const VoxState* st, const unsigned long long* a,
                                                              const unsigned long long* b, const unsigned* flags,
                                                              const unsigned* below, const unsigned* block_base,
                                                              const unsigned long long* total, float eps,
                                                              uint64_t* new_keys, float* new_pos, long long capacity,
                                                              uint64_t* merged, int64_t* counts) {
  const VoxState p = *st;
  const unsigned long long n = p.n_sort;
  const unsigned long long* k = (p.npasses & 1) ? b : a;
  __shared__ unsigned s_f[kVTile];
  __shared__ unsigned s_scan[kVThreads];
  const unsigned long long base = (unsigned long long)blockIdx.x * kVTile;
  const int t = threadIdx.x;
  if (blockIdx.x == 0 && t == 0) {
    counts[0] = (int64_t)*total;
    counts[1] = (int64_t)p.dropped;
  }
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long idx = base + (unsigned long long)i * kVThreads + t;
    s_f[i * kVThreads + t] = idx < n ? flags[idx] : 0u;
  }
  __syncthreads();
  // thread t scans items [8t, 8t + 8) of the tile
  unsigned local[kVItems], sum = 0;
  for (int i = 0; i < kVItems; ++i) {
    local[i] = sum;
    sum += s_f[t * kVItems + i];
  }
  s_scan[t] = sum;
  __syncthreads();
  for (int off = 1; off < kVThreads; off <<= 1) {
    const unsigned v = t >= off ? s_scan[t - off] : 0u;
    __syncthreads();
    s_scan[t] += v;
    __syncthreads();
  }
  const unsigned before = s_scan[t] - sum + block_base[blockIdx.x];
  for (int i = 0; i < kVItems; ++i) {
    const unsigned long long idx = base + (unsigned long long)t * kVItems + i;
    if (idx >= n || !s_f[t * kVItems + i]) continue;
    const long long pos = (long long)before + local[i];
    if (pos >= capacity) continue;
    const unsigned long long key = load_key(k, idx, p.fill);
    new_keys[pos] = key;
    if (merged) merged[pos + below[idx]] = key;
    const int kx = (int)(key >> (2 * kKeyBits)) - (int)kKeyOff;
    const int ky = (int)((key >> kKeyBits) & kFieldMask) - (int)kKeyOff;
    const int kz = (int)(key & kFieldMask) - (int)kKeyOff;
    new_pos[pos] = (float)kx * eps;
    new_pos[capacity + pos] = (float)ky * eps;
    new_pos[2 * capacity + pos] = (float)kz * eps;
  }
}

// The existing keys' entries of the grown set (the sorted union of the existing keys and
// the new ones, disjoint sets): a key's place is its index plus the number of new keys
// below it.
__global__ void __launch_bounds__(256) vox_merge_kernel(const uint64_t* existing, long long n_existing,
                                                        const uint64_t* new_keys, const unsigned long long* total,
                                                        long long capacity, uint64_t* merged) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_existing) return;
  const long long n_new = min((long long)*total, capacity);
  const uint64_t key = existing[i];
  merged[i + count_below(new_keys, n_new, key)] = key;
}

struct VoxLayout {
  size_t state, partials, keys_a, keys_b, counts, totals, flags, below, block_sums, total, bytes;
  int n_blocks, n_part;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

VoxLayout vox_layout(long long n) {
  VoxLayout L{};
  const long long n1 = n > 0 ? n : 1;
  L.n_blocks = (int)((n1 + kVTile - 1) / kVTile);
  L.n_part = (int)((n1 + kVThreads - 1) / kVThreads);
  size_t o = 0;
  L.state = o; o = align256(o + sizeof(VoxState));
  L.partials = o; o = align256(o + sizeof(VoxPartial) * (size_t)L.n_part);
  L.keys_a = o; o = align256(o + 8ull * n1);
  L.keys_b = o; o = align256(o + 8ull * n1);
  L.counts = o; o = align256(o + 4ull * kVRadix * L.n_blocks);
  L.totals = o; o = align256(o + 4ull * kVRadix);
  L.flags = o; o = align256(o + 4ull * n1);
  L.below = o; o = align256(o + 4ull * n1);
  L.block_sums = o; o = align256(o + 4ull * L.n_blocks);
  L.total = o; o = align256(o + 8);
  L.bytes = o;
  return L;
}

// Growth bookkeeping: rows of per-anchor entries widened by n_new anchors inserted at
// anchor `at` (the end of the partition that receives them).  One thread per output
// float; rows of the source and the inserted block are read contiguously.
__global__ void __launch_bounds__(256) insert_rows_kernel(const float* src, float* dst, long long n_old, int width,
                                                          long long at, long long n_new, const float* ins,
                                                          long long ins_stride, float fill) {
  const long long len_new = (n_old + n_new) * width;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= len_new) return;
  const int r = blockIdx.y;
  const long long lo = at * width, hi = (at + n_new) * width;
  float v;
  if (i < lo)
    v = src[(long long)r * n_old * width + i];
  else if (i >= hi)
    v = src[(long long)r * n_old * width + i - n_new * width];
  else
    v = ins ? ins[(long long)r * ins_stride + (i - lo)] : fill;
  dst[(long long)r * len_new + i] = v;
}

}  // namespace

glam_status launch_insert_rows(const float* src, float* dst, int rows, long long n_old, int width, long long at,
                               long long n_new, const float* ins, long long ins_stride, float fill, hipStream_t s) {
  const long long len_new = (n_old + n_new) * width;
  if (rows == 0 || len_new == 0) return GLAM_OK;
  hipLaunchKernelGGL(insert_rows_kernel, dim3((unsigned)((len_new + 255) / 256), (unsigned)rows), dim3(256), 0, s,
                     src, dst, n_old, width, at, n_new, ins, ins_stride, fill);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

size_t voxelize_workspace(long long n) { return vox_layout(n).bytes; }

glam_status launch_voxelize(const float* points, long long n, float eps, const uint64_t* existing,
                            long long n_existing, uint64_t* new_keys, float* new_pos, long long capacity,
                            uint64_t* merged, int64_t* counts, void* ws, hipStream_t s) {
  const VoxLayout L = vox_layout(n);
  if (L.n_blocks > (1 << 21) || n_existing >= (1ll << 32)) return GLAM_ERR_UNSUPPORTED;
  char* w = static_cast<char*>(ws);
  auto* st = reinterpret_cast<VoxState*>(w + L.state);
  auto* part = reinterpret_cast<VoxPartial*>(w + L.partials);
  auto* ka = reinterpret_cast<unsigned long long*>(w + L.keys_a);
  auto* kb = reinterpret_cast<unsigned long long*>(w + L.keys_b);
  auto* cnt = reinterpret_cast<unsigned*>(w + L.counts);
  auto* dtot = reinterpret_cast<unsigned*>(w + L.totals);
  auto* flags = reinterpret_cast<unsigned*>(w + L.flags);
  auto* below = reinterpret_cast<unsigned*>(w + L.below);
  auto* bsum = reinterpret_cast<unsigned*>(w + L.block_sums);
  auto* total = reinterpret_cast<unsigned long long*>(w + L.total);
  const int nb = L.n_blocks;
  int n_part = 0;
  if (n > 0) {
    n_part = L.n_part;
    hipLaunchKernelGGL(vox_quantise_kernel, dim3((unsigned)n_part), dim3(kVThreads), 0, s, points, n, eps, ka, part);
  }
  hipLaunchKernelGGL(vox_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, part, n_part, n, st);
  for (int p = 0; p < kVMaxPasses; ++p) {
    hipLaunchKernelGGL(vox_count_kernel, dim3(nb), dim3(kVThreads), 0, s, st, p, nb, ka, kb, cnt);
    hipLaunchKernelGGL(vox_scan_kernel, dim3(kVRadix), dim3(256), 0, s, st, p, nb, cnt, dtot);
    hipLaunchKernelGGL(vox_scatter_kernel, dim3(nb), dim3(kVThreads), 0, s, st, p, nb, ka, kb, cnt, dtot);
  }
  hipLaunchKernelGGL(vox_flag_kernel, dim3(nb), dim3(kVThreads), 0, s, st, ka, kb, existing, n_existing, flags,
                     below, bsum);
  hipLaunchKernelGGL(vox_block_scan_kernel, dim3(1), dim3(1024), 0, s, bsum, nb, total);
  hipLaunchKernelGGL(vox_place_kernel, dim3(nb), dim3(kVThreads), 0, s, st, ka, kb, flags, below, bsum, total, eps,
                     new_keys, new_pos, capacity, merged, counts);
  if (merged && n_existing > 0)
    hipLaunchKernelGGL(vox_merge_kernel, dim3((unsigned)((n_existing + 255) / 256)), dim3(256), 0, s, existing,
                       n_existing, new_keys, total, capacity, merged);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace glam
