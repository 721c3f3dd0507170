// The optimiser step of a mapping iteration: Adam over every parameter group in one
// launch, and the keyframe sampler (host) that picks the views of an iteration.
//
// Adam is elementwise and HBM-bound: 16 bytes read (param, grad, m, v) and 12 bytes
// written (param, m, v) per parameter.  A thread takes four consecutive elements with
// 16-byte loads and stores; the groups (any number of plain arrays and the packed MLP
// sets, up to GLAM_ADAM_MAX_GROUPS) share one grid, each workgroup finding its group in
// a block-offset table passed by value.  The learning rate of an element is periodic
// in its index, so the MLP sets of all partitions form one group with one segment per
// MLP.
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

constexpr int kAdamThreads = 256, kAdamPer = 4;  // elements per thread
constexpr long long kAdamBlock = (long long)kAdamThreads * kAdamPer;

struct AdamGroups {
  int n;
  long long block_begin[GLAM_ADAM_MAX_GROUPS + 1];  // first workgroup of each group
  glam_adam_group g[GLAM_ADAM_MAX_GROUPS];
};

// Learning rate at position r of the period.
__device__ __forceinline__ float group_lr(const glam_adam_group& g, int r) {
  float lr = g.lr[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) lr = (k < g.n_seg && r >= g.seg_end[k - 1]) ? g.lr[k] : lr;
  return lr;
}

__device__ __forceinline__ int next_pos(int r, int period) { return r + 1 == period ? 0 : r + 1; }

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                         float c1, float c2, float eps) {
  m = fmaf(b1, m, (1.f - b1) * g);
  v = fmaf(b2, v, (1.f - b2) * (g * g));
  // the step divides by sqrt(v_hat) + eps with the hardware reciprocal (1 ulp)
  p -= (lr * (m * c1)) * __builtin_amdgcn_rcpf(sqrtf(v * c2) + eps);
}

__global__ void __launch_bounds__(kAdamThreads) adam_kernel(AdamGroups groups, float b1, float b2, float c1,
                                                             float c2, float eps) {
  int gi = 0;
  while (gi + 1 < groups.n && groups.block_begin[gi + 1] <= (long long)blockIdx.x) ++gi;
  const glam_adam_group& g = groups.g[gi];
  const long long i0 = ((long long)blockIdx.x - groups.block_begin[gi]) * kAdamBlock + (long long)threadIdx.x * kAdamPer;
  if (i0 >= g.n) return;
  const int r0 = g.period == 1 ? 0 : (int)(i0 % g.period);  // one 64-bit remainder per thread
  if (i0 + kAdamPer <= g.n) {
    // 16-byte accesses: the arrays are 16-byte aligned and i0 is a multiple of four
    float4 p = *reinterpret_cast<const float4*>(g.param + i0);
    const float4 gr = *reinterpret_cast<const float4*>(g.grad + i0);
    float4 m = *reinterpret_cast<const float4*>(g.m + i0);
    float4 v = *reinterpret_cast<const float4*>(g.v + i0);
    const int r1 = next_pos(r0, g.period), r2 = next_pos(r1, g.period), r3 = next_pos(r2, g.period);
    adam_one(p.x, gr.x, m.x, v.x, group_lr(g, r0), b1, b2, c1, c2, eps);
    adam_one(p.y, gr.y, m.y, v.y, group_lr(g, r1), b1, b2, c1, c2, eps);
    adam_one(p.z, gr.z, m.z, v.z, group_lr(g, r2), b1, b2, c1, c2, eps);
    adam_one(p.w, gr.w, m.w, v.w, group_lr(g, r3), b1, b2, c1, c2, eps);
    *reinterpret_cast<float4*>(g.param + i0) = p;
    *reinterpret_cast<float4*>(g.m + i0) = m;
    *reinterpret_cast<float4*>(g.v + i0) = v;
  } else {
    int r = r0;
    for (long long i = i0; i < g.n; ++i, r = next_pos(r, g.period)) {
      float p = g.param[i], m = g.m[i], v = g.v[i];
      adam_one(p, g.grad[i], m, v, group_lr(g, r), b1, b2, c1, c2, eps);
      g.param[i] = p;
      g.m[i] = m;
      g.v[i] = v;
    }
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two 32x32 -> 64-bit
// multiplications with the Weyl-sequence key schedule.
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u, w0 = 0x9E3779B9u, w1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += w0;
      k[1] += w1;
    }
    const uint64_t p0 = (uint64_t)m0 * c[0], p1 = (uint64_t)m1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

}  // namespace

bool adam_groups_ok(const glam_adam_group* groups, int n_groups) {
  if (!groups || n_groups < 1 || n_groups > GLAM_ADAM_MAX_GROUPS) return false;
  for (int i = 0; i < n_groups; ++i) {
    const glam_adam_group& g = groups[i];
    if (g.n < 0 || g.period <= 0 || g.n_seg < 1 || g.n_seg > 4) return false;
    if (g.n > 0) {
      const void* ptrs[4] = {g.param, g.grad, g.m, g.v};
      for (const void* p : ptrs)
        if (!p || (reinterpret_cast<uintptr_t>(p) & 15u)) return false;
    }
    int prev = 0;
    for (int k = 0; k < g.n_seg; ++k) {
      if (g.seg_end[k] <= prev || !(g.lr[k] >= 0.f) || !std::isfinite(g.lr[k])) return false;
      prev = g.seg_end[k];
    }
    if (prev != g.period) return false;
  }
  return true;
}

glam_status launch_adam(const glam_adam_group* groups, int n_groups, int step, float b1, float b2, float eps,
                        hipStream_t s) {
  AdamGroups ag{};
  ag.n = n_groups;
  long long b = 0;
  for (int i = 0; i < n_groups; ++i) {
    ag.block_begin[i] = b;
    ag.g[i] = groups[i];
    b += (groups[i].n + kAdamBlock - 1) / kAdamBlock;
  }
  ag.block_begin[n_groups] = b;
  if (b == 0) return GLAM_OK;
  if (b >= (1ll << 31)) return GLAM_ERR_UNSUPPORTED;
  // bias corrections in double on the host
  const double c1 = 1.0 / (1.0 - std::pow((double)b1, step)), c2 = 1.0 / (1.0 - std::pow((double)b2, step));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)b), dim3(kAdamThreads), 0, s, ag, b1, b2, (float)c1, (float)c2,
                     eps);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

void sample_keyframes(int n, int k_recent, float p_recent, int count, uint64_t seed, uint64_t counter, int32_t* out) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  // recent when the first word is below p_recent 2^32
  const double t = std::floor((double)p_recent * 4294967296.0);
  const uint64_t thr = t <= 0.0 ? 0ull : (t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t);
  const bool all_recent = n <= k_recent;
  for (int j = 0; j < count; ++j) {
    const uint64_t c = counter + (uint64_t)j;
    const uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), 0u, 0u};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    int idx;
    if (all_recent) {
      idx = (int)(((uint64_t)w[1] * (uint64_t)n) >> 32);
    } else if ((uint64_t)w[0] < thr) {
      idx = n - k_recent + (int)(((uint64_t)w[1] * (uint64_t)k_recent) >> 32);
    } else {
      idx = (int)(((uint64_t)w[1] * (uint64_t)(n - k_recent)) >> 32);
    }
    out[j] = idx;
  }
}

}  // namespace glam
