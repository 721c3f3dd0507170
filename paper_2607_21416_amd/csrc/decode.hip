// View-conditioned anchor decode (Eq. 2) with one MLP set per partition (Eq. 6), and
// its adjoint, on FP32 MFMA (v_mfma_f32_16x16x4_f32).
//
// A wave decodes 16 anchors of one view.  The three MLPs share their input
// z = [f_a, d_ac, delta_ac], so their first layers are evaluated as one 96-row
// product H^T[96][16] = W1[96][F+4] Z^T[F+4][16] (six 16x16 output tiles).  The output
// layout of the MFMA puts hidden rows 4g..4g+3 of a tile in lane group g (lanes
// 16g..16g+15, one anchor per lane), register r = row 4g+r.  The second layer consumes
// H^T straight from those registers: K-step r of a tile feeds lane group g the hidden
// row 4g+r, and the matching A operand (W2) is read with the same permutation, so no
// transpose through LDS is needed.  Outputs Y^T land in LDS, where one lane per
// Gaussian applies the activations and writes the structure-of-arrays Gaussians.
//
// MFMA operand layout (16x16x4, one block): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, D[i][j] in lane j + 16(i/4), register i%4.
//
// The adjoint recomputes the forward for a 16-anchor chunk, applies the activation
// adjoints, and runs dH = W2^T dY, dZ = W1^T dPre on MFMA the same way.  The weight
// gradients dW2 = dY^T H and dW1 = dPre^T Z are contractions over anchors (K = 16 per
// chunk), accumulated in registers over all chunks and views a wave handles, reduced
// across the workgroup in LDS, and written as one partial per workgroup; a final
// kernel sums the partials of each partition.  Anchor gradients are summed over the
// views of the partition in registers, so every anchor is written exactly once.
#include "common.hpp"
#include "kernels.hpp"

namespace glam {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kHid = 32;

// Packed offsets of one partition's MLP set (same order as the ABI documents).
struct MlpOff {
  int w1[3], b1[3], w2[3], b2[3], out[3], yoff[3];
  int total;
};

__host__ __device__ constexpr MlpOff mlp_offsets(int F, int K) {
  MlpOff o{};
  const int n_in = F + 4;
  const int outs[3] = {K, 3 * K, 7 * K};
  const int yoffs[3] = {0, K, 4 * K};
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    o.w1[l] = off;
    o.b1[l] = off + kHid * n_in;
    o.w2[l] = o.b1[l] + kHid;
    o.b2[l] = o.w2[l] + outs[l] * kHid;
    o.out[l] = outs[l];
    o.yoff[l] = yoffs[l];
    off = o.b2[l] + outs[l];
  }
  o.total = off;
  return o;
}

// The weights as staged in LDS: rows padded by one word (W1 rows F+5, W2 rows 33) so
// that lanes reading one column of consecutive rows fall in different banks.
struct LdsOff {
  int w1[3], b1[3], w2[3], b2[3];
  int total;
};

__host__ __device__ constexpr LdsOff lds_offsets(int F, int K) {
  LdsOff o{};
  const int w1s = F + 5, w2s = kHid + 1;
  const int outs[3] = {K, 3 * K, 7 * K};
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    o.w1[l] = off;
    o.b1[l] = off + kHid * w1s;
    o.w2[l] = o.b1[l] + kHid;
    o.b2[l] = o.w2[l] + outs[l] * w2s;
    off = o.b2[l] + outs[l];
  }
  o.total = off;
  return o;
}

template <int F, int K>
struct Cfg {
  static constexpr int NIN = F + 4;
  static constexpr int KS1 = NIN / 4;       // K-steps of layer 1
  static constexpr int ZS = NIN + 1;        // LDS row stride of Z
  static constexpr int NY = 11 * K;         // outputs per anchor
  static constexpr int YS = NY + 1;         // LDS row stride of Y
  static constexpr int HS = 3 * kHid + 1;   // LDS row stride of H
  static constexpr int OT0 = (K + 15) / 16, OT1 = (3 * K + 15) / 16, OT2 = (7 * K + 15) / 16;
  static constexpr int P = mlp_offsets(F, K).total;
  static constexpr int W1S = F + 5;         // LDS row stride of W1
  static constexpr int W2S = kHid + 1;      // LDS row stride of W2
  static constexpr int PA = (lds_offsets(F, K).total + 3) & ~3;  // LDS words of the weights
  static_assert(NIN % 4 == 0, "F + 4 must be a multiple of 4");
};

// Copies one packed MLP set into the padded LDS layout.
template <int F, int K>
__device__ __forceinline__ void load_weights(const float* pm, float* s, int t, int nthreads) {
  using C = Cfg<F, K>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr LdsOff L = lds_offsets(F, K);
  for (int i = t; i < C::P; i += nthreads) {
    const int l = i < O.w1[1] ? 0 : (i < O.w1[2] ? 1 : 2);
    const int j = i - O.w1[l];
    int dst;
    if (j < kHid * C::NIN) {
      dst = L.w1[l] + (j / C::NIN) * C::W1S + j % C::NIN;
    } else if (j < kHid * C::NIN + kHid) {
      dst = L.b1[l] + (j - kHid * C::NIN);
    } else if (j < O.b2[l] - O.w1[l]) {
      const int jj = j - kHid * C::NIN - kHid;
      dst = L.w2[l] + (jj / kHid) * C::W2S + jj % kHid;
    } else {
      dst = L.b2[l] + (j - (O.b2[l] - O.w1[l]));
    }
    s[dst] = pm[i];
  }
}

__device__ __forceinline__ void camera_centre(const glam_camera& c, float xc[3]) {
  for (int i = 0; i < 3; ++i) xc[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
}

// Z rows of 16 anchors [a0, a0+16) of one view into z (zero rows past the partition).
template <int F, int K>
__device__ __forceinline__ void build_z(const glam_anchors& an, const glam_view_info& vw, int a0, float* z, int l) {
  using C = Cfg<F, K>;
  const int A = vw.anchor_count;
  for (int idx = l; idx < 16 * F; idx += 64) {
    const int ai = idx / F, k = idx % F, a = a0 + ai;
    z[ai * C::ZS + k] = a < A ? an.feat[(size_t)(vw.anchor_begin + a) * F + k] : 0.f;
  }
  if (l < 16) {
    const int a = a0 + l;
    float d[3] = {0.f, 0.f, 0.f}, delta = 0.f;
    if (a < A) {
      float xc[3];
      camera_centre(vw.cam, xc);
      const int ga = vw.anchor_begin + a;
      for (int i = 0; i < 3; ++i) d[i] = an.pos[(size_t)i * an.A + ga] - xc[i];
      delta = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const float inv = 1.f / delta;
      for (int i = 0; i < 3; ++i) d[i] *= inv;
    }
    z[l * C::ZS + F + 0] = d[0];
    z[l * C::ZS + F + 1] = d[1];
    z[l * C::ZS + F + 2] = d[2];
    z[l * C::ZS + F + 3] = delta;
  }
}

// Layer 1 for all three MLPs: H^T tiles (ReLU applied), lane layout of the MFMA output.
template <int F, int K>
__device__ __forceinline__ void layer1(const float* p, const float* z, int l, f4 H[6]) {
  using C = Cfg<F, K>;
  constexpr LdsOff O = lds_offsets(F, K);
  const int li = l & 15, lg = l >> 4;
#pragma unroll
  for (int mt = 0; mt < 6; ++mt) {
    const int h = mt * 16 + li, ml = h >> 5, hi = h & 31;
    const float* W1 = p + O.w1[ml] + hi * C::W1S;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < C::KS1; ++ks) acc = mfma(W1[ks * 4 + lg], z[li * C::ZS + ks * 4 + lg], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int hr = mt * 16 + 4 * lg + r;
      acc[r] = fmaxf(acc[r] + p[O.b1[hr >> 5] + (hr & 31)], 0.f);
    }
    H[mt] = acc;
  }
}

// Layer 2 of MLP ml: Y^T tiles from the H^T registers (permuted K), stored to y.
template <int F, int K, int ML, int OT>
__device__ __forceinline__ void layer2(const float* p, const f4 H[6], float* y, int l) {
  using C = Cfg<F, K>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr LdsOff Ls = lds_offsets(F, K);
  const int li = l & 15, lg = l >> 4;
  constexpr int out = O.out[ML];
#pragma unroll
  for (int ot = 0; ot < OT; ++ot) {
    const int o = ot * 16 + li;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int hc = t2 * 16 + 4 * lg + r;
        const float a = o < out ? p[Ls.w2[ML] + o * C::W2S + hc] : 0.f;
        acc = mfma(a, H[2 * ML + t2][r], acc);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = ot * 16 + 4 * lg + r;
      if (orow < out) y[li * C::YS + O.yoff[ML] + orow] = acc[r] + p[Ls.b2[ML] + orow];
    }
  }
}

// Orders one wave's LDS writes before its later reads by other lanes of the wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One block stages its partition's weights once and then runs `chunks` consecutive
// groups of 64 anchors; each wave owns 16 anchors of a group and its own LDS rows, so
// after the weights are in place the waves proceed independently.
template <int F, int K>
__global__ void __launch_bounds__(256) decode_kernel(glam_anchors an, const float* __restrict__ mlp,
                                                     const glam_view_info* views, int sigmoid_op, int chunks,
                                                     glam_gaussians out) {
  using C = Cfg<F, K>;
  extern __shared__ float smem[];
  const glam_view_info vw = views[blockIdx.y];
  const int A = vw.anchor_count;
  const int block0 = blockIdx.x * chunks * 64;
  if (block0 >= A) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  float* s_p = smem;
  float* s_z = s_p + C::PA + w * 16 * C::ZS;
  float* s_y = smem + C::PA + 4 * 16 * C::ZS + w * 16 * C::YS;
  const float* pm = mlp + (size_t)vw.cam.partition * C::P;
  load_weights<F, K>(pm, s_p, t, 256);
  __syncthreads();
  const long long n = out.n;
  const size_t GK = (size_t)an.A * K;
  for (int c = 0; c < chunks; ++c) {
    const int a0 = block0 + c * 64 + w * 16;
    if (a0 >= A) break;
    build_z<F, K>(an, vw, a0, s_z, l);
    wave_sync();
    f4 H[6];
    layer1<F, K>(s_p, s_z, l, H);
    layer2<F, K, 0, C::OT0>(s_p, H, s_y, l);
    layer2<F, K, 1, C::OT1>(s_p, H, s_y, l);
    layer2<F, K, 2, C::OT2>(s_p, H, s_y, l);
    wave_sync();
    for (int gi = l; gi < 16 * K; gi += 64) {
      const int ai = gi / K, j = gi % K, a = a0 + ai;
      if (a >= A) continue;
      const int ga = vw.anchor_begin + a;
      const float* y = s_y + ai * C::YS;
      const long long g = vw.g_begin + (long long)a * K + j;
      const float yo = y[j];
      out.opacity[g] = sigmoid_op ? sigmoid(yo) : tanhf(yo);
      for (int c3 = 0; c3 < 3; ++c3) out.rgb[c3 * n + g] = sigmoid(y[K + 3 * j + c3]);
      const float es = expf(an.log_scale[ga]);
      for (int k = 0; k < 3; ++k) out.scale[k * n + g] = es * sigmoid(y[4 * K + 7 * j + k]);
      const float* q = y + 4 * K + 7 * j + 3;
      const float inv = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] + 1e-24f);
      for (int k = 0; k < 4; ++k) out.quat[k * n + g] = q[k] * inv;
      const size_t go = (size_t)ga * K + j;
      for (int i = 0; i < 3; ++i) out.mean[i * n + g] = fmaf(es, an.offs[i * GK + go], an.pos[(size_t)i * an.A + ga]);
    }
    // the next group's inputs overwrite rows this group's outputs were read from
    wave_sync();
  }
}

// ---------------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------------

template <int F, int K>
struct BwdAcc {
  f4 dW2[2 * (Cfg<F, K>::OT0 + Cfg<F, K>::OT1 + Cfg<F, K>::OT2)];
  f4 dW1[6 * ((Cfg<F, K>::NIN + 15) / 16)];
  float db2[(11 * K + 63) / 64];
  float db1[2];
};

// dH^T of MLP ML: A[i][k] = W2[k][i] over the outputs (K-steps of 4), B = dY^T from LDS.
template <int F, int K, int ML>
__device__ __forceinline__ void dhidden(const float* p, const float* dy, int l, f4 dH[6]) {
  using C = Cfg<F, K>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr int out = O.out[ML];
  constexpr int ks_n = (out + 3) / 4;
  const int li = l & 15, lg = l >> 4;
#pragma unroll
  for (int ht = 0; ht < 2; ++ht) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < ks_n; ++ks) {
      const int o = ks * 4 + lg;
      const float a = o < out ? p[lds_offsets(F, K).w2[ML] + o * C::W2S + ht * 16 + li] : 0.f;
      const float b = o < out ? dy[li * C::YS + O.yoff[ML] + o] : 0.f;
      acc = mfma(a, b, acc);
    }
    dH[2 * ML + ht] = acc;
  }
}

// dW2 of MLP ML += dY^T H over the 16 anchors of the chunk (A from dY, B from H in LDS).
template <int F, int K, int ML, int OT, int BASE>
__device__ __forceinline__ void acc_dW2(const float* dy, const float* hs, int l, f4* dW2) {
  using C = Cfg<F, K>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr int out = O.out[ML];
  const int li = l & 15, lg = l >> 4;
#pragma unroll
  for (int ot = 0; ot < OT; ++ot) {
    const int o = ot * 16 + li;
#pragma unroll
    for (int ht = 0; ht < 2; ++ht) {
      f4 acc = dW2[BASE + ot * 2 + ht];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int an = ks * 4 + lg;
        const float a = o < out ? dy[an * C::YS + O.yoff[ML] + o] : 0.f;
        const float b = hs[an * C::HS + ML * 32 + ht * 16 + li];
        acc = mfma(a, b, acc);
      }
      dW2[BASE + ot * 2 + ht] = acc;
    }
  }
}

template <int F, int K, int ML, int OT, int BASE>
__device__ __forceinline__ void store_dW2(const f4* dW2, float* red, int l) {
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr int out = O.out[ML];
  const int li = l & 15, lg = l >> 4;
#pragma unroll
  for (int ot = 0; ot < OT; ++ot)
#pragma unroll
    for (int ht = 0; ht < 2; ++ht)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = ot * 16 + 4 * lg + r;
        if (o < out) atomicAdd(&red[O.w2[ML] + o * kHid + ht * 16 + li], dW2[BASE + ot * 2 + ht][r]);
      }
}

// Work split of the adjoint: partition m owns workgroups [first[m], first[m+1]) of a 1-D
// grid (about one workgroup per CU, shared in proportion to the partitions' anchor
// counts); leader[m] is the first of the partition's (consecutive) views.
constexpr int kMaxBwdParts = 256;
constexpr int kBwdWaves = 4;
struct BwdGrid {
  int n_parts;
  int first[kMaxBwdParts + 1];
  int leader[kMaxBwdParts];
  int n_views_of[kMaxBwdParts];
};

// Orders this wave's LDS traffic (the waves of a workgroup run independently).

template <int F, int K>
__global__ void __launch_bounds__(64 * kBwdWaves) decode_bwd_kernel(glam_anchors an, const float* __restrict__ mlp,
                                                                    const glam_view_info* views, int sigmoid_op,
                                                                    glam_gaussians dg, BwdGrid grid, float* dfeat,
                                                                    float* doffs, float* dlog_scale, float* partial) {
  using C = Cfg<F, K>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr int NT2 = 2 * (C::OT0 + C::OT1 + C::OT2);
  constexpr int NC1 = (C::NIN + 15) / 16;
  extern __shared__ float smem[];
  // partition of this workgroup
  int m = 0;
  while (m + 1 < grid.n_parts && grid.first[m + 1] <= (int)blockIdx.x) ++m;
  const int b_local = blockIdx.x - grid.first[m], nb = grid.first[m + 1] - grid.first[m];
  const int v0 = grid.leader[m], v1 = v0 + grid.n_views_of[m];
  const glam_view_info lead = views[v0];
  const int A = lead.anchor_count;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lg = l >> 4;
  float* s_p = smem;
  float* base = smem + C::PA + w * (16 * C::ZS + 16 * C::YS + 16 * C::HS + 16);
  float* s_z = base;
  float* s_y = s_z + 16 * C::ZS;
  float* s_h = s_y + 16 * C::YS;
  float* s_ds = s_h + 16 * C::HS;
  const float* pm = mlp + (size_t)lead.cam.partition * C::P;
  load_weights<F, K>(pm, s_p, t, 64 * kBwdWaves);
  __syncthreads();
  f4 dW2[NT2];
  f4 dW1[6 * NC1];
  float db2[(C::NY + 63) / 64];
  float db1[2];
#pragma unroll
  for (int i = 0; i < NT2; ++i) dW2[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 6 * NC1; ++i) dW1[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < (C::NY + 63) / 64; ++i) db2[i] = 0.f;
  db1[0] = db1[1] = 0.f;
  const long long n = dg.n;
  const size_t GK = (size_t)an.A * K;
  const int n_chunks = (A + 15) / 16;
  // each wave walks its chunks independently: no workgroup barrier until the end
  for (int chunk = b_local * kBwdWaves + w; chunk < n_chunks; chunk += nb * kBwdWaves) {
    const int a0 = chunk * 16;
    f4 dZ[F / 16];
#pragma unroll
    for (int i = 0; i < F / 16; ++i) dZ[i] = f4{0.f, 0.f, 0.f, 0.f};
    float doff[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (l < 16) s_ds[l] = 0.f;
    for (int v = v0; v < v1; ++v) {
      const glam_view_info vw = views[v];
      build_z<F, K>(an, vw, a0, s_z, l);  // zero rows past the partition
      wave_sync();
      f4 H[6];
      layer1<F, K>(s_p, s_z, l, H);
      layer2<F, K, 0, C::OT0>(s_p, H, s_y, l);
      layer2<F, K, 1, C::OT1>(s_p, H, s_y, l);
      layer2<F, K, 2, C::OT2>(s_p, H, s_y, l);
      // H to LDS (anchor-major) for the dW2 contraction
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_h[li * C::HS + mt * 16 + 4 * lg + r] = H[mt][r];
      wave_sync();
      // activation adjoints, one lane per Gaussian; dY overwrites Y in place
      for (int q = 0; q < 3; ++q) {
        const int gi = l + 64 * q;
        if (gi >= 16 * K) break;
        const int ai = gi / K, j = gi % K, a = a0 + ai;
        float* y = s_y + ai * C::YS;
        if (a >= A) {
          y[j] = 0.f;
          for (int c = 0; c < 3; ++c) y[K + 3 * j + c] = 0.f;
          for (int k = 0; k < 7; ++k) y[4 * K + 7 * j + k] = 0.f;
          continue;
        }
        const int ga = vw.anchor_begin + a;
        const long long g = vw.g_begin + (long long)a * K + j;
        const float es = expf(an.log_scale[ga]);
        float ds = 0.f;
        const float yo = y[j];
        const float dop = dg.opacity[g];
        if (sigmoid_op) {
          const float al = sigmoid(yo);
          y[j] = dop * al * (1.f - al);
        } else {
          const float al = tanhf(yo);
          y[j] = al > 0.f ? dop * (1.f - al * al) : 0.f;
        }
        for (int c = 0; c < 3; ++c) {
          const float col = sigmoid(y[K + 3 * j + c]);
          y[K + 3 * j + c] = dg.rgb[c * n + g] * col * (1.f - col);
        }
        float* yc = y + 4 * K + 7 * j;
        for (int k = 0; k < 3; ++k) {
          const float sg = sigmoid(yc[k]);
          const float dsc = dg.scale[k * n + g];
          yc[k] = dsc * es * sg * (1.f - sg);
          ds = fmaf(dsc, es * sg, ds);
        }
        const float nr = sqrtf(yc[3] * yc[3] + yc[4] * yc[4] + yc[5] * yc[5] + yc[6] * yc[6] + 1e-24f);
        const float inv = 1.f / nr;
        float dq[4], qd = 0.f;
        for (int k = 0; k < 4; ++k) { dq[k] = dg.quat[k * n + g]; qd = fmaf(yc[3 + k] * inv, dq[k], qd); }
        for (int k = 0; k < 4; ++k) yc[3 + k] = (dq[k] - yc[3 + k] * inv * qd) * inv;
        const size_t go = (size_t)ga * K + j;
        for (int i = 0; i < 3; ++i) {
          const float dm = dg.mean[i * n + g];
          doff[q][i] = fmaf(es, dm, doff[q][i]);
          ds = fmaf(es * an.offs[i * GK + go], dm, ds);
        }
        atomicAdd(&s_ds[ai], ds);
      }
      wave_sync();
      // dH = W2^T dY, masked by the ReLU (H > 0 exactly where pre > 0)
      f4 dP[6];
      dhidden<F, K, 0>(s_p, s_y, l, dP);
      dhidden<F, K, 1>(s_p, s_y, l, dP);
      dhidden<F, K, 2>(s_p, s_y, l, dP);
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dP[mt][r] = H[mt][r] > 0.f ? dP[mt][r] : 0.f;
      // dZ (feature rows only) = W1^T dPre, K-steps over hidden rows in register order
#pragma unroll
      for (int ft = 0; ft < F / 16; ++ft) {
        f4 acc = dZ[ft];
#pragma unroll
        for (int mt = 0; mt < 6; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int h = mt * 16 + 4 * lg + r;
            const float a = s_p[lds_offsets(F, K).w1[h >> 5] + (h & 31) * C::W1S + ft * 16 + li];
            acc = mfma(a, dP[mt][r], acc);
          }
        dZ[ft] = acc;
      }
      // dW2 += dY^T H, db2 += sum dY
      acc_dW2<F, K, 0, C::OT0, 0>(s_y, s_h, l, dW2);
      acc_dW2<F, K, 1, C::OT1, 2 * C::OT0>(s_y, s_h, l, dW2);
      acc_dW2<F, K, 2, C::OT2, 2 * (C::OT0 + C::OT1)>(s_y, s_h, l, dW2);
#pragma unroll
      for (int i = 0; i < (C::NY + 63) / 64; ++i) {
        const int o = l + 64 * i;
        if (o < C::NY)
          for (int an_ = 0; an_ < 16; ++an_) db2[i] += s_y[an_ * C::YS + o];
      }
      wave_sync();
      // dPre to LDS (reusing the H buffer) for dW1 += dPre^T Z, db1 += sum dPre
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_h[li * C::HS + mt * 16 + 4 * lg + r] = dP[mt][r];
      wave_sync();
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
#pragma unroll
        for (int ct = 0; ct < NC1; ++ct) {
          f4 acc = dW1[mt * NC1 + ct];
          const int col = ct * 16 + li;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int an_ = ks * 4 + lg;
            const float a = s_h[an_ * C::HS + mt * 16 + li];
            const float b = col < C::NIN ? s_z[an_ * C::ZS + col] : 0.f;
            acc = mfma(a, b, acc);
          }
          dW1[mt * NC1 + ct] = acc;
        }
      for (int i = 0; i < 2; ++i) {
        const int h = l + 64 * i;
        if (h < 96)
          for (int an_ = 0; an_ < 16; ++an_) db1[i] += s_h[an_ * C::HS + h];
      }
      wave_sync();
    }
    // anchor gradients of this chunk (all views summed)
#pragma unroll
    for (int ft = 0; ft < F / 16; ++ft)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + li;
        if (a < A) dfeat[(size_t)(lead.anchor_begin + a) * F + ft * 16 + 4 * lg + r] = dZ[ft][r];
      }
    if (l < 16 && a0 + l < A) dlog_scale[lead.anchor_begin + a0 + l] = s_ds[l];
    for (int q = 0; q < 3; ++q) {
      const int gi = l + 64 * q;
      if (gi >= 16 * K) break;
      const int ai = gi / K, j = gi % K, a = a0 + ai;
      if (a >= A) continue;
      const size_t go = (size_t)(lead.anchor_begin + a) * K + j;
      for (int i = 0; i < 3; ++i) doffs[i * GK + go] = doff[q][i];
    }
    wave_sync();
  }
  // workgroup reduction of the weight gradients into the packed layout
  __syncthreads();
  float* red = s_p;
  for (int i = t; i < C::P; i += 64 * kBwdWaves) red[i] = 0.f;
  __syncthreads();
  store_dW2<F, K, 0, C::OT0, 0>(dW2, red, l);
  store_dW2<F, K, 1, C::OT1, 2 * C::OT0>(dW2, red, l);
  store_dW2<F, K, 2, C::OT2, 2 * (C::OT0 + C::OT1)>(dW2, red, l);
#pragma unroll
  for (int i = 0; i < (C::NY + 63) / 64; ++i) {
    const int o = l + 64 * i;
    if (o < C::NY) {
      const int ml = o < K ? 0 : (o < 4 * K ? 1 : 2);
      atomicAdd(&red[O.b2[ml] + o - O.yoff[ml]], db2[i]);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 6; ++mt)
#pragma unroll
    for (int ct = 0; ct < NC1; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h = mt * 16 + 4 * lg + r, col = ct * 16 + li;
        if (col < C::NIN) atomicAdd(&red[O.w1[h >> 5] + (h & 31) * C::NIN + col], dW1[mt * NC1 + ct][r]);
      }
  for (int i = 0; i < 2; ++i) {
    const int h = l + 64 * i;
    if (h < 96) atomicAdd(&red[O.b1[h >> 5] + (h & 31)], db1[i]);
  }
  __syncthreads();
  float* dst = partial + (size_t)blockIdx.x * C::P;
  for (int i = t; i < C::P; i += 64 * kBwdWaves) dst[i] = red[i];
}

// dmlp[m] = sum of partition m's workgroup partials (zero for partitions without
// views).  Block: 16 parameters x 16 partial groups, contiguous 64-byte reads.
__global__ void __launch_bounds__(256) mlp_grad_reduce_kernel(const float* partial, BwdGrid grid, int P, int M,
                                                              float* dmlp) {
  __shared__ float s[16][17];
  const int c = threadIdx.x & 15, r = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + c;
  const int slot = blockIdx.y;  // index into grid (partitions with views)
  float acc = 0.f;
  if (i < P)
    for (int b = grid.first[slot] + r; b < grid.first[slot + 1]; b += 16) acc += partial[(size_t)b * P + i];
  s[r][c] = acc;
  __syncthreads();
  if (r == 0 && i < P) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += s[k][c];
    dmlp[(size_t)grid.leader[slot] * P + i] = t;  // leader holds the partition index here
  }
}

__global__ void zero_f32_kernel(float* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

template <int F, int K>
size_t fwd_smem() {
  using C = Cfg<F, K>;
  return sizeof(float) * (C::PA + 4 * 16 * C::ZS + 4 * 16 * C::YS);
}

template <int F, int K>
size_t bwd_smem() {
  using C = Cfg<F, K>;
  return sizeof(float) * (C::PA + kBwdWaves * (16 * C::ZS + 16 * C::YS + 16 * C::HS + 16));
}

// Raises a kernel's dynamic LDS limit above the 64 KiB default.  Not a stream operation;
// skipped while the stream is being captured (the first, eager call has set it).
bool set_smem_limit(const void* fn, size_t bytes, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
  if (cs != hipStreamCaptureStatusNone) return true;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

int max_anchors(const glam_views& v) {
  int mx = 0;
  for (int i = 0; i < v.n; ++i) mx = v.host[i].anchor_count > mx ? v.host[i].anchor_count : mx;
  return mx;
}

// One workgroup per CU in total, shared by the partitions in proportion to their anchor
// counts (at least one each, never more than their 16-anchor chunks / 8 waves).
int total_bwd_blocks() { return cu_count(); }

bool bwd_grid(const glam_views& v, BwdGrid& g) {
  g.n_parts = 0;
  long long total_anchors = 0;
  for (int i = 0; i < v.n; ++i) {
    const glam_view_info& vi = v.host[i];
    if (i > 0 && v.host[i - 1].cam.partition == vi.cam.partition) {
      ++g.n_views_of[g.n_parts - 1];
      continue;
    }
    if (g.n_parts == kMaxBwdParts) return false;
    g.leader[g.n_parts] = i;
    g.n_views_of[g.n_parts] = 1;
    ++g.n_parts;
    total_anchors += vi.anchor_count;
  }
  const int budget = total_bwd_blocks();
  int b = 0;
  for (int k = 0; k < g.n_parts; ++k) {
    const int A = v.host[g.leader[k]].anchor_count;
    const int cap = (A + 16 * kBwdWaves - 1) / (16 * kBwdWaves);
    int nb = total_anchors > 0 ? (int)((double)budget * A / (double)total_anchors + 0.5) : 1;
    nb = nb < 1 ? 1 : (nb > cap ? (cap < 1 ? 1 : cap) : nb);
    g.first[k] = b;
    b += nb;
  }
  g.first[g.n_parts] = b;
  return true;
}

template <int F, int K>
glam_status run_decode(const glam_anchors& a, const float* mlp, const glam_views& v, bool sig,
                       const glam_gaussians& out, hipStream_t s) {
  const int mx = max_anchors(v);
  if (mx == 0 || v.n == 0) return GLAM_OK;
  const size_t sm = fwd_smem<F, K>();
  if (!set_smem_limit((const void*)decode_kernel<F, K>, sm, s)) return GLAM_ERR_HIP;
  // groups of 64 anchors per block: enough blocks to fill every CU four times over,
  // each staging the weights as few times as that allows
  const int groups = (mx + 63) / 64;
  const long long target = 4LL * cu_count();
  int chunks = (int)(((long long)groups * v.n + target - 1) / target);
  chunks = chunks < 1 ? 1 : (chunks > 16 ? 16 : chunks);
  const int nbx = (groups + chunks - 1) / chunks;
  hipLaunchKernelGGL((decode_kernel<F, K>), dim3(nbx, v.n), dim3(256), sm, s, a, mlp, v.dev, sig ? 1 : 0, chunks,
                     out);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

template <int F, int K>
glam_status run_decode_bwd(const glam_anchors& a, const float* mlp, int n_parts, const glam_views& v, bool sig,
                           const glam_gaussians& dg, float* dfeat, float* doffs, float* dls, float* dmlp, void* ws,
                           hipStream_t s) {
  using C = Cfg<F, K>;
  BwdGrid g;
  if (!bwd_grid(v, g)) return GLAM_ERR_UNSUPPORTED;
  float* partial = static_cast<float*>(ws);
  // partitions without views get zero gradients
  const long long nm = (long long)n_parts * C::P;
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, dmlp, nm);
  if (g.first[g.n_parts] > 0) {
    const size_t sm = bwd_smem<F, K>();
    if (!set_smem_limit((const void*)decode_bwd_kernel<F, K>, sm, s)) return GLAM_ERR_HIP;
    hipLaunchKernelGGL((decode_bwd_kernel<F, K>), dim3(g.first[g.n_parts]), dim3(64 * kBwdWaves), sm, s, a, mlp,
                       v.dev, sig ? 1 : 0, dg, g, dfeat, doffs, dls, partial);
    // the reduction writes dmlp[partition of slot k]: pass partitions in place of leaders
    BwdGrid r = g;
    for (int k = 0; k < g.n_parts; ++k) r.leader[k] = v.host[g.leader[k]].cam.partition;
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((C::P + 15) / 16, g.n_parts), dim3(256), 0, s, partial, r, C::P,
                       n_parts, dmlp);
  }
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace

#define GLAM_DECODE_CASES(X) X(32, 10) X(16, 4)

glam_status launch_decode(const glam_anchors& a, const float* mlp, const glam_views& v, bool sig,
                          const glam_gaussians& out, hipStream_t s) {
#define X(F_, K_) if (a.F == F_ && a.K == K_) return run_decode<F_, K_>(a, mlp, v, sig, out, s);
  GLAM_DECODE_CASES(X)
#undef X
  return GLAM_ERR_UNSUPPORTED;
}

size_t decode_bwd_workspace(const glam_anchors& a, const glam_views& v, int n_parts) {
  (void)n_parts;
  const MlpOff o = mlp_offsets(a.F, a.K);
  BwdGrid g;
  if (!bwd_grid(v, g)) return 0;
  return sizeof(float) * (size_t)o.total * (size_t)(g.first[g.n_parts] > 0 ? g.first[g.n_parts] : 1);
}

glam_status launch_decode_bwd(const glam_anchors& a, const float* mlp, int n_parts, const glam_views& v, bool sig,
                              const glam_gaussians& dg, float* dfeat, float* doffs, float* dls, float* dmlp, void* ws,
                              hipStream_t s) {
#define X(F_, K_) \
  if (a.F == F_ && a.K == K_) return run_decode_bwd<F_, K_>(a, mlp, n_parts, v, sig, dg, dfeat, doffs, dls, dmlp, ws, s);
  GLAM_DECODE_CASES(X)
#undef X
  return GLAM_ERR_UNSUPPORTED;
}

bool decode_supported(int F, int K) {
#define X(F_, K_) if (F == F_ && K == K_) return true;
  GLAM_DECODE_CASES(X)
#undef X
  return false;
}

}  // namespace glam
