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
#include "projection.hpp"

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

// LDS word of packed weight i (the padded layout of lds_offsets), from compile-time
// constants only: no table is indexed at run time.
template <int F, int K>
__host__ __device__ constexpr int lds_word(int i) {
  constexpr int nin = F + 4, w1s = F + 5, w2s = kHid + 1;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr LdsOff L = lds_offsets(F, K);
  const bool m0 = i < O.w1[1], m1 = !m0 && i < O.w1[2];
  const int base = m0 ? O.w1[0] : (m1 ? O.w1[1] : O.w1[2]);
  const int lbase = m0 ? L.w1[0] : (m1 ? L.w1[1] : L.w1[2]);
  const int out = m0 ? K : (m1 ? 3 * K : 7 * K);
  const int j = i - base;
  if (j < kHid * nin) return lbase + (j / nin) * w1s + j % nin;  // W1 row j / nin
  const int j1 = j - kHid * nin;
  if (j1 < kHid) return lbase + kHid * w1s + j1;  // b1
  const int j2 = j1 - kHid;
  if (j2 < out * kHid) return lbase + kHid * w1s + kHid + (j2 / kHid) * w2s + j2 % kHid;  // W2 row j2 / kHid
  return lbase + kHid * w1s + kHid + out * w2s + (j2 - out * kHid);  // b2
}

// lds_word against the offset tables, for every packed weight (checked when compiling).
template <int F, int K>
constexpr bool lds_word_matches() {
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr LdsOff L = lds_offsets(F, K);
  for (int i = 0; i < O.total; ++i) {
    const int l = i < O.w1[1] ? 0 : (i < O.w1[2] ? 1 : 2);
    const int j = i - O.w1[l];
    int dst;
    if (j < kHid * (F + 4)) dst = L.w1[l] + (j / (F + 4)) * (F + 5) + j % (F + 4);
    else if (j < kHid * (F + 4) + kHid) dst = L.b1[l] + (j - kHid * (F + 4));
    else if (j < O.b2[l] - O.w1[l]) dst = L.w2[l] + ((j - kHid * (F + 4) - kHid) / kHid) * (kHid + 1) +
                                            (j - kHid * (F + 4) - kHid) % kHid;
    else dst = L.b2[l] + (j - (O.b2[l] - O.w1[l]));
    if (dst != lds_word<F, K>(i)) return false;
  }
  return true;
}

// Copies one packed MLP set into the padded LDS layout, by a workgroup of 256 threads:
// every thread's loads are issued before its first store, so the copy costs about one
// memory latency instead of one per word.
template <int F, int K>
__device__ __forceinline__ void load_weights(const float* pm, float* s, int t) {
  using C = Cfg<F, K>;
  static_assert(lds_word_matches<F, K>(), "LDS layout of the weights");
  constexpr int kN = (C::P + 255) / 256;
  float v[kN];
#pragma unroll
  for (int n = 0; n < kN; ++n) {
    const int i = t + 256 * n;
    v[n] = i < C::P ? pm[i] : 0.f;
  }
#pragma unroll
  for (int n = 0; n < kN; ++n) {
    const int i = t + 256 * n;
    if (i < C::P) s[lds_word<F, K>(i)] = v[n];
  }
}

// The camera centre -R^T t (compensated: camera translations of kilometres keep every
// digit of the anchors' directions and distances from it).
__device__ __forceinline__ void camera_centre(const glam_camera& c, float xc[3]) {
  for (int i = 0; i < 3; ++i) xc[i] = -dot3_add(c.R[i], c.R[3 + i], c.R[6 + i], c.t[0], c.t[1], c.t[2], 0.f);
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

// Work split of the decode and its adjoint over partitions: partition slot k (a run of
// consecutive views of one partition) owns workgroups [first[k], first[k+1]) of a 1-D
// grid, shared in proportion to the partitions' anchor counts; its views are
// [leader[k], leader[k+1]).  The adjoint's workgroups of a slot differentiate one MLP
// each: the first (split[k] & 0xffff) the opacity MLP, the next (split[k] >> 16) the
// colour MLP, the rest the covariance MLP.
constexpr int kMaxBwdParts = 256;
struct BwdGrid {
  int n_parts;
  int first[kMaxBwdParts + 1];
  int leader[kMaxBwdParts + 1];
  int split[kMaxBwdParts];
};

// A workgroup stages its partition's weights once; each wave then takes 16-anchor
// chunks and, for every view of the partition, decodes the chunk's Gaussians.  What
// does not depend on the view (features, the features' share of layer 1, positions,
// scales, offsets) is loaded and computed once per chunk.
template <int F, int K>
__global__ void __launch_bounds__(256) decode_kernel(glam_anchors an, const float* __restrict__ mlp,
                                                     const glam_view_info* views, int sigmoid_op, BwdGrid grid,
                                                     glam_gaussians out, int fuse_project, int tl,
                                                     int sigma3, glam_projected proj) {
  using C = Cfg<F, K>;
  constexpr LdsOff L = lds_offsets(F, K);
  extern __shared__ float smem[];
  int m = 0;
  while (m + 1 < grid.n_parts && grid.first[m + 1] <= (int)blockIdx.x) ++m;
  const int b_local = (int)blockIdx.x - grid.first[m], nb = grid.first[m + 1] - grid.first[m];
  const int v0 = grid.leader[m], v1 = grid.leader[m + 1];
  const glam_view_info lead = views[v0];
  const int A = lead.anchor_count;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lg = l >> 4;
  float* s_p = smem;
  float* s_z = s_p + C::PA + w * 16 * C::ZS;
  float* s_y = smem + C::PA + 4 * 16 * C::ZS + w * 16 * C::YS;
  load_weights<F, K>(mlp + (size_t)lead.cam.partition * C::P, s_p, t);
  __syncthreads();
  const long long n = out.n;
  const size_t GK = (size_t)an.A * K;
  const int n_chunks = (A + 15) / 16;
  for (int chunk = b_local * 4 + w; chunk < n_chunks; chunk += nb * 4) {
    const int a0 = chunk * 16;
    {
      float fv[16 * F / 64];
#pragma unroll
      for (int k = 0; k < 16 * F / 64; ++k) {
        const int idx = l + 64 * k, a = a0 + idx / F;
        fv[k] = a < A ? an.feat[(size_t)(lead.anchor_begin + a) * F + idx % F] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 16 * F / 64; ++k) {
        const int idx = l + 64 * k;
        s_z[(idx / F) * C::ZS + idx % F] = fv[k];
      }
    }
    float apos[3] = {0.f, 0.f, 0.f};
    if (l < 16 && a0 + l < A)
      for (int i = 0; i < 3; ++i) apos[i] = an.pos[(size_t)i * an.A + lead.anchor_begin + a0 + l];
    // per Gaussian of this lane: e^{s_a} and its (view-independent) mean
    float es[3] = {0.f, 0.f, 0.f}, mu[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int gi = l + 64 * q, a = a0 + gi / K;
      if (gi < 16 * K && a < A) {
        const int ga = lead.anchor_begin + a;
        es[q] = expf(an.log_scale[ga]);
        for (int i = 0; i < 3; ++i)
          mu[q][i] = fmaf(es[q], an.offs[i * GK + (size_t)ga * K + gi % K], an.pos[(size_t)i * an.A + ga]);
      }
    }
    wave_sync();
    // the features' share of layer 1 (all K-steps but the last, which holds d and delta)
    f4 PF[6];
#pragma unroll
    for (int mt = 0; mt < 6; ++mt) {
      const int h = mt * 16 + li;
      const float* W1 = s_p + L.w1[h >> 5] + (h & 31) * C::W1S;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < C::KS1 - 1; ++ks) acc = mfma(W1[ks * 4 + lg], s_z[li * C::ZS + ks * 4 + lg], acc);
      PF[mt] = acc;
    }
    for (int v = v0; v < v1; ++v) {
      const glam_view_info vw = views[v];
      if (l < 16) {
        float d[3] = {0.f, 0.f, 0.f}, delta = 0.f;
        if (a0 + l < A) {
          float xc[3];
          camera_centre(vw.cam, xc);
          for (int i = 0; i < 3; ++i) d[i] = apos[i] - xc[i];
          delta = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          const float inv = 1.f / delta;
          for (int i = 0; i < 3; ++i) d[i] *= inv;
        }
        s_z[l * C::ZS + F + 0] = d[0];
        s_z[l * C::ZS + F + 1] = d[1];
        s_z[l * C::ZS + F + 2] = d[2];
        s_z[l * C::ZS + F + 3] = delta;
      }
      wave_sync();
      f4 H[6];
#pragma unroll
      for (int mt = 0; mt < 6; ++mt) {
        const int h = mt * 16 + li;
        const float* W1 = s_p + L.w1[h >> 5] + (h & 31) * C::W1S;
        constexpr int ks = C::KS1 - 1;
        f4 acc = mfma(W1[ks * 4 + lg], s_z[li * C::ZS + ks * 4 + lg], PF[mt]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int hr = mt * 16 + 4 * lg + r;
          acc[r] = fmaxf(acc[r] + s_p[L.b1[hr >> 5] + (hr & 31)], 0.f);
        }
        H[mt] = acc;
      }
      layer2<F, K, 0, C::OT0>(s_p, H, s_y, l);
      layer2<F, K, 1, C::OT1>(s_p, H, s_y, l);
      layer2<F, K, 2, C::OT2>(s_p, H, s_y, l);
      wave_sync();
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int gi = l + 64 * q;
        if (gi >= 16 * K) break;
        const int ai = gi / K, j = gi % K, a = a0 + ai;
        if (a >= A) continue;
        const float* y = s_y + ai * C::YS;
        const long long g = vw.g_begin + (long long)a * K + j;
        const float yo = y[j];
        const float op = sigmoid_op ? sigmoid(yo) : tanhf(yo);
        float rgb[3], sc[3], qn[4];
        for (int c3 = 0; c3 < 3; ++c3) rgb[c3] = sigmoid(y[K + 3 * j + c3]);
        for (int k = 0; k < 3; ++k) sc[k] = es[q] * sigmoid(y[4 * K + 7 * j + k]);
        const float* qv = y + 4 * K + 7 * j + 3;
        const float inv = 1.f / sqrtf(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3] + 1e-24f);
        for (int k = 0; k < 4; ++k) qn[k] = qv[k] * inv;
        out.opacity[g] = op;
        for (int c3 = 0; c3 < 3; ++c3) out.rgb[c3 * n + g] = rgb[c3];
        for (int k = 0; k < 3; ++k) out.scale[k * n + g] = sc[k];
        for (int k = 0; k < 4; ++k) out.quat[k * n + g] = qn[k];
        for (int i = 0; i < 3; ++i) out.mean[i * n + g] = mu[q][i];
        // the projection of the Gaussian just decoded, from the same registers
        if (fuse_project) project_one(vw.cam, mu[q], sc, qn, op, rgb, g, n, tl, sigma3 != 0, proj);
      }
      // the next view's rows overwrite rows these outputs were read from
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------------

// The adjoint is split by MLP: a workgroup differentiates one of the three MLPs, so a
// wave holds only that MLP's weight-gradient accumulators in registers and stages only
// its weights in LDS.  Everything the three MLPs share (the input rows Z and the ReLU
// pattern of their own hidden layer) is cheap to rebuild.  The workgroups of each MLP
// are counted so that the three finish together (the covariance MLP's chunks cost about
// twice the others').
constexpr int kBwdWaves = 4;
constexpr int kBwdBlocksPerCU = 2;  // workgroups resident per CU (registers: two waves per SIMD)

constexpr int align4(int x) { return (x + 3) & ~3; }

// LDS layout of one MLP's adjoint.  Operands of the MFMAs are read four K-steps at a
// time (one 16-byte LDS read): the K order of each product is chosen so that a lane's
// four consecutive K-steps are four consecutive words, with transposed copies where a
// product runs over the other index (W2^T, W1^T; Y and H are kept output-major).  Row
// strides are multiples of four words whose 16 rows fall in distinct banks.
// Feature widths that are not a multiple of 16 are zero-padded to one inside the
// adjoint (FP columns): padded weight columns and inputs are zero, and their gradients
// are dropped, so the packed layout in HBM keeps the width F.
template <int F, int K, int ML>
struct MCfg {
  static constexpr int FP = (F + 15) / 16 * 16;  // feature columns inside the adjoint
  static constexpr int NIN = FP + 4;             // layer-1 inputs inside the adjoint
  static constexpr int NINP = F + 4;             // layer-1 inputs in the packed layout
  static constexpr int OUT = ML == 0 ? K : (ML == 1 ? 3 * K : 7 * K);
  static constexpr int OUTP = (OUT + 15) / 16 * 16;  // outputs padded to 16-row tiles
  static constexpr int OT = OUTP / 16;
  static constexpr int KF = FP / 4;            // feature columns per lane group in layer 1
  static constexpr int NC1 = (NIN + 15) / 16;  // 16-column tiles of W1
  static constexpr int W1S = NIN, W2S = kHid + 4, W2TS = OUTP + 4, W1TS = kHid + 4;
  static constexpr int LW1 = 0, LB1 = kHid * W1S, LW2 = align4(LB1 + kHid), LB2 = LW2 + OUT * W2S;
  static constexpr int LW2T = align4(LB2 + OUT), LW1T = LW2T + kHid * W2TS;
  static constexpr int PW = align4(LW1T + FP * W1TS);
  static constexpr int PM = kHid * NINP + kHid + OUT * kHid + OUT;  // packed parameters
  static constexpr int ZS = NIN, YTS = 20, HTS = 20;
  // per wave: Z [16][NIN] anchor-major; Y^T [OUTP][20] and H^T [32][20] output-major
  static constexpr int WAVE_WORDS = align4(16 * ZS + OUTP * YTS + kHid * HTS + 16);
  static constexpr int SMEM = PW + kBwdWaves * WAVE_WORDS;
  static_assert(NIN % 4 == 0 && FP % 16 == 0 && F % 4 == 0, "layout");
  // internal layer-1 column of packed column c, and back (-1: a padding column)
  static constexpr __host__ __device__ int col_in(int c) { return c < F ? c : c + (FP - F); }
  static constexpr __host__ __device__ int col_packed(int c) { return c < F ? c : (c < FP ? -1 : c - (FP - F)); }
};

template <int F, int K>
constexpr int bwd_smem_words() {
  constexpr int a = MCfg<F, K, 0>::SMEM, b = MCfg<F, K, 1>::SMEM, c = MCfg<F, K, 2>::SMEM;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

__device__ __forceinline__ float4 lds4(const float* p) { return *reinterpret_cast<const float4*>(p); }

__device__ __forceinline__ f4 mfma4(const float4& a, const float4& b, f4 acc) {
  acc = mfma(a.x, b.x, acc);
  acc = mfma(a.y, b.y, acc);
  acc = mfma(a.z, b.z, acc);
  return mfma(a.w, b.w, acc);
}

template <int F, int K, int ML>
__device__ void decode_bwd_mlp(const glam_anchors& an, const float* __restrict__ mlp,
                               const glam_view_info* views, int sigmoid_op, const glam_gaussians& dg,
                               const BwdGrid& grid, int m, int b_local, int nb, float* doffs, float* dfeat_part,
                               float* dls_part, float* partial, float* smem) {
  using C = MCfg<F, K, ML>;
  constexpr MlpOff O = mlp_offsets(F, K);
  constexpr int OUT = C::OUT;
  const int v0 = grid.leader[m], v1 = grid.leader[m + 1];
  const glam_view_info lead = views[v0];
  const int A = lead.anchor_count;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lg = l >> 4;
  float* s_p = smem;
  float* s_z = smem + C::PW + w * C::WAVE_WORDS;
  float* s_yt = s_z + 16 * C::ZS;
  float* s_ht = s_yt + C::OUTP * C::YTS;
  float* s_ds = s_ht + kHid * C::HTS;
  const long long n = dg.n;
  const size_t GK = (size_t)an.A * K;
  const int n_chunks = (A + 15) / 16;
  // view-independent inputs of a chunk (features, anchor positions and, per Gaussian of
  // this lane, the log-scale and offsets), loaded into registers one chunk ahead so
  // that their latency hides behind the current chunk's work
  struct ChunkIn {
    float fv[16 * F / 64];
    float apos[3];
    float ls[3];
    float off[3][3];
  };
  auto load_chunk = [&](int chunk, ChunkIn& in) {
    const int a0 = chunk * 16;
#pragma unroll
    for (int k = 0; k < 16 * F / 64; ++k) {
      const int idx = l + 64 * k, ai = idx / F, a = a0 + ai;
      in.fv[k] = a < A ? an.feat[(size_t)(lead.anchor_begin + a) * F + idx % F] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
      in.apos[i] = l < 16 && a0 + l < A ? an.pos[(size_t)i * an.A + lead.anchor_begin + a0 + l] : 0.f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int gi = l + 64 * q, ai = gi / K, a = a0 + ai;
      const bool ok = ML != 1 && gi < 16 * K && a < A;
      const int ga = lead.anchor_begin + (ok ? a : 0);
      in.ls[q] = ok ? an.log_scale[ga] : 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) in.off[q][i] = ok && ML == 0 ? an.offs[i * GK + (size_t)ga * K + gi % K] : 0.f;
    }
  };
  // (wide features: no prefetch, the registers would spill); the first chunk's loads
  // are issued before the weights are staged, so that the two latencies overlap
  constexpr bool kPrefetch = F <= 32;
  const int chunk_step = nb * kBwdWaves;
  ChunkIn nxt;
  if (kPrefetch && b_local * kBwdWaves + w < n_chunks) load_chunk(b_local * kBwdWaves + w, nxt);
  {  // this MLP's weights: W1, b1, W2 (rows padded to 36), b2, and the transposes W2^T, W1^T
    const float* pm = mlp + (size_t)lead.cam.partition * O.total + O.w1[ML];
    // every load in flight before the first store (one memory latency, not one per word)
    constexpr int kN = (C::PM + 64 * kBwdWaves - 1) / (64 * kBwdWaves);
    float vw[kN];
#pragma unroll
    for (int n = 0; n < kN; ++n) {
      const int i = t + 64 * kBwdWaves * n;
      vw[n] = i < C::PM ? pm[i] : 0.f;
    }
#pragma unroll
    for (int n = 0; n < kN; ++n) {
      const int i = t + 64 * kBwdWaves * n;
      if (i >= C::PM) break;
      const float v = vw[n];
      if (i < kHid * C::NINP) {
        const int h = i / C::NINP, c = i % C::NINP;
        s_p[C::LW1 + h * C::W1S + C::col_in(c)] = v;
        if (c < F) s_p[C::LW1T + c * C::W1TS + h] = v;
      } else if (i < kHid * C::NINP + kHid) {
        s_p[C::LB1 + (i - kHid * C::NINP)] = v;
      } else if (i < kHid * C::NINP + kHid + OUT * kHid) {
        const int j = i - kHid * C::NINP - kHid, o = j / kHid, h = j % kHid;
        s_p[C::LW2 + o * C::W2S + h] = v;
        s_p[C::LW2T + h * C::W2TS + o] = v;
      } else {
        s_p[C::LB2 + (i - kHid * C::NINP - kHid - OUT * kHid)] = v;
      }
    }
    if (C::FP > F) {  // padding columns of W1 and rows of W1^T
      for (int i = t; i < kHid * (C::FP - F); i += 64 * kBwdWaves)
        s_p[C::LW1 + (i / (C::FP - F)) * C::W1S + F + i % (C::FP - F)] = 0.f;
      for (int i = t; i < (C::FP - F) * C::W1TS; i += 64 * kBwdWaves) s_p[C::LW1T + F * C::W1TS + i] = 0.f;
    }
    for (int i = t; i < kHid * (C::OUTP - OUT); i += 64 * kBwdWaves)
      s_p[C::LW2T + (i / (C::OUTP - OUT)) * C::W2TS + OUT + i % (C::OUTP - OUT)] = 0.f;
    // padded output rows of this wave's Y^T stay zero
    for (int i = l; i < (C::OUTP - OUT) * C::YTS; i += 64) s_yt[OUT * C::YTS + i] = 0.f;
  }
  __syncthreads();
  const float* W1 = s_p + C::LW1;
  const float* W2 = s_p + C::LW2;
  const float* W2T = s_p + C::LW2T;
  const float* W1T = s_p + C::LW1T;
  f4 dW2[2 * C::OT];
  f4 dW1[2 * C::NC1];
  float db2[(OUT + 63) / 64];
  float db1 = 0.f;
#pragma unroll
  for (int i = 0; i < 2 * C::OT; ++i) dW2[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 2 * C::NC1; ++i) dW1[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < (OUT + 63) / 64; ++i) db2[i] = 0.f;
  // each wave walks its chunks independently: no workgroup barrier until the end
  for (int chunk = b_local * kBwdWaves + w; chunk < n_chunks; chunk += chunk_step) {
    const int a0 = chunk * 16;
    ChunkIn cur;
    if (kPrefetch) {
      cur = nxt;
      if (chunk + chunk_step < n_chunks) load_chunk(chunk + chunk_step, nxt);
    } else {
      load_chunk(chunk, cur);
    }
    // features into Z
#pragma unroll
    for (int k = 0; k < 16 * F / 64; ++k) {
      const int idx = l + 64 * k;
      s_z[(idx / F) * C::ZS + idx % F] = cur.fv[k];
    }
    if (C::FP > F)  // zero padding features
      for (int i = l; i < 16 * (C::FP - F); i += 64) s_z[(i / (C::FP - F)) * C::ZS + F + i % (C::FP - F)] = 0.f;
    float apos[3] = {cur.apos[0], cur.apos[1], cur.apos[2]};
    float es[3], off[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int gi = l + 64 * q, a = a0 + gi / K;
      es[q] = ML != 1 && gi < 16 * K && a < A ? expf(cur.ls[q]) : 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) off[q][i] = cur.off[q][i];
    }
    wave_sync();
    // the features' share of layer 1 (lane group g takes feature columns [g KF, g KF + KF))
    f4 PF[2], dPsum[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const float* wr = W1 + (mt * 16 + li) * C::W1S + C::KF * lg;
      const float* zr = s_z + li * C::ZS + C::KF * lg;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q4 = 0; q4 < C::KF / 4; ++q4) acc = mfma4(lds4(wr + 4 * q4), lds4(zr + 4 * q4), acc);
      PF[mt] = acc;
      dPsum[mt] = f4{0.f, 0.f, 0.f, 0.f};
    }
    float doff[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (l < 16) s_ds[l] = 0.f;
    for (int v = v0; v < v1; ++v) {
      const glam_view_info vw = views[v];
      // this view's incoming Gaussian gradients, in flight while the MLP is recomputed
      float pg[3][7];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int gi = l + 64 * q, a = a0 + gi / K;
        const bool ok = gi < 16 * K && a < A;
        const long long g = vw.g_begin + (long long)a * K + gi % K;
#pragma unroll
        for (int k = 0; k < 7; ++k) pg[q][k] = 0.f;
        if (ok) {
          if (ML == 0) {
            pg[q][0] = dg.opacity[g];
            for (int i = 0; i < 3; ++i) pg[q][1 + i] = dg.mean[i * n + g];
          } else if (ML == 1) {
            for (int c = 0; c < 3; ++c) pg[q][c] = dg.rgb[c * n + g];
          } else {
            for (int k = 0; k < 3; ++k) pg[q][k] = dg.scale[k * n + g];
            for (int k = 0; k < 4; ++k) pg[q][3 + k] = dg.quat[k * n + g];
          }
        }
      }
      // direction and distance from this view's camera centre (zero rows past the partition)
      if (l < 16) {
        float d[3] = {0.f, 0.f, 0.f}, delta = 0.f;
        if (a0 + l < A) {
          float xc[3];
          camera_centre(vw.cam, xc);
          for (int i = 0; i < 3; ++i) d[i] = apos[i] - xc[i];
          delta = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          const float inv = 1.f / delta;
          for (int i = 0; i < 3; ++i) d[i] *= inv;
        }
        s_z[l * C::ZS + C::FP + 0] = d[0];
        s_z[l * C::ZS + C::FP + 1] = d[1];
        s_z[l * C::ZS + C::FP + 2] = d[2];
        s_z[l * C::ZS + C::FP + 3] = delta;
      }
      wave_sync();
      // layer 1 completed with the d, delta columns (lane group g: column FP + g)
      f4 H[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        f4 acc = mfma(W1[(mt * 16 + li) * C::W1S + C::FP + lg], s_z[li * C::ZS + C::FP + lg], PF[mt]);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = fmaxf(acc[r] + s_p[C::LB1 + mt * 16 + 4 * lg + r], 0.f);
        H[mt] = acc;
      }
      // layer 2 into Y^T (K-step (t2, r) of lane group g: hidden row 16 t2 + 4 g + r)
#pragma unroll
      for (int ot = 0; ot < C::OT; ++ot) {
        const int o = ot * 16 + li;
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
          const float4 a = o < OUT ? lds4(W2 + o * C::W2S + t2 * 16 + 4 * lg) : make_float4(0.f, 0.f, 0.f, 0.f);
          acc = mfma4(a, make_float4(H[t2][0], H[t2][1], H[t2][2], H[t2][3]), acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = ot * 16 + 4 * lg + r;
          if (orow < OUT) s_yt[orow * C::YTS + li] = acc[r] + s_p[C::LB2 + orow];
        }
      }
      // H^T for dW2
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_ht[(mt * 16 + 4 * lg + r) * C::HTS + li] = H[mt][r];
      wave_sync();
      // activation adjoints, one lane per Gaussian; dY overwrites Y in place
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int gi = l + 64 * q;
        if (gi >= 16 * K) break;
        const int ai = gi / K, j = gi % K, a = a0 + ai;
        float* y = s_yt + ai;  // output o of this anchor at y[o * YTS]
        constexpr int S = C::YTS;
        if (a >= A) {
          if (ML == 0) y[j * S] = 0.f;
          if (ML == 1)
            for (int c = 0; c < 3; ++c) y[(3 * j + c) * S] = 0.f;
          if (ML == 2)
            for (int k = 0; k < 7; ++k) y[(7 * j + k) * S] = 0.f;
          continue;
        }
        if (ML == 0) {
          const float yo = y[j * S];
          const float dop = pg[q][0];
          if (sigmoid_op) {
            const float al = sigmoid(yo);
            y[j * S] = dop * al * (1.f - al);
          } else {
            const float al = tanhf(yo);
            y[j * S] = al > 0.f ? dop * (1.f - al * al) : 0.f;
          }
          // the mean is x_a + e^{s_a} o: offsets and log-scale
          float ds = 0.f;
          for (int i = 0; i < 3; ++i) {
            const float dm = pg[q][1 + i];
            doff[q][i] = fmaf(es[q], dm, doff[q][i]);
            ds = fmaf(es[q] * off[q][i], dm, ds);
          }
          atomicAdd(&s_ds[ai], ds);
        } else if (ML == 1) {
          for (int c = 0; c < 3; ++c) {
            const float col = sigmoid(y[(3 * j + c) * S]);
            y[(3 * j + c) * S] = pg[q][c] * col * (1.f - col);
          }
        } else {
          float yc[7];
          for (int k = 0; k < 7; ++k) yc[k] = y[(7 * j + k) * S];
          float ds = 0.f;
          for (int k = 0; k < 3; ++k) {
            const float sg = sigmoid(yc[k]);
            const float dsc = pg[q][k];
            y[(7 * j + k) * S] = dsc * es[q] * sg * (1.f - sg);
            ds = fmaf(dsc, es[q] * sg, ds);
          }
          const float nr = sqrtf(yc[3] * yc[3] + yc[4] * yc[4] + yc[5] * yc[5] + yc[6] * yc[6] + 1e-24f);
          const float inv = 1.f / nr;
          float qd = 0.f;
          for (int k = 0; k < 4; ++k) qd = fmaf(yc[3 + k] * inv, pg[q][3 + k], qd);
          for (int k = 0; k < 4; ++k) y[(7 * j + 3 + k) * S] = (pg[q][3 + k] - yc[3 + k] * inv * qd) * inv;
          atomicAdd(&s_ds[ai], ds);
        }
      }
      wave_sync();
      // dH^T = W2^T dY^T (K-step (m, r) of lane group g: output 16 m + 4 g + r), masked
      // by the ReLU (H > 0 exactly where the pre-activation is)
      f4 dP[2];
#pragma unroll
      for (int ht = 0; ht < 2; ++ht) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        const float* wr = W2T + (ht * 16 + li) * C::W2TS + 4 * lg;
#pragma unroll
        for (int mo = 0; mo < C::OT; ++mo) {
          const float* yr = s_yt + (16 * mo + 4 * lg) * C::YTS + li;
          acc = mfma4(lds4(wr + 16 * mo),
                      make_float4(yr[0], yr[C::YTS], yr[2 * C::YTS], yr[3 * C::YTS]), acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = H[ht][r] > 0.f ? acc[r] : 0.f;
        dP[ht] = acc;
      }
      // the features' gradients and weight gradients are linear in dPre: sum it over views
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) dPsum[mt] += dP[mt];
      // dW2 += dY^T H over the chunk's 16 anchors (K-step k of lane group g: anchor 4 g + k)
#pragma unroll
      for (int ot = 0; ot < C::OT; ++ot) {
        const float4 a = lds4(s_yt + (ot * 16 + li) * C::YTS + 4 * lg);
#pragma unroll
        for (int ht = 0; ht < 2; ++ht)
          dW2[ot * 2 + ht] = mfma4(a, lds4(s_ht + (ht * 16 + li) * C::HTS + 4 * lg), dW2[ot * 2 + ht]);
      }
#pragma unroll
      for (int i = 0; i < (OUT + 63) / 64; ++i) {
        const int o = l + 64 * i;
        if (o < OUT) {
          const float* yr = s_yt + o * C::YTS;
          float acc = 0.f;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const float4 y4 = lds4(yr + 4 * q4);
            acc += (y4.x + y4.y) + (y4.z + y4.w);
          }
          db2[i] += acc;
        }
      }
      wave_sync();
      // dPre^T (reusing the H^T rows) for the d, delta columns of dW1, this view
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_ht[(mt * 16 + 4 * lg + r) * C::HTS + li] = dP[mt][r];
      wave_sync();
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        constexpr int ct = C::FP / 16;
        const int col = ct * 16 + li;
        const float* zc = s_z + 4 * lg * C::ZS + col;
        const float4 b = col < C::NIN ? make_float4(zc[0], zc[C::ZS], zc[2 * C::ZS], zc[3 * C::ZS])
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
        dW1[mt * C::NC1 + ct] = mfma4(lds4(s_ht + (mt * 16 + li) * C::HTS + 4 * lg), b, dW1[mt * C::NC1 + ct]);
      }
      wave_sync();
    }
    // per chunk, from the view sum of dPre: feature columns of dW1, db1, and the
    // features' gradients dZ = W1_f^T dPre
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) s_ht[(mt * 16 + 4 * lg + r) * C::HTS + li] = dPsum[mt][r];
    wave_sync();
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const float4 a = lds4(s_ht + (mt * 16 + li) * C::HTS + 4 * lg);
#pragma unroll
      for (int ct = 0; ct < C::FP / 16; ++ct) {
        const float* zc = s_z + 4 * lg * C::ZS + ct * 16 + li;
        dW1[mt * C::NC1 + ct] =
            mfma4(a, make_float4(zc[0], zc[C::ZS], zc[2 * C::ZS], zc[3 * C::ZS]), dW1[mt * C::NC1 + ct]);
      }
    }
    if (l < kHid) {
      const float* hr = s_ht + l * C::HTS;
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const float4 h4 = lds4(hr + 4 * q4);
        db1 += (h4.x + h4.y) + (h4.z + h4.w);
      }
    }
    f4 dZ[C::FP / 16];
#pragma unroll
    for (int ft = 0; ft < C::FP / 16; ++ft) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      const float* wr = W1T + (ft * 16 + li) * C::W1TS + 4 * lg;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc = mfma4(lds4(wr + 16 * mt), make_float4(dPsum[mt][0], dPsum[mt][1], dPsum[mt][2], dPsum[mt][3]), acc);
      dZ[ft] = acc;
    }
    // this MLP's share of the anchor gradients (all views summed)
#pragma unroll
    for (int ft = 0; ft < C::FP / 16; ++ft)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + li, f = ft * 16 + 4 * lg + r;
        if (a < A && f < F) dfeat_part[(size_t)(lead.anchor_begin + a) * F + f] = dZ[ft][r];
      }
    if (ML != 1 && l < 16 && a0 + l < A) dls_part[lead.anchor_begin + a0 + l] = s_ds[l];
    if (ML == 0)
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
  // workgroup reduction of this MLP's weight gradients into the packed layout: each wave
  // stores its share (one value per parameter) in a slice of LDS of its own, then every
  // parameter is summed over the slices from zero in wave order, so the sums are
  // reproducible
  static_assert(kBwdWaves * C::PM <= C::SMEM, "reduction slices fit the workgroup's LDS");
  __syncthreads();
  float* red = smem + w * C::PM;  // packed offsets relative to this MLP's first parameter
  constexpr int RW2 = kHid * C::NINP + kHid, RB2 = RW2 + OUT * kHid, RB1 = kHid * C::NINP;
#pragma unroll
  for (int ot = 0; ot < C::OT; ++ot)
#pragma unroll
    for (int ht = 0; ht < 2; ++ht)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = ot * 16 + 4 * lg + r;
        if (o < OUT) red[RW2 + o * kHid + ht * 16 + li] = dW2[ot * 2 + ht][r];
      }
#pragma unroll
  for (int i = 0; i < (OUT + 63) / 64; ++i) {
    const int o = l + 64 * i;
    if (o < OUT) red[RB2 + o] = db2[i];
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int ct = 0; ct < C::NC1; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h = mt * 16 + 4 * lg + r, col = C::col_packed(ct * 16 + li);
        if (col >= 0 && col < C::NINP) red[h * C::NINP + col] = dW1[mt * C::NC1 + ct][r];
      }
  if (l < kHid) red[RB1 + l] = db1;
  __syncthreads();
  // one partial row per workgroup, of which it fills its MLP's parameters
  float* dst = partial + (size_t)blockIdx.x * O.total + O.w1[ML];
  for (int i = t; i < C::PM; i += 64 * kBwdWaves) {
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < kBwdWaves; ++ww) acc += smem[ww * C::PM + i];
    dst[i] = acc;
  }
}

template <int F, int K>
__global__ void __launch_bounds__(64 * kBwdWaves) __attribute__((amdgpu_waves_per_eu(kBwdBlocksPerCU)))
decode_bwd_kernel(glam_anchors an, const float* __restrict__ mlp,
                                                                    const glam_view_info* views, int sigmoid_op,
                                                                    glam_gaussians dg, BwdGrid grid, float* doffs,
                                                                    float* dfeat_part, float* dls_part,
                                                                    float* partial) {
  extern __shared__ float smem[];
  const size_t AF = (size_t)an.A * F;
  int m = 0;
  while (m + 1 < grid.n_parts && grid.first[m + 1] <= (int)blockIdx.x) ++m;
  const int b = (int)blockIdx.x - grid.first[m], nb = grid.first[m + 1] - grid.first[m];
  const int n0 = grid.split[m] & 0xffff, n1 = grid.split[m] >> 16;
  if (b < n0)
    decode_bwd_mlp<F, K, 0>(an, mlp, views, sigmoid_op, dg, grid, m, b, n0, doffs, dfeat_part, dls_part, partial,
                            smem);
  else if (b < n0 + n1)
    decode_bwd_mlp<F, K, 1>(an, mlp, views, sigmoid_op, dg, grid, m, b - n0, n1, doffs, dfeat_part + AF, dls_part,
                            partial, smem);
  else
    decode_bwd_mlp<F, K, 2>(an, mlp, views, sigmoid_op, dg, grid, m, b - n0 - n1, nb - n0 - n1, doffs,
                            dfeat_part + 2 * AF, dls_part + an.A, partial, smem);
}

// dmlp[m] = sum of the partials of partition m's workgroups that differentiate the MLP
// owning each parameter (its colour MLP's parameters start at col0, its covariance
// MLP's at cov0).  Block: 16 parameters x 16 partial groups, contiguous 64-byte reads.
__device__ void mlp_grad_reduce(const float* partial, const BwdGrid& grid, int P, int col0, int cov0, float* dmlp,
                                int bx, int slot) {
  __shared__ float s[16][17];
  const int c = threadIdx.x & 15, r = threadIdx.x >> 4;
  const int i = bx * 16 + c;  // slot: index into grid (partitions with views)
  float acc = 0.f;
  if (i < P) {
    const int n0 = grid.split[slot] & 0xffff, n1 = grid.split[slot] >> 16;
    const int lo = grid.first[slot] + (i < col0 ? 0 : (i < cov0 ? n0 : n0 + n1));
    const int hi = i < col0 ? grid.first[slot] + n0 : (i < cov0 ? grid.first[slot] + n0 + n1 : grid.first[slot + 1]);
    // rows lo + r, lo + r + 16, ... in order, eight loads in flight at a time
    constexpr int kBatch = 8;
    for (int b = lo + r; b < hi; b += 16 * kBatch) {
      float v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) v[k] = b + 16 * k < hi ? partial[(size_t)(b + 16 * k) * P + i] : 0.f;
#pragma unroll
      for (int k = 0; k < kBatch; ++k)
        if (b + 16 * k < hi) acc += v[k];
    }
  }
  s[r][c] = acc;
  __syncthreads();
  if (r == 0 && i < P) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += s[k][c];
    dmlp[(size_t)grid.leader[slot] * P + i] = t;  // leader holds the partition index here
  }
}

// Anchor ranges that some view covers, sorted by start.
struct Covered {
  int n;
  int begin[kMaxBwdParts];
  int end[kMaxBwdParts];
};

// dfeat = sum of the three MLPs' parts, dlog_scale = mean part + scale part; anchors of
// partitions without views get zero gradients (offsets included).
template <int F, int K>
__device__ void anchor_grad_combine(const float* dfeat_part, const float* dls_part, int A, const Covered& cov,
                                    float* dfeat, float* doffs, float* dls, long long block) {
  const long long i = block * blockDim.x + threadIdx.x;
  const long long AF = (long long)A * F;
  if (i >= AF) return;
  const int a = (int)(i / F);
  int lo = 0, hi = cov.n - 1;  // last range starting at or before a
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cov.begin[mid] <= a) lo = mid; else hi = mid - 1;
  }
  const bool in = cov.n > 0 && cov.begin[lo] <= a && a < cov.end[lo];
  dfeat[i] = in ? dfeat_part[i] + dfeat_part[AF + i] + dfeat_part[2 * AF + i] : 0.f;
  if (i % F == 0) {
    dls[a] = in ? dls_part[a] + dls_part[A + a] : 0.f;
    if (!in)
      for (int k = 0; k < 3 * K; ++k) doffs[(size_t)(k / K) * A * K + (size_t)a * K + k % K] = 0.f;
  }
}

// The two reductions after the decode adjoint in one launch: blocks [0, n_red) sum the
// weight-gradient partials (16 parameters x one partition each), the rest combine the
// anchor gradients.
template <int F, int K>
__global__ void __launch_bounds__(256) decode_bwd_finish_kernel(const float* partial, BwdGrid grid, int P, int col0,
                                                                int cov0, float* dmlp, int red_x, int n_red,
                                                                const float* dfeat_part, const float* dls_part, int A,
                                                                Covered cov, float* dfeat, float* doffs, float* dls) {
  const int b = (int)blockIdx.x;
  if (b < n_red)
    mlp_grad_reduce(partial, grid, P, col0, cov0, dmlp, b % red_x, b / red_x);
  else
    anchor_grad_combine<F, K>(dfeat_part, dls_part, A, cov, dfeat, doffs, dls, (long long)(b - n_red));
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

// Workgroups of the adjoint in total: kBwdBlocksPerCU resident on every CU.
int total_bwd_blocks() { return cu_count() * kBwdBlocksPerCU; }

// Relative cost of one 16-anchor chunk in the adjoint of each MLP (measured per wave at
// K = 10: the opacity MLP also carries the gradients of the offsets and of the
// Gaussians' means, the covariance MLP has seven outputs per Gaussian).
constexpr double kMlpChunkCost[3] = {1.1, 1.0, 1.9};

// Workgroups needed for MLP j so that no wave's chunks cost more than T.
long long mlp_blocks_for(long long n_chunks, double T, int j) {
  const long long per = (long long)(T / kMlpChunkCost[j] + 1e-9);  // chunks one wave may take
  if (per < 1) return 1ll << 40;
  const long long waves = (n_chunks + per - 1) / per;
  return (waves + kBwdWaves - 1) / kBwdWaves;
}

// The split of a slot's budget of workgroups over the three MLPs that minimises the
// cost of the longest wave (chunks are dealt to a MLP's waves round-robin, so its
// waves take ceil(chunks / waves) at most): the least makespan T whose workgroup
// counts fit the budget, by bisection (the counts only grow as T shrinks).
void split_mlps(long long n_chunks, int budget, int c[3]) {
  c[0] = c[1] = c[2] = 1;
  if (n_chunks <= 0 || budget <= 3) return;
  auto fits = [&](double T) {
    long long s = 0;
    for (int j = 0; j < 3; ++j) s += mlp_blocks_for(n_chunks, T, j);
    return s <= budget;
  };
  double lo = 0.0, hi = kMlpChunkCost[2] * (double)n_chunks;  // one wave each always fits
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lo + hi);
    (fits(mid) ? hi : lo) = mid;
  }
  for (int j = 0; j < 3; ++j) c[j] = (int)mlp_blocks_for(n_chunks, hi, j);
}

// The slots (runs of consecutive views of one partition) and their workgroups.  The
// forward gives each slot its share of `budget` (never more workgroups than 4-wave
// groups of 16-anchor chunks); the adjoint (adjoint = true) splits each slot's share
// over the three MLPs with split_mlps.
bool bwd_grid(const glam_views& v, BwdGrid& g, int budget, bool adjoint) {
  g.n_parts = 0;
  long long total_anchors = 0;
  for (int i = 0; i < v.n; ++i) {
    const glam_view_info& vi = v.host[i];
    if (i > 0 && v.host[i - 1].cam.partition == vi.cam.partition) continue;
    if (g.n_parts == kMaxBwdParts) return false;
    g.leader[g.n_parts] = i;
    ++g.n_parts;
    total_anchors += vi.anchor_count;
  }
  g.leader[g.n_parts] = v.n;
  int b = 0;
  for (int k = 0; k < g.n_parts; ++k) {
    const int A = v.host[g.leader[k]].anchor_count;
    int nb = total_anchors > 0 ? (int)((double)budget * A / (double)total_anchors + 0.5) : 1;
    g.first[k] = b;
    if (adjoint) {
      int c[3];
      split_mlps((A + 15) / 16, nb < 3 ? 3 : nb, c);
      g.split[k] = c[0] | (c[1] << 16);
      nb = c[0] + c[1] + c[2];
    } else {
      const int cap = (A + 16 * kBwdWaves - 1) / (16 * kBwdWaves);
      nb = nb < 1 ? 1 : (nb > cap ? (cap < 1 ? 1 : cap) : nb);
      g.split[k] = 0;
    }
    b += nb;
  }
  g.first[g.n_parts] = b;
  return true;
}

template <int F, int K>
glam_status run_decode(const glam_anchors& a, const float* mlp, const glam_views& v, bool sig, bool sigma3,
                       const glam_gaussians& out, const glam_projected* proj, hipStream_t s) {
  if (max_anchors(v) == 0 || v.n == 0) return GLAM_OK;
  BwdGrid g;
  if (!bwd_grid(v, g, 2 * cu_count(), false)) return GLAM_ERR_UNSUPPORTED;  // two workgroups per CU
  const size_t sm = fwd_smem<F, K>();
  if (!set_smem_limit((const void*)decode_kernel<F, K>, sm, s)) return GLAM_ERR_HIP;
  const glam_projected none{};
  hipLaunchKernelGGL((decode_kernel<F, K>), dim3(g.first[g.n_parts]), dim3(256), sm, s, a, mlp, v.dev, sig ? 1 : 0, g,
                     out, proj ? 1 : 0, tile_log2(v.tile_w), sigma3 ? 1 : 0, proj ? *proj : none);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

// Workspace of the adjoint: weight-gradient partials (one row of P per workgroup),
// per-MLP anchor feature gradients [3][A][F] and log-scale parts [2][A].
struct BwdWs {
  size_t partial, dfeat, dls, total;
};

BwdWs bwd_ws(int F, int K, int A, int blocks) {
  const MlpOff o = mlp_offsets(F, K);
  BwdWs w;
  const size_t u = blocks > 0 ? (size_t)blocks : 1;
  w.partial = 0;
  w.dfeat = (u * (size_t)o.total * 4 + 255) & ~size_t(255);
  w.dls = w.dfeat + ((3 * (size_t)A * F * 4 + 255) & ~size_t(255));
  w.total = w.dls + ((2 * (size_t)A * 4 + 255) & ~size_t(255));
  return w;
}

template <int F, int K>
glam_status run_decode_bwd(const glam_anchors& a, const float* mlp, int n_parts, const glam_views& v, bool sig,
                           const glam_gaussians& dg, float* dfeat, float* doffs, float* dls, float* dmlp, void* ws,
                           hipStream_t s) {
  constexpr int P = mlp_offsets(F, K).total;
  BwdGrid g;
  if (!bwd_grid(v, g, total_bwd_blocks(), true)) return GLAM_ERR_UNSUPPORTED;
  const int blocks = g.first[g.n_parts];
  const BwdWs W = bwd_ws(F, K, a.A, blocks);
  char* w = static_cast<char*>(ws);
  float* partial = reinterpret_cast<float*>(w + W.partial);
  float* dfp = reinterpret_cast<float*>(w + W.dfeat);
  float* dlp = reinterpret_cast<float*>(w + W.dls);
  // partitions without views get zero gradients (the views' partitions are distinct runs,
  // so every partition has one when there are as many runs as partitions)
  if (g.n_parts < n_parts) {
    const long long nm = (long long)n_parts * P;
    hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, dmlp, nm);
  }
  if (blocks > 0) {
    const size_t sm = sizeof(float) * bwd_smem_words<F, K>();
    if (!set_smem_limit((const void*)decode_bwd_kernel<F, K>, sm, s)) return GLAM_ERR_HIP;
    hipLaunchKernelGGL((decode_bwd_kernel<F, K>), dim3(blocks), dim3(64 * kBwdWaves), sm, s, a, mlp, v.dev,
                       sig ? 1 : 0, dg, g, doffs, dfp, dlp, partial);
  }
  // the reduction writes dmlp[partition of slot k]: pass partitions in place of leaders
  BwdGrid r = g;
  for (int k = 0; k < g.n_parts; ++k) r.leader[k] = v.host[g.leader[k]].cam.partition;
  const int red_x = (P + 15) / 16, n_red = blocks > 0 ? red_x * g.n_parts : 0;
  Covered cov;
  cov.n = 0;
  for (int k = 0; k < g.n_parts; ++k) {
    const glam_view_info& vi = v.host[g.leader[k]];
    if (vi.anchor_count == 0) continue;
    int pos = cov.n++;
    while (pos > 0 && cov.begin[pos - 1] > vi.anchor_begin) {
      cov.begin[pos] = cov.begin[pos - 1];
      cov.end[pos] = cov.end[pos - 1];
      --pos;
    }
    cov.begin[pos] = vi.anchor_begin;
    cov.end[pos] = vi.anchor_begin + vi.anchor_count;
  }
  const long long AF = (long long)a.A * F;
  const long long n_comb = a.A > 0 ? (AF + 255) / 256 : 0;
  if (n_red + n_comb > 0)
    hipLaunchKernelGGL((decode_bwd_finish_kernel<F, K>), dim3((unsigned)(n_red + n_comb)), dim3(256), 0, s, partial, r,
                       P, mlp_offsets(F, K).w1[1], mlp_offsets(F, K).w1[2], dmlp, red_x, n_red, dfp, dlp, a.A, cov,
                       dfeat, doffs, dls);
  return hipGetLastError() == hipSuccess ? GLAM_OK : GLAM_ERR_HIP;
}

}  // namespace

#define GLAM_DECODE_CASES(X) X(32, 10) X(16, 4) X(8, 10) X(64, 10)

glam_status launch_decode(const glam_anchors& a, const float* mlp, const glam_views& v, bool sig, bool sigma3,
                          const glam_gaussians& out, const glam_projected* proj, hipStream_t s) {
#define X(F_, K_) if (a.F == F_ && a.K == K_) return run_decode<F_, K_>(a, mlp, v, sig, sigma3, out, proj, s);
  GLAM_DECODE_CASES(X)
#undef X
  return GLAM_ERR_UNSUPPORTED;
}

size_t decode_bwd_workspace(const glam_anchors& a, const glam_views& v, int n_parts) {
  (void)n_parts;
  BwdGrid g;
  if (!bwd_grid(v, g, total_bwd_blocks(), true)) return 0;
  return bwd_ws(a.F, a.K, a.A, g.first[g.n_parts]).total;
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
