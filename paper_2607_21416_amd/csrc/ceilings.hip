// Measured ceilings of the chip, for the roofline fractions the benchmark reports:
// FP32 FMA issue, v_exp_f32 issue, LDS read bandwidth, HBM copy and triad bandwidth,
// FP32 matrix-core (MFMA) throughput, and device-scope FP32 atomic throughput on
// distinct and on one contended address.  Each call runs its kernel once to warm up,
// then times one launch with HIP events and returns the rate; it allocates (and frees)
// its own device buffers and synchronises, so it is a measuring tool, not part of the
// render library.  Every loop has a fixed trip count and every access stays inside its
// buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glam_ceilings.h"

namespace {

constexpr int kThreads = 256;

int cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n <= 0)
    n = 256;
  return n;
}

// eight independent FMA chains per lane
__global__ void __launch_bounds__(kThreads) fma_kernel(float* out, int iters, float a, float b) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  if (s == 1234.5f) out[blockIdx.x * kThreads + threadIdx.x] = s;  // keeps the chains live
}

// eight independent chains x <- 2^(-x) per lane (v_exp_f32 with a negated source; the
// iteration stays in [0.5, 1])
__global__ void __launch_bounds__(kThreads) exp_kernel(float* out, int iters) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.1f * (float)(k + 1);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  if (s == 1234.5f) out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// 16-byte LDS reads, consecutive lanes on consecutive 16-byte words (no bank conflicts),
// over a 32 KB buffer per workgroup
constexpr int kLdsWords4 = 2048;  // float4 words
__global__ void __launch_bounds__(kThreads) lds_kernel(float* out, int iters) {
  __shared__ float4 buf[kLdsWords4];
  for (int i = threadIdx.x; i < kLdsWords4; i += kThreads) buf[i] = make_float4(i, 1.f, 2.f, 3.f);
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int idx = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 v = buf[(idx + k * kThreads) & (kLdsWords4 - 1)];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
    idx = (idx + 64) & (kLdsWords4 - 1);
  }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == 1234.5f) out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                        long long n4) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(kThreads) triad_kernel(const float4* __restrict__ b, const float4* __restrict__ c,
                                                         float4* __restrict__ a, float s, long long n4) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) {
    const float4 x = b[i], y = c[i];
    a[i] = make_float4(fmaf(s, y.x, x.x), fmaf(s, y.y, x.y), fmaf(s, y.z, x.z), fmaf(s, y.w, x.w));
  }
}

typedef float f4v __attribute__((ext_vector_type(4)));

// four independent 16x16x4 FP32 MFMA accumulators per wave
__global__ void __launch_bounds__(kThreads) mfma_kernel(float* out, int iters) {
  f4v acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  const float a = 1e-3f * (float)(threadIdx.x & 63), b = 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (s == 1234.5f) out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// device-scope FP32 atomic adds, results unused: lane t of the grid adds to word
// (t + i * threads) mod n on iteration i (distinct addresses), or all to word 0
__global__ void __launch_bounds__(kThreads) atomic_kernel(float* buf, long long n, int iters, int contended) {
  const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long threads = (long long)gridDim.x * kThreads;
  for (int i = 0; i < iters; ++i) {
    const long long w = contended ? 0 : (t + (long long)i * threads) % n;
    atomicAdd(&buf[w], 1.0f);
  }
}

// Times the second of two launches of f(stream); returns milliseconds or -1 on error.
template <class F>
double time_ms(F f) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  f();
  (void)hipEventRecord(a, 0);
  f();
  (void)hipEventRecord(b, 0);
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipGetLastError() == hipSuccess;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ok ? (double)ms : -1.0;
}

}  // namespace

extern "C" {

double glamc_fma_tflops(void) {
  const int blocks = cus() * 8, iters = 4096;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float)) != hipSuccess) return -1.0;
  const double ms = time_ms([&] { hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, iters, 0.999f, 1e-3f); });
  (void)hipFree(out);
  return ms > 0 ? 2.0 * 8.0 * iters * blocks * kThreads / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_exp_trate(void) {
  const int blocks = cus() * 8, iters = 1024;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float)) != hipSuccess) return -1.0;
  const double ms = time_ms([&] { hipLaunchKernelGGL(exp_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, iters); });
  (void)hipFree(out);
  return ms > 0 ? 8.0 * iters * blocks * kThreads / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_lds_read_tbs(void) {
  const int blocks = cus() * 4, iters = 2048;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float)) != hipSuccess) return -1.0;
  const double ms = time_ms([&] { hipLaunchKernelGGL(lds_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, iters); });
  (void)hipFree(out);
  return ms > 0 ? 16.0 * 8.0 * iters * blocks * kThreads / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_hbm_copy_tbs(long long bytes) {
  const long long n4 = bytes / 16;
  if (n4 <= 0) return -1.0;
  float4 *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, n4 * 16) != hipSuccess) return -1.0;
  if (hipMalloc(&dst, n4 * 16) != hipSuccess) { (void)hipFree(src); return -1.0; }
  (void)hipMemset(src, 0, n4 * 16);
  const int blocks = cus() * 16;
  const double ms = time_ms([&] { hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kThreads), 0, 0, src, dst, n4); });
  (void)hipFree(src);
  (void)hipFree(dst);
  return ms > 0 ? 2.0 * 16.0 * n4 / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_hbm_triad_tbs(long long bytes) {
  const long long n4 = bytes / 16;
  if (n4 <= 0) return -1.0;
  float4 *a = nullptr, *b = nullptr, *c = nullptr;
  if (hipMalloc(&a, n4 * 16) != hipSuccess) return -1.0;
  if (hipMalloc(&b, n4 * 16) != hipSuccess) { (void)hipFree(a); return -1.0; }
  if (hipMalloc(&c, n4 * 16) != hipSuccess) { (void)hipFree(a); (void)hipFree(b); return -1.0; }
  (void)hipMemset(b, 0, n4 * 16);
  (void)hipMemset(c, 0, n4 * 16);
  const int blocks = cus() * 16;
  const double ms =
      time_ms([&] { hipLaunchKernelGGL(triad_kernel, dim3(blocks), dim3(kThreads), 0, 0, b, c, a, 0.5f, n4); });
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(c);
  return ms > 0 ? 3.0 * 16.0 * n4 / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_mfma_fp32_tflops(void) {
  const int blocks = cus() * 8, iters = 2048;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float)) != hipSuccess) return -1.0;
  const double ms = time_ms([&] { hipLaunchKernelGGL(mfma_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, iters); });
  (void)hipFree(out);
  // per wave and MFMA: 16 x 16 x 4 multiply-adds
  const double waves = (double)blocks * kThreads / 64.0;
  return ms > 0 ? waves * 4.0 * iters * 2.0 * 16 * 16 * 4 / (ms * 1e-3) / 1e12 : -1.0;
}

double glamc_atomic_grate(int contended) {
  const long long n = 1ll << 24;
  float* buf = nullptr;
  if (hipMalloc(&buf, n * sizeof(float)) != hipSuccess) return -1.0;
  (void)hipMemset(buf, 0, n * sizeof(float));
  // contended: 2^20 adds to one word (each served in turn); distinct: 2^27 adds
  const int blocks = contended ? 64 : cus() * 8;
  const int iters = contended ? 64 : (int)((1ll << 27) / ((long long)blocks * kThreads));
  const double ms =
      time_ms([&] { hipLaunchKernelGGL(atomic_kernel, dim3(blocks), dim3(kThreads), 0, 0, buf, n, iters, contended); });
  (void)hipFree(buf);
  return ms > 0 ? (double)blocks * kThreads * iters / (ms * 1e-3) / 1e9 : -1.0;
}

}  // extern "C"
