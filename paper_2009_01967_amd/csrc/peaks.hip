// Attainable peaks of the MI355X units the linewidth kernels use, measured by
// register-only loops (MFMA bf16 / fp32 / fp64, FP32 and FP64 vector FMA) and
// by a streaming copy (HBM).  Not part of the method: the benchmark reports
// these beside the published peaks.  C ABI, one call per unit; each returns
// the rate (FLOP/s or bytes/s) or a negative value on a HIP error.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

constexpr int kChains = 8;  // independent accumulators per wave (hides MFMA latency)

// Each wave: iters x kChains MFMAs on register operands; one value per wave is
// stored so that nothing is optimised away.
__global__ void __launch_bounds__(256) k_mfma_bf16(float* out, int iters, float seed) {
  bf16x8 a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(seed * (threadIdx.x + i));
    b[i] = (__bf16)(seed * (i + 1));
  }
  f32x4 acc[kChains] = {};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

__global__ void __launch_bounds__(256) k_mfma_f32(float* out, int iters, float seed) {
  const float a = seed * threadIdx.x, b = seed * 3.0f;
  f32x4 acc[kChains] = {};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

__global__ void __launch_bounds__(256) k_mfma_f64(float* out, int iters, float seed) {
  const double a = seed * threadIdx.x, b = seed * 3.0;
  f64x4 acc[kChains] = {};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = (float)s;
}

// Vector FMA: 16 independent chains per lane.
template <typename R>
__global__ void __launch_bounds__(256) k_valu_fma(float* out, int iters, float seed) {
  R x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = (R)(seed * (threadIdx.x + c));
  const R m = (R)0.999999, d = (R)1e-7;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = x[c] * m + d;
  R s = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) s += x[c];
  if (s == (R)12345.0) out[blockIdx.x] = (float)s;  // practically never: keeps the loop
}

__global__ void __launch_bounds__(256) k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Time `reps` launches of `launch` (after one warm-up) with events; returns ms per launch.
template <class F>
double time_ms(F launch, int reps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  launch();
  (void)hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, nullptr);
  float ms = -1.0f;
  const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                  hipGetLastError() == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok ? ms / reps : -1.0;
}

constexpr int kBlocks = 256 * 8;  // 8 blocks per CU: two waves per SIMD
constexpr int kIters = 4096;

template <class K>
double mfma_rate(K kernel, double flop_per_inst) {
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)kBlocks * 4 * sizeof(float)) != hipSuccess) return -1.0;
  const double ms = time_ms([&] { hipLaunchKernelGGL(kernel, dim3(kBlocks), dim3(256), 0, nullptr, out, kIters, 1e-3f); }, 5);
  (void)hipFree(out);
  if (ms <= 0.0) return -1.0;
  const double insts = (double)kBlocks * 4 * kIters * kChains;  // per wave
  return insts * flop_per_inst / (ms * 1e-3);
}

}  // namespace

extern "C" {

// Dense MFMA rates in FLOP/s: bf16 16x16x32, fp32 16x16x4, fp64 16x16x4.
double mi355x_peak_mfma_bf16() { return mfma_rate(k_mfma_bf16, 2.0 * 16 * 16 * 32); }
double mi355x_peak_mfma_f32() { return mfma_rate(k_mfma_f32, 2.0 * 16 * 16 * 4); }
double mi355x_peak_mfma_f64() { return mfma_rate(k_mfma_f64, 2.0 * 16 * 16 * 4); }

// Vector FMA rate in FLOP/s (2 per FMA), FP32 (non-packed, as the library is built) or FP64.
double mi355x_peak_valu(int fp64) {
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)kBlocks * sizeof(float)) != hipSuccess) return -1.0;
  const int iters = 8192;
  const double ms = time_ms(
      [&] {
        if (fp64)
          hipLaunchKernelGGL(k_valu_fma<double>, dim3(kBlocks), dim3(256), 0, nullptr, out, iters, 1e-3f);
        else
          hipLaunchKernelGGL(k_valu_fma<float>, dim3(kBlocks), dim3(256), 0, nullptr, out, iters, 1e-3f);
      },
      5);
  (void)hipFree(out);
  if (ms <= 0.0) return -1.0;
  return (double)kBlocks * 256 * iters * 16 * 2.0 / (ms * 1e-3);
}

// Streaming copy of `bytes` (rounded down to 16) device to device: bytes/s
// counted as read + written.
double mi355x_peak_hbm(size_t bytes) {
  const size_t n = bytes / 16;
  uint4 *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n * 16) != hipSuccess) return -1.0;
  if (hipMalloc(&b, n * 16) != hipSuccess) {
    (void)hipFree(a);
    return -1.0;
  }
  (void)hipMemset(a, 1, n * 16);
  const double ms = time_ms([&] { hipLaunchKernelGGL(k_copy, dim3(256 * 16), dim3(256), 0, nullptr, b, a, n); }, 5);
  (void)hipFree(a);
  (void)hipFree(b);
  if (ms <= 0.0) return -1.0;
  return 2.0 * (double)n * 16 / (ms * 1e-3);
}

}  // extern "C"
