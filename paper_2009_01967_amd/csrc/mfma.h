// Operand types and MFMA helpers shared by the GEMM-shaped projection kernels.
//
// Lane layouts of the gfx950 MFMA instructions used here (checked on the device):
//   f32 16x16x4:   lane l supplies A[l%16][l/16] and B[l/16][l%16];
//                  accumulator register r of lane l is C[4*(l/16) + r][l%16]
//   f64 16x16x4:   same inputs; accumulator register r of lane l is C[l/16 + 4*r][l%16]
//   bf16 16x16x32: lane l supplies A[l%16][8*(l/16) .. +7] and B[8*(l/16) .. +7][l%16];
//                  accumulators as f32 16x16x4
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "../../include/kaldo.h"

namespace kaldo {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

template <int P>
struct Operand;
template <>
struct Operand<KALDO_FP64> {
  using T = double;
  using Acc = f64x4;
  static constexpr int split = 1;
};
template <>
struct Operand<KALDO_FP32> {
  using T = float;
  using Acc = f32x4;
  static constexpr int split = 1;
};
template <>
struct Operand<KALDO_BF16X3> {
  using T = __bf16;
  using Acc = f32x4;
  static constexpr int split = 2;  // hi and lo planes
};

// Global-memory view of a pointer into a device buffer.  Inside kernels that
// take their buffers from a table in memory (the persistent batch kernel) the
// compiler cannot tell the address space and issues flat loads and stores;
// those count against the LDS wait counter as well, so every wait for an LDS
// read would also wait for the memory operations in flight.  Through this view
// they are global_* instructions.  Only for device memory (never LDS).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Store v into an operand plane; for BF16X3 as hi = bf16(v), lo = bf16(v - hi).
template <int P>
__device__ __forceinline__ void store_operand(typename Operand<P>::T* hi, typename Operand<P>::T* lo, size_t o,
                                              double v) {
  if constexpr (P == KALDO_BF16X3) {
    const float f = (float)v;
    const __bf16 h = (__bf16)f;
    gmem(hi)[o] = h;
    gmem(lo)[o] = (__bf16)(f - (float)h);
  } else {
    gmem(hi)[o] = (typename Operand<P>::T)v;
  }
}

// Store the adjacent pair (v0, v1) at o, o + 1 (o even) with one write per plane.
template <int P>
__device__ __forceinline__ void store_operand2(typename Operand<P>::T* hi, typename Operand<P>::T* lo, size_t o,
                                               double v0, double v1) {
  if constexpr (P == KALDO_BF16X3) {
    const float f0 = (float)v0, f1 = (float)v1;
    const __bf16 h0 = (__bf16)f0, h1 = (__bf16)f1;
    const __bf16 l0 = (__bf16)(f0 - (float)h0), l1 = (__bf16)(f1 - (float)h1);
    typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
    *gmem(reinterpret_cast<bf16x2*>(hi + o)) = bf16x2{h0, h1};
    *gmem(reinterpret_cast<bf16x2*>(lo + o)) = bf16x2{l0, l1};
  } else if constexpr (P == KALDO_FP32) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    *gmem(reinterpret_cast<f32x2*>(hi + o)) = f32x2{(float)v0, (float)v1};
  } else {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    *gmem(reinterpret_cast<f64x2*>(hi + o)) = f64x2{v0, v1};
  }
}

// Arguments x^2 / (2 sigma^2) of the Gaussian beyond which an element's weight
// is dropped: 6 sigma for the mixed precisions (relative weight < 2e-8), 8.9
// sigma for FP64 (< 5e-18, below its rounding).
template <int P>
__host__ __device__ constexpr double gauss_cut() {
  return P == KALDO_FP64 ? 40.0 : 18.0;
}

// Squared scaled mismatch u^2 beyond which a delta of kind `kind` is dropped:
// the Gaussian cut above, exactly 1 for the triangle (zero outside its base),
// never for the Lorentzian (its tails are kept).
template <int P>
__host__ __device__ constexpr double delta_cut(int kind) {
  return kind == KALDO_DELTA_GAUSS ? gauss_cut<P>() : (kind == KALDO_DELTA_TRIANGLE ? 1.0 : 1e300);
}

// Shape of the energy delta of kind DK as a function of the mismatch u in
// units of the kind's scale s (Gaussian: s = sqrt(2) sigma, exp(-u^2);
// Lorentzian: s = sigma the half width, 1 / (1 + u^2); triangle: s = sigma the
// half base, max(0, 1 - |u|)).  The normalisation (1 / (sqrt(pi) s),
// 1 / (pi s), 1 / s) is applied when the sums are collected.  u is formed in
// FP64 (a difference of near-equal scaled frequencies); the shape is evaluated
// in R.
template <typename R, int DK>
__device__ __forceinline__ R delta_shape(double u) {
  if constexpr (DK == KALDO_DELTA_GAUSS) {
    if constexpr (sizeof(R) == 8) return exp(-u * u);
    else return __expf((float)(-u * u));
  } else if constexpr (DK == KALDO_DELTA_LORENTZ) {
    if constexpr (sizeof(R) == 8) return 1.0 / (1.0 + u * u);
    else {
      const float x = (float)u;
      return __builtin_amdgcn_rcpf(fmaf(x, x, 1.0f));
    }
  } else {
    const R t = (R)1 - fabs((R)u);
    return t > (R)0 ? t : (R)0;
  }
}

// Host: the scale s (rad/ps) and the normalisation of the delta of kind `kind`
// for the width sigma_omega (rad/ps).
inline void delta_scale(int kind, double sigma_omega, double& scale, double& norm) {
  const double pi = 3.141592653589793238462643383279;
  if (kind == KALDO_DELTA_GAUSS) {
    scale = sqrt(2.0) * sigma_omega;
    norm = 1.0 / (sqrt(pi) * scale);
  } else if (kind == KALDO_DELTA_LORENTZ) {
    scale = sigma_omega;
    norm = 1.0 / (pi * scale);
  } else {
    scale = sigma_omega;
    norm = 1.0 / scale;
  }
}

// Store 16 bytes of elements v[0 .. 16 / sizeof(T)) at o (a multiple of that
// count) with one write per plane.
template <int P>
__device__ __forceinline__ void store_operand_vec(typename Operand<P>::T* hi, typename Operand<P>::T* lo, size_t o,
                                                  const double* v) {
  if constexpr (P == KALDO_BF16X3) {
    typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8v;
    bf16x8v h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float f = (float)v[q];
      h[q] = (__bf16)f;
      l[q] = (__bf16)(f - (float)h[q]);
    }
    *reinterpret_cast<bf16x8v*>(hi + o) = h;
    *reinterpret_cast<bf16x8v*>(lo + o) = l;
  } else if constexpr (P == KALDO_FP32) {
    *reinterpret_cast<float4*>(hi + o) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  } else {
    *reinterpret_cast<double2*>(hi + o) = make_double2(v[0], v[1]);
  }
}

// accumulator row of register r in lane l for a 16x16 tile
template <int P>
__device__ __forceinline__ int acc_row(int lane, int r) {
  return P == KALDO_FP64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
}

}  // namespace kaldo
