// Small device helpers shared by the kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace kaldo {

template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// a += b * c
template <typename R>
__device__ __forceinline__ void cfma(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}

// a += b * conj(c)
template <typename R>
__device__ __forceinline__ void cfma_conj(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(-b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}

// exp(2 pi i * num / den) computed from an exactly reduced fraction.
__device__ __forceinline__ void unit_phase(long long num, long long den, double& c, double& s) {
  long long r = num % den;
  if (r < 0) r += den;
  const double f = 2.0 * (double)r / (double)den;
  sincospi(f, &s, &c);
}

__device__ __forceinline__ int imod(int a, int m) {
  int r = a % m;
  return r < 0 ? r + m : r;
}

inline unsigned blocks_for(long long n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// Index of -q_k on the Gamma-centred grid (k = (m0 G1 + m1) G2 + m2).
__host__ __device__ inline int k_mirror(int k, int G0, int G1, int G2) {
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  return (((G0 - m0) % G0) * G1 + (G1 - m1) % G1) * G2 + (G2 - m2) % G2;
}

}  // namespace kaldo
