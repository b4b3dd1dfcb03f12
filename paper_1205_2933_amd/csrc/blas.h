// Device helpers: wavefront/workgroup reductions and complex arithmetic.
#pragma once

#include <hip/hip_runtime.h>

namespace mgdwf {

// Sum over a 64-lane wavefront with xor shuffles (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup sum for a block of BS threads (multiple of 64); result valid in
// thread 0.  Contains barriers: every thread of the block must call it.
template <int BS>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[BS / 64];
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += red[i];
  }
  return s;
}

// ---- complex helpers for double2 / float2 (x = re, y = im)
template <class C2> struct real_of;
template <> struct real_of<double2> { using type = double; };
template <> struct real_of<float2> { using type = float; };

template <class C2>
__device__ __forceinline__ C2 cmk(typename real_of<C2>::type re, typename real_of<C2>::type im) {
  C2 r; r.x = re; r.y = im; return r;
}
template <class C2> __device__ __forceinline__ C2 cadd(C2 a, C2 b) { return cmk<C2>(a.x + b.x, a.y + b.y); }
template <class C2> __device__ __forceinline__ C2 csub(C2 a, C2 b) { return cmk<C2>(a.x - b.x, a.y - b.y); }
template <class C2> __device__ __forceinline__ C2 cmul(C2 a, C2 b) {
  return cmk<C2>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <class C2> __device__ __forceinline__ C2 cmulc(C2 a, C2 b) {
  return cmk<C2>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc += a * b, as four fused multiply-adds into the accumulator
template <class C2> __device__ __forceinline__ void cfma(C2& acc, C2 a, C2 b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(-a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <class C2> __device__ __forceinline__ void cfmac(C2& acc, C2 a, C2 b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(-a.y, b.x, acc.y);
}
// i * a
template <class C2> __device__ __forceinline__ C2 ci(C2 a) { return cmk<C2>(-a.y, a.x); }
template <class C2> __device__ __forceinline__ C2 cscale(C2 a, typename real_of<C2>::type s) {
  return cmk<C2>(a.x * s, a.y * s);
}

// ---- host-side launch wrappers for reductions (core.hip)
void finalize_sum(const double* partial, int nparts, int ncomp, double* out, hipStream_t st);
template <class C2>
void multidot(const C2* const* avec_dev, int nv, const C2* b, long long n, double* partial,
              int nparts, double* out, hipStream_t st);

}  // namespace mgdwf
