// Internal declarations of the MI355X multigrid library for the Shamir
// domain-wall operator.  Not part of the public C ABI (include/mgdwf.h).
//
// Internal layouts (all device memory, owned by the context):
//   fine field, one right-hand side:  element (c, x4, s) at (c * V4 + x4) * Ls + s,
//     c = spin * 3 + colour in 0..11, stored as double2 / float2 (re, im).
//     A wavefront's 64 lanes take 64 consecutive (x4, s) pairs, so every load
//     of one spin-colour component is one contiguous, fully coalesced segment.
//   nrhs fields are stacked: field r starts at r * 12 * V5 elements.
//   gauge field:  element (mu, a, b, x4) at ((mu * 9 + a * 3 + b) * V4 + x4).
//   coarse vector: element (X4, chi, k) at (X4 * 2 + chi) * Nv + k  (one RHS),
//     nrhs vectors stacked with stride 2 * Nv * Vc.
//   coarse operator: block (X4, d) at (X4 * 9 + d) * n2 * n2, row-major n2 x n2,
//     n2 = 2 * Nv; d = 0 self, 1 + 2 mu for +mu, 2 + 2 mu for -mu.
//   block basis Vhat: Nv fine fields in the fine-field layout; column (B, chi, k)
//     is field k restricted to block B and to the spins of chirality chi.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mgdwf.h"

namespace mgdwf {

struct Geometry {
  int L[4];      // x, y, z, t
  int Ls;
  int V4;        // 4D volume
  int V5;        // V4 * Ls
  int bc[4];     // +1 periodic, -1 antiperiodic in direction mu
  int ftile = -1;  // FP32 Dslash tiling (index into its table; -1: the default)
  int ctile = 0;   // 16-bit coarse apply MFMA shape (0: 16x16x16, 1: 16x16x32)
};

struct CoarseGeometry {
  int block[4];
  int Lc[4];
  int Vc;        // number of coarse sites
  int Nv;        // columns per chirality
  int n2;        // 2 * Nv
  int bvol;      // 4D sites per block
};

// Error carrying a status code through the C++ layers; converted to an
// mgdwf_status at the C boundary.
struct Error {
  mgdwf_status code;
  std::string msg;
};

[[noreturn]] void fail(mgdwf_status code, const std::string& msg);

#define MG_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      ::mgdwf::fail(MGDWF_ERR_HIP, std::string(#call) + ": " +                \
                                       hipGetErrorString(e_));                \
  } while (0)

#define MG_LAUNCH_CHECK() MG_HIP(hipGetLastError())

// Device buffer owned by the library (RAII).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

inline int ceil_div(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

// One coarse stencil (D_c or its adjoint) in every storage precision.
//   m64, m32:        complex blocks, column major, block (X, d) at (X * 9 + d) * n2 * n2
//   re16/im16/sc16:  FP16 real and imaginary parts, row major, one FP32 scale per block
//   reb/imb/scb:     the same in BF16
struct CoarseStore {
  DevBuf m64, m32, re16, im16, sc16, reb, imb, scb;
};

// Remap a linear workgroup index so that each XCD (workgroups are dealt to
// the 8 XCDs round robin) processes one contiguous slice of the index range:
// neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int nx = 8;
  int per = nblocks / nx;
  int full = per * nx;
  if (bid >= full) return bid;  // ragged tail keeps its index
  return (bid % nx) * per + bid / nx;
}

// ---------------------------------------------------------------- kernels API
// layout / conversion
void pack_fermion_f64(const double2* canon, double2* field, const Geometry& g, int nrhs, hipStream_t st);
void unpack_fermion_f64(const double2* field, double2* canon, const Geometry& g, int nrhs, hipStream_t st);
void pack_gauge(const double2* canon, double2* g64, float2* g32, const Geometry& g, hipStream_t st);
void convert_f64_to_f32(const double2* in, float2* out, long long n, hipStream_t st);
void convert_f32_to_f64(const float2* in, double2* out, long long n, hipStream_t st);

// Dslash:  out = D in  (dagger: D^+).  mode 0: out = D in;  mode 1: out = b - D in.
template <class R2>
void dslash(const R2* in, R2* out, const R2* b, const R2* gauge, const Geometry& g, double M5,
            double mf, bool dagger, int mode, int nrhs, hipStream_t st);

}  // namespace mgdwf
