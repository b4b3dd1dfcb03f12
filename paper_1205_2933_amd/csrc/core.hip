// Buffers, errors, layout conversion and deterministic reductions.
#include "mg_internal.h"
#include "blas.h"

namespace mgdwf {

void fail(mgdwf_status code, const std::string& msg) { throw Error{code, msg}; }

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) return;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    fail(MGDWF_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
  }
  bytes = n;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------ layout packing

// canonical fermion (i5 * 12 + c) <-> internal (c * V5 + i5), i5 = x4 * Ls + s
__global__ void k_pack_fermion(const double2* __restrict__ canon, double2* __restrict__ field,
                               long long V5, int nrhs) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = V5 * nrhs;
  if (i >= tot) return;
  long long r = i / V5, i5 = i - r * V5;
  const double2* src = canon + r * 12 * V5 + i5 * 12;
  double2* dst = field + r * 12 * V5 + i5;
#pragma unroll
  for (int c = 0; c < 12; ++c) dst[c * V5] = src[c];
}

__global__ void k_unpack_fermion(const double2* __restrict__ field, double2* __restrict__ canon,
                                 long long V5, int nrhs) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = V5 * nrhs;
  if (i >= tot) return;
  long long r = i / V5, i5 = i - r * V5;
  const double2* src = field + r * 12 * V5 + i5;
  double2* dst = canon + r * 12 * V5 + i5 * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) dst[c] = src[c * V5];
}

void pack_fermion_f64(const double2* canon, double2* field, const Geometry& g, int nrhs, hipStream_t st) {
  long long n = (long long)g.V5 * nrhs;
  hipLaunchKernelGGL(k_pack_fermion, dim3(ceil_div(n, 256)), dim3(256), 0, st, canon, field,
                     (long long)g.V5, nrhs);
  MG_LAUNCH_CHECK();
}

void unpack_fermion_f64(const double2* field, double2* canon, const Geometry& g, int nrhs, hipStream_t st) {
  long long n = (long long)g.V5 * nrhs;
  hipLaunchKernelGGL(k_unpack_fermion, dim3(ceil_div(n, 256)), dim3(256), 0, st, field, canon,
                     (long long)g.V5, nrhs);
  MG_LAUNCH_CHECK();
}

// canonical gauge ((x4*4 + mu)*9 + ab) -> internal ((mu*9 + ab)*V4 + x4), FP64 and FP32
__global__ void k_pack_gauge(const double2* __restrict__ canon, double2* __restrict__ g64,
                             float2* __restrict__ g32, Geometry g) {
  const int V4 = g.V4;
  int x4 = blockIdx.x * blockDim.x + threadIdx.x;
  if (x4 >= V4) return;
  const int co[4] = {x4 % g.L[0], (x4 / g.L[0]) % g.L[1], (x4 / (g.L[0] * g.L[1])) % g.L[2],
                     x4 / (g.L[0] * g.L[1] * g.L[2])};
  for (int j = 0; j < 36; ++j) {
    double2 v = canon[(long long)x4 * 36 + j];
    long long o = (long long)j * V4 + x4;
    g64[o] = v;
    g32[o] = make_float2((float)v.x, (float)v.y);
    // second FP32 copy, site major ([x4][mu][a][b], the canonical order): the
    // 36 entries of a site are contiguous for the wavefront-per-site kernel
    g32[36LL * V4 + (long long)x4 * 36 + j] = make_float2((float)v.x, (float)v.y);
    // third, component major with the boundary phase folded into the links
    // of each direction's last slice (every hop across that face uses them)
    const int mu = j / 9;
    const float ph = co[mu] == g.L[mu] - 1 ? (float)g.bc[mu] : 1.0f;
    g32[72LL * V4 + o] = make_float2(ph * (float)v.x, ph * (float)v.y);
  }
}

void pack_gauge(const double2* canon, double2* g64, float2* g32, const Geometry& g, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_gauge, dim3(ceil_div(g.V4, 256)), dim3(256), 0, st, canon, g64, g32, g);
  MG_LAUNCH_CHECK();
}

__global__ void k_f64_to_f32(const double2* __restrict__ in, float2* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double2 v = in[i];
    out[i] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void k_f32_to_f64(const float2* __restrict__ in, double2* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    float2 v = in[i];
    out[i] = make_double2(v.x, v.y);
  }
}

void convert_f64_to_f32(const double2* in, float2* out, long long n, hipStream_t st) {
  int nb = std::min(ceil_div(n, 256), 8192);
  if (nb < 1) return;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(nb), dim3(256), 0, st, in, out, n);
  MG_LAUNCH_CHECK();
}

void convert_f32_to_f64(const float2* in, double2* out, long long n, hipStream_t st) {
  int nb = std::min(ceil_div(n, 256), 8192);
  if (nb < 1) return;
  hipLaunchKernelGGL(k_f32_to_f64, dim3(nb), dim3(256), 0, st, in, out, n);
  MG_LAUNCH_CHECK();
}

// ------------------------------------------------------------ reductions

// Sum of nparts rows of `ncomp` doubles each into out[ncomp]; one workgroup per
// component, fixed summation order (bitwise reproducible).
__global__ void k_finalize(const double* __restrict__ partial, int nparts, int ncomp,
                           double* __restrict__ out) {
  int comp = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[(long long)i * ncomp + comp];
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) out[comp] = acc;
}

void finalize_sum(const double* partial, int nparts, int ncomp, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(ncomp), dim3(256), 0, st, partial, nparts, ncomp, out);
  MG_LAUNCH_CHECK();
}

// partial[b][m] (complex, 2 doubles) = sum over this block's elements of conj(a_m) b,
// and partial[b][nv] = |b|^2 when with_norm.  Element-wise the vectors are
// length n complex numbers.
template <class C2>
__global__ void k_multidot(const C2* const* __restrict__ avec, int nv, const C2* __restrict__ b,
                           long long n, int with_norm, double* __restrict__ partial) {
  constexpr int MAXV = 18;
  double re[MAXV], im[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) { re[m] = 0.0; im[m] = 0.0; }
  double nn = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    C2 bv = b[i];
    double bx = bv.x, by = bv.y;
    nn += bx * bx + by * by;
#pragma unroll
    for (int m = 0; m < MAXV; ++m) {
      if (m < nv) {
        C2 av = avec[m][i];
        re[m] += (double)av.x * bx + (double)av.y * by;
        im[m] += (double)av.x * by - (double)av.y * bx;
      }
    }
  }
  int ncomp = 2 * nv + 1;
  for (int m = 0; m < nv; ++m) {
    double sr = block_sum<256>(re[m]);
    double si = block_sum<256>(im[m]);
    if (threadIdx.x == 0) {
      partial[(long long)blockIdx.x * ncomp + 2 * m] = sr;
      partial[(long long)blockIdx.x * ncomp + 2 * m + 1] = si;
    }
  }
  if (with_norm) {
    double s = block_sum<256>(nn);
    if (threadIdx.x == 0) partial[(long long)blockIdx.x * ncomp + 2 * nv] = s;
  } else if (threadIdx.x == 0) {
    partial[(long long)blockIdx.x * ncomp + 2 * nv] = 0.0;
  }
}

template <class C2>
void multidot(const C2* const* avec_dev, int nv, const C2* b, long long n, double* partial,
              int nparts, double* out, hipStream_t st) {
  if (nv > 18) fail(MGDWF_ERR_INVALID_ARG, "multidot supports at most 18 vectors");
  hipLaunchKernelGGL(k_multidot<C2>, dim3(nparts), dim3(256), 0, st, avec_dev, nv, b, n, 1, partial);
  MG_LAUNCH_CHECK();
  finalize_sum(partial, nparts, 2 * nv + 1, out, st);
}

template void multidot<double2>(const double2* const*, int, const double2*, long long, double*, int,
                                double*, hipStream_t);
template void multidot<float2>(const float2* const*, int, const float2*, long long, double*, int,
                               double*, hipStream_t);

}  // namespace mgdwf
