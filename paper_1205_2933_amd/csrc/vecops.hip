// Vector kernels of the solvers (multi-RHS, device-resident scalars).
//
// Every vector argument holds nrhs stacked vectors of n complex numbers each
// (stride n); gridDim.y = nrhs.  Scalars live in a device array `sl` with a
// fixed slot table per right-hand side: slot(rhs, i) = sl[rhs * NSLOT + i].
// Reductions are two-stage: a per-workgroup partial, then k_finalize; the
// summation order is fixed, so results are bitwise reproducible.
#include <cstdint>
#include <type_traits>

#include "mg_internal.h"
#include "blas.h"
#include "vecops.h"

namespace mgdwf {

namespace {

__device__ __forceinline__ double slot(const double* sl, int rhs, int i) { return sl[rhs * NSLOT + i]; }

// out[rhs * NSLOT + dst + comp] = sum_i partial[(rhs * nparts + i) * ncomp + comp]
__global__ void k_finalize_rhs(const double* __restrict__ partial, int nparts, int ncomp,
                               double* __restrict__ sl, int dst) {
  const int comp = blockIdx.x, rhs = blockIdx.y;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[((long long)rhs * nparts + i) * ncomp + comp];
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) sl[rhs * NSLOT + dst + comp] = acc;
}

// x (+)= alpha p;  r -= alpha q;  alpha = sl[num] / sl[den] (real);  partial |r|^2.
template <class C2>
__global__ __launch_bounds__(256) void k_mr_update(C2* __restrict__ x, C2* __restrict__ r, const C2* __restrict__ p,
                                                   const C2* __restrict__ q, long long n, const double* __restrict__ sl,
                                                   int num, int den, int first, double* __restrict__ partial) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double dd = slot(sl, rhs, den);
  const T alpha = (T)(dd > 0.0 ? slot(sl, rhs, num) / dd : 0.0);
  double nr = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 pv = p[off + i], qv = q[off + i];
    C2 xv = first ? cmk<C2>(0, 0) : x[off + i];
    x[off + i] = cadd(xv, cscale(pv, alpha));
    C2 rv = csub(r[off + i], cscale(qv, alpha));
    r[off + i] = rv;
    nr += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  if (partial) {
    double s = block_sum<256>(nr);
    if (threadIdx.x == 0) partial[(long long)rhs * gridDim.x + blockIdx.x] = s;
  }
}

// r_out = r_in - alpha q, alpha = sl[num] / sl[den]  (the residual half of an MR step;
// r_in may equal r_out).
template <class C2>
__global__ __launch_bounds__(256) void k_res_update(C2* __restrict__ rout, const C2* rin, const C2* __restrict__ q,
                                                    long long n, const double* __restrict__ sl, int num, int den) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double dd = slot(sl, rhs, den);
  const T alpha = (T)(dd > 0.0 ? slot(sl, rhs, num) / dd : 0.0);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    rout[off + i] = csub(rin[off + i], cscale(q[off + i], alpha));
}

// FP32 forms of k_res_update and k_lincomb for vectors of even length with
// 16-byte aligned storage: each lane moves two complex numbers per access
// (np = n / 2 pairs per RHS), the same arithmetic per element.
__global__ __launch_bounds__(256) void k_res_update_pair(float4* rout, const float4* rin, const float4* __restrict__ q,
                                                         long long np, const double* __restrict__ sl, int num, int den) {
  const int rhs = blockIdx.y;
  const long long off = rhs * np;
  const double dd = slot(sl, rhs, den);
  const float alpha = (float)(dd > 0.0 ? slot(sl, rhs, num) / dd : 0.0);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (long long)gridDim.x * blockDim.x) {
    const float4 a = rin[off + i], b = q[off + i];
    const float2 lo = csub(make_float2(a.x, a.y), cscale(make_float2(b.x, b.y), alpha));
    const float2 hi = csub(make_float2(a.z, a.w), cscale(make_float2(b.z, b.w), alpha));
    rout[off + i] = make_float4(lo.x, lo.y, hi.x, hi.y);
  }
}

__global__ __launch_bounds__(256) void k_lincomb_pair(float4* __restrict__ x, const float2* const* __restrict__ ps,
                                                      int nv, long long np, const double* __restrict__ sl, int num,
                                                      int acc0) {
  constexpr int MAXV = 16;
  const int rhs = blockIdx.y;
  const long long off = rhs * np;
  float al[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) {
    const double d = m < nv ? slot(sl, rhs, num + 2 * m + 1) : 0.0;
    al[m] = (float)(d > 0.0 ? slot(sl, rhs, num + 2 * m) / d : 0.0);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (long long)gridDim.x * blockDim.x) {
    float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
    if (acc0) {
      const float4 v = x[off + i];
      lo = make_float2(v.x, v.y);
      hi = make_float2(v.z, v.w);
    }
#pragma unroll
    for (int m = 0; m < MAXV; ++m)
      if (m < nv) {
        const float4 v = reinterpret_cast<const float4*>(ps[m])[off + i];
        lo = cadd(lo, cscale(make_float2(v.x, v.y), al[m]));
        hi = cadd(hi, cscale(make_float2(v.z, v.w), al[m]));
      }
    x[off + i] = make_float4(lo.x, lo.y, hi.x, hi.y);
  }
}

// x = sum_m alpha_m p_m (acc: x += ...), alpha_m = sl[num + 2m] / sl[num + 2m + 1]  (m < nv)
template <class C2>
__global__ __launch_bounds__(256) void k_lincomb(C2* __restrict__ x, const C2* const* __restrict__ ps, int nv,
                                                 long long n, const double* __restrict__ sl, int num, int acc0) {
  using T = typename real_of<C2>::type;
  constexpr int MAXV = 16;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  T al[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) {
    const double d = m < nv ? slot(sl, rhs, num + 2 * m + 1) : 0.0;
    al[m] = (T)(d > 0.0 ? slot(sl, rhs, num + 2 * m) / d : 0.0);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 acc = acc0 ? x[off + i] : cmk<C2>(0, 0);
#pragma unroll
    for (int m = 0; m < MAXV; ++m)
      if (m < nv) acc = cadd(acc, cscale(ps[m][off + i], al[m]));
    x[off + i] = acc;
  }
}

// p = r + beta p, beta = sl[num] / sl[den]  (CG direction update); partial |p|^2
template <class C2>
__global__ __launch_bounds__(256) void k_cg_dir(C2* __restrict__ p, const C2* __restrict__ r, long long n,
                                                const double* __restrict__ sl, int num, int den,
                                                double* __restrict__ partial) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double dd = slot(sl, rhs, den);
  const T beta = (T)(dd > 0.0 ? slot(sl, rhs, num) / dd : 0.0);
  double np = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 v = cadd(r[off + i], cscale(p[off + i], beta));
    p[off + i] = v;
    np += (double)v.x * v.x + (double)v.y * v.y;
  }
  if (partial) {
    double s = block_sum<256>(np);
    if (threadIdx.x == 0) partial[(long long)rhs * gridDim.x + blockIdx.x] = s;
  }
}

// Multi-dot: partial[rhs][blk][2m..] = <a_m, b> (complex) for m < nv, then |b|^2 and
// <b, c> (complex) when c is non-null.  Layout of the ncomp = 2 nv + 3 components:
// [re0, im0, ..., |b|^2, re_bc, im_bc].
template <class C2>
__global__ __launch_bounds__(256) void k_multidot(const C2* const* __restrict__ avec, int nv, const C2* __restrict__ b,
                                                  const C2* __restrict__ c, long long n,
                                                  double* __restrict__ partial) {
  constexpr int MAXV = 16;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  double re[MAXV], im[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) { re[m] = 0.0; im[m] = 0.0; }
  double nn = 0.0, cr = 0.0, cim = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 bv = b[off + i];
    const double bx = bv.x, by = bv.y;
    nn += bx * bx + by * by;
    if (c) {
      C2 cv = c[off + i];
      cr += bx * cv.x + by * cv.y;
      cim += bx * cv.y - by * cv.x;
    }
#pragma unroll
    for (int m = 0; m < MAXV; ++m) {
      if (m < nv) {
        C2 av = avec[m][off + i];
        re[m] += (double)av.x * bx + (double)av.y * by;
        im[m] += (double)av.x * by - (double)av.y * bx;
      }
    }
  }
  const int ncomp = 2 * nv + 3;
  double* out = partial + ((long long)rhs * gridDim.x + blockIdx.x) * ncomp;
  for (int m = 0; m < nv; ++m) {
    double sr = block_sum<256>(re[m]);
    double si = block_sum<256>(im[m]);
    if (threadIdx.x == 0) { out[2 * m] = sr; out[2 * m + 1] = si; }
  }
  double s0 = block_sum<256>(nn), s1 = block_sum<256>(cr), s2 = block_sum<256>(cim);
  if (threadIdx.x == 0) { out[2 * nv] = s0; out[2 * nv + 1] = s1; out[2 * nv + 2] = s2; }
}

// q -= sum_m beta_m q_m;  z -= sum_m beta_m z_m;  beta_m = <q_m, q> / |q_m|^2 with
// <q_m, q> at slots dots + 2m and |q_m|^2 at slots nrm + m.
template <class C2>
__global__ __launch_bounds__(256) void k_orth_update(C2* __restrict__ q, C2* __restrict__ z, const C2* const* __restrict__ qs,
                                                     const C2* const* __restrict__ zs, int nv, long long n,
                                                     const double* __restrict__ sl, int dots, int nrm) {
  using T = typename real_of<C2>::type;
  constexpr int MAXV = 16;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  T br[MAXV], bi[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) {
    if (m < nv) {
      const double d = slot(sl, rhs, nrm + m);
      const double inv = d > 0.0 ? 1.0 / d : 0.0;
      br[m] = (T)(slot(sl, rhs, dots + 2 * m) * inv);
      bi[m] = (T)(slot(sl, rhs, dots + 2 * m + 1) * inv);
    } else { br[m] = 0; bi[m] = 0; }
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 qv = q[off + i];
#pragma unroll
    for (int m = 0; m < MAXV; ++m)
      if (m < nv) qv = csub(qv, cmul(cmk<C2>(br[m], bi[m]), qs[m][off + i]));
    q[off + i] = qv;
    if (z) {  // z follows q unless the caller keeps the coefficients instead
      C2 zv = z[off + i];
#pragma unroll
      for (int m = 0; m < MAXV; ++m)
        if (m < nv) zv = csub(zv, cmul(cmk<C2>(br[m], bi[m]), zs[m][off + i]));
      z[off + i] = zv;
    }
  }
}

// e += alpha z; r -= alpha q;  alpha = <q, r> / |q|^2 (slots cr, ci over nq); partial |r|^2
template <class C2>
__global__ __launch_bounds__(256) void k_gcr_update(C2* __restrict__ e, C2* __restrict__ r, const C2* __restrict__ z,
                                                    const C2* __restrict__ q, long long n, const double* __restrict__ sl,
                                                    int cr_, int nq, int first, double* __restrict__ partial) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double d = slot(sl, rhs, nq);
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  const C2 alpha = cmk<C2>((T)(slot(sl, rhs, cr_) * inv), (T)(slot(sl, rhs, cr_ + 1) * inv));
  double nr = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if (e) {  // without e only the residual moves
      C2 ev = first ? cmk<C2>(0, 0) : e[off + i];
      e[off + i] = cadd(ev, cmul(alpha, z[off + i]));
    }
    C2 rv = csub(r[off + i], cmul(alpha, q[off + i]));
    r[off + i] = rv;
    nr += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  if (partial) {
    double s = block_sum<256>(nr);
    if (threadIdx.x == 0) partial[(long long)rhs * gridDim.x + blockIdx.x] = s;
  }
}

// Minimal-residual step on a Hermitian operator N with the direction r itself:
// x = (first ? 0 : x) + alpha rin, rnew = rin - alpha p, p = N rin,
// alpha = <p, rin> / |p|^2 (complex <p, rin> at slots cr, cr + 1, |p|^2 at nq).
// rnew must not alias rin.
template <class C2>
__global__ __launch_bounds__(256) void k_mrh_update(C2* __restrict__ x, C2* __restrict__ rnew,
                                                    const C2* __restrict__ rin, const C2* __restrict__ p, long long n,
                                                    const double* __restrict__ sl, int cr_, int nq, int first) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double d = slot(sl, rhs, nq);
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  const C2 alpha = cmk<C2>((T)(slot(sl, rhs, cr_) * inv), (T)(slot(sl, rhs, cr_ + 1) * inv));
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const C2 rv = rin[off + i];
    const C2 xv = first ? cmk<C2>(0, 0) : x[off + i];
    x[off + i] = cadd(xv, cmul(alpha, rv));
    rnew[off + i] = csub(rv, cmul(alpha, p[off + i]));
  }
}

// x = sum_m c[rhs][m] p_m with complex coefficients c (FP64, [rhs][16]), m < nv
template <class C2>
__global__ __launch_bounds__(256) void k_lincomb_c(C2* __restrict__ x, const C2* const* __restrict__ ps, int nv,
                                                   long long n, const double2* __restrict__ coef) {
  using T = typename real_of<C2>::type;
  constexpr int MAXV = 16;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  C2 cf[MAXV];
#pragma unroll
  for (int m = 0; m < MAXV; ++m) {
    const double2 v = m < nv ? coef[rhs * MAXV + m] : make_double2(0.0, 0.0);
    cf[m] = cmk<C2>((T)v.x, (T)v.y);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    C2 acc = cmk<C2>(0, 0);
#pragma unroll
    for (int m = 0; m < MAXV; ++m)
      if (m < nv) acc = cadd(acc, cmul(cf[m], ps[m][off + i]));
    x[off + i] = acc;
  }
}

// y = x * sl[num] / sqrt(sl[den])  or plain scale by 1/sqrt(sl[den]) when num < 0
template <class C2>
__global__ void k_scale_slot(C2* __restrict__ y, const C2* __restrict__ x, long long n, const double* __restrict__ sl,
                             int den) {
  using T = typename real_of<C2>::type;
  const int rhs = blockIdx.y;
  const long long off = rhs * n;
  const double d = slot(sl, rhs, den);
  const T s = (T)(d > 0.0 ? 1.0 / sqrt(d) : 0.0);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[off + i] = cscale(x[off + i], s);
}

template <class A2, class B2>
__global__ void k_convert(const A2* __restrict__ in, B2* __restrict__ out, long long n) {
  using T = typename real_of<B2>::type;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    A2 v = in[i];
    out[i] = cmk<B2>((T)v.x, (T)v.y);
  }
}

// y += x (x possibly in another precision)
template <class A2, class B2>
__global__ void k_add_to(B2* __restrict__ y, const A2* __restrict__ x, long long n) {
  using T = typename real_of<B2>::type;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    A2 v = x[i];
    B2 w = y[i];
    y[i] = cmk<B2>(w.x + (T)v.x, w.y + (T)v.y);
  }
}

template <class C2>
__global__ void k_zero(C2* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = cmk<C2>(0, 0);
}

// (R5 v)(x4, s) = v(x4, Ls-1-s), internal fine layout, nrhs fields
template <class C2>
__global__ void k_reflect5(const C2* __restrict__ in, C2* __restrict__ out, long long V5, int Ls, long long nf) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nf * 12 * V5; i += (long long)gridDim.x * blockDim.x) {
    long long i5 = i % V5;
    long long rest = i - i5;
    long long x4 = i5 / Ls;
    int s = (int)(i5 - x4 * Ls);
    out[i] = in[rest + x4 * Ls + (Ls - 1 - s)];
  }
}

}  // namespace

int vec_blocks(long long n) { return std::max(1, std::min(ceil_div(n, 256), VEC_BLOCKS)); }

void finalize_rhs(const double* partial, int nparts, int ncomp, double* sl, int dst, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_rhs, dim3(ncomp, nrhs), dim3(256), 0, st, partial, nparts, ncomp, sl, dst);
  MG_LAUNCH_CHECK();
}

template <class C2>
void mr_update(C2* x, C2* r, const C2* p, const C2* q, long long n, int nrhs, const double* sl, int num, int den,
               bool first, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_mr_update<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, x, r, p, q, n, sl, num, den,
                     first ? 1 : 0, partial);
  MG_LAUNCH_CHECK();
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <class C2>
void res_update(C2* rout, const C2* rin, const C2* q, long long n, int nrhs, const double* sl, int num, int den,
                hipStream_t st) {
  if constexpr (std::is_same<C2, float2>::value) {
    if (n % 2 == 0 && aligned16(rout) && aligned16(rin) && aligned16(q)) {
      hipLaunchKernelGGL(k_res_update_pair, dim3(vec_blocks(n / 2), nrhs), dim3(256), 0, st,
                         reinterpret_cast<float4*>(rout), reinterpret_cast<const float4*>(rin),
                         reinterpret_cast<const float4*>(q), n / 2, sl, num, den);
      MG_LAUNCH_CHECK();
      return;
    }
  }
  hipLaunchKernelGGL(k_res_update<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, rout, rin, q, n, sl, num, den);
  MG_LAUNCH_CHECK();
}

template <class C2>
void lincomb(C2* x, const C2* const* ps, int nv, long long n, int nrhs, const double* sl, int num, bool acc,
             hipStream_t st) {
  if (nv > 16) fail(MGDWF_ERR_INVALID_ARG, "at most 16 smoother steps");
  if constexpr (std::is_same<C2, float2>::value) {
    if (n % 2 == 0 && aligned16(x)) {  // the vectors ps[m] are workspaces: 256-byte aligned
      hipLaunchKernelGGL(k_lincomb_pair, dim3(vec_blocks(n / 2), nrhs), dim3(256), 0, st,
                         reinterpret_cast<float4*>(x), ps, nv, n / 2, sl, num, acc ? 1 : 0);
      MG_LAUNCH_CHECK();
      return;
    }
  }
  hipLaunchKernelGGL(k_lincomb<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, x, ps, nv, n, sl, num, acc ? 1 : 0);
  MG_LAUNCH_CHECK();
}

template <class C2>
void cg_dir(C2* p, const C2* r, long long n, int nrhs, const double* sl, int num, int den, double* partial,
            hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, p, r, n, sl, num, den, partial);
  MG_LAUNCH_CHECK();
}

template <class C2>
void multidot_rhs(const C2* const* avec, int nv, const C2* b, const C2* c, long long n, int nrhs, double* partial,
                  double* sl, int dst, hipStream_t st) {
  if (nv > 16) fail(MGDWF_ERR_INVALID_ARG, "at most 16 Krylov vectors per restart");
  hipLaunchKernelGGL(k_multidot<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, avec, nv, b, c, n, partial);
  MG_LAUNCH_CHECK();
  finalize_rhs(partial, vec_blocks(n), 2 * nv + 3, sl, dst, nrhs, st);
}

template <class C2>
void orth_update(C2* q, C2* z, const C2* const* qs, const C2* const* zs, int nv, long long n, int nrhs,
                 const double* sl, int dots, int nrm, hipStream_t st) {
  if (nv == 0) return;
  hipLaunchKernelGGL(k_orth_update<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, q, z, qs, zs, nv, n, sl, dots, nrm);
  MG_LAUNCH_CHECK();
}

template <class C2>
void lincomb_c(C2* x, const C2* const* ps, int nv, long long n, int nrhs, const double2* coef, hipStream_t st) {
  if (nv > 16) fail(MGDWF_ERR_INVALID_ARG, "at most 16 Krylov vectors per restart");
  hipLaunchKernelGGL(k_lincomb_c<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, x, ps, nv, n, coef);
  MG_LAUNCH_CHECK();
}

template <class C2>
void gcr_update(C2* e, C2* r, const C2* z, const C2* q, long long n, int nrhs, const double* sl, int cr, int nq,
                bool first, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_gcr_update<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, e, r, z, q, n, sl, cr, nq,
                     first ? 1 : 0, partial);
  MG_LAUNCH_CHECK();
}

template <class C2>
void mrh_update(C2* x, C2* rnew, const C2* rin, const C2* p, long long n, int nrhs, const double* sl, int cr, int nq,
                bool first, hipStream_t st) {
  hipLaunchKernelGGL(k_mrh_update<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, x, rnew, rin, p, n, sl, cr, nq,
                     first ? 1 : 0);
  MG_LAUNCH_CHECK();
}

template <class C2>
void scale_by_rsqrt_slot(C2* y, const C2* x, long long n, int nrhs, const double* sl, int den, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_slot<C2>, dim3(vec_blocks(n), nrhs), dim3(256), 0, st, y, x, n, sl, den);
  MG_LAUNCH_CHECK();
}

template <class A2, class B2>
void convert(const A2* in, B2* out, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<A2, B2>), dim3(vec_blocks(n)), dim3(256), 0, st, in, out, n);
  MG_LAUNCH_CHECK();
}

template <class A2, class B2>
void add_to(B2* y, const A2* x, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_add_to<A2, B2>), dim3(vec_blocks(n)), dim3(256), 0, st, y, x, n);
  MG_LAUNCH_CHECK();
}

template <class C2>
void zero(C2* y, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<C2>, dim3(vec_blocks(n)), dim3(256), 0, st, y, n);
  MG_LAUNCH_CHECK();
}

template <class C2>
void reflect5(const C2* in, C2* out, const Geometry& g, int nf, hipStream_t st) {
  hipLaunchKernelGGL(k_reflect5<C2>, dim3(vec_blocks(12LL * g.V5 * nf)), dim3(256), 0, st, in, out, (long long)g.V5,
                     g.Ls, (long long)nf);
  MG_LAUNCH_CHECK();
}

#define MG_INST(C2)                                                                                              \
  template void mr_update<C2>(C2*, C2*, const C2*, const C2*, long long, int, const double*, int, int, bool,    \
                              double*, hipStream_t);                                                             \
  template void cg_dir<C2>(C2*, const C2*, long long, int, const double*, int, int, double*, hipStream_t);      \
  template void res_update<C2>(C2*, const C2*, const C2*, long long, int, const double*, int, int, hipStream_t); \
  template void lincomb_c<C2>(C2*, const C2* const*, int, long long, int, const double2*, hipStream_t);        \
  template void lincomb<C2>(C2*, const C2* const*, int, long long, int, const double*, int, bool, hipStream_t);        \
  template void multidot_rhs<C2>(const C2* const*, int, const C2*, const C2*, long long, int, double*, double*, \
                                 int, hipStream_t);                                                              \
  template void orth_update<C2>(C2*, C2*, const C2* const*, const C2* const*, int, long long, int,              \
                                const double*, int, int, hipStream_t);                                          \
  template void gcr_update<C2>(C2*, C2*, const C2*, const C2*, long long, int, const double*, int, int, bool,   \
                               double*, hipStream_t);                                                            \
  template void scale_by_rsqrt_slot<C2>(C2*, const C2*, long long, int, const double*, int, hipStream_t);       \
  template void mrh_update<C2>(C2*, C2*, const C2*, const C2*, long long, int, const double*, int, int, bool,    \
                               hipStream_t);                                                                    \
  template void zero<C2>(C2*, long long, hipStream_t);                                                           \
  template void reflect5<C2>(const C2*, C2*, const Geometry&, int, hipStream_t);
MG_INST(double2)
MG_INST(float2)
#undef MG_INST
template void convert<double2, float2>(const double2*, float2*, long long, hipStream_t);
template void convert<float2, double2>(const float2*, double2*, long long, hipStream_t);
template void convert<double2, double2>(const double2*, double2*, long long, hipStream_t);
template void convert<float2, float2>(const float2*, float2*, long long, hipStream_t);
template void add_to<float2, double2>(double2*, const float2*, long long, hipStream_t);
template void add_to<double2, double2>(double2*, const double2*, long long, hipStream_t);
template void add_to<float2, float2>(float2*, const float2*, long long, hipStream_t);

}  // namespace mgdwf
