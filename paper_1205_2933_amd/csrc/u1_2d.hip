// The two-dimensional U(1) domain-wall operator (the paper's first test
// problem, Sec. 3 and Fig. 2: a quenched U(1) field in two dimensions, blocks
// spanning the fifth dimension) and the fine-level operations that depend on
// which model a handle holds.
//
// The 2D operator, with g_x = sigma_1, g_y = sigma_2, g_5 = sigma_3 (P_+ keeps
// spin 0, P_- spin 1):
//   (D psi)(x,s) = (3 - M5) psi(x,s)
//     - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) conj(U_mu(x-mu)) psi(x-mu,s) ]
//     - P_- psi(x,s+1) - P_+ psi(x,s-1),
// the fifth-dimension hops across the walls carrying -m_f instead of 1 (so
// +m_f in D), the adjoint exchanging the signs of g_mu and the roles of P_+
// and P_-.  This is the 4D Shamir form of the library with two directions.
//
// Internal layouts of the 2D model:
//   fine field: element (x2, spin, s) at (x2 * 2 + spin) * Ls + s, x2 = y * Lx + x;
//     field r of nrhs at r * 2 * Lx * Ly * Ls.  This is the coarse-vector
//     layout [site][chirality][k] with Nv = Ls (chirality = spin), so the
//     chirality-split block basis, R, P and the probed Galerkin operator of
//     the third level (level2.hip) serve the 2D fine level unchanged.
//   gauge: element (mu, x2) at mu * Lx * Ly + x2 (FP64 in U64, FP32 in U32).
#include <functional>

#include "blas.h"
#include "ctx.h"
#include "vecops.h"

namespace mgdwf {

namespace {

struct D2Args {
  int Lx, Ly, Ls, V2, V5;
  int bcx, bcy;       // +1 periodic, -1 antiperiodic
  double diag, mf;    // 3 - M5, m_f
};

// (1 + sg g_x) h and (1 + sg g_y) h for a two-spinor h = (h0, h1)
template <class F2>
__device__ __forceinline__ void proj_x(F2& o0, F2& o1, F2 h0, F2 h1, int sg) {
  if (sg > 0) { o0 = cadd(o0, cadd(h0, h1)); o1 = cadd(o1, cadd(h1, h0)); }
  else        { o0 = cadd(o0, csub(h0, h1)); o1 = cadd(o1, csub(h1, h0)); }
}
template <class F2>
__device__ __forceinline__ void proj_y(F2& o0, F2& o1, F2 h0, F2 h1, int sg) {
  // g_y h = (-i h1, i h0)
  if (sg > 0) { o0 = cadd(o0, csub(h0, ci(h1))); o1 = cadd(o1, cadd(h1, ci(h0))); }
  else        { o0 = cadd(o0, cadd(h0, ci(h1))); o1 = cadd(o1, csub(h1, ci(h0))); }
}

// One thread per (site, s) and right-hand side; MODE 0: out = D in (D^+ for
// DAG), MODE 1: out = b - D in.  With partial, the |out|^2 of each workgroup
// goes to partial[rhs * gridDim.x + blockIdx.x].
template <class F2, bool DAG, int MODE>
__global__ __launch_bounds__(256) void k_dwf2d(const F2* __restrict__ in, F2* __restrict__ out,
                                               const F2* __restrict__ b, const F2* __restrict__ U, D2Args a,
                                               double* __restrict__ partial) {
  using T = typename real_of<F2>::type;
  const int rhs = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  double nrm = 0.0;
  if (i < a.V5) {
    const long long base = (long long)rhs * 2 * a.V5;
    const F2* f = in + base;
    const int x2 = i / a.Ls, s = i - x2 * a.Ls;
    const int x = x2 % a.Lx, y = x2 / a.Lx;
    auto at = [&](int site, int sp, int ss) { return f[((long long)site * 2 + sp) * a.Ls + ss]; };
    const F2 p0 = at(x2, 0, s), p1 = at(x2, 1, s);
    F2 h0 = cmk<F2>(0, 0), h1 = cmk<F2>(0, 0);
    const int sf = DAG ? 1 : -1;  // forward hop: (1 + sf g_mu), backward: (1 - sf g_mu)
    // x direction
    {
      const int xf = x + 1 == a.Lx ? 0 : x + 1, xb = x == 0 ? a.Lx - 1 : x - 1;
      const int nf = y * a.Lx + xf, nb = y * a.Lx + xb;
      const T phf = (x + 1 == a.Lx) ? (T)a.bcx : (T)1, phb = (x == 0) ? (T)a.bcx : (T)1;
      const F2 uf = cscale(U[x2], phf), ub = cscale(U[nb], phb);
      proj_x(h0, h1, cmul(uf, at(nf, 0, s)), cmul(uf, at(nf, 1, s)), sf);
      proj_x(h0, h1, cmulc(ub, at(nb, 0, s)), cmulc(ub, at(nb, 1, s)), -sf);
    }
    // y direction
    {
      const int yf = y + 1 == a.Ly ? 0 : y + 1, yb = y == 0 ? a.Ly - 1 : y - 1;
      const int nf = yf * a.Lx + x, nb = yb * a.Lx + x;
      const T phf = (y + 1 == a.Ly) ? (T)a.bcy : (T)1, phb = (y == 0) ? (T)a.bcy : (T)1;
      const F2 uf = cscale(U[a.V2 + x2], phf), ub = cscale(U[a.V2 + nb], phb);
      proj_y(h0, h1, cmul(uf, at(nf, 0, s)), cmul(uf, at(nf, 1, s)), sf);
      proj_y(h0, h1, cmulc(ub, at(nb, 0, s)), cmulc(ub, at(nb, 1, s)), -sf);
    }
    F2 o0 = csub(cscale(p0, (T)a.diag), cscale(h0, (T)0.5));
    F2 o1 = csub(cscale(p1, (T)a.diag), cscale(h1, (T)0.5));
    // fifth dimension: the spin taken from s + 1 (P_- for D, P_+ for D^+) and
    // the one taken from s - 1, each with -1 or, across the wall, +m_f
    const int su = s + 1 == a.Ls ? 0 : s + 1, sd = s == 0 ? a.Ls - 1 : s - 1;
    const T cu = (s + 1 == a.Ls) ? (T)a.mf : (T)-1, cd = (s == 0) ? (T)a.mf : (T)-1;
    if (!DAG) {
      o1 = cadd(o1, cscale(at(x2, 1, su), cu));
      o0 = cadd(o0, cscale(at(x2, 0, sd), cd));
    } else {
      o0 = cadd(o0, cscale(at(x2, 0, su), cu));
      o1 = cadd(o1, cscale(at(x2, 1, sd), cd));
    }
    const long long e0 = base + (long long)x2 * 2 * a.Ls + s, e1 = e0 + a.Ls;
    if (MODE == 1) {
      o0 = csub(b[e0], o0);
      o1 = csub(b[e1], o1);
    }
    out[e0] = o0;
    out[e1] = o1;
    nrm = (double)o0.x * o0.x + (double)o0.y * o0.y + (double)o1.x * o1.x + (double)o1.y * o1.y;
  }
  if (partial) {
    const double t = block_sum<256>(nrm);
    if (threadIdx.x == 0) partial[rhs * gridDim.x + blockIdx.x] = t;
  }
}

// canonical ((x2 * Ls + s) * 2 + spin) <-> internal ((x2 * 2 + spin) * Ls + s)
__global__ void k_pack2d(const double2* __restrict__ canon, double2* __restrict__ field, int Ls, long long n,
                         int unpack) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long site = e / (2 * Ls);
    const int r = (int)(e - site * 2 * Ls);
    const int s = r >> 1, sp = r & 1;
    const long long f = (site * 2 + sp) * Ls + s;
    if (unpack) field[e] = canon[f];  // here `canon` is the internal field, `field` the canonical output
    else field[f] = canon[e];
  }
}

// canonical (x2 * 2 + mu) -> internal (mu * V2 + x2), FP64 and FP32
__global__ void k_pack_gauge2d(const double2* __restrict__ canon, double2* __restrict__ g64,
                               float2* __restrict__ g32, int V2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * V2) return;
  const int x2 = e >> 1, mu = e & 1;
  const double2 v = canon[e];
  g64[mu * V2 + x2] = v;
  g32[mu * V2 + x2] = make_float2((float)v.x, (float)v.y);
}

D2Args args_of(const mgdwf_ctx* c) {
  D2Args a;
  a.Lx = c->g.L[0];
  a.Ly = c->g.L[1];
  a.Ls = c->g.Ls;
  a.V2 = c->g.V4;
  a.V5 = c->g.V5;
  a.bcx = c->g.bc[0];
  a.bcy = c->g.bc[1];
  a.diag = 3.0 - c->M5;
  a.mf = c->mf;
  return a;
}

int nblk(long long n) { return (int)std::max<long long>(1, std::min<long long>(ceil_div(n, 256), 4096)); }

template <class F2> const F2* gauge_for(const mgdwf_ctx* c);
template <> const double2* gauge_for<double2>(const mgdwf_ctx* c) { return c->U64.as<double2>(); }
template <> const float2* gauge_for<float2>(const mgdwf_ctx* c) { return c->U32.as<float2>(); }

template <class F2>
void dwf2d(const mgdwf_ctx* c, const F2* in, F2* out, const F2* b, bool dag, int mode, int nrhs, double* partial,
           hipStream_t st) {
  const D2Args a = args_of(c);
  const dim3 grid(ceil_div(a.V5, 256), nrhs);
  const F2* U = gauge_for<F2>(c);
  if (!dag && mode == 0) hipLaunchKernelGGL((k_dwf2d<F2, false, 0>), grid, dim3(256), 0, st, in, out, b, U, a, partial);
  else if (!dag) hipLaunchKernelGGL((k_dwf2d<F2, false, 1>), grid, dim3(256), 0, st, in, out, b, U, a, partial);
  else if (mode == 0) hipLaunchKernelGGL((k_dwf2d<F2, true, 0>), grid, dim3(256), 0, st, in, out, b, U, a, partial);
  else hipLaunchKernelGGL((k_dwf2d<F2, true, 1>), grid, dim3(256), 0, st, in, out, b, U, a, partial);
  MG_LAUNCH_CHECK();
}

}  // namespace

// ---------------------------------------------------------------- model dispatch

void pack_field(const mgdwf_ctx* c, const double2* canon, double2* field, int nrhs) {
  if (c->model == 0) {
    pack_fermion_f64(canon, field, c->g, nrhs, c->st);
    return;
  }
  const long long n = 2LL * c->g.V5 * nrhs;
  hipLaunchKernelGGL(k_pack2d, dim3(nblk(n)), dim3(256), 0, c->st, canon, field, c->g.Ls, n, 0);
  MG_LAUNCH_CHECK();
}

void unpack_field(const mgdwf_ctx* c, const double2* field, double2* canon, int nrhs) {
  if (c->model == 0) {
    unpack_fermion_f64(field, canon, c->g, nrhs, c->st);
    return;
  }
  const long long n = 2LL * c->g.V5 * nrhs;
  hipLaunchKernelGGL(k_pack2d, dim3(nblk(n)), dim3(256), 0, c->st, field, canon, c->g.Ls, n, 1);
  MG_LAUNCH_CHECK();
}

void pack_gauge_field(mgdwf_ctx* c, const double2* canon) {
  if (c->model == 0) {
    const long long n = 36LL * c->g.V4;
    c->U64.alloc(n * sizeof(double2));
    c->U32.alloc(3 * n * sizeof(float2));  // component-major links, a site-major copy, a phase-folded copy
    pack_gauge(canon, c->U64.as<double2>(), c->U32.as<float2>(), c->g, c->st);
    return;
  }
  const int V2 = c->g.V4;
  c->U64.alloc(2LL * V2 * sizeof(double2));
  c->U32.alloc(2LL * V2 * sizeof(float2));
  hipLaunchKernelGGL(k_pack_gauge2d, dim3(ceil_div(2LL * V2, 256)), dim3(256), 0, c->st, canon, c->U64.as<double2>(),
                     c->U32.as<float2>(), V2);
  MG_LAUNCH_CHECK();
}

template <class F2>
int fine_nblocks(const mgdwf_ctx* c, int nrhs) {
  return c->model == 0 ? dslash_nblocks<F2>(c->g, nrhs) : ceil_div(c->g.V5, 256);
}

template <class F2>
void fine_dslash(const mgdwf_ctx* c, const F2* in, F2* out, const F2* b, bool dag, int mode, int nrhs,
                 double* partial, hipStream_t st) {
  if (c->model == 0)
    dslash_ex<F2>(in, out, b, gauge_for<F2>(c), c->g, c->M5, c->mf, dag, mode, nrhs, partial, st);
  else
    dwf2d<F2>(c, in, out, b, dag, mode, nrhs, partial, st);
}

template <class F2>
void fine_restrict(mgdwf_ctx* c, const F2* V, const F2* in, F2* out, int nrhs) {
  if (c->model == 0)
    restrict_op<F2, F2>(V, in, out, c->buf<double>("rpart", restrict_partial_doubles(c->cg, nrhs)), c->g, c->cg,
                        nrhs, c->st);
  else
    restrict2<F2>(V, in, out, c->fg, c->cg, nrhs, c->st);
}

template <class F2>
void fine_prolong(mgdwf_ctx* c, const F2* V, const F2* cc, F2* out, bool acc, int nrhs) {
  if (c->model == 0) prolong_op<F2, F2>(V, cc, out, acc, c->g, c->cg, nrhs, c->st);
  else prolong2<F2>(V, cc, out, acc, c->fg, c->cg, nrhs, c->st);
}

bool fine_orthonormalise(mgdwf_ctx* c) {
  if (c->model == 0) return orthonormalise_basis(c->V64.as<double2>(), c->g, c->cg, c->st);
  return orthonormalise_level2(c->V64.as<double2>(), c->fg, c->cg, c->buf<int>("orth_err", 1), c->st);
}

// A_c = P^+ D^+D P of the 2D model, read off per source block (probing the
// fine D^+D with the block's basis columns, restricting, scattering into the
// 33-offset form whose offsets along the two unit directions z, t stay zero).
void build_sq_coarse_2d(mgdwf_ctx* c) {
  const CoarseGeometry& cg = c->cg;
  const long long nf = c->fine_len();
  const int np = cg.n2;
  double2* probes = c->buf<double2>("dc_probe", (size_t)np * nf);
  double2* applied = c->buf<double2>("dc_applied", (size_t)np * nf);
  double2* tmp = c->buf<double2>("dc_tmp", (size_t)np * nf);
  double2* rr = c->buf<double2>("dc_rr", (size_t)np * cg.Vc * cg.n2);
  auto normal = [&](const double2* x, double2* y, int n) {
    dwf2d<double2>(c, x, tmp, nullptr, false, 0, n, nullptr, c->st);
    dwf2d<double2>(c, tmp, y, nullptr, true, 0, n, nullptr, c->st);
  };
  build_galerkin_op(normal, c->V64.as<double2>(), c->Asq.m64.as<double2>(), probes, applied, rr, c->fg, cg, c->st);
  c->fine_applies += 2LL * cg.Vc;
}

template int fine_nblocks<double2>(const mgdwf_ctx*, int);
template int fine_nblocks<float2>(const mgdwf_ctx*, int);
template void fine_dslash<double2>(const mgdwf_ctx*, const double2*, double2*, const double2*, bool, int, int,
                                   double*, hipStream_t);
template void fine_dslash<float2>(const mgdwf_ctx*, const float2*, float2*, const float2*, bool, int, int, double*,
                                  hipStream_t);
template void fine_restrict<double2>(mgdwf_ctx*, const double2*, const double2*, double2*, int);
template void fine_restrict<float2>(mgdwf_ctx*, const float2*, const float2*, float2*, int);
template void fine_prolong<double2>(mgdwf_ctx*, const double2*, const double2*, double2*, bool, int);
template void fine_prolong<float2>(mgdwf_ctx*, const float2*, const float2*, float2*, bool, int);

}  // namespace mgdwf
