// Shamir domain-wall operator on gfx950.
//
// Operator (the paper's Sec. 2 fifth-dimension paragraph and Sec. 4 stencil):
//   (D psi)(x,s) = (5 - M5) psi(x,s)
//       - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu,s)]
//       - P_- psi(x,s+1) - P_+ psi(x,s-1),    P_- psi(x,Ls) = -m_f P_- psi(x,0),
//                                             P_+ psi(x,-1) = -m_f P_+ psi(x,Ls-1).
// D^+ exchanges (1 - g_mu) <-> (1 + g_mu) and P_+ <-> P_- in the fifth-dimension hop.
//
// Mapping: one thread per 5D site (x4, s); a 256-thread workgroup covers 256
// consecutive (x4, s) pairs of the layout (c * V4 + x4) * Ls + s, so each of
// the 12 spin-colour loads of a neighbour is one coalesced segment per
// wavefront, and the Ls lanes of one 4D site read the same link (one cache
// line serves them all).  The 4D hop is done on half spinors: (1 +- g_mu)
// has rank 2 in spin, so two SU(3) mat-vecs per direction instead of four.
// Workgroup indices are remapped so each XCD sweeps a contiguous slab of the
// lattice and neighbour re-reads hit its own L2.
#include "mg_internal.h"
#include "blas.h"

namespace mgdwf {

namespace {

template <class C2>
struct Spinor {
  C2 v[4][3];
};

// Half spinor of (1 + eps g_mu) psi in the chiral basis; returns the upper two
// spin components h0, h1 (the lower two are a fixed 2x2 map of them).
template <int MU, int EPS, class C2>
__device__ __forceinline__ void project(const Spinor<C2>& p, C2 h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {        // g_x: h0 = p0 - eps i p3, h1 = p1 - eps i p2
      h[0][c] = csub(p.v[0][c], cscale(ci(p.v[3][c]), (float)EPS));
      h[1][c] = csub(p.v[1][c], cscale(ci(p.v[2][c]), (float)EPS));
    } else if (MU == 1) { // g_y: h0 = p0 - eps p3, h1 = p1 + eps p2
      h[0][c] = csub(p.v[0][c], cscale(p.v[3][c], (float)EPS));
      h[1][c] = cadd(p.v[1][c], cscale(p.v[2][c], (float)EPS));
    } else if (MU == 2) { // g_z: h0 = p0 - eps i p2, h1 = p1 + eps i p3
      h[0][c] = csub(p.v[0][c], cscale(ci(p.v[2][c]), (float)EPS));
      h[1][c] = cadd(p.v[1][c], cscale(ci(p.v[3][c]), (float)EPS));
    } else {              // g_t: h0 = p0 + eps p2, h1 = p1 + eps p3
      h[0][c] = cadd(p.v[0][c], cscale(p.v[2][c], (float)EPS));
      h[1][c] = cadd(p.v[1][c], cscale(p.v[3][c], (float)EPS));
    }
  }
}

// acc += (1 + eps g_mu) reconstructed from the transported half spinor u.
template <int MU, int EPS, class C2>
__device__ __forceinline__ void accumulate(Spinor<C2>& acc, const C2 u[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc.v[0][c] = cadd(acc.v[0][c], u[0][c]);
    acc.v[1][c] = cadd(acc.v[1][c], u[1][c]);
    if (MU == 0) {        // lower = eps (i u1, i u0)
      acc.v[2][c] = cadd(acc.v[2][c], cscale(ci(u[1][c]), (float)EPS));
      acc.v[3][c] = cadd(acc.v[3][c], cscale(ci(u[0][c]), (float)EPS));
    } else if (MU == 1) { // lower = eps (u1, -u0)
      acc.v[2][c] = cadd(acc.v[2][c], cscale(u[1][c], (float)EPS));
      acc.v[3][c] = csub(acc.v[3][c], cscale(u[0][c], (float)EPS));
    } else if (MU == 2) { // lower = eps (i u0, -i u1)
      acc.v[2][c] = cadd(acc.v[2][c], cscale(ci(u[0][c]), (float)EPS));
      acc.v[3][c] = csub(acc.v[3][c], cscale(ci(u[1][c]), (float)EPS));
    } else {              // lower = eps (u0, u1)
      acc.v[2][c] = cadd(acc.v[2][c], cscale(u[0][c], (float)EPS));
      acc.v[3][c] = cadd(acc.v[3][c], cscale(u[1][c], (float)EPS));
    }
  }
}

template <class C2>
__device__ __forceinline__ void load_spinor(Spinor<C2>& p, const C2* __restrict__ f, long long stride,
                                            long long i5) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p.v[sp][c] = f[(sp * 3 + c) * stride + i5];
}

// u = U h  (DAGU false) or U^+ h (DAGU true) for both half-spinor rows;
// link (mu, a, b) lives at (mu*9 + a*3 + b) * V4 + x4.
template <bool DAGU, class C2>
__device__ __forceinline__ void transport(const C2* __restrict__ gauge, int mu, long long V4, int x4,
                                          const C2 h[2][3], C2 u[2][3]) {
  C2 U[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) U[a][b] = gauge[(mu * 9 + a * 3 + b) * V4 + x4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C2 s = cmk<C2>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (DAGU) cfmac(s, U[b][a], h[r][b]);
        else cfma(s, U[a][b], h[r][b]);
      }
      u[r][a] = s;
    }
}

template <int MU, int EPS_F, int EPS_B, class C2>
__device__ __forceinline__ void hop_dir(Spinor<C2>& acc, const C2* __restrict__ in,
                                        const C2* __restrict__ gauge, long long V5, long long V4,
                                        int Ls, int s, int x4, int xf, int xb, float phf, float phb) {
  Spinor<C2> p;
  C2 h[2][3], u[2][3];
  // forward neighbour: U_mu(x) psi(x + mu)
  load_spinor(p, in, V5, (long long)xf * Ls + s);
  project<MU, EPS_F>(p, h);
  transport<false>(gauge, MU, V4, x4, h, u);
  if (phf != 1.0f) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) u[r][c] = cscale(u[r][c], phf);
  }
  accumulate<MU, EPS_F>(acc, u);
  // backward neighbour: U_mu(x - mu)^+ psi(x - mu)
  load_spinor(p, in, V5, (long long)xb * Ls + s);
  project<MU, EPS_B>(p, h);
  transport<true>(gauge, MU, V4, xb, h, u);
  if (phb != 1.0f) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) u[r][c] = cscale(u[r][c], phb);
  }
  accumulate<MU, EPS_B>(acc, u);
}

struct DslashArgs {
  int L[4];
  int Ls;
  int V4;
  int V5;
  float ph[4];   // boundary phase per direction (+1 / -1)
  double diag;   // 5 - M5
  double mf;
};

// MODE 0: out = D in;  MODE 1: out = b - D in.  partial (if non-null) gets the
// per-workgroup sum of |out|^2 at index blockIdx.y * gridDim.x + blockIdx.x.
template <class C2, bool DAG, int MODE>
__global__ __launch_bounds__(256) void k_dslash(const C2* __restrict__ in, C2* __restrict__ out,
                                                const C2* __restrict__ b, const C2* __restrict__ gauge,
                                                DslashArgs a, double* __restrict__ partial) {
  using T = typename real_of<C2>::type;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const long long i5 = (long long)bid * 256 + threadIdx.x;
  const long long V5 = a.V5, V4 = a.V4;
  const long long roff = (long long)blockIdx.y * 12 * V5;
  in += roff;
  out += roff;
  if (MODE == 1) b += roff;
  double nrm = 0.0;
  if (i5 < V5) {
    const int Ls = a.Ls;
    const int x4 = (int)(i5 / Ls);
    const int s = (int)(i5 - (long long)x4 * Ls);
    int co[4];
    {
      int r = x4;
      co[0] = r % a.L[0]; r /= a.L[0];
      co[1] = r % a.L[1]; r /= a.L[1];
      co[2] = r % a.L[2]; co[3] = r / a.L[2];
    }
    int stride[4] = {1, a.L[0], a.L[0] * a.L[1], a.L[0] * a.L[1] * a.L[2]};
    int xf[4], xb[4];
    float phf[4], phb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      bool top = co[mu] == a.L[mu] - 1, bot = co[mu] == 0;
      xf[mu] = top ? x4 - (a.L[mu] - 1) * stride[mu] : x4 + stride[mu];
      xb[mu] = bot ? x4 + (a.L[mu] - 1) * stride[mu] : x4 - stride[mu];
      phf[mu] = top ? a.ph[mu] : 1.0f;
      phb[mu] = bot ? a.ph[mu] : 1.0f;
    }
    Spinor<C2> acc;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sp][c] = cmk<C2>(0, 0);
    // D: forward (1 - g), backward (1 + g);  D^+: the other way round
    constexpr int EF = DAG ? 1 : -1;
    constexpr int EB = DAG ? -1 : 1;
    hop_dir<0, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, xf[0], xb[0], phf[0], phb[0]);
    hop_dir<1, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, xf[1], xb[1], phf[1], phb[1]);
    hop_dir<2, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, xf[2], xb[2], phf[2], phb[2]);
    hop_dir<3, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, xf[3], xb[3], phf[3], phb[3]);

    // fifth dimension: spins coupled to s+1 are {2,3} for D, {0,1} for D^+
    const int up0 = DAG ? 0 : 2;
    const int dn0 = DAG ? 2 : 0;
    const long long base = (long long)x4 * Ls;
    const int sp1 = (s == Ls - 1) ? 0 : s + 1;
    const int sm1 = (s == 0) ? Ls - 1 : s - 1;
    const T cup = (s == Ls - 1) ? (T)a.mf : (T)-1;
    const T cdn = (s == 0) ? (T)a.mf : (T)-1;
    const T half = (T)-0.5;
    const T dg = (T)a.diag;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long cc = (long long)(sp * 3 + c) * V5;
        C2 self = in[cc + i5];
        C2 r = cadd(cscale(self, dg), cscale(acc.v[sp][c], half));
        if (sp == up0 || sp == up0 + 1) r = cadd(r, cscale(in[cc + base + sp1], cup));
        if (sp == dn0 || sp == dn0 + 1) r = cadd(r, cscale(in[cc + base + sm1], cdn));
        if (MODE == 1) r = csub(b[cc + i5], r);
        out[cc + i5] = r;
        nrm += (double)r.x * r.x + (double)r.y * r.y;
      }
  }
  if (partial) {
    double sum = block_sum<256>(nrm);
    if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
}

// Face-split operator for the coarse-operator build (FP64): the nine pieces of
// D applied to P_chi psi (the chirality-chi spins of psi):
//   out[0]          diagonal, fifth-dimension hop and every 4D hop that stays
//                   inside the site's block;
//   out[1 + 2 mu]   the +mu hop of sites on the upper block face;
//   out[2 + 2 mu]   the -mu hop of sites on the lower block face.
// Uses the same half-spinor helpers as k_dslash.
struct SplitArgs {
  int L[4];
  int b[4];
  int Ls;
  int V4;
  int V5;
  float ph[4];
  double diag;
  double mf;
  int chi;
};

__device__ __forceinline__ void load_masked(Spinor<double2>& p, const double2* __restrict__ f, long long V5,
                                            long long j5, int chi) {
  load_spinor(p, f, V5, j5);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if ((sp >> 1) != chi) p.v[sp][c] = make_double2(0.0, 0.0);
}

template <int MU>
__device__ __forceinline__ void split_dir(Spinor<double2>& self, double2* __restrict__ out, const double2* __restrict__ in,
                                          const double2* __restrict__ gauge, const SplitArgs& a, long long i5, int x4,
                                          int s, const int co[4], const int stride[4]) {
  const long long V5 = a.V5, V4 = a.V4;
  const bool top = co[MU] == a.L[MU] - 1, bot = co[MU] == 0;
  const int xf = top ? x4 - (a.L[MU] - 1) * stride[MU] : x4 + stride[MU];
  const int xb = bot ? x4 + (a.L[MU] - 1) * stride[MU] : x4 - stride[MU];
  const double phf = top ? a.ph[MU] : 1.0, phb = bot ? a.ph[MU] : 1.0;
  const bool upper_face = (co[MU] % a.b[MU]) == a.b[MU] - 1;
  const bool lower_face = (co[MU] % a.b[MU]) == 0;
  Spinor<double2> p, f;
  double2 h[2][3], u[2][3];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) f.v[sp][c] = make_double2(0.0, 0.0);
    if (dir == 0) {  // -1/2 (1 - g_mu) U_mu(x) psi(x + mu)
      load_masked(p, in, V5, (long long)xf * a.Ls + s, a.chi);
      project<MU, -1>(p, h);
      transport<false>(gauge, MU, V4, x4, h, u);
      accumulate<MU, -1>(f, u);
    } else {         // -1/2 (1 + g_mu) U_mu(x - mu)^+ psi(x - mu)
      load_masked(p, in, V5, (long long)xb * a.Ls + s, a.chi);
      project<MU, 1>(p, h);
      transport<true>(gauge, MU, V4, xb, h, u);
      accumulate<MU, 1>(f, u);
    }
    const double sc = -0.5 * (dir == 0 ? phf : phb);
    const bool face = dir == 0 ? upper_face : lower_face;
    double2* o = out + (long long)(1 + 2 * MU + dir) * 12 * V5;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 v = cscale(f.v[sp][c], sc);
        if (face) {
          o[(sp * 3 + c) * V5 + i5] = v;
        } else {
          o[(sp * 3 + c) * V5 + i5] = make_double2(0.0, 0.0);
          self.v[sp][c] = cadd(self.v[sp][c], v);
        }
      }
  }
}

__global__ __launch_bounds__(256) void k_dslash_split(const double2* __restrict__ in, double2* __restrict__ out,
                                                      const double2* __restrict__ gauge, SplitArgs a) {
  const long long i5 = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long V5 = a.V5;
  if (i5 >= V5) return;
  const int Ls = a.Ls;
  const int x4 = (int)(i5 / Ls), s = (int)(i5 - (long long)x4 * Ls);
  int co[4];
  {
    int r = x4;
    co[0] = r % a.L[0]; r /= a.L[0];
    co[1] = r % a.L[1]; r /= a.L[1];
    co[2] = r % a.L[2]; co[3] = r / a.L[2];
  }
  const int stride[4] = {1, a.L[0], a.L[0] * a.L[1], a.L[0] * a.L[1] * a.L[2]};
  Spinor<double2> self, p, pu, pd;
  load_masked(p, in, V5, i5, a.chi);
  const long long base = (long long)x4 * Ls;
  const int sp1 = (s == Ls - 1) ? 0 : s + 1, sm1 = (s == 0) ? Ls - 1 : s - 1;
  const double cup = (s == Ls - 1) ? a.mf : -1.0, cdn = (s == 0) ? a.mf : -1.0;
  load_masked(pu, in, V5, base + sp1, a.chi);
  load_masked(pd, in, V5, base + sm1, a.chi);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double2 r = cscale(p.v[sp][c], a.diag);
      if (sp >= 2) r = cadd(r, cscale(pu.v[sp][c], cup));  // D: P_- couples to s+1
      else r = cadd(r, cscale(pd.v[sp][c], cdn));          //    P_+ couples to s-1
      self.v[sp][c] = r;
    }
  split_dir<0>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<1>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<2>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<3>(self, out, in, gauge, a, i5, x4, s, co, stride);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) out[(sp * 3 + c) * V5 + i5] = self.v[sp][c];
}

}  // namespace

int dslash_nblocks(const Geometry& g) { return ceil_div(g.V5, 256); }

template <class C2>
void dslash_ex(const C2* in, C2* out, const C2* b, const C2* gauge, const Geometry& g, double M5,
               double mf, bool dagger, int mode, int nrhs, double* partial, hipStream_t st) {
  DslashArgs a;
  for (int m = 0; m < 4; ++m) { a.L[m] = g.L[m]; a.ph[m] = (float)g.bc[m]; }
  a.Ls = g.Ls; a.V4 = g.V4; a.V5 = g.V5; a.diag = 5.0 - M5; a.mf = mf;
  dim3 grid(dslash_nblocks(g), nrhs), blk(256);
#define MG_DS(DAG, MODE) \
  hipLaunchKernelGGL((k_dslash<C2, DAG, MODE>), grid, blk, 0, st, in, out, b, gauge, a, partial)
  if (!dagger && mode == 0) MG_DS(false, 0);
  else if (!dagger && mode == 1) MG_DS(false, 1);
  else if (dagger && mode == 0) MG_DS(true, 0);
  else MG_DS(true, 1);
#undef MG_DS
  MG_LAUNCH_CHECK();
}

template <class C2>
void dslash(const C2* in, C2* out, const C2* b, const C2* gauge, const Geometry& g, double M5,
            double mf, bool dagger, int mode, int nrhs, hipStream_t st) {
  dslash_ex<C2>(in, out, b, gauge, g, M5, mf, dagger, mode, nrhs, nullptr, st);
}

void dslash_split(const double2* in, double2* out9, const double2* gauge, const Geometry& g, const int block[4],
                  double M5, double mf, int chi, hipStream_t st) {
  SplitArgs a;
  for (int m = 0; m < 4; ++m) { a.L[m] = g.L[m]; a.b[m] = block[m]; a.ph[m] = (float)g.bc[m]; }
  a.Ls = g.Ls; a.V4 = g.V4; a.V5 = g.V5; a.diag = 5.0 - M5; a.mf = mf; a.chi = chi;
  hipLaunchKernelGGL(k_dslash_split, dim3(ceil_div(g.V5, 256)), dim3(256), 0, st, in, out9, gauge, a);
  MG_LAUNCH_CHECK();
}

template void dslash<double2>(const double2*, double2*, const double2*, const double2*, const Geometry&,
                              double, double, bool, int, int, hipStream_t);
template void dslash<float2>(const float2*, float2*, const float2*, const float2*, const Geometry&,
                             double, double, bool, int, int, hipStream_t);
template void dslash_ex<double2>(const double2*, double2*, const double2*, const double2*,
                                 const Geometry&, double, double, bool, int, int, double*, hipStream_t);
template void dslash_ex<float2>(const float2*, float2*, const float2*, const float2*, const Geometry&,
                                double, double, bool, int, int, double*, hipStream_t);

}  // namespace mgdwf
