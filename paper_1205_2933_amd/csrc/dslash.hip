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

// Face-split operator for the coarse-operator builds (FP64): the nine pieces
// of D (or of D^+ with DAG) applied to P_chi psi (the chirality-chi spins of
// psi; all spins when chi < 0):
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
      if (chi >= 0 && (sp >> 1) != chi) p.v[sp][c] = make_double2(0.0, 0.0);
}

template <int MU, bool DAG>
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
    constexpr int EF = DAG ? 1 : -1, EB = DAG ? -1 : 1;
    if (dir == 0) {  // -1/2 (1 -+ g_mu) U_mu(x) psi(x + mu)
      load_masked(p, in, V5, (long long)xf * a.Ls + s, a.chi);
      project<MU, EF>(p, h);
      transport<false>(gauge, MU, V4, x4, h, u);
      accumulate<MU, EF>(f, u);
    } else {         // -1/2 (1 +- g_mu) U_mu(x - mu)^+ psi(x - mu)
      load_masked(p, in, V5, (long long)xb * a.Ls + s, a.chi);
      project<MU, EB>(p, h);
      transport<true>(gauge, MU, V4, xb, h, u);
      accumulate<MU, EB>(f, u);
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

template <bool DAG>
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
      // D: P_- couples to s+1 and P_+ to s-1; D^+ the other way round
      if ((sp >= 2) != DAG) r = cadd(r, cscale(pu.v[sp][c], cup));
      else r = cadd(r, cscale(pd.v[sp][c], cdn));
      self.v[sp][c] = r;
    }
  split_dir<0, DAG>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<1, DAG>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<2, DAG>(self, out, in, gauge, a, i5, x4, s, co, stride);
  split_dir<3, DAG>(self, out, in, gauge, a, i5, x4, s, co, stride);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) out[(sp * 3 + c) * V5 + i5] = self.v[sp][c];
}

// ---------------------------------------------------------------- t-march kernel
// Same operator, organised for reuse in the cache hierarchy.  A workgroup owns
// a 4 x 2 x 2 tile of (x, y, z) sites times all Ls and walks a chunk of
// t-slices.  The backward t-hop of slice t, (1 +- g_t) U_t(x, t-1)^+ psi(t-1),
// is the transported half spinor computed from slice t-1 in the previous step
// (kept in registers, with the link loaded once for both t-hops), so per slice
// only psi(t+1) is new to the workgroup; the x, y, z neighbours are the current
// slice, which every workgroup touches at about the same time, so they come
// from L2.  Workgroups are ordered tile-fastest then chunk, and remapped so each
// XCD takes a contiguous range (one chunk of t over a contiguous set of tiles).
constexpr int TMX = 4, TMY = 2, TMZ = 2, TMS = TMX * TMY * TMZ;

struct TMArgs {
  DslashArgs d;
  int ntx, nty, ntz;  // tiles per direction
  int tc;             // t-slices per chunk
  int fold = 0;       // 1: one-dimensional grid over (t-chunk, rhs, tile), t-chunk outermost
                      // 2: one-dimensional grid of XCD units (one t-chunk; see k_dslash_tx)
  int nrhs = 1;
  int zs = 1;         // fold 2: z-slabs per right-hand side
};

__device__ __forceinline__ double block_sum_dyn(double v) {
  __shared__ double red[16];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

template <class C2>
__device__ __forceinline__ void load_link(const C2* __restrict__ gauge, int mu, long long V4, int x4, C2 U[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) U[a][b] = gauge[(mu * 9 + a * 3 + b) * V4 + x4];
}

template <bool DAGU, class C2>
__device__ __forceinline__ void mul_link(const C2 U[3][3], const C2 h[2][3], C2 u[2][3], float ph) {
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
      u[r][a] = cscale(s, ph);
    }
}

template <class C2, bool DAG, int MODE>
__global__ __launch_bounds__(256) void k_dslash_tm(const C2* __restrict__ in, C2* __restrict__ out,
                                                    const C2* __restrict__ b, const C2* __restrict__ gauge, TMArgs ta,
                                                    double* __restrict__ partial) {
  using T = typename real_of<C2>::type;
  const DslashArgs& a = ta.d;
  const int ntiles = ta.ntx * ta.nty * ta.ntz;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = bid / ntiles, tile = bid - chunk * ntiles;
  const int tx = tile % ta.ntx, ty = (tile / ta.ntx) % ta.nty, tz = tile / (ta.ntx * ta.nty);
  const int Ls = a.Ls;
  const int site = threadIdx.x / Ls, s = threadIdx.x - site * Ls;
  const int x = tx * TMX + (site & 3), y = ty * TMY + ((site >> 2) & 1), z = tz * TMZ + (site >> 3);
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const long long roff = (long long)blockIdx.y * 12 * V5;
  in += roff;
  out += roff;
  if (MODE == 1) b += roff;
  const int x3 = (z * Ly + y) * Lx + x;
  // x, y, z neighbours inside a slice, with boundary phases
  int nf3[3], nb3[3];
  float phf[3], phb[3];
  {
    const int co[3] = {x, y, z};
    const int Lm[3] = {Lx, Ly, Lz};
    const int st[3] = {1, Lx, Lx * Ly};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool top = co[mu] == Lm[mu] - 1, bot = co[mu] == 0;
      nf3[mu] = top ? x3 - (Lm[mu] - 1) * st[mu] : x3 + st[mu];
      nb3[mu] = bot ? x3 + (Lm[mu] - 1) * st[mu] : x3 - st[mu];
      phf[mu] = top ? a.ph[mu] : 1.0f;
      phb[mu] = bot ? a.ph[mu] : 1.0f;
    }
  }
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const int t0 = chunk * ta.tc;
  const int t1 = min(t0 + ta.tc, Lt);
  C2 h[2][3], hb[2][3], U[3][3];
  Spinor<C2> p;
  {  // backward t-hop of the first slice, from slice t0 - 1
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    const int x4m = tm * V3 + x3;
    load_spinor(p, in, V5, (long long)x4m * Ls + s);
    project<3, EB>(p, h);
    load_link(gauge, 3, V4, x4m, U);
    mul_link<true>(U, h, hb, t0 == 0 ? a.ph[3] : 1.0f);
  }
  const int up0 = DAG ? 0 : 2;
  const int dn0 = DAG ? 2 : 0;
  const T half = (T)-0.5;
  const T dg = (T)a.diag;
  double nrm = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int x4 = t * V3 + x3;
    const long long i5 = (long long)x4 * Ls + s;
    Spinor<C2> acc;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sp][c] = cmk<C2>(0, 0);
    const int tb = t * V3;
    hop_dir<0, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, tb + nf3[0], tb + nb3[0], phf[0], phb[0]);
    hop_dir<1, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, tb + nf3[1], tb + nb3[1], phf[1], phb[1]);
    hop_dir<2, EF, EB>(acc, in, gauge, V5, V4, Ls, s, x4, tb + nf3[2], tb + nb3[2], phf[2], phb[2]);
    // forward t-hop: U_t(x, t) psi(x, t+1)
    const bool top = t == Lt - 1;
    const int x4f = (top ? 0 : t + 1) * V3 + x3;
    load_spinor(p, in, V5, (long long)x4f * Ls + s);
    project<3, EF>(p, h);
    load_link(gauge, 3, V4, x4, U);
    {
      C2 u[2][3];
      mul_link<false>(U, h, u, top ? a.ph[3] : 1.0f);
      accumulate<3, EF>(acc, u);
    }
    accumulate<3, EB>(acc, hb);
    // this slice's own spinor: diagonal, fifth-dimension hop, and the next backward t-hop
    load_spinor(p, in, V5, i5);
    const long long base = (long long)x4 * Ls;
    const int sp1 = (s == Ls - 1) ? 0 : s + 1;
    const int sm1 = (s == 0) ? Ls - 1 : s - 1;
    const T cup = (s == Ls - 1) ? (T)a.mf : (T)-1;
    const T cdn = (s == 0) ? (T)a.mf : (T)-1;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long cc = (long long)(sp * 3 + c) * V5;
        C2 r = cadd(cscale(p.v[sp][c], dg), cscale(acc.v[sp][c], half));
        if (sp == up0 || sp == up0 + 1) r = cadd(r, cscale(in[cc + base + sp1], cup));
        if (sp == dn0 || sp == dn0 + 1) r = cadd(r, cscale(in[cc + base + sm1], cdn));
        if (MODE == 1) r = csub(b[cc + i5], r);
        out[cc + i5] = r;
        nrm += (double)r.x * r.x + (double)r.y * r.y;
      }
    project<3, EB>(p, h);
    mul_link<true>(U, h, hb, 1.0f);  // slice t+1 never crosses the boundary inside a chunk
  }
  if (partial) {
    const double sum = block_sum_dyn(nrm);
    if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
}

// ---------------------------------------------------------------- t-march, s-pairs (FP32)
// Each thread computes the two sites (x4, 2j) and (x4, 2j+1): one 16-byte load
// brings both s-values of a spin-colour component (they are adjacent in the
// layout), and every link is loaded once for both outputs.  A workgroup owns a
// 4 x 4 x 2 tile of (x, y, z) sites; the t-march is as in k_dslash_tm.
constexpr int TPX = 4, TPY = 4, TPZ = 2, TPS = TPX * TPY * TPZ;

__device__ __forceinline__ void load_pair(Spinor<float2>& p0, Spinor<float2>& p1, const float2* __restrict__ f,
                                          long long stride, long long i5) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4 v = *reinterpret_cast<const float4*>(f + (sp * 3 + c) * stride + i5);
      p0.v[sp][c] = make_float2(v.x, v.y);
      p1.v[sp][c] = make_float2(v.z, v.w);
    }
}

template <int MU, int EPS, bool DAGU>
__device__ __forceinline__ void hop_pair(Spinor<float2>& a0, Spinor<float2>& a1, const float2* __restrict__ in,
                                         const float2* __restrict__ gauge, long long V5, long long V4, long long j5,
                                         int xlink, float ph) {
  Spinor<float2> p0, p1;
  float2 U[3][3], h[2][3], u[2][3];
  load_pair(p0, p1, in, V5, j5);
  load_link(gauge, MU, V4, xlink, U);
  project<MU, EPS>(p0, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a0, u);
  project<MU, EPS>(p1, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a1, u);
}

template <bool DAG, int MODE>
__global__ __launch_bounds__(256) void k_dslash_tp(const float2* __restrict__ in, float2* __restrict__ out,
                                                   const float2* __restrict__ b, const float2* __restrict__ gauge,
                                                   TMArgs ta, double* __restrict__ partial) {
  const DslashArgs& a = ta.d;
  const int ntiles = ta.ntx * ta.nty * ta.ntz;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = bid / ntiles, tile = bid - chunk * ntiles;
  const int tx = tile % ta.ntx, ty = (tile / ta.ntx) % ta.nty, tz = tile / (ta.ntx * ta.nty);
  const int Ls = a.Ls, np = Ls >> 1;
  const int site = threadIdx.x / np, jp = threadIdx.x - site * np;
  const int s0 = 2 * jp;  // this thread's sites: s0 and s0 + 1
  const int x = tx * TPX + (site & 3), y = ty * TPY + ((site >> 2) & 3), z = tz * TPZ + (site >> 4);
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const long long roff = (long long)blockIdx.y * 12 * V5;
  in += roff;
  out += roff;
  if (MODE == 1) b += roff;
  const int x3 = (z * Ly + y) * Lx + x;
  int nf3[3], nb3[3];
  float phf[3], phb[3];
  {
    const int co[3] = {x, y, z};
    const int Lm[3] = {Lx, Ly, Lz};
    const int st[3] = {1, Lx, Lx * Ly};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool top = co[mu] == Lm[mu] - 1, bot = co[mu] == 0;
      nf3[mu] = top ? x3 - (Lm[mu] - 1) * st[mu] : x3 + st[mu];
      nb3[mu] = bot ? x3 + (Lm[mu] - 1) * st[mu] : x3 - st[mu];
      phf[mu] = top ? a.ph[mu] : 1.0f;
      phb[mu] = bot ? a.ph[mu] : 1.0f;
    }
  }
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const int t0 = chunk * ta.tc;
  const int t1 = min(t0 + ta.tc, Lt);
  float2 hb0[2][3], hb1[2][3], U[3][3], h[2][3];
  Spinor<float2> p0, p1;
  {
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    const int x4m = tm * V3 + x3;
    load_pair(p0, p1, in, V5, (long long)x4m * Ls + s0);
    load_link(gauge, 3, V4, x4m, U);
    const float ph = t0 == 0 ? a.ph[3] : 1.0f;
    project<3, EB>(p0, h);
    mul_link<true>(U, h, hb0, ph);
    project<3, EB>(p1, h);
    mul_link<true>(U, h, hb1, ph);
  }
  const int up0 = DAG ? 0 : 2;   // spins coupled to s+1
  const int dn0 = DAG ? 2 : 0;   // spins coupled to s-1
  const float dg = (float)a.diag, mf = (float)a.mf;
  double nrm = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int x4 = t * V3 + x3;
    const long long i5 = (long long)x4 * Ls + s0;
    const int tb = t * V3;
    Spinor<float2> a0, a1;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) { a0.v[sp][c] = make_float2(0.f, 0.f); a1.v[sp][c] = make_float2(0.f, 0.f); }
    hop_pair<0, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[0]) * Ls + s0, x4, phf[0]);
    hop_pair<0, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[0]) * Ls + s0, tb + nb3[0], phb[0]);
    hop_pair<1, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[1]) * Ls + s0, x4, phf[1]);
    hop_pair<1, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[1]) * Ls + s0, tb + nb3[1], phb[1]);
    hop_pair<2, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[2]) * Ls + s0, x4, phf[2]);
    hop_pair<2, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[2]) * Ls + s0, tb + nb3[2], phb[2]);
    {  // forward t-hop, then the carried backward t-hop
      const bool top = t == Lt - 1;
      const int x4f = (top ? 0 : t + 1) * V3 + x3;
      load_pair(p0, p1, in, V5, (long long)x4f * Ls + s0);
      load_link(gauge, 3, V4, x4, U);
      const float ph = top ? a.ph[3] : 1.0f;
      float2 u[2][3];
      project<3, EF>(p0, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a0, u);
      project<3, EF>(p1, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a1, u);
      accumulate<3, EB>(a0, hb0);
      accumulate<3, EB>(a1, hb1);
    }
    load_pair(p0, p1, in, V5, i5);  // psi(x4, s0), psi(x4, s0 + 1)
    // neighbours in s outside the pair: s0 - 1 (for s0) and s0 + 2 (for s0 + 1)
    const long long base = (long long)x4 * Ls;
    const int sm = s0 == 0 ? Ls - 1 : s0 - 1;
    const int sp2 = s0 + 2 == Ls ? 0 : s0 + 2;
    const float cdn0 = s0 == 0 ? mf : -1.f;          // s0 - 1 across the wall
    const float cup1 = s0 + 2 == Ls ? mf : -1.f;     // s0 + 2 across the wall
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long cc = (long long)(sp * 3 + c) * V5;
        float2 r0 = cadd(cscale(p0.v[sp][c], dg), cscale(a0.v[sp][c], -0.5f));
        float2 r1 = cadd(cscale(p1.v[sp][c], dg), cscale(a1.v[sp][c], -0.5f));
        if (sp == up0 || sp == up0 + 1) {
          r0 = csub(r0, p1.v[sp][c]);                               // s0 <- s0 + 1 (inside the pair)
          r1 = cadd(r1, cscale(in[cc + base + sp2], cup1));         // s0 + 1 <- s0 + 2
        }
        if (sp == dn0 || sp == dn0 + 1) {
          r0 = cadd(r0, cscale(in[cc + base + sm], cdn0));          // s0 <- s0 - 1
          r1 = csub(r1, p0.v[sp][c]);                               // s0 + 1 <- s0
        }
        if (MODE == 1) {
          const float4 bb = *reinterpret_cast<const float4*>(b + cc + i5);
          r0 = make_float2(bb.x - r0.x, bb.y - r0.y);
          r1 = make_float2(bb.z - r1.x, bb.w - r1.y);
        }
        *reinterpret_cast<float4*>(out + cc + i5) = make_float4(r0.x, r0.y, r1.x, r1.y);
        nrm += (double)r0.x * r0.x + (double)r0.y * r0.y + (double)r1.x * r1.x + (double)r1.y * r1.y;
      }
    project<3, EB>(p0, h);
    mul_link<true>(U, h, hb0, 1.0f);
    project<3, EB>(p1, h);
    mul_link<true>(U, h, hb1, 1.0f);
  }
  if (partial) {
    const double sum = block_sum_dyn(nrm);
    if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
}

// hop_pair with the link read from LDS: entry (a, b) at Ul[(a * 3 + b) * stride]
template <int MU, int EPS, bool DAGU>
__device__ __forceinline__ void hop_pair_l(Spinor<float2>& a0, Spinor<float2>& a1, const float2* __restrict__ in,
                                           long long V5, long long j5, const float2* Ul, int stride, float ph) {
  Spinor<float2> p0, p1;
  float2 U[3][3], h[2][3], u[2][3];
  load_pair(p0, p1, in, V5, j5);
#pragma unroll
  for (int q = 0; q < 9; ++q) U[q / 3][q % 3] = Ul[q * stride];
  project<MU, EPS>(p0, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a0, u);
  project<MU, EPS>(p1, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a1, u);
}

// ---------------------------------------------------------------- t-march, carried own slice (FP32)
// As k_dslash_tp, with the spinor of slice t+1 loaded once: the forward
// t-hop of slice t uses it, and in the same registers it gives slice t+1's
// diagonal and fifth-dimension terms and the half spinor of slice t+2's
// backward t-hop.  Seven spinor loads per step instead of eight.  The tile
// (TX x TY x TZ sites of x, y, z) is a template parameter so several shapes
// can be timed on the device.
//
// acc holds -2 x (the own terms) plus the hop sum, so out = -acc / 2 exactly
// as D = (own terms) - 1/2 (hops).
__device__ __forceinline__ void own_pair(Spinor<float2>& a0, Spinor<float2>& a1, const Spinor<float2>& p0,
                                         const Spinor<float2>& p1, const float2* __restrict__ in, long long V5,
                                         long long base, int s0, int Ls, float dg, float mf, int up0, int dn0) {
  const int sm = s0 == 0 ? Ls - 1 : s0 - 1;
  const int sp2 = s0 + 2 == Ls ? 0 : s0 + 2;
  const float cdn0 = s0 == 0 ? mf : -1.f;       // s0 - 1 across the wall
  const float cup1 = s0 + 2 == Ls ? mf : -1.f;  // s0 + 2 across the wall
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long cc = (long long)(sp * 3 + c) * V5 + base;
      float2 r0 = cscale(p0.v[sp][c], dg), r1 = cscale(p1.v[sp][c], dg);
      if (sp == up0 || sp == up0 + 1) {
        r0 = csub(r0, p1.v[sp][c]);                     // s0 <- s0 + 1
        r1 = cadd(r1, cscale(in[cc + sp2], cup1));      // s0 + 1 <- s0 + 2
      }
      if (sp == dn0 || sp == dn0 + 1) {
        r0 = cadd(r0, cscale(in[cc + sm], cdn0));       // s0 <- s0 - 1
        r1 = csub(r1, p0.v[sp][c]);                     // s0 + 1 <- s0
      }
      a0.v[sp][c] = cscale(r0, -2.f);
      a1.v[sp][c] = cscale(r1, -2.f);
    }
}

template <bool DAG, int MODE, int TX, int TY, int TZ, int PAD, bool LL>
__global__ __launch_bounds__(TX * TY * TZ * 8, PAD > 0 ? 1 : 2) void k_dslash_tq(const float2* __restrict__ in,
                                                               float2* __restrict__ out,
                                                               const float2* __restrict__ b,
                                                               const float2* __restrict__ gauge, TMArgs ta,
                                                               double* __restrict__ partial) {
  if (PAD > 0) {  // LDS reserved only to cap workgroups per CU (one per CU when PAD > 80 KB)
    __shared__ float pad[PAD > 0 ? PAD / 4 : 1];
    if (ta.d.Ls < 0) pad[threadIdx.x] = 0.f;  // never true: keeps the allocation
    if (ta.d.Ls < 0) out[threadIdx.x].x = pad[threadIdx.x ^ 1];
  }
  const DslashArgs& a = ta.d;
  const int ntiles = ta.ntx * ta.nty * ta.ntz;
  // fold 0: grid (chunks x tiles, rhs), chunk-major per rhs.  fold 1: the
  // rhs folds into x with the t-chunk outermost, so the contiguous range of
  // workgroups each XCD receives covers whole t-chunks of every rhs.
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int chunk, tile, rhs, pidx;
  if (ta.fold) {
    const int per_chunk = ta.nrhs * ntiles;
    chunk = bid / per_chunk;
    const int r2 = bid - chunk * per_chunk;
    rhs = r2 / ntiles;
    tile = r2 - rhs * ntiles;
    pidx = rhs * (gridDim.x / ta.nrhs) + chunk * ntiles + tile;
  } else {
    chunk = bid / ntiles;
    tile = bid - chunk * ntiles;
    rhs = blockIdx.y;
    pidx = blockIdx.y * gridDim.x + blockIdx.x;
  }
  const int tx = tile % ta.ntx, ty = (tile / ta.ntx) % ta.nty, tz = tile / (ta.ntx * ta.nty);
  const int Ls = a.Ls, np = Ls >> 1;
  const int site = threadIdx.x / np, jp = threadIdx.x - site * np;
  const int s0 = 2 * jp;
  const int x = tx * TX + site % TX, y = ty * TY + (site / TX) % TY, z = tz * TZ + site / (TX * TY);
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const long long roff = (long long)rhs * 12 * V5;
  in += roff;
  out += roff;
  if (MODE == 1) b += roff;
  const int x3 = (z * Ly + y) * Lx + x;
  int nf3[3], nb3[3];
  float phf[3], phb[3];
  {
    const int co[3] = {x, y, z};
    const int Lm[3] = {Lx, Ly, Lz};
    const int st[3] = {1, Lx, Lx * Ly};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool top = co[mu] == Lm[mu] - 1, bot = co[mu] == 0;
      nf3[mu] = top ? x3 - (Lm[mu] - 1) * st[mu] : x3 + st[mu];
      nb3[mu] = bot ? x3 + (Lm[mu] - 1) * st[mu] : x3 - st[mu];
      phf[mu] = top ? a.ph[mu] : 1.0f;
      phb[mu] = bot ? a.ph[mu] : 1.0f;
    }
  }
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const int up0 = DAG ? 0 : 2;   // spins coupled to s+1
  const int dn0 = DAG ? 2 : 0;   // spins coupled to s-1
  const float dg = (float)a.diag, mf = (float)a.mf;
  const int t0 = chunk * ta.tc;
  const int t1 = min(t0 + ta.tc, Lt);
  // LL: the links of the slice are staged in LDS once per step -- U_mu(x) of
  // the tile's sites for mu = x, y, z, t, and U_mu(x - mu) on the three minus
  // faces -- instead of every s-pair thread loading its seven links.
  constexpr int NS = TX * TY * TZ;
  constexpr int NF0 = TY * TZ, NF1 = TX * TZ, NF2 = TX * TY;
  constexpr int NL = LL ? 36 * NS + 9 * (NF0 + NF1 + NF2) : 1;
  __shared__ float2 sU[NL];
  int lf[3], lb[3], sb[3];  // LDS offsets of the forward / backward links, backward strides
  {
    const int lc[3] = {site % TX, (site / TX) % TY, site / (TX * TY)};
    const int ts[3] = {1, TX, TX * TY};
    const int fo[3] = {36 * NS, 36 * NS + 9 * NF0, 36 * NS + 9 * (NF0 + NF1)};
    const int fi[3] = {lc[1] + TY * lc[2], lc[0] + TX * lc[2], lc[0] + TX * lc[1]};
    const int nfc[3] = {NF0, NF1, NF2};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      lf[mu] = mu * 9 * NS + site;
      if (lc[mu] > 0) { lb[mu] = mu * 9 * NS + site - ts[mu]; sb[mu] = NS; }
      else { lb[mu] = fo[mu] + fi[mu]; sb[mu] = nfc[mu]; }
    }
  }
  float2 hp0[2][3], hp1[2][3], U[3][3], h[2][3], u[2][3];
  Spinor<float2> p0, p1, a0, a1;
  {  // slice t0: own terms, and the backward t-hop from slice t0 - 1
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    const int x4m = tm * V3 + x3;
    load_pair(p0, p1, in, V5, (long long)x4m * Ls + s0);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    const long long base = (long long)(t0 * V3 + x3) * Ls;
    load_pair(p0, p1, in, V5, base + s0);
    own_pair(a0, a1, p0, p1, in, V5, base, s0, Ls, dg, mf, up0, dn0);
    load_link(gauge, 3, V4, x4m, U);
    const float ph = t0 == 0 ? a.ph[3] : 1.0f;
    mul_link<true>(U, hp0, u, ph);
    accumulate<3, EB>(a0, u);
    mul_link<true>(U, hp1, u, ph);
    accumulate<3, EB>(a1, u);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
  }
  float nrmf = 0.f;  // per-thread |out|^2 in FP32 (a few hundred terms), FP64 across the workgroup
  for (int t = t0; t < t1; ++t) {
    const int x4 = t * V3 + x3;
    const int tb = t * V3;
    if (LL) {
      __syncthreads();  // every thread is done with the previous slice's links
      const int bx = tx * TX, by = ty * TY, bz = tz * TZ;
      for (int i = threadIdx.x; i < 36 * NS; i += blockDim.x) {  // own sites, mu = x, y, z, t
        const int mab = i / NS, q = i - mab * NS;
        const int xx = bx + q % TX, yy = by + (q / TX) % TY, zz = bz + q / (TX * TY);
        sU[i] = gauge[(long long)mab * V4 + tb + (zz * Ly + yy) * Lx + xx];
      }
      for (int i = threadIdx.x; i < 9 * (NF0 + NF1 + NF2); i += blockDim.x) {  // minus faces
        int mu, r;
        if (i < 9 * NF0) { mu = 0; r = i; }
        else if (i < 9 * (NF0 + NF1)) { mu = 1; r = i - 9 * NF0; }
        else { mu = 2; r = i - 9 * (NF0 + NF1); }
        const int nf = mu == 0 ? NF0 : (mu == 1 ? NF1 : NF2);
        const int ab = r / nf, f = r - ab * nf;
        int xx, yy, zz;
        if (mu == 0) { xx = bx == 0 ? Lx - 1 : bx - 1; yy = by + f % TY; zz = bz + f / TY; }
        else if (mu == 1) { xx = bx + f % TX; yy = by == 0 ? Ly - 1 : by - 1; zz = bz + f / TX; }
        else { xx = bx + f % TX; yy = by + f / TX; zz = bz == 0 ? Lz - 1 : bz - 1; }
        sU[36 * NS + (mu == 0 ? 0 : (mu == 1 ? 9 * NF0 : 9 * (NF0 + NF1))) + r] =
            gauge[(long long)(mu * 9 + ab) * V4 + tb + (zz * Ly + yy) * Lx + xx];
      }
      __syncthreads();
      hop_pair_l<0, EF, false>(a0, a1, in, V5, (long long)(tb + nf3[0]) * Ls + s0, sU + lf[0], NS, phf[0]);
      hop_pair_l<0, EB, true>(a0, a1, in, V5, (long long)(tb + nb3[0]) * Ls + s0, sU + lb[0], sb[0], phb[0]);
      hop_pair_l<1, EF, false>(a0, a1, in, V5, (long long)(tb + nf3[1]) * Ls + s0, sU + lf[1], NS, phf[1]);
      hop_pair_l<1, EB, true>(a0, a1, in, V5, (long long)(tb + nb3[1]) * Ls + s0, sU + lb[1], sb[1], phb[1]);
      hop_pair_l<2, EF, false>(a0, a1, in, V5, (long long)(tb + nf3[2]) * Ls + s0, sU + lf[2], NS, phf[2]);
      hop_pair_l<2, EB, true>(a0, a1, in, V5, (long long)(tb + nb3[2]) * Ls + s0, sU + lb[2], sb[2], phb[2]);
    } else {
      hop_pair<0, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[0]) * Ls + s0, x4, phf[0]);
      hop_pair<0, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[0]) * Ls + s0, tb + nb3[0], phb[0]);
      hop_pair<1, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[1]) * Ls + s0, x4, phf[1]);
      hop_pair<1, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[1]) * Ls + s0, tb + nb3[1], phb[1]);
      hop_pair<2, EF, false>(a0, a1, in, gauge, V5, V4, (long long)(tb + nf3[2]) * Ls + s0, x4, phf[2]);
      hop_pair<2, EB, true>(a0, a1, in, gauge, V5, V4, (long long)(tb + nb3[2]) * Ls + s0, tb + nb3[2], phb[2]);
    }
    // forward t-hop with slice t+1
    const bool top = t == Lt - 1;
    const long long basef = (long long)((top ? 0 : t + 1) * V3 + x3) * Ls;
    load_pair(p0, p1, in, V5, basef + s0);
    if (LL) {
#pragma unroll
      for (int q = 0; q < 9; ++q) U[q / 3][q % 3] = sU[(27 + q) * NS + site];
    } else {
      load_link(gauge, 3, V4, x4, U);
    }
    {
      const float ph = top ? a.ph[3] : 1.0f;
      project<3, EF>(p0, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a0, u);
      project<3, EF>(p1, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a1, u);
    }
    const long long i5 = (long long)x4 * Ls + s0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long cc = (long long)(sp * 3 + c) * V5;
        float2 r0 = cscale(a0.v[sp][c], -0.5f), r1 = cscale(a1.v[sp][c], -0.5f);
        if (MODE == 1) {
          const float4 bb = *reinterpret_cast<const float4*>(b + cc + i5);
          r0 = make_float2(bb.x - r0.x, bb.y - r0.y);
          r1 = make_float2(bb.z - r1.x, bb.w - r1.y);
        }
        *reinterpret_cast<float4*>(out + cc + i5) = make_float4(r0.x, r0.y, r1.x, r1.y);
        if (partial) nrmf += r0.x * r0.x + r0.y * r0.y + r1.x * r1.x + r1.y * r1.y;
      }
    if (t + 1 < t1) {  // slice t+1: own terms, backward t-hop from slice t (never across the boundary here)
      own_pair(a0, a1, p0, p1, in, V5, basef, s0, Ls, dg, mf, up0, dn0);
      mul_link<true>(U, hp0, u, 1.0f);
      accumulate<3, EB>(a0, u);
      mul_link<true>(U, hp1, u, 1.0f);
      accumulate<3, EB>(a1, u);
      project<3, EB>(p0, hp0);
      project<3, EB>(p1, hp1);
    }
  }
  if (partial) {
    const double sum = block_sum_dyn((double)nrmf);
    if (threadIdx.x == 0) partial[pidx] = sum;
  }
}

// ---------------------------------------------------------------- one wavefront per site pair (FP32)
// k_dslash_tq spends more vector-memory instructions on links than on
// spinors: each of its lanes loads every link entry itself (63 of about 170
// loads per wavefront step), and it loads the s - 1 and s + 2 neighbours of
// its s-pair again.  Here a wavefront holds only two 4D sites, A = (x, y, z, t)
// with x even and B = A + x, for R = 32 / P right-hand sides and all
// Ls = 2 P fifth-dimension sites: lane = half * 32 + r * P + j holds s = 2j
// and 2j + 1 of right-hand side r at A (half 0) or B (half 1).  Each half
// then shares one link, which one load instruction fetches for both halves
// (lanes 0..8 and 32..40, one complex entry each) and the LDS crossbar
// (ds_bpermute) hands to the other lanes; the s - 1 and s + 2 neighbours are
// the neighbouring lanes' registers.  Per wavefront step that leaves the 84
// spinor loads (six spatial neighbours and slice t + 1, 16 bytes a lane), 8
// link loads and 12 stores.  The t-march, the carried slice t + 1 and the
// carried backward t-hop are those of k_dslash_tq.  Workgroups are four
// wavefronts; the wavefront items are ordered in bricks of BX x BY x BZ
// (x pairs, y, z) so that the wavefronts one XCD runs at a time share their
// neighbours in its L2.
struct WSArgs {
  DslashArgs d;
  int nxp;      // Lx / 2 site pairs
  int ngrp;     // groups of R right-hand sides
  int nchunk;   // t chunks
  int tc;       // t-slices per chunk
  int nrhs;
  int bx, by, bz;  // brick of wavefront items: x pairs, y, z
};

// The link U_mu at site x4a for half 0 and x4b for half 1, in every lane of
// its half: one load instruction, nine crossbar reads of each real part.
__device__ __forceinline__ void link_pair(const float2* __restrict__ gs, int x4a, int x4b, int mu, int lane,
                                          float2 U[3][3]) {
  const int q = min(lane & 31, 8);  // lanes past the ninth repeat it: one load instruction, no branch
  const int x4 = (lane & 32) ? x4b : x4a;
  const float2 v = gs[((long long)x4 * 4 + mu) * 9 + q];
  const int src = (lane & 32) << 2;  // byte address of lane 0 of this half
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    U[e / 3][e % 3].x = __int_as_float(__builtin_amdgcn_ds_bpermute(src + 4 * e, __float_as_int(v.x)));
    U[e / 3][e % 3].y = __int_as_float(__builtin_amdgcn_ds_bpermute(src + 4 * e, __float_as_int(v.y)));
  }
}

__device__ __forceinline__ float2 lane_read(int addr, float2 v) {
  return make_float2(__int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v.x))),
                     __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v.y))));
}

// Spinor pair loads and stores addressed as a wavefront-uniform base (one
// per spin-colour component, in scalar registers) plus a 32-bit per-lane
// byte offset, so no 64-bit per-lane address is formed or kept per component.
// The component base is made opaque to the optimiser in a scalar register,
// so the address stays (scalar base) + (32-bit lane offset) instead of being
// re-associated into one 64-bit per-lane address per component.
typedef const char __attribute__((address_space(1)))* gbase_t;  // global memory
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef const nf4 __attribute__((address_space(1)))* gf4_t;
typedef nf4 __attribute__((address_space(1)))* gf4w_t;

__device__ __forceinline__ gbase_t sbase(const char* base, long long cs, int k) {
  gbase_t b = (gbase_t)(base + k * cs);
  asm volatile("" : "+s"(b));
  return b;
}

__device__ __forceinline__ void load_pair_o(Spinor<float2>& p0, Spinor<float2>& p1, const char* base, long long cs,
                                            unsigned off) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const nf4 v = *(gf4_t)(sbase(base, cs, sp * 3 + c) + off);
      p0.v[sp][c] = make_float2(v.x, v.y);
      p1.v[sp][c] = make_float2(v.z, v.w);
    }
}

template <int MU, int EPS, bool DAGU>
__device__ __forceinline__ void hop_pair_u(Spinor<float2>& a0, Spinor<float2>& a1, const char* base, long long cs,
                                           unsigned off, const float2 U[3][3], float ph) {
  Spinor<float2> p0, p1;
  float2 h[2][3], u[2][3];
  load_pair_o(p0, p1, base, cs, off);
  project<MU, EPS>(p0, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a0, u);
  project<MU, EPS>(p1, h);
  mul_link<DAGU>(U, h, u, ph);
  accumulate<MU, EPS>(a1, u);
}

// own_pair with the s0 - 1 and s0 + 2 values read from the lanes that hold
// them (addresses up_addr, dn_addr) instead of from memory; UP0 / DN0 are
// the first of the two spins coupled to s + 1 / s - 1
template <int UP0, int DN0>
__device__ __forceinline__ void own_pair_x(Spinor<float2>& a0, Spinor<float2>& a1, const Spinor<float2>& p0,
                                           const Spinor<float2>& p1, int up_addr, int dn_addr, float cup1,
                                           float cdn0, float dg) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 r0 = cscale(p0.v[sp][c], dg), r1 = cscale(p1.v[sp][c], dg);
      if (sp == UP0 || sp == UP0 + 1) {
        const float2 nup = lane_read(up_addr, p0.v[sp][c]);  // s0 + 2 = the next lane's s0
        r0 = csub(r0, p1.v[sp][c]);          // s0 <- s0 + 1
        r1 = cadd(r1, cscale(nup, cup1));    // s0 + 1 <- s0 + 2
      }
      if (sp == DN0 || sp == DN0 + 1) {
        const float2 ndn = lane_read(dn_addr, p1.v[sp][c]);  // s0 - 1 = the previous lane's s0 + 1
        r0 = cadd(r0, cscale(ndn, cdn0));    // s0 <- s0 - 1
        r1 = csub(r1, p0.v[sp][c]);          // s0 + 1 <- s0
      }
      a0.v[sp][c] = cscale(r0, -2.f);
      a1.v[sp][c] = cscale(r1, -2.f);
    }
}

template <bool DAG, int MODE, int P>
__global__ __launch_bounds__(256, 2) void k_dslash_ws(const float2* __restrict__ in, float2* __restrict__ out,
                                                      const float2* __restrict__ b, const float2* __restrict__ gauge,
                                                      WSArgs wa, double* __restrict__ partial) {
  constexpr int R = 32 / P;
  const DslashArgs& a = wa.d;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const int Ls = a.Ls;
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const float2* __restrict__ gs = gauge + 36LL * V4;  // site-major copy
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // wavefront item -> (x pair, y, z) in bricks, right-hand-side group, t chunk;
  // one workgroup's four items share the group and the chunk
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int item = bid * 4 + wave;
  const int nsp = wa.nxp * Ly * Lz;                 // items per (group, chunk)
  const int cg = item / nsp, sp3 = item - cg * nsp;
  const int grp = cg % wa.ngrp, chunk = cg / wa.ngrp;
  const int bvol = wa.bx * wa.by * wa.bz;
  const int brick = sp3 / bvol, ib = sp3 - brick * bvol;
  const int nbx = wa.nxp / wa.bx, nby = Ly / wa.by;
  const int xp = (brick % nbx) * wa.bx + ib % wa.bx;
  const int y = ((brick / nbx) % nby) * wa.by + (ib / wa.bx) % wa.by;
  const int z = (brick / (nbx * nby)) * wa.bz + ib / (wa.bx * wa.by);
  // lane -> half (site), right-hand side, s-pair
  const int half = lane >> 5, r = (lane & 31) / P, jl = lane % P;
  const int s0 = 2 * jl;
  const int rhs = grp * R + r;
  const bool valid = rhs < wa.nrhs;
  // uniform bases (the group's first right-hand side) and per-lane byte offsets
  const long long cs = V5 * (long long)sizeof(float2);  // bytes between spin-colour components
  const long long g0 = (long long)grp * R * 12 * V5;
  const char* inb = reinterpret_cast<const char*>(in + g0);
  char* outb = reinterpret_cast<char*>(out + g0);
  const char* bb0 = MODE == 1 ? reinterpret_cast<const char*>(b + g0) : nullptr;
  const unsigned roff = (unsigned)((valid ? r : (wa.nrhs - 1 - grp * R)) * 12 * cs);
  auto lo = [&](long long j5) { return roff + (unsigned)(j5 * (long long)sizeof(float2)); };
  const int xa = 2 * xp;
  const int x = xa + half;
  const int x3a = (z * Ly + y) * Lx + xa;           // site A (wave uniform)
  const int x3 = x3a + half;
  // neighbours (per lane) and the backward-link sites (per half, wave uniform)
  const int xf = x + 1 == Lx ? 0 : x + 1, xb = x == 0 ? Lx - 1 : x - 1;
  const int yf = y + 1 == Ly ? 0 : y + 1, yb = y == 0 ? Ly - 1 : y - 1;
  const int zf = z + 1 == Lz ? 0 : z + 1, zb = z == 0 ? Lz - 1 : z - 1;
  const int nf3[3] = {(z * Ly + y) * Lx + xf, (z * Ly + yf) * Lx + x, (zf * Ly + y) * Lx + x};
  const int nb3[3] = {(z * Ly + y) * Lx + xb, (z * Ly + yb) * Lx + x, (zb * Ly + y) * Lx + x};
  const int xam = xa == 0 ? Lx - 1 : xa - 1;       // A - x; B - x is A
  const int bl3a[3] = {(z * Ly + y) * Lx + xam, (z * Ly + yb) * Lx + xa, (zb * Ly + y) * Lx + xa};
  const int bl3b[3] = {x3a, (z * Ly + yb) * Lx + xa + 1, (zb * Ly + y) * Lx + xa + 1};
  const float phf[3] = {x == Lx - 1 ? a.ph[0] : 1.0f, y == Ly - 1 ? a.ph[1] : 1.0f, z == Lz - 1 ? a.ph[2] : 1.0f};
  const float phb[3] = {x == 0 ? a.ph[0] : 1.0f, y == 0 ? a.ph[1] : 1.0f, z == 0 ? a.ph[2] : 1.0f};
  // fifth-dimension neighbours in the lanes of the same (site, rhs)
  const int lbase = lane - jl;
  const int up_addr = 4 * (lbase + (jl + 1 == P ? 0 : jl + 1));
  const int dn_addr = 4 * (lbase + (jl == 0 ? P - 1 : jl - 1));
  const float cup1 = s0 + 2 == Ls ? (float)a.mf : -1.f;  // s0 + 2 across the wall
  const float cdn0 = s0 == 0 ? (float)a.mf : -1.f;       // s0 - 1 across the wall
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const float dg = (float)a.diag;
  const int t0 = chunk * wa.tc;
  const int t1 = min(t0 + wa.tc, Lt);
  float2 hp0[2][3], hp1[2][3], U[3][3], h[2][3], u[2][3];
  Spinor<float2> p0, p1, a0, a1;
  {  // slice t0: own terms, and the backward t-hop from slice t0 - 1
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    load_pair_o(p0, p1, inb, cs, lo((long long)(tm * V3 + x3) * Ls + s0));
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    const long long base = (long long)(t0 * V3 + x3) * Ls;
    load_pair_o(p0, p1, inb, cs, lo(base + s0));
    own_pair_x<DAG ? 0 : 2, DAG ? 2 : 0>(a0, a1, p0, p1, up_addr, dn_addr, cup1, cdn0, dg);
    link_pair(gs, tm * V3 + x3a, tm * V3 + x3a + 1, 3, lane, U);
    const float ph = t0 == 0 ? a.ph[3] : 1.0f;
    mul_link<true>(U, hp0, u, ph);
    accumulate<3, EB>(a0, u);
    mul_link<true>(U, hp1, u, ph);
    accumulate<3, EB>(a1, u);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
  }
  float nrmf = 0.f;
  for (int t = t0; t < t1; ++t) {
    const int tb = t * V3;
    link_pair(gs, tb + x3a, tb + x3a + 1, 0, lane, U);
    hop_pair_u<0, EF, false>(a0, a1, inb, cs, lo((long long)(tb + nf3[0]) * Ls + s0), U, phf[0]);
    __builtin_amdgcn_sched_barrier(0);  // one hop at a time: the next hop's loads wait
    link_pair(gs, tb + bl3a[0], tb + bl3b[0], 0, lane, U);
    hop_pair_u<0, EB, true>(a0, a1, inb, cs, lo((long long)(tb + nb3[0]) * Ls + s0), U, phb[0]);
    __builtin_amdgcn_sched_barrier(0);
    link_pair(gs, tb + x3a, tb + x3a + 1, 1, lane, U);
    hop_pair_u<1, EF, false>(a0, a1, inb, cs, lo((long long)(tb + nf3[1]) * Ls + s0), U, phf[1]);
    __builtin_amdgcn_sched_barrier(0);
    link_pair(gs, tb + bl3a[1], tb + bl3b[1], 1, lane, U);
    hop_pair_u<1, EB, true>(a0, a1, inb, cs, lo((long long)(tb + nb3[1]) * Ls + s0), U, phb[1]);
    __builtin_amdgcn_sched_barrier(0);
    link_pair(gs, tb + x3a, tb + x3a + 1, 2, lane, U);
    hop_pair_u<2, EF, false>(a0, a1, inb, cs, lo((long long)(tb + nf3[2]) * Ls + s0), U, phf[2]);
    __builtin_amdgcn_sched_barrier(0);
    link_pair(gs, tb + bl3a[2], tb + bl3b[2], 2, lane, U);
    hop_pair_u<2, EB, true>(a0, a1, inb, cs, lo((long long)(tb + nb3[2]) * Ls + s0), U, phb[2]);
    __builtin_amdgcn_sched_barrier(0);
    // forward t-hop with slice t + 1
    const bool top = t == Lt - 1;
    const long long basef = (long long)((top ? 0 : t + 1) * V3 + x3) * Ls;
    load_pair_o(p0, p1, inb, cs, lo(basef + s0));
    link_pair(gs, tb + x3a, tb + x3a + 1, 3, lane, U);
    {
      const float ph = top ? a.ph[3] : 1.0f;
      project<3, EF>(p0, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a0, u);
      project<3, EF>(p1, h);
      mul_link<false>(U, h, u, ph);
      accumulate<3, EF>(a1, u);
    }
    // Lanes past the last right-hand side read that one's fields, so they
    // compute its values bit for bit and their stores repeat them: no branch
    // around the stores; they are left out of the norm.
    const unsigned o5 = lo((long long)(tb + x3) * Ls + s0);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float2 r0 = cscale(a0.v[sp][c], -0.5f), r1 = cscale(a1.v[sp][c], -0.5f);
        if (MODE == 1) {
          const nf4 bb = *(gf4_t)(sbase(bb0, cs, sp * 3 + c) + o5);
          r0 = make_float2(bb.x - r0.x, bb.y - r0.y);
          r1 = make_float2(bb.z - r1.x, bb.w - r1.y);
        }
        *(gf4w_t)(sbase(outb, cs, sp * 3 + c) + o5) = nf4{r0.x, r0.y, r1.x, r1.y};
        if (partial) nrmf += r0.x * r0.x + r0.y * r0.y + r1.x * r1.x + r1.y * r1.y;
      }
    if (t + 1 < t1) {  // slice t + 1: own terms, backward t-hop from slice t
      own_pair_x<DAG ? 0 : 2, DAG ? 2 : 0>(a0, a1, p0, p1, up_addr, dn_addr, cup1, cdn0, dg);
      mul_link<true>(U, hp0, u, 1.0f);
      accumulate<3, EB>(a0, u);
      mul_link<true>(U, hp1, u, 1.0f);
      accumulate<3, EB>(a1, u);
      project<3, EB>(p0, hp0);
      project<3, EB>(p1, hp1);
    }
  }
  if (partial) {
    // per right-hand side: the P lanes of each half, then the two halves,
    // then the four wavefronts of the workgroup (all in the same group)
    double v = valid ? (double)nrmf : 0.0;
#pragma unroll
    for (int off = 1; off < P; off <<= 1) v += __shfl_xor(v, off, 64);
    v += __shfl_xor(v, 32, 64);
    __shared__ double red[4][R];
    if (lane < 32 && jl == 0) red[wave][r] = v;
    __syncthreads();
    if ((int)threadIdx.x < R) {
      const int rr = grp * R + (int)threadIdx.x;
      if (rr < wa.nrhs) {
        const double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        // partial index: (rhs, block within the group's range of this chunk)
        const int nbs = nsp / 4;
        partial[(long long)rr * (nbs * wa.nchunk) + chunk * nbs + sp3 / 4] = s;
      }
    }
  }
}

// ---------------------------------------------------------------- t-march, spatial neighbours through LDS (FP32)
// k_dslash_tq brings every spatial neighbour, both fifth-dimension
// neighbours and every link through the vector-memory data path: per s-pair
// thread and t-slice about 1.9 KB returned to registers for 0.4 KB of
// algorithmic traffic, and that path (TD ~92 % busy) set its speed while L2
// and HBM had headroom.  Here the workgroup keeps its tile's slice t in LDS:
// each thread writes its own spinor pair there (the forward t-hop of the
// previous slice already loaded it), the slice's links are staged there once
// (each multiplied by its boundary phase, which is exact and belongs to the
// link: the forward hop of x and the backward hop of x + mu cross the same
// face), and the x, y, z neighbours inside the tile, the s - 1 and s + 2
// values of the fifth-dimension hop and all links are read from LDS.  Only
// neighbours across the tile faces and slice t + 1 are loaded from memory
// (the neighbouring tiles run on the same XCD at the same time, so the faces
// are L2 hits); those are addressed as a scalar base per component plus a
// 32-bit lane offset, as in k_dslash_ws.  With a 4 x 4 x 2 tile that is about 0.6 KB per thread and
// slice.  One LDS buffer, two barriers per slice; 60 KB per workgroup at
// 4 x 4 x 2, so two workgroups share a CU.
// LDS pointers typed as such, so a neighbour read is a ds_read and is never
// merged with the memory path of a face neighbour into one flat load
typedef float xf2 __attribute__((ext_vector_type(2)));
typedef const nf4 __attribute__((address_space(3)))* lds_f4_t;
typedef nf4 __attribute__((address_space(3)))* lds_f4w_t;
typedef const xf2 __attribute__((address_space(3)))* lds_f2_t;

__device__ __forceinline__ void lds_pair(Spinor<float2>& p0, Spinor<float2>& p1, lds_f4_t sp, int cst) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const nf4 v = sp[k * cst];
    p0.v[k / 3][k % 3] = make_float2(v.x, v.y);
    p1.v[k / 3][k % 3] = make_float2(v.z, v.w);
  }
}

template <bool DAGU>
__device__ __forceinline__ void mul_link_1(const float2 U[3][3], const float2 h[2][3], float2 u[2][3]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (DAGU) cfmac(s, U[b][a], h[r][b]);
        else cfma(s, U[a][b], h[r][b]);
      }
      u[r][a] = s;
    }
}

// Materialises the accumulators where it stands: the optimiser would
// otherwise sink every hop's arithmetic below the last hop's load branches,
// with six hops' neighbour spinors live at once (hundreds of spilled registers).
__device__ __forceinline__ void pin_acc(Spinor<float2>& a) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    float& re = a.v[k / 3][k % 3].x;
    float& im = a.v[k / 3][k % 3].y;
    asm volatile("" : "+v"(re), "+v"(im));
  }
}

// The links a tile's slice t needs, into LDS: U_mu(x) of its sites for mu =
// x, y, z, t ([mu * 9 + ab][site]) and U_mu(x - mu) on the three minus faces,
// each multiplied by the boundary phase of the face it crosses.  Entries go in
// pairs of x-neighbours (one 16-byte load; on the x face, whose pairs are
// y-neighbours, two 8-byte loads), and every thread issues its loads before
// writing any (batches of four pairs), so a slice costs one memory round trip
// rather than one per loop pass.  Needs even TX and TY (x extent even too).
template <int TX, int TY, int TZ>
__device__ __forceinline__ void stage_links(float2* sU, const float2* __restrict__ gauge, const DslashArgs& a,
                                            long long V4, int tb, int t, int bx, int by, int bz) {
  constexpr int NS = TX * TY * TZ;
  constexpr int NF0 = TY * TZ, NF1 = TX * TZ, NF2 = TX * TY;
  static_assert(TX % 2 == 0 && TY % 2 == 0, "link pairs need even TX and TY");
  constexpr int NU = (36 * NS + 9 * (NF0 + NF1 + NF2)) / 2;
  constexpr int B = 4;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  for (int base = 0; base < NU; base += B * (int)blockDim.x) {
    float2 v0[B], v1[B];
    float f0[B], f1[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int u = base + j * (int)blockDim.x + (int)threadIdx.x;
      v0[j] = v1[j] = make_float2(0.f, 0.f);
      f0[j] = f1[j] = 1.f;
      if (u < 18 * NS) {
        const int i = 2 * u, mab = i / NS, q = i - mab * NS, mu = mab / 9;
        const int xx = bx + q % TX, yy = by + (q / TX) % TY, zz = bz + q / (TX * TY);
        const float4 w = *reinterpret_cast<const float4*>(gauge + (long long)mab * V4 + tb + (zz * Ly + yy) * Lx + xx);
        v0[j] = make_float2(w.x, w.y);
        v1[j] = make_float2(w.z, w.w);
        if (mu == 0) f1[j] = xx + 1 == Lx - 1 ? a.ph[0] : 1.f;  // xx is even: only the second can be on the face
        else {
          const bool cross = mu == 1 ? yy == Ly - 1 : (mu == 2 ? zz == Lz - 1 : t == Lt - 1);
          f0[j] = f1[j] = cross ? a.ph[mu] : 1.f;
        }
      } else if (u < NU) {
        const int r0 = 2 * (u - 18 * NS);
        int mu, r;
        if (r0 < 9 * NF0) { mu = 0; r = r0; }
        else if (r0 < 9 * (NF0 + NF1)) { mu = 1; r = r0 - 9 * NF0; }
        else { mu = 2; r = r0 - 9 * (NF0 + NF1); }
        const int nf = mu == 0 ? NF0 : (mu == 1 ? NF1 : NF2);
        const int ab = r / nf, f = r - ab * nf;
        const long long cb = (long long)(mu * 9 + ab) * V4 + tb;
        bool cross;
        if (mu == 0) {
          cross = bx == 0;
          const int xx = cross ? Lx - 1 : bx - 1;
          v0[j] = gauge[cb + ((bz + f / TY) * Ly + by + f % TY) * Lx + xx];
          v1[j] = gauge[cb + ((bz + (f + 1) / TY) * Ly + by + (f + 1) % TY) * Lx + xx];
        } else {
          int xx = bx + f % TX, yy, zz;
          if (mu == 1) { cross = by == 0; yy = cross ? Ly - 1 : by - 1; zz = bz + f / TX; }
          else { cross = bz == 0; yy = by + f / TX; zz = cross ? Lz - 1 : bz - 1; }
          const float4 w = *reinterpret_cast<const float4*>(gauge + cb + (zz * Ly + yy) * Lx + xx);
          v0[j] = make_float2(w.x, w.y);
          v1[j] = make_float2(w.z, w.w);
        }
        f0[j] = f1[j] = cross ? a.ph[mu] : 1.f;
      }
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int u = base + j * (int)blockDim.x + (int)threadIdx.x;
      if (u < NU) {
        sU[2 * u] = cscale(v0[j], f0[j]);
        sU[2 * u + 1] = cscale(v1[j], f1[j]);
      }
    }
  }
}

// As stage_links, from the phase-folded link copy (gauge + 72 V4: links on
// the last slice of a direction already multiplied by its boundary phase)
// and with direct global-to-LDS copies (global_load_lds): each lane's 16 or 4
// bytes land at a wavefront-uniform LDS base + lane x size without passing
// through registers, so the copies for slice t + 1 are in flight during slice
// t's arithmetic.  The caller waits (vmcnt) before the barrier that precedes
// their use.  Own links and the y and z faces go in 16-byte x-pairs, the x
// face (pairs are y-neighbours there) in 4-byte words.
typedef __attribute__((address_space(3))) void* lds_void_t;

template <int TX, int TY, int TZ>
__device__ __forceinline__ void stage_links_async(float2* sU, const float2* __restrict__ gp, const DslashArgs& a,
                                                  long long V4, int tb, int bx, int by, int bz) {
  constexpr int NS = TX * TY * TZ;
  constexpr int NF0 = TY * TZ, NF1 = TX * TZ, NF2 = TX * TY;
  static_assert(TX % 2 == 0, "link pairs need even TX");
  constexpr int NOWN = 18 * NS;              // 16-byte units of own links
  constexpr int NYZ = 9 * (NF1 + NF2) / 2;   // 16-byte units of the y and z faces
  constexpr int NXW = 2 * 9 * NF0;           // 4-byte words of the x face
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const int lane = (int)threadIdx.x & 63;
  const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), nw = (int)blockDim.x >> 6;
  for (int g0 = w0 * 64; g0 < NOWN; g0 += nw * 64) {
    const int u = g0 + lane;
    if (u < NOWN) {
      const int i = 2 * u, mab = i / NS, q = i - mab * NS;
      const int xx = bx + q % TX, yy = by + (q / TX) % TY, zz = bz + q / (TX * TY);
      __builtin_amdgcn_global_load_lds((const void*)(gp + (long long)mab * V4 + tb + (zz * Ly + yy) * Lx + xx),
                                       (lds_void_t)(void*)(sU + 2 * g0), 16, 0, 0);
    }
  }
  float2* sYZ = sU + 36 * NS + 9 * NF0;
  for (int g0 = w0 * 64; g0 < NYZ; g0 += nw * 64) {
    const int u = g0 + lane;
    if (u < NYZ) {
      const int r0 = 2 * u;
      const int mu = r0 < 9 * NF1 ? 1 : 2;
      const int r = mu == 1 ? r0 : r0 - 9 * NF1;
      const int nf = mu == 1 ? NF1 : NF2;
      const int ab = r / nf, f = r - ab * nf;
      const int xx = bx + f % TX;
      int yy, zz;
      if (mu == 1) { yy = by == 0 ? Ly - 1 : by - 1; zz = bz + f / TX; }
      else { yy = by + f / TX; zz = bz == 0 ? Lz - 1 : bz - 1; }
      __builtin_amdgcn_global_load_lds((const void*)(gp + (long long)(mu * 9 + ab) * V4 + tb + (zz * Ly + yy) * Lx + xx),
                                       (lds_void_t)(void*)(sYZ + 2 * g0), 16, 0, 0);
    }
  }
  float2* sX = sU + 36 * NS;
  const int xx = bx == 0 ? Lx - 1 : bx - 1;
  for (int g0 = w0 * 64; g0 < NXW; g0 += nw * 64) {
    const int d = g0 + lane;
    if (d < NXW) {
      const int e = d >> 1, ab = e / NF0, f = e - ab * NF0;
      const char* src = reinterpret_cast<const char*>(gp + (long long)ab * V4 + tb +
                                                      ((bz + f / TY) * Ly + by + f % TY) * Lx + xx) + 4 * (d & 1);
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t)(void*)(reinterpret_cast<char*>(sX) + 4 * g0),
                                       4, 0, 0);
    }
  }
}

// One spatial hop of an s-pair: the neighbour from LDS when it is in the
// tile (sp), else from memory (row j5 of in); link (phase included) from LDS.
template <int MU, int EPS, bool DAGU>
__device__ __forceinline__ void hop_x(Spinor<float2>& a0, Spinor<float2>& a1, bool inside, lds_f4_t sp, int cst,
                                      const char* inb, long long cs, unsigned off, lds_f2_t Ul, int ustride) {
  Spinor<float2> q0, q1;
  float2 U[3][3], h[2][3], u[2][3];
  if (inside) lds_pair(q0, q1, sp, cst);
  else load_pair_o(q0, q1, inb, cs, off);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const xf2 v = Ul[q * ustride];
    U[q / 3][q % 3] = make_float2(v.x, v.y);
  }
  project<MU, EPS>(q0, h);
  mul_link_1<DAGU>(U, h, u);
  accumulate<MU, EPS>(a0, u);
  project<MU, EPS>(q1, h);
  mul_link_1<DAGU>(U, h, u);
  accumulate<MU, EPS>(a1, u);
  pin_acc(a0);
  pin_acc(a1);
}

// Own terms of an s-pair (diagonal and fifth-dimension hop) with the s0 - 1
// and s0 + 2 values read from LDS: row jm's second and row jq's first s-value.
__device__ __forceinline__ void own_pair_x(Spinor<float2>& a0, Spinor<float2>& a1, const Spinor<float2>& p0,
                                           const Spinor<float2>& p1, lds_f4_t row_m, lds_f4_t row_q,
                                           int cst, int s0, int Ls, float dg, float mf, int up0, int dn0) {
  const float cdn0 = s0 == 0 ? mf : -1.f;       // s0 - 1 across the wall
  const float cup1 = s0 + 2 == Ls ? mf : -1.f;  // s0 + 2 across the wall
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = sp * 3 + c;
      float2 r0 = cscale(p0.v[sp][c], dg), r1 = cscale(p1.v[sp][c], dg);
      if (sp == up0 || sp == up0 + 1) {
        const nf4 v = row_q[k * cst];
        r0 = csub(r0, p1.v[sp][c]);                                  // s0 <- s0 + 1
        r1 = cadd(r1, cscale(make_float2(v.x, v.y), cup1));          // s0 + 1 <- s0 + 2
      }
      if (sp == dn0 || sp == dn0 + 1) {
        const nf4 v = row_m[k * cst];
        r0 = cadd(r0, cscale(make_float2(v.z, v.w), cdn0));          // s0 <- s0 - 1
        r1 = csub(r1, p0.v[sp][c]);                                  // s0 + 1 <- s0
      }
      a0.v[sp][c] = cscale(r0, -2.f);
      a1.v[sp][c] = cscale(r1, -2.f);
    }
}

template <bool DAG, int MODE, int TX, int TY, int TZ, bool AL>
__global__ __launch_bounds__(TX * TY * TZ * 8, TX * TY * TZ >= 64 ? 1 : 2) void k_dslash_tx(
    const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ b,
    const float2* __restrict__ gauge, TMArgs ta, double* __restrict__ partial) {
  constexpr int NS = TX * TY * TZ;
  constexpr int NF0 = TY * TZ, NF1 = TX * TZ, NF2 = TX * TY;
  __shared__ float4 sP[12 * NS * 8];                    // slice t: [component][site][s-pair]
  constexpr int NL = 36 * NS + 9 * (NF0 + NF1 + NF2);
  __shared__ __align__(16) float2 sU[AL ? 2 : 1][NL];     // as in k_dslash_tq's staged links (AL: two slices)
  const float2* gp = gauge + 72LL * ta.d.V4;             // phase-folded copy
  const DslashArgs& a = ta.d;
  const int ntiles = ta.ntx * ta.nty * ta.ntz;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int chunk, tile, rhs, pidx;
  if (ta.fold == 2) {
    // XCD units: unit u = (rhs, z-slab of ntiles / zs tiles) goes whole to
    // XCD u % 8 (workgroups are dealt to the eight XCDs in turn), so x, y and
    // most z faces are read from the XCD's own L2; each XCD runs its units
    // one after another.  One t-chunk.
    const int S = ntiles / ta.zs;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int u = xcd + 8 * (j / S);
    rhs = u / ta.zs;
    tile = (u - rhs * ta.zs) * S + j % S;
    chunk = 0;
    pidx = rhs * ntiles + tile;
  } else if (ta.fold) {
    const int per_chunk = ta.nrhs * ntiles;
    chunk = bid / per_chunk;
    const int r2 = bid - chunk * per_chunk;
    rhs = r2 / ntiles;
    tile = r2 - rhs * ntiles;
    pidx = rhs * (gridDim.x / ta.nrhs) + chunk * ntiles + tile;
  } else {
    chunk = bid / ntiles;
    tile = bid - chunk * ntiles;
    rhs = blockIdx.y;
    pidx = blockIdx.y * gridDim.x + blockIdx.x;
  }
  const int tx = tile % ta.ntx, ty = (tile / ta.ntx) % ta.nty, tz = tile / (ta.ntx * ta.nty);
  const int Ls = a.Ls, np = Ls >> 1;
  const int site = threadIdx.x / np, jp = threadIdx.x - site * np;
  const int s0 = 2 * jp;
  const int lc[3] = {site % TX, (site / TX) % TY, site / (TX * TY)};
  const int x = tx * TX + lc[0], y = ty * TY + lc[1], z = tz * TZ + lc[2];
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const long long roff = (long long)rhs * 12 * V5;
  const char* inb = reinterpret_cast<const char*>(in + roff);
  const char* outb = reinterpret_cast<const char*>(out + roff);
  const char* bb0 = MODE == 1 ? reinterpret_cast<const char*>(b + roff) : nullptr;
  const long long cs = V5 * (long long)sizeof(float2);  // component stride in bytes
  const int x3 = (z * Ly + y) * Lx + x;
  constexpr int TS[3] = {1, TX, TX * TY};
  constexpr int TE[3] = {TX, TY, TZ};
  const int cst = NS * np;  // component stride of sP in float4
  const int me = site * np + jp;
  int nf3[3], nb3[3], sf[3], sb3[3], lf[3], lb[3], ub[3];
  bool inF[3], inB[3];
  {
    const int co[3] = {x, y, z};
    const int Lm[3] = {Lx, Ly, Lz};
    const int st[3] = {1, Lx, Lx * Ly};
    const int fo[3] = {36 * NS, 36 * NS + 9 * NF0, 36 * NS + 9 * (NF0 + NF1)};
    const int fi[3] = {lc[1] + TY * lc[2], lc[0] + TX * lc[2], lc[0] + TX * lc[1]};
    const int nfc[3] = {NF0, NF1, NF2};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool top = co[mu] == Lm[mu] - 1, bot = co[mu] == 0;
      nf3[mu] = top ? x3 - (Lm[mu] - 1) * st[mu] : x3 + st[mu];
      nb3[mu] = bot ? x3 + (Lm[mu] - 1) * st[mu] : x3 - st[mu];
      inF[mu] = lc[mu] + 1 < TE[mu];
      inB[mu] = lc[mu] > 0;
      sf[mu] = inF[mu] ? me + TS[mu] * np : me;
      sb3[mu] = inB[mu] ? me - TS[mu] * np : me;
      lf[mu] = mu * 9 * NS + site;
      if (inB[mu]) { lb[mu] = mu * 9 * NS + site - TS[mu]; ub[mu] = NS; }
      else { lb[mu] = fo[mu] + fi[mu]; ub[mu] = nfc[mu]; }
    }
  }
  const int jm = jp == 0 ? np - 1 : jp - 1, jq = jp + 1 == np ? 0 : jp + 1;
  const lds_f4_t lP = (lds_f4_t)(void*)sP;
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const int up0 = DAG ? 0 : 2;   // spins coupled to s+1
  const int dn0 = DAG ? 2 : 0;   // spins coupled to s-1
  const float dg = (float)a.diag, mf = (float)a.mf;
  const int t0 = chunk * ta.tc;
  const int t1 = min(t0 + ta.tc, Lt);
  const int bx = tx * TX, by = ty * TY, bz = tz * TZ;
  float2 hp0[2][3], hp1[2][3], U[3][3], h[2][3], u[2][3];
  Spinor<float2> p0, p1, a0, a1;
  {  // half spinor of slice t0 - 1 for the backward t-hop, its link (phase included), slice t0
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    load_pair_o(p0, p1, inb, cs, (unsigned)((tm * V3 + x3) * Ls + s0) * 8u);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    if (AL) {
      load_link(gp, 3, V4, tm * V3 + x3, U);
      stage_links_async<TX, TY, TZ>(sU[t0 & 1], gp, a, V4, t0 * V3, bx, by, bz);
    } else {
      load_link(gauge, 3, V4, tm * V3 + x3, U);
    }
    if (!AL && t0 == 0) {
      const float ph = a.ph[3];
#pragma unroll
      for (int q = 0; q < 9; ++q) U[q / 3][q % 3] = cscale(U[q / 3][q % 3], ph);
    }
    load_pair_o(p0, p1, inb, cs, (unsigned)((t0 * V3 + x3) * Ls + s0) * 8u);
  }
  float nrmf = 0.f;
  for (int t = t0; t < t1; ++t) {
    const int x4 = t * V3 + x3;
    const int tb = t * V3;
    if (AL) __builtin_amdgcn_s_waitcnt(0);  // this wavefront's copies of slice t's links have landed
    __syncthreads();  // every thread is done with the previous slice's LDS
    const lds_f2_t lU = (lds_f2_t)(void*)sU[AL ? (t & 1) : 0];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const float2 v0 = p0.v[k / 3][k % 3], v1 = p1.v[k / 3][k % 3];
      ((lds_f4w_t)(void*)sP)[k * cst + me] = nf4{v0.x, v0.y, v1.x, v1.y};
    }
    if (AL) {
      // the slice is written: wait for this wavefront's LDS stores (no fence:
      // nothing else of this wavefront needs to land first) and meet
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
      __builtin_amdgcn_s_barrier();
    } else {
      stage_links<TX, TY, TZ>(sU[0], gauge, a, V4, tb, t, bx, by, bz);
      __syncthreads();
    }
    // own terms, backward t-hop (half spinor and link carried from slice t - 1)
    own_pair_x(a0, a1, p0, p1, lP + site * np + jm, lP + site * np + jq, cst, s0, Ls, dg, mf, up0, dn0);
    mul_link_1<true>(U, hp0, u);
    accumulate<3, EB>(a0, u);
    mul_link_1<true>(U, hp1, u);
    accumulate<3, EB>(a1, u);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    hop_x<0, EF, false>(a0, a1, inF[0], lP + sf[0], cst, inb, cs, (unsigned)((tb + nf3[0]) * Ls + s0) * 8u, lU + lf[0], NS);
    hop_x<0, EB, true>(a0, a1, inB[0], lP + sb3[0], cst, inb, cs, (unsigned)((tb + nb3[0]) * Ls + s0) * 8u, lU + lb[0], ub[0]);
    hop_x<1, EF, false>(a0, a1, inF[1], lP + sf[1], cst, inb, cs, (unsigned)((tb + nf3[1]) * Ls + s0) * 8u, lU + lf[1], NS);
    hop_x<1, EB, true>(a0, a1, inB[1], lP + sb3[1], cst, inb, cs, (unsigned)((tb + nb3[1]) * Ls + s0) * 8u, lU + lb[1], ub[1]);
    hop_x<2, EF, false>(a0, a1, inF[2], lP + sf[2], cst, inb, cs, (unsigned)((tb + nf3[2]) * Ls + s0) * 8u, lU + lf[2], NS);
    hop_x<2, EB, true>(a0, a1, inB[2], lP + sb3[2], cst, inb, cs, (unsigned)((tb + nb3[2]) * Ls + s0) * 8u, lU + lb[2], ub[2]);
    // forward t-hop with slice t + 1 (its own slice next); the link is the
    // next slice's backward t-hop link
    const bool top = t == Lt - 1;
    load_pair_o(p0, p1, inb, cs, (unsigned)(((top ? 0 : t + 1) * V3 + x3) * Ls + s0) * 8u);
    // the next slice's links, copied behind the spinor load (vmcnt is in
    // order: waiting for the spinor does not wait for them); they land during
    // this slice's forward hop and stores, and the next barrier waits for them
    if (AL && t + 1 < t1) stage_links_async<TX, TY, TZ>(sU[(t + 1) & 1], gp, a, V4, tb + V3, bx, by, bz);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const xf2 v = lU[(27 + q) * NS + site];
      U[q / 3][q % 3] = make_float2(v.x, v.y);
    }
    project<3, EF>(p0, h);
    mul_link_1<false>(U, h, u);
    accumulate<3, EF>(a0, u);
    project<3, EF>(p1, h);
    mul_link_1<false>(U, h, u);
    accumulate<3, EF>(a1, u);
    const unsigned o5 = (unsigned)(x4 * Ls + s0) * 8u;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float2 r0 = cscale(a0.v[sp][c], -0.5f), r1 = cscale(a1.v[sp][c], -0.5f);
        if (MODE == 1) {
          const nf4 bb = AL ? __builtin_nontemporal_load((gf4_t)(sbase(bb0, cs, sp * 3 + c) + o5))
                            : *(gf4_t)(sbase(bb0, cs, sp * 3 + c) + o5);
          r0 = make_float2(bb.x - r0.x, bb.y - r0.y);
          r1 = make_float2(bb.z - r1.x, bb.w - r1.y);
        }
        // AL: results and b stream past L2 (read or written once), which then
        // keeps more of the input slices that neighbouring tiles read as faces
        if (AL) __builtin_nontemporal_store(nf4{r0.x, r0.y, r1.x, r1.y}, (gf4w_t)(sbase(outb, cs, sp * 3 + c) + o5));
        else *(gf4w_t)(sbase(outb, cs, sp * 3 + c) + o5) = nf4{r0.x, r0.y, r1.x, r1.y};
        if (partial) nrmf += r0.x * r0.x + r0.y * r0.y + r1.x * r1.x + r1.y * r1.y;
      }
  }
  if (partial) {
    const double sum = block_sum_dyn((double)nrmf);
    if (threadIdx.x == 0) partial[pidx] = sum;
  }
}

// ---------------------------------------------------------------- t-march, software-pipelined (FP32)
// k_dslash_tq computes each hop right after loading it, so every hop waits
// out a full memory round trip: with one wavefront per SIMD nothing else hides
// it.  Here the loads of hop k+1 are issued as soon as hop k's spinor is
// projected to half spinors (the raw registers are free again), and the SU(3)
// products of hop k run while they are in flight.  Hop order per t-slice:
// +x, -x, +y, -y, +z, -z, then +t, whose spinor (slice t+1) also gives slice
// t+1's own terms and backward t-hop as in k_dslash_tq; the first hop of slice
// t+1 is issued once slice t is stored.  Scheduling barriers keep the
// compiler from sinking the early loads back to their uses.
struct HopRaw {
  float4 q[12];  // spin-colour component k of the pair (s0, s0 + 1)
  float2 U[9];   // link entries (a, b) at 3a + b
};

__device__ __forceinline__ void issue_hop(HopRaw& r, const float2* __restrict__ in, const float2* __restrict__ gauge,
                                          long long V5, long long V4, long long j5, int mu, int xlink) {
#pragma unroll
  for (int k = 0; k < 12; ++k) r.q[k] = *reinterpret_cast<const float4*>(in + k * V5 + j5);
#pragma unroll
  for (int q = 0; q < 9; ++q) r.U[q] = gauge[(mu * 9 + q) * V4 + xlink];
}

__device__ __forceinline__ void unpack_pair(const HopRaw& r, Spinor<float2>& p0, Spinor<float2>& p1) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4 v = r.q[sp * 3 + c];
      p0.v[sp][c] = make_float2(v.x, v.y);
      p1.v[sp][c] = make_float2(v.z, v.w);
    }
}

// half spinors of both s-values and the link, copied out of the raw buffer
template <int MU, int EPS>
__device__ __forceinline__ void take_hop(const HopRaw& r, float2 h0[2][3], float2 h1[2][3], float2 U[3][3]) {
  Spinor<float2> p0, p1;
  unpack_pair(r, p0, p1);
  project<MU, EPS>(p0, h0);
  project<MU, EPS>(p1, h1);
#pragma unroll
  for (int q = 0; q < 9; ++q) U[q / 3][q % 3] = r.U[q];
}

template <int MU, int EPS, bool DAGU>
__device__ __forceinline__ void finish_hop(Spinor<float2>& a0, Spinor<float2>& a1, const float2 U[3][3],
                                           const float2 h0[2][3], const float2 h1[2][3], float ph) {
  float2 u[2][3];
  mul_link<DAGU>(U, h0, u, ph);
  accumulate<MU, EPS>(a0, u);
  mul_link<DAGU>(U, h1, u, ph);
  accumulate<MU, EPS>(a1, u);
}

// The fifth-dimension neighbours of the pair outside it (s0 - 1 for the spins
// coupled to s-1, s0 + 2 for those coupled to s+1), six components each.
__device__ __forceinline__ void issue_own(float2 ex[12], const float2* __restrict__ in, long long V5, long long base,
                                          int s0, int Ls, int up0, int dn0) {
  const int sm = s0 == 0 ? Ls - 1 : s0 - 1;
  const int sp2 = s0 + 2 == Ls ? 0 : s0 + 2;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    ex[k] = in[(long long)((up0 + k / 3) * 3 + k % 3) * V5 + base + sp2];
    ex[6 + k] = in[(long long)((dn0 + k / 3) * 3 + k % 3) * V5 + base + sm];
  }
}

// own_pair with the out-of-pair neighbours already loaded by issue_own
__device__ __forceinline__ void own_pair_pre(Spinor<float2>& a0, Spinor<float2>& a1, const Spinor<float2>& p0,
                                             const Spinor<float2>& p1, const float2 ex[12], int s0, int Ls,
                                             float dg, float mf, int up0, int dn0) {
  const float cdn0 = s0 == 0 ? mf : -1.f;       // s0 - 1 across the wall
  const float cup1 = s0 + 2 == Ls ? mf : -1.f;  // s0 + 2 across the wall
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 r0 = cscale(p0.v[sp][c], dg), r1 = cscale(p1.v[sp][c], dg);
      if (sp == up0 || sp == up0 + 1) {
        r0 = csub(r0, p1.v[sp][c]);                                 // s0 <- s0 + 1
        r1 = cadd(r1, cscale(ex[(sp - up0) * 3 + c], cup1));        // s0 + 1 <- s0 + 2
      }
      if (sp == dn0 || sp == dn0 + 1) {
        r0 = cadd(r0, cscale(ex[6 + (sp - dn0) * 3 + c], cdn0));    // s0 <- s0 - 1
        r1 = csub(r1, p0.v[sp][c]);                                 // s0 + 1 <- s0
      }
      a0.v[sp][c] = cscale(r0, -2.f);
      a1.v[sp][c] = cscale(r1, -2.f);
    }
}

#define MG_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

template <bool DAG, int MODE, int TX, int TY, int TZ, int PAD>
__global__ __launch_bounds__(TX * TY * TZ * 8, 1) void k_dslash_tw(const float2* __restrict__ in,
                                                                   float2* __restrict__ out,
                                                                   const float2* __restrict__ b,
                                                                   const float2* __restrict__ gauge, TMArgs ta,
                                                                   double* __restrict__ partial) {
  if (PAD > 0) {  // LDS reserved only to cap workgroups per CU (one per CU when PAD > 80 KB)
    __shared__ float pad[PAD > 0 ? PAD / 4 : 1];
    if (ta.d.Ls < 0) pad[threadIdx.x] = 0.f;  // never true: keeps the allocation
    if (ta.d.Ls < 0) out[threadIdx.x].x = pad[threadIdx.x ^ 1];
  }
  const DslashArgs& a = ta.d;
  const int ntiles = ta.ntx * ta.nty * ta.ntz;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int chunk, tile, rhs, pidx;
  if (ta.fold) {
    const int per_chunk = ta.nrhs * ntiles;
    chunk = bid / per_chunk;
    const int r2 = bid - chunk * per_chunk;
    rhs = r2 / ntiles;
    tile = r2 - rhs * ntiles;
    pidx = rhs * (gridDim.x / ta.nrhs) + chunk * ntiles + tile;
  } else {
    chunk = bid / ntiles;
    tile = bid - chunk * ntiles;
    rhs = blockIdx.y;
    pidx = blockIdx.y * gridDim.x + blockIdx.x;
  }
  const int tx = tile % ta.ntx, ty = (tile / ta.ntx) % ta.nty, tz = tile / (ta.ntx * ta.nty);
  const int Ls = a.Ls, np = Ls >> 1;
  const int site = threadIdx.x / np, jp = threadIdx.x - site * np;
  const int s0 = 2 * jp;
  const int x = tx * TX + site % TX, y = ty * TY + (site / TX) % TY, z = tz * TZ + site / (TX * TY);
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2], Lt = a.L[3];
  const long long V5 = a.V5, V4 = a.V4;
  const int V3 = Lx * Ly * Lz;
  const long long roff = (long long)rhs * 12 * V5;
  in += roff;
  out += roff;
  if (MODE == 1) b += roff;
  const int x3 = (z * Ly + y) * Lx + x;
  int nf3[3], nb3[3];
  float phf[3], phb[3];
  {
    const int co[3] = {x, y, z};
    const int Lm[3] = {Lx, Ly, Lz};
    const int st[3] = {1, Lx, Lx * Ly};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool top = co[mu] == Lm[mu] - 1, bot = co[mu] == 0;
      nf3[mu] = top ? x3 - (Lm[mu] - 1) * st[mu] : x3 + st[mu];
      nb3[mu] = bot ? x3 + (Lm[mu] - 1) * st[mu] : x3 - st[mu];
      phf[mu] = top ? a.ph[mu] : 1.0f;
      phb[mu] = bot ? a.ph[mu] : 1.0f;
    }
  }
  constexpr int EF = DAG ? 1 : -1;
  constexpr int EB = DAG ? -1 : 1;
  const int up0 = DAG ? 0 : 2;   // spins coupled to s+1
  const int dn0 = DAG ? 2 : 0;   // spins coupled to s-1
  const float dg = (float)a.diag, mf = (float)a.mf;
  const int t0 = chunk * ta.tc;
  const int t1 = min(t0 + ta.tc, Lt);
  float2 hp0[2][3], hp1[2][3], U[3][3], h0[2][3], h1[2][3];
  Spinor<float2> p0, p1, a0, a1;
  HopRaw r;
  float2 ex[12];
  {  // slice t0: own terms, and the backward t-hop from slice t0 - 1
    const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
    const int x4m = tm * V3 + x3;
    load_pair(p0, p1, in, V5, (long long)x4m * Ls + s0);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    const long long base = (long long)(t0 * V3 + x3) * Ls;
    load_pair(p0, p1, in, V5, base + s0);
    own_pair(a0, a1, p0, p1, in, V5, base, s0, Ls, dg, mf, up0, dn0);
    load_link(gauge, 3, V4, x4m, U);
    const float ph = t0 == 0 ? a.ph[3] : 1.0f;
    finish_hop<3, EB, true>(a0, a1, U, hp0, hp1, ph);
    project<3, EB>(p0, hp0);
    project<3, EB>(p1, hp1);
    const int tb = t0 * V3;
    issue_hop(r, in, gauge, V5, V4, (long long)(tb + nf3[0]) * Ls + s0, 0, tb + x3);
  }
  float nrmf = 0.f;  // per-thread |out|^2 in FP32, FP64 across the workgroup
  for (int t = t0; t < t1; ++t) {
    const int x4 = t * V3 + x3;
    const int tb = t * V3;
    const bool top = t == Lt - 1;
    const long long basef = (long long)((top ? 0 : t + 1) * V3 + x3) * Ls;
    // hops +x .. -z: project hop k, issue hop k+1, finish hop k
#define MG_TW_STAGE(MU, E, DAGU, PH, NEXT)  \
    take_hop<MU, E>(r, h0, h1, U);          \
    MG_SCHED_FENCE();                       \
    NEXT;                                   \
    MG_SCHED_FENCE();                       \
    finish_hop<MU, E, DAGU>(a0, a1, U, h0, h1, PH);
    MG_TW_STAGE(0, EF, false, phf[0], issue_hop(r, in, gauge, V5, V4, (long long)(tb + nb3[0]) * Ls + s0, 0, tb + nb3[0]))
    MG_TW_STAGE(0, EB, true, phb[0], issue_hop(r, in, gauge, V5, V4, (long long)(tb + nf3[1]) * Ls + s0, 1, x4))
    MG_TW_STAGE(1, EF, false, phf[1], issue_hop(r, in, gauge, V5, V4, (long long)(tb + nb3[1]) * Ls + s0, 1, tb + nb3[1]))
    MG_TW_STAGE(1, EB, true, phb[1], issue_hop(r, in, gauge, V5, V4, (long long)(tb + nf3[2]) * Ls + s0, 2, x4))
    MG_TW_STAGE(2, EF, false, phf[2], issue_hop(r, in, gauge, V5, V4, (long long)(tb + nb3[2]) * Ls + s0, 2, tb + nb3[2]))
    MG_TW_STAGE(2, EB, true, phb[2], issue_hop(r, in, gauge, V5, V4, basef + s0, 3, x4);
                issue_own(ex, in, V5, basef, s0, Ls, up0, dn0))
#undef MG_TW_STAGE
    // +t: slice t+1's spinor stays in p0, p1 for its own terms
    unpack_pair(r, p0, p1);
    project<3, EF>(p0, h0);
    project<3, EF>(p1, h1);
#pragma unroll
    for (int q = 0; q < 9; ++q) U[q / 3][q % 3] = r.U[q];
    finish_hop<3, EF, false>(a0, a1, U, h0, h1, top ? a.ph[3] : 1.0f);
    const long long i5 = (long long)x4 * Ls + s0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long cc = (long long)(sp * 3 + c) * V5;
        float2 r0 = cscale(a0.v[sp][c], -0.5f), r1 = cscale(a1.v[sp][c], -0.5f);
        if (MODE == 1) {
          const float4 bb = *reinterpret_cast<const float4*>(b + cc + i5);
          r0 = make_float2(bb.x - r0.x, bb.y - r0.y);
          r1 = make_float2(bb.z - r1.x, bb.w - r1.y);
        }
        *reinterpret_cast<float4*>(out + cc + i5) = make_float4(r0.x, r0.y, r1.x, r1.y);
        if (partial) nrmf += r0.x * r0.x + r0.y * r0.y + r1.x * r1.x + r1.y * r1.y;
      }
    if (t + 1 < t1) {  // slice t+1: first hop in flight, then own terms and backward t-hop
      const int tb1 = tb + V3;
      MG_SCHED_FENCE();
      issue_hop(r, in, gauge, V5, V4, (long long)(tb1 + nf3[0]) * Ls + s0, 0, tb1 + x3);
      MG_SCHED_FENCE();
      own_pair_pre(a0, a1, p0, p1, ex, s0, Ls, dg, mf, up0, dn0);
      finish_hop<3, EB, true>(a0, a1, U, hp0, hp1, 1.0f);
      project<3, EB>(p0, hp0);
      project<3, EB>(p1, hp1);
    }
  }
  if (partial) {
    const double sum = block_sum_dyn((double)nrmf);
    if (threadIdx.x == 0) partial[pidx] = sum;
  }
}
#undef MG_SCHED_FENCE

}  // namespace

// FP32 t-march tilings: x, y, z tile, workgroups aimed at per right-hand side
// (sets the t-slices per workgroup), which kernel, workgroup order and
// occupancy.  Entry 0 is the default; mgdwf_tune times the others on the
// device.  Measured on 16^3 x 32 x 16 at 12 RHS the shapes and orders are
// within 10 % of each other.  With two workgroups per CU the kernel fetches
// 3.8x its algorithmic bytes from beyond L2 (tile faces re-read by the
// neighbouring workgroups); one workgroup per CU halves the L2 footprint and
// the fetch (1.9x) but gains only 3 %, and staging the links in LDS (which
// removes most of the link loads) is 25 % slower -- the kernel is limited by
// the issue and latency of its 16-byte spinor loads, not by DRAM bytes.  The
// software-pipelined k_dslash_tw keeps a hop's loads in flight under the
// previous hop's arithmetic and is within 1-6 % of k_dslash_tq.
struct FTile {
  int tx, ty, tz, target;
  bool eight_loads;  // k_dslash_tp (reloads the own slice) instead of k_dslash_tq
  int fold;          // workgroup order (TMArgs::fold)
  bool one_per_cu = false;  // reserve LDS so that one workgroup runs per CU
  bool lds_links = false;   // stage each slice's links in LDS
  bool pipelined = false;   // k_dslash_tw (loads one hop ahead)
  bool ws = false;          // k_dslash_ws: tx, ty, tz = brick of (x pairs, y, z), target = t-slices per chunk
  bool xchg = false;        // k_dslash_tx: spatial neighbours inside the tile through LDS
  bool alinks = false;      // with xchg: next slice's links copied to LDS directly, during this slice
};
constexpr FTile kFTiles[] = {
    // LDS exchange with asynchronous links first: the default where it applies
    {8, 4, 2, 768, false, 2, false, false, false, false, true, true},
    {8, 4, 2, 768, false, 0, false, false, false, false, true, true},
    {8, 4, 2, 1536, false, 0, false, false, false, false, true, true},
    {8, 4, 2, 384, false, 0, false, false, false, false, true, true},
    {4, 4, 4, 768, false, 0, false, false, false, false, true, true},
    {4, 4, 2, 1536, false, 0, false, false, false, false, true, true},
    {4, 4, 2, 3072, false, 0, false, false, false, false, true, true},
    {8, 4, 2, 3072, false, 1, false, false, false, false, true, true},
    {4, 4, 4, 768, false, 2, false, false, false, false, true, true},
    {4, 4, 2, 1536, false, 2, false, false, false, false, true, true},
    // t-march kernels loading every neighbour from memory
    {4, 4, 2, 256, false, 0, true}, {4, 4, 2, 512, false, 0, true}, {4, 4, 2, 256, false, 0},
    {4, 4, 2, 512, false, 0},       {8, 2, 2, 512, false, 0},       {8, 4, 2, 256, false, 0},
    {4, 4, 4, 512, false, 0},       {4, 8, 2, 512, false, 0},       {4, 4, 2, 1024, false, 1},
    {4, 4, 2, 512, true, 0},        {4, 4, 2, 256, false, 0, true, true},
    {4, 4, 2, 256, false, 0, true, false, true}, {4, 4, 2, 256, false, 0, false, false, true},
    {4, 4, 2, 512, false, 0, true, false, true},
    // one wavefront per site pair
    {2, 2, 2, 2, false, 0, false, false, false, true}, {4, 4, 4, 2, false, 0, false, false, false, true},
    {8, 16, 1, 2, false, 0, false, false, false, true},
    // LDS exchange, links staged synchronously
    {4, 4, 2, 256, false, 0, false, false, false, false, true},
};
constexpr int NFTILE = sizeof(kFTiles) / sizeof(kFTiles[0]);

// A tiling applies when x, y, z divide by the tile and Ls is even, 4..16,
// with whole wavefronts per workgroup.
static bool ftile_ok(const Geometry& g, int i) {
  if (i < 0 || i >= NFTILE) return false;
  const FTile& f = kFTiles[i];
  if (f.ws) {  // two sites per wavefront in x; 2 P = Ls with P = 4 or 8; whole workgroups per (group, chunk)
    const int nxp = g.L[0] / 2;
    const long long group_bytes = 32LL / (g.Ls / 2) * 12 * (long long)g.V5 * 8;  // R fields: 32-bit lane offsets
    return g.L[0] % 2 == 0 && nxp % f.tx == 0 && g.L[1] % f.ty == 0 && g.L[2] % f.tz == 0 &&
           (g.Ls == 8 || g.Ls == 16) && (nxp * g.L[1] * g.L[2]) % 4 == 0 && group_bytes < (1LL << 32);
  }
  const int thr = f.tx * f.ty * f.tz * g.Ls / 2;
  if (f.xchg && (long long)g.V5 * 8 >= (1LL << 32)) return false;  // 32-bit lane offsets
  return g.L[0] % f.tx == 0 && g.L[1] % f.ty == 0 && g.L[2] % f.tz == 0 && g.Ls % 2 == 0 && g.Ls >= 4 &&
         g.Ls <= 16 && thr % 64 == 0;
}

static int ftile_of(const Geometry& g) {
  if (ftile_ok(g, g.ftile)) return g.ftile;
  for (int i = 0; i < NFTILE; ++i)
    if (ftile_ok(g, i)) return i;
  return -1;
}

static int ftile_ntiles(const Geometry& g, int i) {
  const FTile& f = kFTiles[i];
  if (f.ws) return g.L[0] / 2 * g.L[1] * g.L[2] / 4;  // workgroups per (group, chunk)
  return (g.L[0] / f.tx) * (g.L[1] / f.ty) * (g.L[2] / f.tz);
}

// z-slabs per right-hand side for XCD units: the smallest divisor zs of the
// tile count in z with nrhs * zs a multiple of the eight XCDs (0: none).
static int xcd_units_zs(int ntz, int nrhs) {
  for (int zs = 1; zs <= ntz; ++zs)
    if (ntz % zs == 0 && (nrhs * zs) % 8 == 0) return zs;
  return 0;
}

// t-slices per workgroup.  target: site-pair kernel, the chunk itself;
// LDS-exchange kernels with asynchronous links, the workgroups wanted over
// all right-hand sides (long chunks when many right-hand sides fill the chip:
// fewer chunk starts, whose first slice is loaded twice); others, the
// workgroups wanted per right-hand side.
static int ftile_chunk(const Geometry& g, int i, int nrhs) {
  const FTile& f = kFTiles[i];
  if (f.ws) return std::min(g.L[3], f.target);
  const int per = f.alinks ? ftile_ntiles(g, i) * std::max(1, nrhs) : ftile_ntiles(g, i);
  const int want_chunks = std::max(1, std::min(g.L[3], ceil_div(f.target, per)));
  return ceil_div(g.L[3], want_chunks);
}

int dslash_ftile_count() { return NFTILE; }

bool dslash_ftile_desc(const Geometry& g, int i, int nrhs, int desc[4], int* flags) {
  if (!ftile_ok(g, i)) return false;
  desc[0] = kFTiles[i].tx;
  desc[1] = kFTiles[i].ty;
  desc[2] = kFTiles[i].tz;
  desc[3] = ftile_chunk(g, i, nrhs);
  *flags = (kFTiles[i].eight_loads ? 1 : 0) | (kFTiles[i].fold == 1 ? 2 : 0) | (kFTiles[i].fold == 2 ? 512 : 0) |
           (kFTiles[i].one_per_cu ? 4 : 0) |
           (kFTiles[i].lds_links ? 8 : 0) | (kFTiles[i].pipelined ? 16 : 0) | (kFTiles[i].ws ? 32 : 0) |
           (kFTiles[i].xchg ? 64 : 0) | (kFTiles[i].alinks ? 256 : 0);
  return true;
}

// The t-march kernel covers lattices whose x, y, z extents tile by 4, 2, 2 and
// whose Ls is a multiple of 4 (whole wavefronts) up to 16; others use k_dslash.
static bool use_tmarch(const Geometry& g) {
  return g.L[0] % TMX == 0 && g.L[1] % TMY == 0 && g.L[2] % TMZ == 0 && g.Ls % 4 == 0 && g.Ls <= 16;
}

// t-slices per chunk: enough chunks that about four workgroups share each CU.
static int tmarch_chunk(const Geometry& g) {
  const int ntiles = (g.L[0] / TMX) * (g.L[1] / TMY) * (g.L[2] / TMZ);
  const int want_chunks = std::max(1, std::min(g.L[3], ceil_div(1024, ntiles)));
  return ceil_div(g.L[3], want_chunks);
}

template <int TX, int TY, int TZ, int PAD, bool LL>
static void launch_tq(const float2* in, float2* out, const float2* b, const float2* gauge, const TMArgs& ta,
                      double* partial, bool dagger, int mode, dim3 grid, dim3 blk, hipStream_t st) {
#define MG_TQ(DAG, MODE) \
  hipLaunchKernelGGL((k_dslash_tq<DAG, MODE, TX, TY, TZ, PAD, LL>), grid, blk, 0, st, in, out, b, gauge, ta, partial)
  if (!dagger && mode == 0) MG_TQ(false, 0);
  else if (!dagger && mode == 1) MG_TQ(false, 1);
  else if (dagger && mode == 0) MG_TQ(true, 0);
  else MG_TQ(true, 1);
#undef MG_TQ
}

static void launch_tpair(const float2* in, float2* out, const float2* b, const float2* gauge, const TMArgs& ta,
                         double* partial, bool dagger, int mode, dim3 grid, dim3 blk, int which, hipStream_t st) {
  const FTile& f = kFTiles[which];
  if (f.eight_loads) {
#define MG_TP(DAG, MODE) \
  hipLaunchKernelGGL((k_dslash_tp<DAG, MODE>), grid, blk, 0, st, in, out, b, gauge, ta, partial)
    if (!dagger && mode == 0) MG_TP(false, 0);
    else if (!dagger && mode == 1) MG_TP(false, 1);
    else if (dagger && mode == 0) MG_TP(true, 0);
    else MG_TP(true, 1);
#undef MG_TP
    return;
  }
  constexpr int P1 = 96 * 1024;
  if (f.xchg) {
#define MG_TX(X, Y, Z, AL)                                                                                   \
  if (f.tx == X && f.ty == Y && f.tz == Z && f.alinks == AL) {                                               \
    if (!dagger && mode == 0) hipLaunchKernelGGL((k_dslash_tx<false, 0, X, Y, Z, AL>), grid, blk, 0, st, in, out, b, gauge, ta, partial); \
    else if (!dagger && mode == 1) hipLaunchKernelGGL((k_dslash_tx<false, 1, X, Y, Z, AL>), grid, blk, 0, st, in, out, b, gauge, ta, partial); \
    else if (dagger && mode == 0) hipLaunchKernelGGL((k_dslash_tx<true, 0, X, Y, Z, AL>), grid, blk, 0, st, in, out, b, gauge, ta, partial); \
    else hipLaunchKernelGGL((k_dslash_tx<true, 1, X, Y, Z, AL>), grid, blk, 0, st, in, out, b, gauge, ta, partial); \
    return;                                                                                                  \
  }
    MG_TX(4, 4, 2, false)
    MG_TX(4, 4, 2, true)
    MG_TX(8, 4, 2, true)
    MG_TX(4, 4, 4, true)
#undef MG_TX
    fail(MGDWF_ERR_INVALID_ARG, "no LDS-exchange kernel for this Dslash tiling");
  }
  if (f.pipelined && f.tx == 4 && f.ty == 4 && f.tz == 2) {
#define MG_TW(DAG, MODE, PAD) \
  hipLaunchKernelGGL((k_dslash_tw<DAG, MODE, 4, 4, 2, PAD>), grid, blk, 0, st, in, out, b, gauge, ta, partial)
    if (f.one_per_cu) {
      if (!dagger && mode == 0) MG_TW(false, 0, P1);
      else if (!dagger && mode == 1) MG_TW(false, 1, P1);
      else if (dagger && mode == 0) MG_TW(true, 0, P1);
      else MG_TW(true, 1, P1);
    } else {
      if (!dagger && mode == 0) MG_TW(false, 0, 0);
      else if (!dagger && mode == 1) MG_TW(false, 1, 0);
      else if (dagger && mode == 0) MG_TW(true, 0, 0);
      else MG_TW(true, 1, 0);
    }
#undef MG_TW
    return;
  }
#define MG_TQL(X, Y, Z)                                                                        \
  if (f.tx == X && f.ty == Y && f.tz == Z) {                                                   \
    if (f.one_per_cu) launch_tq<X, Y, Z, P1, false>(in, out, b, gauge, ta, partial, dagger, mode, grid, blk, st); \
    else launch_tq<X, Y, Z, 0, false>(in, out, b, gauge, ta, partial, dagger, mode, grid, blk, st);   \
    return;                                                                                    \
  }
  if (f.lds_links) {
    if (f.tx == 4 && f.ty == 4 && f.tz == 2) {
      launch_tq<4, 4, 2, P1, true>(in, out, b, gauge, ta, partial, dagger, mode, grid, blk, st);
      return;
    }
  }
  MG_TQL(4, 4, 2)
  MG_TQL(8, 4, 2)
  MG_TQL(4, 4, 4)
  MG_TQL(8, 2, 2)
  MG_TQL(4, 8, 2)
#undef MG_TQL
  fail(MGDWF_ERR_INVALID_ARG, "no kernel for this Dslash tiling");
}
static void launch_tpair(const double2*, double2*, const double2*, const double2*, const TMArgs&, double*, bool, int,
                         dim3, dim3, int, hipStream_t) {
  fail(MGDWF_ERR_INVALID_ARG, "the s-pair kernel is FP32 only");
}

static void launch_ws(const float2* in, float2* out, const float2* b, const float2* gauge, const WSArgs& wa,
                      double* partial, bool dagger, int mode, dim3 grid, int P, hipStream_t st) {
#define MG_WS(DAG, MODE, PP) \
  hipLaunchKernelGGL((k_dslash_ws<DAG, MODE, PP>), grid, dim3(256), 0, st, in, out, b, gauge, wa, partial)
#define MG_WSP(PP)                                \
  if (!dagger && mode == 0) MG_WS(false, 0, PP);  \
  else if (!dagger && mode == 1) MG_WS(false, 1, PP); \
  else if (dagger && mode == 0) MG_WS(true, 0, PP);   \
  else MG_WS(true, 1, PP);
  if (P == 8) { MG_WSP(8) }
  else if (P == 4) { MG_WSP(4) }
  else fail(MGDWF_ERR_INVALID_ARG, "no wavefront-per-site-pair kernel for this Ls");
#undef MG_WSP
#undef MG_WS
}
static void launch_ws(const double2*, double2*, const double2*, const double2*, const WSArgs&, double*, bool, int,
                      dim3, int, hipStream_t) {
  fail(MGDWF_ERR_INVALID_ARG, "the wavefront-per-site-pair kernel is FP32 only");
}

// Kernel choice: FP32 takes the s-pair t-march where the lattice tiles, else the
// t-march, else the plain kernel; FP64 takes the plain kernel, whose register
// budget (about 250) keeps two wavefronts per SIMD where the t-march keeps one.
enum DslashKind { DS_PLAIN, DS_TMARCH, DS_TPAIR };

template <class C2>
static DslashKind dslash_kind(const Geometry& g) {
  if (sizeof(typename real_of<C2>::type) == 8) return DS_PLAIN;
  if (ftile_of(g) >= 0) return DS_TPAIR;
  if (use_tmarch(g)) return DS_TMARCH;
  return DS_PLAIN;
}

template <class C2>
int dslash_nblocks(const Geometry& g, int nrhs) {
  switch (dslash_kind<C2>(g)) {
    case DS_TPAIR: {
      const int i = ftile_of(g);
      return ftile_ntiles(g, i) * ceil_div(g.L[3], ftile_chunk(g, i, nrhs));
    }
    case DS_TMARCH:
      return (g.L[0] / TMX) * (g.L[1] / TMY) * (g.L[2] / TMZ) * ceil_div(g.L[3], tmarch_chunk(g));
    default:
      return ceil_div(g.V5, 256);
  }
}
template int dslash_nblocks<double2>(const Geometry&, int);
template int dslash_nblocks<float2>(const Geometry&, int);

template <class C2>
void dslash_ex(const C2* in, C2* out, const C2* b, const C2* gauge, const Geometry& g, double M5,
               double mf, bool dagger, int mode, int nrhs, double* partial, hipStream_t st) {
  DslashArgs a;
  for (int m = 0; m < 4; ++m) { a.L[m] = g.L[m]; a.ph[m] = (float)g.bc[m]; }
  a.Ls = g.Ls; a.V4 = g.V4; a.V5 = g.V5; a.diag = 5.0 - M5; a.mf = mf;
  const DslashKind kind = dslash_kind<C2>(g);
  if (kind == DS_TPAIR && kFTiles[ftile_of(g)].ws) {
    const int i = ftile_of(g);
    const FTile& f = kFTiles[i];
    WSArgs wa;
    wa.d = a;
    wa.nxp = g.L[0] / 2;
    wa.tc = ftile_chunk(g, i, nrhs);
    wa.nchunk = ceil_div(g.L[3], wa.tc);
    wa.nrhs = nrhs;
    wa.bx = f.tx; wa.by = f.ty; wa.bz = f.tz;
    const int P = g.Ls / 2, R = 32 / P;
    wa.ngrp = ceil_div(nrhs, R);
    const dim3 grid(ftile_ntiles(g, i) * wa.ngrp * wa.nchunk);
    launch_ws(in, out, b, gauge, wa, partial, dagger, mode, grid, P, st);
    MG_LAUNCH_CHECK();
    return;
  }
  if (kind == DS_TPAIR) {
    const int i = ftile_of(g);
    const FTile& f = kFTiles[i];
    TMArgs ta;
    ta.d = a;
    ta.ntx = g.L[0] / f.tx; ta.nty = g.L[1] / f.ty; ta.ntz = g.L[2] / f.tz;
    ta.tc = ftile_chunk(g, i, nrhs);
    ta.fold = f.fold;
    ta.nrhs = nrhs;
    if (f.fold == 2) {  // the smallest z-slab count giving whole rounds of eight units; else plain order
      ta.zs = xcd_units_zs(ta.ntz, nrhs);
      if (ta.zs == 0 || ta.tc < g.L[3]) { ta.fold = 0; ta.zs = 1; }
    }
    const int nb = dslash_nblocks<C2>(g, nrhs);
    const dim3 grid = ta.fold ? dim3(nb * nrhs, 1) : dim3(nb, nrhs);
    launch_tpair(in, out, b, gauge, ta, partial, dagger, mode, grid, dim3(f.tx * f.ty * f.tz * g.Ls / 2), i, st);
    MG_LAUNCH_CHECK();
    return;
  }
  if (kind == DS_TMARCH) {
    TMArgs ta;
    ta.d = a;
    ta.ntx = g.L[0] / TMX; ta.nty = g.L[1] / TMY; ta.ntz = g.L[2] / TMZ;
    ta.tc = tmarch_chunk(g);
    dim3 grid(dslash_nblocks<C2>(g, nrhs), nrhs), blk(TMS * g.Ls);
#define MG_TM(DAG, MODE) \
  hipLaunchKernelGGL((k_dslash_tm<C2, DAG, MODE>), grid, blk, 0, st, in, out, b, gauge, ta, partial)
    if (!dagger && mode == 0) MG_TM(false, 0);
    else if (!dagger && mode == 1) MG_TM(false, 1);
    else if (dagger && mode == 0) MG_TM(true, 0);
    else MG_TM(true, 1);
#undef MG_TM
    MG_LAUNCH_CHECK();
    return;
  }
  dim3 grid(dslash_nblocks<C2>(g, nrhs), nrhs), blk(256);
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
                  double M5, double mf, int chi, hipStream_t st, bool dagger) {
  SplitArgs a;
  for (int m = 0; m < 4; ++m) { a.L[m] = g.L[m]; a.b[m] = block[m]; a.ph[m] = (float)g.bc[m]; }
  a.Ls = g.Ls; a.V4 = g.V4; a.V5 = g.V5; a.diag = 5.0 - M5; a.mf = mf; a.chi = chi;
  if (dagger)
    hipLaunchKernelGGL(k_dslash_split<true>, dim3(ceil_div(g.V5, 256)), dim3(256), 0, st, in, out9, gauge, a);
  else
    hipLaunchKernelGGL(k_dslash_split<false>, dim3(ceil_div(g.V5, 256)), dim3(256), 0, st, in, out9, gauge, a);
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
