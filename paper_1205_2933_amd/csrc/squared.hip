// Coarse operator of the squared operator, A_c = P^+ D^+ D P: construction and
// 33-point application.
//
// Paper, Sec. 3 (first paragraph): the multigrid and the CG control act on
// the squared operator D^+D; Sec. 4 (last paragraph): its coarse operator
// couples a coarse site to sites up to two hops away.  With 4D blocks of
// extent >= 2 spanning the fifth dimension, A_c couples X to X + o for 33
// offsets o: self, the eight unit neighbours +-mu and the 24 diagonal ones
// +-mu +-nu (mu < nu).  The two hops of one direction land on opposite faces
// of the block between them, so no coupling two blocks away in one
// direction exists.
//
// Construction, one basis column j = (chi, k) at a time for every block at
// once: the face-split D applied to the chirality-chi part of basis field k
// gives nine fields W_e (e = 0: the hops into each block from the block
// itself, with the diagonal and fifth-dimension terms; e = 1+2mu / 2+2mu:
// the hops into each block from its +mu / -mu neighbour).  The face-split
// D^+ of W_e gives nine fields Z_d (the hops into each block from its
// neighbour d).  Z_d restricted to block X is D^+_{X, X+d} D_{X+d, X+d+e} V_j,
// so R Z_d is column j of A_c[X][o] with o = delta_d + delta_e; pairs with
// o = +-2 mu are zero (opposite faces) and skipped.  The same assignment by
// direction keeps coarse extents 1 and 2 exact, as for the 9-point operator.
//
// A_c is Hermitian, so one stencil serves both A_c and its adjoint.  Storage:
// column-major 2Nv x 2Nv blocks [X][o], FP64 and an FP32 copy.
#include <algorithm>

#include "mg_internal.h"
#include "blas.h"
#include "vecops.h"

namespace mgdwf {

void dslash_split(const double2* in, double2* out9, const double2* gauge, const Geometry& g, const int block[4],
                  double M5, double mf, int chi, hipStream_t st, bool dagger);

namespace {

struct SqArgs {
  int Lc[4];
  int Vc;
  int n2;
  int off[33][4];  // offsets in (x, y, z, t)
};

// Offset index table: 0 self; 1 + 2 mu = +mu; 2 + 2 mu = -mu; then for mu < nu
// the four diagonals (+mu+nu, +mu-nu, -mu+nu, -mu-nu).
void offset_table(int off[33][4]) {
  int n = 0;
  for (int m = 0; m < 4; ++m) off[n][m] = 0;
  ++n;
  for (int mu = 0; mu < 4; ++mu)
    for (int sg : {1, -1}) {
      for (int m = 0; m < 4; ++m) off[n][m] = 0;
      off[n][mu] = sg;
      ++n;
    }
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu)
      for (int s1 : {1, -1})
        for (int s2 : {1, -1}) {
          for (int m = 0; m < 4; ++m) off[n][m] = 0;
          off[n][mu] = s1;
          off[n][nu] = s2;
          ++n;
        }
}

// index of delta_d + delta_e in the table, -1 for +-2 mu
int pair_offset(const int off[33][4], int d, int e) {
  int v[4] = {0, 0, 0, 0};
  for (int q : {d, e})
    if (q > 0) v[(q - 1) >> 1] += (q & 1) ? 1 : -1;
  for (int i = 0; i < 33; ++i) {
    bool eq = true;
    for (int m = 0; m < 4; ++m) eq = eq && off[i][m] == v[m];
    if (eq) return i;
  }
  return -1;
}

SqArgs sq_args(const CoarseGeometry& cg) {
  SqArgs a;
  for (int m = 0; m < 4; ++m) a.Lc[m] = cg.Lc[m];
  a.Vc = cg.Vc;
  a.n2 = cg.n2;
  offset_table(a.off);
  return a;
}

__device__ __forceinline__ int sq_neighbour(const SqArgs& a, int X, int o) {
  int c[4];
  int r = X;
  c[0] = r % a.Lc[0]; r /= a.Lc[0];
  c[1] = r % a.Lc[1]; r /= a.Lc[1];
  c[2] = r % a.Lc[2]; c[3] = r / a.Lc[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) c[m] = (c[m] + a.off[o][m] + a.Lc[m]) % a.Lc[m];
  return ((c[3] * a.Lc[2] + c[2]) * a.Lc[1] + c[1]) * a.Lc[0] + c[0];
}

// Ac[X][oi[d]] column j += coarse[d][X][row] for the nine d of one e
struct PairIdx {
  int oi[9];
};

__global__ void k_sq_scatter(const double2* __restrict__ coarse, double2* __restrict__ Ac, int Vc, int n2, int j,
                             PairIdx pi) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = 9LL * Vc * n2;
  if (i >= tot) return;
  const int row = (int)(i % n2);
  const long long t = i / n2;
  const int X = (int)(t % Vc), d = (int)(t / Vc);
  const int o = pi.oi[d];
  if (o < 0) return;
  double2* dst = Ac + (((long long)X * 33 + o) * n2 + j) * n2 + row;
  const double2 v = coarse[i];
  *dst = make_double2(dst->x + v.x, dst->y + v.y);
}

__global__ void k_zero64(double2* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

__global__ void k_sq_to_f32(const double2* __restrict__ in, float2* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// y[rhs](X) = sum_o A[X][o] x[rhs](X + o) for up to NR right-hand sides.
// Workgroup = one coarse site, nine wavefronts; wavefront w takes the
// offsets o = w, w + 9, w + 18, w + 27 (< 33); lane = output row.  Per offset
// the wavefront first copies the neighbour's coarse vectors of all NR
// right-hand sides into its own LDS panel ([col][rhs], zero past the last
// right-hand side), so the inner loop reads one coalesced matrix column per
// step from memory and the NR vector entries as LDS broadcasts.  The nine
// partial sums are added in a fixed order through LDS.
template <class MC2, class VC2, int NR>
__global__ __launch_bounds__(576) void k_sq_apply(const MC2* __restrict__ M, const VC2* __restrict__ x,
                                                  VC2* __restrict__ y, SqArgs a, int nrhs, int rhs0) {
  using T = typename real_of<VC2>::type;
  __shared__ VC2 xs[9][64 * NR];  // per wavefront: [col][rhs]; reused for the reduction at the end
  const int X = blockIdx.x;
  const int n2 = a.n2;
  const int w = threadIdx.x >> 6, row = threadIdx.x & 63;
  const int nr = min(NR, nrhs - rhs0);
  const long long vs = (long long)a.Vc * n2;
  VC2* panel = xs[w];
  VC2 acc[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) acc[j] = cmk<VC2>(0, 0);
  for (int k = 0; k < 4; ++k) {  // every wavefront takes four turns (the barriers need them all)
    const int o = w + 9 * k;
    const bool act = o < 33;
    if (act) {
      const int Y = sq_neighbour(a, X, o);
      const VC2* xv = x + (long long)rhs0 * vs + (long long)Y * n2;
      for (int e = row; e < NR * n2; e += 64) {
        const int j = e / n2, c = e - j * n2;
        panel[c * NR + j] = j < nr ? xv[(long long)j * vs + c] : cmk<VC2>(0, 0);
      }
    }
    __syncthreads();
    if (act && row < n2) {
      const MC2* Mo = M + ((long long)X * 33 + o) * n2 * n2;
      auto column = [&](int c) {
        const MC2 m = Mo[c * n2 + row];
        const VC2 mv = cmk<VC2>((T)m.x, (T)m.y);
#pragma unroll
        for (int j = 0; j < NR; ++j) cfma(acc[j], mv, panel[c * NR + j]);
      };
      if constexpr (sizeof(T) == 4 && NR >= 8) {
        // FP32: columns in flight, measured on 512 sites x 48 dof: at 12 RHS
        // 148 us with 16, 158 with 8, 202 with 4, 262 with none; at one
        // right-hand side 57 us with 8 and 66 with 16.  FP64 runs faster
        // without (307 against 338 us with 4)
#pragma unroll 16
        for (int c = 0; c < n2; ++c) column(c);
      } else if constexpr (sizeof(T) == 4) {
#pragma unroll 8
        for (int c = 0; c < n2; ++c) column(c);
      } else {
        for (int c = 0; c < n2; ++c) column(c);
      }
    }
    __syncthreads();
  }
  T (*red)[64][2] = reinterpret_cast<T (*)[64][2]>(&xs[0][0]);  // [rhs][row][re, im]
  for (int q = 0; q < 9; ++q) {
    if (w == q)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        if (q == 0) { red[j][row][0] = acc[j].x; red[j][row][1] = acc[j].y; }
        else { red[j][row][0] += acc[j].x; red[j][row][1] += acc[j].y; }
      }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nr * n2; i += blockDim.x) {
    const int j = i / n2, r = i % n2;
    y[(long long)(rhs0 + j) * vs + (long long)X * n2 + r] = cmk<VC2>(red[j][r][0], red[j][r][1]);
  }
}

// Canonical layout [X][o][row][col] from the internal column-major blocks.
__global__ void k_sq_canonical(const double2* __restrict__ in, double2* __restrict__ out, long long nblk, int n2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblk * n2 * n2) return;
  const long long blk = i / ((long long)n2 * n2);
  const int rc = (int)(i - blk * n2 * n2);
  const int row = rc / n2, col = rc % n2;
  out[i] = in[blk * n2 * n2 + (long long)col * n2 + row];
}

}  // namespace

size_t sq_coarse_entries(const CoarseGeometry& cg) { return (size_t)cg.Vc * 33 * cg.n2 * cg.n2; }

// Build A_c (FP64) into Ac; work9 and zwork9: 9 fine FP64 fields each; cwork:
// 9 Vc n2 complex; partial: restriction scratch for 9 right-hand sides.
void build_sq_coarse_op(const double2* Vhat, const double2* gauge, double2* Ac, double2* work9, double2* zwork9,
                        double2* cwork, double* partial, const Geometry& g, const CoarseGeometry& cg, double M5,
                        double mf, hipStream_t st) {
  const long long field = 12LL * g.V5;
  const long long nA = (long long)sq_coarse_entries(cg);
  hipLaunchKernelGGL(k_zero64, dim3(std::min<long long>(ceil_div(nA, 256), 8192)), dim3(256), 0, st, Ac, nA);
  MG_LAUNCH_CHECK();
  int off[33][4];
  offset_table(off);
  for (int chi = 0; chi < 2; ++chi)
    for (int k = 0; k < cg.Nv; ++k) {
      const int j = chi * cg.Nv + k;
      dslash_split(Vhat + k * field, work9, gauge, g, cg.block, M5, mf, chi, st, false);  // W_e, e = 0..8
      for (int e = 0; e < 9; ++e) {
        PairIdx pi;
        bool any = false;
        for (int d = 0; d < 9; ++d) {
          pi.oi[d] = pair_offset(off, d, e);
          any = any || pi.oi[d] >= 0;
        }
        if (!any) continue;
        dslash_split(work9 + (long long)e * field, zwork9, gauge, g, cg.block, M5, mf, -1, st, true);
        restrict_op<double2, double2>(Vhat, zwork9, cwork, partial, g, cg, 9, st);
        const long long tot = 9LL * cg.Vc * cg.n2;
        hipLaunchKernelGGL(k_sq_scatter, dim3(ceil_div(tot, 256)), dim3(256), 0, st, cwork, Ac, cg.Vc, cg.n2, j, pi);
        MG_LAUNCH_CHECK();
      }
    }
}

void sq_to_f32(const double2* Ac, float2* Ac32, const CoarseGeometry& cg, hipStream_t st) {
  const long long n = (long long)sq_coarse_entries(cg);
  hipLaunchKernelGGL(k_sq_to_f32, dim3(std::min<long long>(ceil_div(n, 256), 8192)), dim3(256), 0, st, Ac, Ac32, n);
  MG_LAUNCH_CHECK();
}

void sq_canonical(const double2* Ac, double2* out, const CoarseGeometry& cg, hipStream_t st) {
  const long long nblk = 33LL * cg.Vc, tot = nblk * cg.n2 * cg.n2;
  hipLaunchKernelGGL(k_sq_canonical, dim3(ceil_div(tot, 256)), dim3(256), 0, st, Ac, out, nblk, cg.n2);
  MG_LAUNCH_CHECK();
}

// The right-hand sides go in launches of at most NRMAX; each launch uses the
// smallest compiled panel width that holds its count (the inner loop runs
// over the whole width).
template <class MC2, class VC2, int NR>
static void sq_launch(const MC2* A, const VC2* x, VC2* y, const SqArgs& a, int Vc, int nrhs, int r0, hipStream_t st) {
  hipLaunchKernelGGL((k_sq_apply<MC2, VC2, NR>), dim3(Vc), dim3(576), 0, st, A, x, y, a, nrhs, r0);
  MG_LAUNCH_CHECK();
}

void sq_apply64(const double2* Ac, const double2* x, double2* y, const CoarseGeometry& cg, int nrhs, hipStream_t st) {
  if (cg.n2 > 64) fail(MGDWF_ERR_INVALID_ARG, "2*nvec above 64 is not supported");
  const SqArgs a = sq_args(cg);
  for (int r0 = 0; r0 < nrhs; r0 += 8) {
    const int nr = std::min(8, nrhs - r0);
    if (nr == 1) sq_launch<double2, double2, 1>(Ac, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr == 2) sq_launch<double2, double2, 2>(Ac, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr <= 4) sq_launch<double2, double2, 4>(Ac, x, y, a, cg.Vc, nrhs, r0, st);
    else sq_launch<double2, double2, 8>(Ac, x, y, a, cg.Vc, nrhs, r0, st);
  }
}

void sq_apply32(const float2* Ac32, const float2* x, float2* y, const CoarseGeometry& cg, int nrhs, hipStream_t st) {
  if (cg.n2 > 64) fail(MGDWF_ERR_INVALID_ARG, "2*nvec above 64 is not supported");
  const SqArgs a = sq_args(cg);
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = std::min(16, nrhs - r0);
    if (nr == 1) sq_launch<float2, float2, 1>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr == 2) sq_launch<float2, float2, 2>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr <= 4) sq_launch<float2, float2, 4>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr <= 8) sq_launch<float2, float2, 8>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
    else if (nr <= 12) sq_launch<float2, float2, 12>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
    else sq_launch<float2, float2, 16>(Ac32, x, y, a, cg.Vc, nrhs, r0, st);
  }
}

}  // namespace mgdwf
