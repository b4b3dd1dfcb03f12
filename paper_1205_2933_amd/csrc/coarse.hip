// Coarse operator D_c = R D P: construction and 9-point application.
//
// Paper, Sec. 2 (third V-cycle step): the coarse problem uses R A P.  Sec. 4:
// coarsening the unsquared operator keeps a one-hop stencil; with blocks that
// span the fifth dimension, a coarse site couples to itself and its eight 4D
// neighbours only.
//
// Construction: column j = (chi', k') of every block is obtained at once for
// all blocks: the face-split operator applied to the chirality-chi' part of
// basis field k' gives nine fields -- the self part (diagonal, fifth-dimension
// hops and block-interior hops) and the eight block-face hops; restricting
// field d gives column j of Dc[B][d] for every block B.  A hop from x to x+mu
// belongs to d = +mu exactly when x is on the upper face of its block, a hop
// to x-mu to d = -mu exactly when x is on the lower face, which keeps the
// stencil exact when a coarse extent is 1 or 2 (neighbours coincide).
//
// Internal storage of a block: column major, element (row r, col c) of
// Dc[X][d] at ((X * 9 + d) * n2 + c) * n2 + r, so that lane r of a wavefront
// reads consecutive addresses for a fixed column.
#include "mg_internal.h"
#include "blas.h"

namespace mgdwf {

// from transfer.hip
template <class C2, class CC2>
void restrict_op(const C2* V, const C2* x, CC2* coarse, double* partial, const Geometry& g,
                 const CoarseGeometry& cg, int nrhs, hipStream_t st);
// from dslash.hip
void dslash_split(const double2* in, double2* out9, const double2* gauge, const Geometry& g, const int block[4],
                  double M5, double mf, int chi, hipStream_t st);

namespace {

// Dc column j for all (X, d): coarse[d][X][row] (from the restriction of field d)
// -> Dc[((X*9 + d)*n2 + j)*n2 + row].
__global__ void k_scatter_column(const double2* __restrict__ coarse, double2* __restrict__ Dc, int Vc,
                                 int n2, int j) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = 9LL * Vc * n2;
  if (i >= tot) return;
  int row = (int)(i % n2);
  long long t = i / n2;
  int X = (int)(t % Vc), d = (int)(t / Vc);
  Dc[(((long long)X * 9 + d) * n2 + j) * n2 + row] = coarse[i];
}

struct CoarseArgs {
  int Lc[4];
  int Vc;
  int n2;
};

__device__ __forceinline__ int coarse_neighbour(const CoarseArgs& a, int X, int d) {
  if (d == 0) return X;
  const int mu = (d - 1) >> 1;
  const int sgn = (d & 1) ? 1 : -1;  // d = 1 + 2 mu is +mu
  int c[4];
  int r = X;
  c[0] = r % a.Lc[0]; r /= a.Lc[0];
  c[1] = r % a.Lc[1]; r /= a.Lc[1];
  c[2] = r % a.Lc[2]; c[3] = r / a.Lc[2];
  c[mu] = (c[mu] + sgn + a.Lc[mu]) % a.Lc[mu];
  return ((c[3] * a.Lc[2] + c[2]) * a.Lc[1] + c[1]) * a.Lc[0] + c[0];
}

// y = D_c x (DAG false) or D_c^+ x; one workgroup (4 wavefronts) per coarse
// site and RHS; wavefront w handles d = w, w+4, w+8; lane = output row.
// Accumulation in FP64 for double2, FP32 for float2.
template <class MC2, class VC2, bool DAG>
__global__ __launch_bounds__(256) void k_coarse_apply(const MC2* __restrict__ Dc, const VC2* __restrict__ x,
                                                      VC2* __restrict__ y, CoarseArgs a) {
  using T = typename real_of<VC2>::type;
  __shared__ T red[4][64][2];
  const int X = blockIdx.x, rhs = blockIdx.y;
  const int n2 = a.n2;
  const int w = threadIdx.x >> 6, row = threadIdx.x & 63;
  const long long voff = (long long)rhs * a.Vc * n2;
  VC2 acc = cmk<VC2>(0, 0);
  if (row < n2) {
    for (int d = w; d < 9; d += 4) {
      if (!DAG) {
        const int Y = coarse_neighbour(a, X, d);
        const MC2* M = Dc + ((long long)X * 9 + d) * n2 * n2;
        const VC2* xv = x + voff + (long long)Y * n2;
        for (int c = 0; c < n2; ++c) {
          MC2 m = M[c * n2 + row];
          cfma(acc, cmk<VC2>((T)m.x, (T)m.y), xv[c]);
        }
      } else {
        // (D_c^+ x)(X) = sum_d Dc[X - delta_d][d]^+ x(X - delta_d)
        const int dopp = (d == 0) ? 0 : (((d - 1) ^ 1) + 1);
        const int Y = coarse_neighbour(a, X, dopp);
        const MC2* M = Dc + ((long long)Y * 9 + d) * n2 * n2;
        const VC2* xv = x + voff + (long long)Y * n2;
        for (int c = 0; c < n2; ++c) {
          MC2 m = M[row * n2 + c];  // element (c, row) of Dc[Y][d]
          cfmac(acc, cmk<VC2>((T)m.x, (T)m.y), xv[c]);
        }
      }
    }
  }
  red[w][row][0] = acc.x;
  red[w][row][1] = acc.y;
  __syncthreads();
  if (threadIdx.x < n2) {
    const int r = threadIdx.x;
    VC2 s = cmk<VC2>(red[0][r][0] + red[1][r][0] + red[2][r][0] + red[3][r][0],
                     red[0][r][1] + red[1][r][1] + red[2][r][1] + red[3][r][1]);
    y[voff + (long long)X * n2 + r] = s;
  }
}

__global__ void k_dc_to_f32(const double2* __restrict__ in, float2* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

}  // namespace

// Build the FP64 coarse operator.  Vhat: orthonormal basis (Nv FP64 fields);
// work9: 9 fine FP64 fields; cwork: 9 * Vc * n2 complex; partial: restriction
// scratch for 9 right-hand sides.
void build_coarse_op(const double2* Vhat, const double2* gauge, double2* Dc, double2* work9, double2* cwork,
                     double* partial, const Geometry& g, const CoarseGeometry& cg, double M5, double mf,
                     hipStream_t st) {
  const long long field = 12LL * g.V5;
  for (int chi = 0; chi < 2; ++chi)
    for (int k = 0; k < cg.Nv; ++k) {
      dslash_split(Vhat + k * field, work9, gauge, g, cg.block, M5, mf, chi, st);
      restrict_op<double2, double2>(Vhat, work9, cwork, partial, g, cg, 9, st);
      const int j = chi * cg.Nv + k;
      long long tot = 9LL * cg.Vc * cg.n2;
      hipLaunchKernelGGL(k_scatter_column, dim3(ceil_div(tot, 256)), dim3(256), 0, st, cwork, Dc, cg.Vc,
                         cg.n2, j);
      MG_LAUNCH_CHECK();
    }
}

void coarse_to_f32(const double2* Dc64, float2* Dc32, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_to_f32, dim3(std::min(ceil_div(n, 256), 8192)), dim3(256), 0, st, Dc64, Dc32, n);
  MG_LAUNCH_CHECK();
}

template <class MC2, class VC2>
void coarse_apply(const MC2* Dc, const VC2* x, VC2* y, bool dagger, const CoarseGeometry& cg, int nrhs,
                  hipStream_t st) {
  if (cg.n2 > 64) fail(MGDWF_ERR_INVALID_ARG, "2*nvec above 64 is not supported");
  CoarseArgs a;
  for (int m = 0; m < 4; ++m) a.Lc[m] = cg.Lc[m];
  a.Vc = cg.Vc; a.n2 = cg.n2;
  dim3 grid(cg.Vc, nrhs);
  if (dagger) hipLaunchKernelGGL((k_coarse_apply<MC2, VC2, true>), grid, dim3(256), 0, st, Dc, x, y, a);
  else hipLaunchKernelGGL((k_coarse_apply<MC2, VC2, false>), grid, dim3(256), 0, st, Dc, x, y, a);
  MG_LAUNCH_CHECK();
}

template void coarse_apply<double2, double2>(const double2*, const double2*, double2*, bool,
                                             const CoarseGeometry&, int, hipStream_t);
template void coarse_apply<float2, float2>(const float2*, const float2*, float2*, bool, const CoarseGeometry&,
                                           int, hipStream_t);

}  // namespace mgdwf
