// A third multigrid level under the squared two-level method (the paper's
// Sec. 2: the coarse solve of the V-cycle's step 3 may itself be the same
// multigrid, applied recursively).  The coarse operator A_c = P^+ D^+D P acts
// on coarse vectors [X][chi][k] (Vc sites, 2 Nv dof); the level below blocks
// the coarse lattice again:
//   * near-null vectors w_j of A_c (CG on A_c w = 0 from random starts, in
//     solver.hip), split by the coarse chirality index chi and orthonormalised
//     per (level-2 block, chi) panel here (k_orth2: Gram-Schmidt applied twice,
//     so the columns are the thin QR factor with positive real diagonal);
//   * R2 = W^+ and P2 = W on coarse vectors (k_restrict2, k_prolong2);
//   * A_cc = R2 A_c P2 read off column by column (k_probe2 + the squared
//     apply + k_restrict2 + k_scatter2) into the same 33-offset stencil form
//     as A_c, so the squared apply kernels serve the third level too.
// Level-2 vectors are [rhs][B][chi][j] (Vcc blocks, 2 Nv2 dof).
#include <algorithm>

#include "blas.h"
#include "ctx.h"
#include "vecops.h"

namespace mgdwf {

namespace {

// coarse site X of (block B, in-block site i); both in x-fastest order
__device__ __forceinline__ int site_of(const CoarseGeometry& c2, const int Lc[4], int B, int i) {
  const int bx = B % c2.Lc[0], by = (B / c2.Lc[0]) % c2.Lc[1], bz = (B / (c2.Lc[0] * c2.Lc[1])) % c2.Lc[2],
            bt = B / (c2.Lc[0] * c2.Lc[1] * c2.Lc[2]);
  const int ix = i % c2.block[0], iy = (i / c2.block[0]) % c2.block[1],
            iz = (i / (c2.block[0] * c2.block[1])) % c2.block[2], it = i / (c2.block[0] * c2.block[1] * c2.block[2]);
  const int x = bx * c2.block[0] + ix, y = by * c2.block[1] + iy, z = bz * c2.block[2] + iz,
            t = bt * c2.block[3] + it;
  return ((t * Lc[2] + z) * Lc[1] + y) * Lc[0] + x;
}

struct L2Geom {
  CoarseGeometry c2;  // level-2 lattice: Lc = blocks per direction, Vc = blocks, Nv = Nv2, block = block size
  int Lc[4];          // the coarse lattice
  int Vc, nv;         // coarse sites, coarse dof per chirality (Nv of level 1)
};

// Two passes of Gram-Schmidt over the panel (B, chi) of the nv2 vectors in
// W ([j][Vc][2][nv]); one workgroup per panel.  err gets 1 if a column is
// numerically dependent on the ones before it.
__global__ __launch_bounds__(256) void k_orth2(double2* __restrict__ W, L2Geom g, int nv2, int* err) {
  const int B = blockIdx.x >> 1, chi = blockIdx.x & 1;
  const int rows = g.c2.bvol * g.nv;
  const long long vs = (long long)g.Vc * 2 * g.nv;
  __shared__ double red[8];
  __shared__ double2 coef;
  auto at = [&](int j, int r) -> double2& {
    const int i = r / g.nv, k = r - i * g.nv;
    const int X = site_of(g.c2, g.Lc, B, i);
    return W[j * vs + ((long long)X * 2 + chi) * g.nv + k];
  };
  auto bsum = [&](double v) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
  };
  for (int j = 0; j < nv2; ++j) {
    double n0 = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      const double2 v = at(j, r);
      n0 += v.x * v.x + v.y * v.y;
    }
    n0 = bsum(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        double re = 0.0, im = 0.0;
        for (int r = threadIdx.x; r < rows; r += blockDim.x) {
          const double2 q = at(i, r), v = at(j, r);
          re += q.x * v.x + q.y * v.y;
          im += q.x * v.y - q.y * v.x;
        }
        re = bsum(re);
        im = bsum(im);
        if (threadIdx.x == 0) coef = make_double2(re, im);
        __syncthreads();
        const double2 cf = coef;
        for (int r = threadIdx.x; r < rows; r += blockDim.x) {
          const double2 q = at(i, r);
          double2& v = at(j, r);
          v.x -= cf.x * q.x - cf.y * q.y;
          v.y -= cf.x * q.y + cf.y * q.x;
        }
        __syncthreads();
      }
    double nn = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      const double2 v = at(j, r);
      nn += v.x * v.x + v.y * v.y;
    }
    nn = bsum(nn);
    if (!(nn > 1e-24 * n0) && threadIdx.x == 0) atomicOr(err, 1);
    const double s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      double2& v = at(j, r);
      v.x *= s;
      v.y *= s;
    }
    __syncthreads();
  }
}

// out[rhs][B][chi][j] = sum_{i in B, k} conj(W_j[X_i][chi][k]) in[rhs][X_i][chi][k];
// one workgroup per (B, rhs), one wavefront per output (chi, j) at a time.
template <class F2>
__global__ __launch_bounds__(256) void k_restrict2(const F2* __restrict__ W, const F2* __restrict__ in,
                                                   F2* __restrict__ out, L2Geom g, int nv2) {
  const int B = blockIdx.x, rhs = blockIdx.y;
  const int rows = g.c2.bvol * g.nv;
  const long long vs = (long long)g.Vc * 2 * g.nv, vs2 = (long long)g.c2.Vc * 2 * nv2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int o = wv; o < 2 * nv2; o += nw) {
    const int chi = o / nv2, j = o - chi * nv2;
    double re = 0.0, im = 0.0;
    for (int r = lane; r < rows; r += 64) {
      const int i = r / g.nv, k = r - i * g.nv;
      const long long e = ((long long)site_of(g.c2, g.Lc, B, i) * 2 + chi) * g.nv + k;
      const F2 w = W[j * vs + e], x = in[rhs * vs + e];
      re += (double)w.x * x.x + (double)w.y * x.y;
      im += (double)w.x * x.y - (double)w.y * x.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) out[rhs * vs2 + ((long long)B * 2 + chi) * nv2 + j] = cmk<F2>(re, im);
  }
}

// out[rhs][X][chi][k] (+)= sum_j W_j[X][chi][k] cc[rhs][B(X)][chi][j]
template <class F2>
__global__ void k_prolong2(const F2* __restrict__ W, const F2* __restrict__ cc, F2* __restrict__ out, L2Geom g,
                           int nv2, int nrhs, bool acc) {
  const long long vs = (long long)g.Vc * 2 * g.nv, vs2 = (long long)g.c2.Vc * 2 * nv2;
  const long long n = vs * nrhs;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int rhs = (int)(e / vs);
    const long long f = e - rhs * vs;
    const int X = (int)(f / (2 * g.nv));
    const int chi = (int)((f / g.nv) & 1);
    const int x = X % g.Lc[0], y = (X / g.Lc[0]) % g.Lc[1], z = (X / (g.Lc[0] * g.Lc[1])) % g.Lc[2],
              t = X / (g.Lc[0] * g.Lc[1] * g.Lc[2]);
    const int B = (((t / g.c2.block[3]) * g.c2.Lc[2] + z / g.c2.block[2]) * g.c2.Lc[1] + y / g.c2.block[1]) *
                      g.c2.Lc[0] + x / g.c2.block[0];
    const F2* cb = cc + rhs * vs2 + ((long long)B * 2 + chi) * nv2;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nv2; ++j) {
      const F2 w = W[j * vs + f], c = cb[j];
      re += (double)w.x * c.x - (double)w.y * c.y;
      im += (double)w.x * c.y + (double)w.y * c.x;
    }
    F2 r = cmk<F2>(re, im);
    if (acc) r = cadd(out[e], r);
    out[e] = r;
  }
}

// probes[(chi, j)] = W_j on (block B, chirality chi), zero elsewhere
__global__ void k_probe2(const double2* __restrict__ W, double2* __restrict__ probes, L2Geom g, int nv2, int B) {
  const long long vs = (long long)g.Vc * 2 * g.nv;
  const long long n = vs * 2 * nv2;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e / vs);
    const long long f = e - p * vs;
    const int chi = p / nv2, j = p - chi * nv2;
    const int X = (int)(f / (2 * g.nv));
    const int c = (int)((f / g.nv) & 1);
    const int x = X % g.Lc[0], y = (X / g.Lc[0]) % g.Lc[1], z = (X / (g.Lc[0] * g.Lc[1])) % g.Lc[2],
              t = X / (g.Lc[0] * g.Lc[1] * g.Lc[2]);
    const int BX = (((t / g.c2.block[3]) * g.c2.Lc[2] + z / g.c2.block[2]) * g.c2.Lc[1] + y / g.c2.block[1]) *
                       g.c2.Lc[0] + x / g.c2.block[0];
    probes[e] = (BX == B && c == chi) ? W[j * vs + f] : make_double2(0.0, 0.0);
  }
}

// Offset index (of the 33: self, +-mu, then for mu < nu the diagonals
// (+,+), (+,-), (-,+), (-,-)) that takes the coupling from destination D to
// source B, or -1 if D is not within one block in at most two directions.
// Where the level-2 extent is 1 or 2, several offsets name the same block:
// the coupling goes to the first of them in that order (a sign of + for an
// extent of 2, no step for an extent of 1), the others stay zero.
__device__ __forceinline__ int offset_index(const CoarseGeometry& c2, int D, int B) {
  int d[4], L[4] = {c2.Lc[0], c2.Lc[1], c2.Lc[2], c2.Lc[3]};
  int dd = D, bb = B;
  int cD[4], cB[4];
  for (int m = 0; m < 4; ++m) { cD[m] = dd % L[m]; dd /= L[m]; cB[m] = bb % L[m]; bb /= L[m]; }
  int nz = 0, dir[2] = {0, 0}, sg[2] = {0, 0};
  for (int m = 0; m < 4; ++m) {
    int s = ((cB[m] - cD[m]) % L[m] + L[m]) % L[m];  // 0 .. L - 1
    if (s == 0) d[m] = 0;
    else if (s == 1) d[m] = 1;                       // extent 2: the + step
    else if (s == L[m] - 1) d[m] = -1;
    else return -1;
    if (d[m] != 0) {
      if (nz == 2) return -1;
      dir[nz] = m;
      sg[nz] = d[m];
      ++nz;
    }
  }
  if (nz == 0) return 0;
  if (nz == 1) return 1 + 2 * dir[0] + (sg[0] < 0 ? 1 : 0);
  const int mu = dir[0], nu = dir[1];
  const int pair = mu == 0 ? nu - 1 : (mu == 1 ? 3 + (nu - 2) : 5);  // (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
  return 9 + 4 * pair + (sg[0] < 0 ? 2 : 0) + (sg[1] < 0 ? 1 : 0);
}

// Column (chi, j) of source block B: rr[(chi, j)][D][chi'][i] -> Acc[D][o][col][row]
__global__ void k_scatter2(const double2* __restrict__ rr, double2* __restrict__ Acc, CoarseGeometry c2, int B) {
  const int n2 = c2.n2;
  const long long vs2 = (long long)c2.Vc * n2;
  const long long n = vs2 * n2;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(e / vs2);
    const long long f = e - col * vs2;
    const int D = (int)(f / n2), row = (int)(f - (long long)D * n2);
    const int o = offset_index(c2, D, B);
    if (o < 0) continue;  // outside the stencil: the coupling is zero by the support of A_c
    Acc[(((long long)D * 33 + o) * n2 + col) * n2 + row] = rr[e];
  }
}

__global__ void k_zero2(double2* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

template <class F2>
__global__ void k_sub(F2* __restrict__ out, const F2* __restrict__ a, const F2* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = csub(a[i], b[i]);
}

L2Geom geom_of(const CoarseGeometry& cg, const CoarseGeometry& c2) {
  L2Geom g;
  g.c2 = c2;
  for (int m = 0; m < 4; ++m) g.Lc[m] = cg.Lc[m];
  g.Vc = cg.Vc;
  g.nv = cg.Nv;
  return g;
}

int nblk(long long n) { return (int)std::max<long long>(1, std::min<long long>(ceil_div(n, 256), 4096)); }

}  // namespace

bool orthonormalise_level2(double2* W, const CoarseGeometry& cg, const CoarseGeometry& c2, int* err_dev,
                           hipStream_t st) {
  MG_HIP(hipMemsetAsync(err_dev, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_orth2, dim3(2 * c2.Vc), dim3(256), 0, st, W, geom_of(cg, c2), c2.Nv, err_dev);
  MG_LAUNCH_CHECK();
  int err = 0;
  MG_HIP(hipMemcpyAsync(&err, err_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  return err == 0;
}

template <class F2>
void restrict2(const F2* W, const F2* in, F2* out, const CoarseGeometry& cg, const CoarseGeometry& c2, int nrhs,
               hipStream_t st) {
  hipLaunchKernelGGL((k_restrict2<F2>), dim3(c2.Vc, nrhs), dim3(256), 0, st, W, in, out, geom_of(cg, c2), c2.Nv);
  MG_LAUNCH_CHECK();
}

template <class F2>
void prolong2(const F2* W, const F2* cc, F2* out, bool acc, const CoarseGeometry& cg, const CoarseGeometry& c2,
              int nrhs, hipStream_t st) {
  const long long n = (long long)cg.Vc * cg.n2 * nrhs;
  hipLaunchKernelGGL((k_prolong2<F2>), dim3(nblk(n)), dim3(256), 0, st, W, cc, out, geom_of(cg, c2), c2.Nv, nrhs,
                     acc);
  MG_LAUNCH_CHECK();
}

template <class F2>
void sub_into(F2* out, const F2* a, const F2* b, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_sub<F2>), dim3(nblk(n)), dim3(256), 0, st, out, a, b, n);
  MG_LAUNCH_CHECK();
}
template void sub_into<double2>(double2*, const double2*, const double2*, long long, hipStream_t);
template void sub_into<float2>(float2*, const float2*, const float2*, long long, hipStream_t);

template void restrict2<double2>(const double2*, const double2*, double2*, const CoarseGeometry&,
                                 const CoarseGeometry&, int, hipStream_t);
template void restrict2<float2>(const float2*, const float2*, float2*, const CoarseGeometry&, const CoarseGeometry&,
                                int, hipStream_t);
template void prolong2<double2>(const double2*, const double2*, double2*, bool, const CoarseGeometry&,
                                const CoarseGeometry&, int, hipStream_t);
template void prolong2<float2>(const float2*, const float2*, float2*, bool, const CoarseGeometry&,
                               const CoarseGeometry&, int, hipStream_t);

void build_level2_op(const double2* Ac, const double2* W, double2* Acc, double2* probes, double2* applied,
                     double2* rr, const CoarseGeometry& cg, const CoarseGeometry& c2, hipStream_t st) {
  build_galerkin_op([&](const double2* x, double2* y, int n) { sq_apply64(Ac, x, y, cg, n, st); }, W, Acc, probes,
                    applied, rr, cg, c2, st);
}

void build_galerkin_op(const std::function<void(const double2*, double2*, int)>& apply, const double2* W,
                       double2* Acc, double2* probes, double2* applied, double2* rr, const CoarseGeometry& cg,
                       const CoarseGeometry& c2, hipStream_t st) {
  const long long entries = (long long)c2.Vc * 33 * c2.n2 * c2.n2;
  hipLaunchKernelGGL(k_zero2, dim3(nblk(entries)), dim3(256), 0, st, Acc, entries);
  MG_LAUNCH_CHECK();
  const L2Geom g = geom_of(cg, c2);
  const int np = c2.n2;  // probes per source block: (chi, j)
  const long long pn = (long long)cg.Vc * cg.n2 * np;
  for (int B = 0; B < c2.Vc; ++B) {
    hipLaunchKernelGGL(k_probe2, dim3(nblk(pn)), dim3(256), 0, st, W, probes, g, c2.Nv, B);
    MG_LAUNCH_CHECK();
    apply(probes, applied, np);
    restrict2<double2>(W, applied, rr, cg, c2, np, st);
    const long long sn = (long long)c2.Vc * c2.n2 * np;
    hipLaunchKernelGGL(k_scatter2, dim3(nblk(sn)), dim3(256), 0, st, rr, Acc, c2, B);
    MG_LAUNCH_CHECK();
  }
}

}  // namespace mgdwf
