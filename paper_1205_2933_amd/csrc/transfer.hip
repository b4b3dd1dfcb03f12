// Restrictor R, prolongator P and the block orthonormalisation of the basis.
//
// Paper, Sec. 1: R maps fine to coarse vectors, P back, with R P = 1 on the
// coarse space.  Sec. 2: the near-null vectors are cut into blocks, one per
// coarse site, and every block spans the whole fifth dimension.  With the
// basis orthonormal on every (block, chirality) panel, R = P^+ and R P = 1.
//
// Basis storage: Nv fine fields in the internal fine layout; column
// (B, chi, k) is field k restricted to block B and to the spins of chi
// (chi = 0: spins 0,1; chi = 1: spins 2,3).
#include "mg_internal.h"
#include "blas.h"

namespace mgdwf {

namespace {

struct BlockArgs {
  int L[4];
  int Ls;
  int V4;
  int V5;
  int b[4];
  int Lc[4];
  int Vc;
  int bvol;
  int Nv;
};

BlockArgs make_args(const Geometry& g, const CoarseGeometry& cg) {
  BlockArgs a;
  for (int m = 0; m < 4; ++m) { a.L[m] = g.L[m]; a.b[m] = cg.block[m]; a.Lc[m] = cg.Lc[m]; }
  a.Ls = g.Ls; a.V4 = g.V4; a.V5 = g.V5; a.Vc = cg.Vc; a.bvol = cg.bvol; a.Nv = cg.Nv;
  return a;
}

// 4D site of the j-th site (block-local lexicographic, x fastest) of coarse site B.
__device__ __forceinline__ int block_site(const BlockArgs& a, int B, int j) {
  int X = B % a.Lc[0]; int r = B / a.Lc[0];
  int Y = r % a.Lc[1]; r /= a.Lc[1];
  int Z = r % a.Lc[2]; int T = r / a.Lc[2];
  int xx = j % a.b[0]; int q = j / a.b[0];
  int yy = q % a.b[1]; q /= a.b[1];
  int zz = q % a.b[2]; int tt = q / a.b[2];
  int x = X * a.b[0] + xx, y = Y * a.b[1] + yy, z = Z * a.b[2] + zz, t = T * a.b[3] + tt;
  return ((t * a.L[2] + z) * a.L[1] + y) * a.L[0] + x;
}

__device__ __forceinline__ int coarse_of(const BlockArgs& a, int x4) {
  int x = x4 % a.L[0]; int r = x4 / a.L[0];
  int y = r % a.L[1]; r /= a.L[1];
  int z = r % a.L[2]; int t = r / a.L[2];
  return ((t / a.b[3] * a.Lc[2] + z / a.b[2]) * a.Lc[1] + y / a.b[1]) * a.Lc[0] + x / a.b[0];
}

constexpr int KC = 8;      // basis vectors per register chunk in R
constexpr int NSPLIT = 4;  // workgroups per coarse site in R

// Partial restriction: workgroup (B, split) sums its share of block B for
// every (chi, k): partial[((rhs * Vc + B) * NSPLIT + split) * 2 * n2 + ...].
template <class C2>
__global__ __launch_bounds__(256) void k_restrict(const C2* __restrict__ V, const C2* __restrict__ x,
                                                  double* __restrict__ partial, BlockArgs a) {
  const int B = blockIdx.x / NSPLIT, split = blockIdx.x % NSPLIT;
  const int rhs = blockIdx.y;
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  x += rhs * field;
  const int n5 = a.bvol * a.Ls;
  const int n2 = 2 * a.Nv;
  double* out = partial + (((long long)rhs * a.Vc + B) * NSPLIT + split) * 2 * n2;
  __shared__ double red[4][2 * KC * 2];
  for (int k0 = 0; k0 < a.Nv; k0 += KC) {
    double acc[2][KC][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) { acc[h][kk][0] = 0.0; acc[h][kk][1] = 0.0; }
    for (int j = split * 256 + threadIdx.x; j < n5; j += 256 * NSPLIT) {
      const int jl = j / a.Ls, s = j - jl * a.Ls;
      const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
      C2 xv[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) xv[c] = x[c * V5 + i5];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        if (k < a.Nv) {
          const C2* Vk = V + (long long)k * field;
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            C2 v = Vk[c * V5 + i5];
            const int h = c / 6;
            acc[h][kk][0] += (double)v.x * xv[c].x + (double)v.y * xv[c].y;
            acc[h][kk][1] += (double)v.x * xv[c].y - (double)v.y * xv[c].x;
          }
        }
      }
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          double v = wave_sum(acc[h][kk][ri]);
          if (l == 0) red[w][(h * KC + kk) * 2 + ri] = v;
        }
    __syncthreads();
    if (threadIdx.x < 2 * KC * 2) {
      const int h = threadIdx.x / (2 * KC), kk = (threadIdx.x / 2) % KC, ri = threadIdx.x & 1;
      const int k = k0 + kk;
      double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
      if (k < a.Nv) out[(h * a.Nv + k) * 2 + ri] = s;
    }
    __syncthreads();
  }
}

// coarse[(rhs * Vc + B) * n2 + row] = sum over splits, in fixed order.
// Multi-RHS restriction: as k_restrict, for RG right-hand sides per workgroup
// (blockIdx.y picks the group).  A thread keeps the rows of its RG right-hand
// sides in registers while it sweeps KR basis columns, so the basis is read
// once per group of right-hand sides and x once per KR columns.  FP32 fields
// are read two s-values per 16-byte load.  Partial sums in the field's
// precision per thread (a handful of rows), FP64 across threads; same partial
// layout as k_restrict.
template <class C2, int RG, int KR>
__global__ __launch_bounds__(256) void k_restrict_mr(const C2* __restrict__ V, const C2* __restrict__ x,
                                                     double* __restrict__ partial, BlockArgs a, int nrhs) {
  using T = typename real_of<C2>::type;
  constexpr int W = sizeof(T) == 4 ? 2 : 1;  // consecutive s per load
  const int B = blockIdx.x / NSPLIT, split = blockIdx.x % NSPLIT;
  const int r0 = blockIdx.y * RG;
  const int nr = min(RG, nrhs - r0);
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  const int n5 = a.bvol * a.Ls;
  const int n2 = 2 * a.Nv;
  __shared__ double red[4][RG * 2 * KR * 2];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  auto load = [&](const C2* f, long long off, C2 out[W]) {
    if constexpr (W == 2) {
      const float4 q = *reinterpret_cast<const float4*>(f + off);
      out[0] = cmk<C2>(q.x, q.y);
      out[1] = cmk<C2>(q.z, q.w);
    } else {
      out[0] = f[off];
    }
  };
  for (int k0 = 0; k0 < a.Nv; k0 += KR) {
    T acc[RG][2][KR][2];
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) { acc[r][h][kk][0] = 0; acc[r][h][kk][1] = 0; }
    for (int j = split * 256 + threadIdx.x; j * W < n5; j += 256 * NSPLIT) {
      const int jj = j * W;
      const int jl = jj / a.Ls, s = jj - jl * a.Ls;
      const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
      C2 xv[RG][12][W];
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          if (r < nr) load(x + (long long)(r0 + r) * field, c * V5 + i5, xv[r][c]);
          else for (int q = 0; q < W; ++q) xv[r][c][q] = cmk<C2>(0, 0);
        }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int k = k0 + kk;
        if (k < a.Nv) {
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            C2 v[W];
            load(V + (long long)k * field, c * V5 + i5, v);
            const int h = c / 6;
#pragma unroll
            for (int r = 0; r < RG; ++r)
#pragma unroll
              for (int q = 0; q < W; ++q) {
                acc[r][h][kk][0] += v[q].x * xv[r][c][q].x + v[q].y * xv[r][c][q].y;
                acc[r][h][kk][1] += v[q].x * xv[r][c][q].y - v[q].y * xv[r][c][q].x;
              }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int kk = 0; kk < KR; ++kk)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri) {
            const double v = wave_sum((double)acc[r][h][kk][ri]);
            if (l == 0) red[w][((r * 2 + h) * KR + kk) * 2 + ri] = v;
          }
    __syncthreads();
    for (int q = threadIdx.x; q < RG * 2 * KR * 2; q += 256) {
      const int r = q / (2 * KR * 2), h = (q / (KR * 2)) % 2, kk = (q / 2) % KR, ri = q & 1;
      const int k = k0 + kk;
      const double sum = red[0][q] + red[1][q] + red[2][q] + red[3][q];
      if (k < a.Nv && r < nr)
        partial[(((long long)(r0 + r) * a.Vc + B) * NSPLIT + split) * 2 * n2 + (h * a.Nv + k) * 2 + ri] = sum;
    }
    __syncthreads();
  }
}

// Multi-RHS restriction, FP32, basis and fields each read once: a 768-thread
// workgroup owns a quarter of block B's rows.  Per chunk of 64 rows the
// workgroup stages the rows of up to RX right-hand sides in LDS (layout
// [rhs][component][row], so a wavefront reads 64 consecutive rows); wave w
// then accumulates basis columns w and w + 12 against every staged
// right-hand side, lane = row.  Sums in FP32 within the workgroup (16 chunks
// x 6 components per lane, then 64 lanes), FP64 across workgroups; same
// partial layout as k_restrict.
constexpr int RX = 12, RW = 12, RT = 64 * RW;
__global__ __launch_bounds__(RT) void k_restrict_lds(const float2* __restrict__ V, const float2* __restrict__ x,
                                                     double* __restrict__ partial, BlockArgs a, int nrhs) {
  constexpr int KW = 2;  // columns per wave: 12 waves x 2 = 24 >= Nv
  __shared__ float2 xs[RX * 12 * 64];
  const int B = blockIdx.x / NSPLIT, split = blockIdx.x % NSPLIT;
  const int r0 = blockIdx.y * RX;
  const int nr = min(RX, nrhs - r0);
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  const int n5 = a.bvol * a.Ls;
  const int n2 = 2 * a.Nv;
  const int per = n5 / NSPLIT;  // rows of this workgroup (n5 divides by 256)
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  float acc[KW][RX][2][2];
#pragma unroll
  for (int j = 0; j < KW; ++j)
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h) { acc[j][r][h][0] = 0.f; acc[j][r][h][1] = 0.f; }
  for (int c0 = 0; c0 < per; c0 += 64) {
    __syncthreads();  // the previous chunk's rows are consumed
    for (int q = threadIdx.x; q < nr * 12 * 64; q += RT) {
      const int row = q & 63, rc = q >> 6;  // rc = r * 12 + component
      const int jj = split * per + c0 + row;
      const int jl = jj / a.Ls, s = jj - jl * a.Ls;
      const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
      const int r = rc / 12, c = rc - r * 12;
      xs[q] = x[(long long)(r0 + r) * field + c * V5 + i5];
    }
    __syncthreads();
    const int jj = split * per + c0 + l;
    const int jl = jj / a.Ls, s = jj - jl * a.Ls;
    const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const int h = c / 6;
      float2 v[KW];
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const int k = w + RW * j;
        v[j] = k < a.Nv ? V[(long long)k * field + c * V5 + i5] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        if (r < nr) {
          const float2 xv = xs[(r * 12 + c) * 64 + l];
#pragma unroll
          for (int j = 0; j < KW; ++j) {
            acc[j][r][h][0] += v[j].x * xv.x + v[j].y * xv.y;
            acc[j][r][h][1] += v[j].x * xv.y - v[j].y * xv.x;
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = w + RW * j;
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          const float sum = wave_sum(acc[j][r][h][ri]);
          if (l == 0 && k < a.Nv && r < nr)
            partial[(((long long)(r0 + r) * a.Vc + B) * NSPLIT + split) * 2 * n2 + (h * a.Nv + k) * 2 + ri] = sum;
        }
  }
}

template <class C2>
__global__ void k_restrict_finalize(const double* __restrict__ partial, C2* __restrict__ coarse,
                                    int Vc, int n2, int nrhs) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = (long long)nrhs * Vc * n2;
  if (i >= tot) return;
  long long site = i / n2;
  int row = (int)(i - site * n2);
  const double* p = partial + site * NSPLIT * 2 * n2;
  double re = 0.0, im = 0.0;
  for (int sp = 0; sp < NSPLIT; ++sp) {
    re += p[sp * 2 * n2 + 2 * row];
    im += p[sp * 2 * n2 + 2 * row + 1];
  }
  C2 v;
  v.x = re; v.y = im;
  coarse[i] = v;
}

// out = P c (ACC false) or out += P c (ACC true); one thread per 5D site.
template <class C2, class CC2, bool ACC>
__global__ __launch_bounds__(256) void k_prolong(const C2* __restrict__ V, const CC2* __restrict__ cvec,
                                                 C2* __restrict__ out, BlockArgs a) {
  using T = typename real_of<C2>::type;
  const long long i5 = (long long)blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  if (i5 >= V5) return;
  out += rhs * field;
  const int n2 = 2 * a.Nv;
  const int x4 = (int)(i5 / a.Ls);
  const CC2* cb = cvec + ((long long)rhs * a.Vc + coarse_of(a, x4)) * n2;
  C2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = cmk<C2>(0, 0);
  for (int k = 0; k < a.Nv; ++k) {
    const C2* Vk = V + (long long)k * field;
    CC2 c0 = cb[k], c1 = cb[a.Nv + k];
    C2 w0 = cmk<C2>((T)c0.x, (T)c0.y), w1 = cmk<C2>((T)c1.x, (T)c1.y);
#pragma unroll
    for (int c = 0; c < 12; ++c) cfma(acc[c], Vk[c * V5 + i5], c < 6 ? w0 : w1);
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (ACC) out[c * V5 + i5] = cadd(out[c * V5 + i5], acc[c]);
    else out[c * V5 + i5] = acc[c];
  }
}

// Multi-RHS prolongation: each thread reads its site's basis rows once and
// applies them to RG right-hand sides (blockIdx.y picks the group).
template <class C2, class CC2, bool ACC, int RG>
__global__ __launch_bounds__(256) void k_prolong_mr(const C2* __restrict__ V, const CC2* __restrict__ cvec,
                                                    C2* __restrict__ out, BlockArgs a, int nrhs) {
  using T = typename real_of<C2>::type;
  const long long i5 = (long long)blockIdx.x * 256 + threadIdx.x;
  const int r0 = blockIdx.y * RG;
  const int nr = min(RG, nrhs - r0);
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  if (i5 >= V5) return;
  const int n2 = 2 * a.Nv;
  const int x4 = (int)(i5 / a.Ls);
  const int cs = coarse_of(a, x4);
  C2 acc[RG][12];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[r][c] = cmk<C2>(0, 0);
  for (int k = 0; k < a.Nv; ++k) {
    C2 v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = V[(long long)k * field + c * V5 + i5];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      if (r < nr) {
        const CC2* cb = cvec + ((long long)(r0 + r) * a.Vc + cs) * n2;
        const CC2 c0 = cb[k], c1 = cb[a.Nv + k];
        const C2 w0 = cmk<C2>((T)c0.x, (T)c0.y), w1 = cmk<C2>((T)c1.x, (T)c1.y);
#pragma unroll
        for (int c = 0; c < 12; ++c) cfma(acc[r][c], v[c], c < 6 ? w0 : w1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    if (r < nr) {
      C2* o = out + (long long)(r0 + r) * field;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        if (ACC) o[c * V5 + i5] = cadd(o[c * V5 + i5], acc[r][c]);
        else o[c * V5 + i5] = acc[r][c];
      }
    }
  }
}

// Prolongation for up to RW right-hand sides in one pass over the basis: one
// thread per fine component (spin-colour c, 5D site), all right-hand sides
// accumulated in registers, so each basis entry is read once per launch
// (k_prolong_mr reads the basis once per group of RG right-hand sides).
// Thread i covers c = i / V5 and i5 = i % V5, the basis layout's own order,
// so the basis loads and the output stores are unit-stride.  When the
// wavefront lies in one block and one chirality (64 consecutive 5D sites of
// one spin-colour component: always so when Ls x block_x is a multiple of 64)
// its coefficients are wave-uniform and come through scalar loads; otherwise
// every lane loads its own through the cache.
template <class C2, class CC2, bool ACC, int RW>
__global__ __launch_bounds__(256) void k_prolong_wide(const C2* __restrict__ V, const CC2* __restrict__ cvec,
                                                      C2* __restrict__ out, BlockArgs a, int nrhs) {
  using T = typename real_of<C2>::type;
  const long long V5 = a.V5;
  const long long field = 12 * V5;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= field) return;
  const int c = (int)(i / V5);
  const long long i5 = i - (long long)c * V5;
  const int n2 = 2 * a.Nv;
  const int cs = coarse_of(a, (int)(i5 / a.Ls));
  const int chi_off = c < 6 ? 0 : a.Nv;  // spins 0, 1: P+ columns; spins 2, 3: P- columns
  C2 acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = cmk<C2>(0, 0);
  const long long cstride = (long long)a.Vc * n2;
  const int cs0 = __builtin_amdgcn_readfirstlane(cs), off0 = __builtin_amdgcn_readfirstlane(chi_off);
  if (__all(cs == cs0 && chi_off == off0)) {
    const CC2* cb = cvec + (long long)cs0 * n2 + off0;  // wave-uniform
    int k = 0;
    for (; k + 4 <= a.Nv; k += 4) {  // four k at a time: wider scalar loads, more loads in flight
      C2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = V[(long long)(k + q) * field + i];
#pragma unroll
      for (int r = 0; r < RW; ++r)
        if (r < nrhs) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const CC2 w = cb[r * cstride + k + q];
            cfma(acc[r], v[q], cmk<C2>((T)w.x, (T)w.y));
          }
        }
    }
    for (; k < a.Nv; ++k) {
      const C2 v = V[(long long)k * field + i];
#pragma unroll
      for (int r = 0; r < RW; ++r)
        if (r < nrhs) {
          const CC2 w = cb[r * cstride + k];
          cfma(acc[r], v, cmk<C2>((T)w.x, (T)w.y));
        }
    }
  } else {
    const CC2* cb = cvec + (long long)cs * n2 + chi_off;
    for (int k = 0; k < a.Nv; ++k) {
      const C2 v = V[(long long)k * field + i];
#pragma unroll
      for (int r = 0; r < RW; ++r)
        if (r < nrhs) {
          const CC2 w = cb[r * cstride + k];
          cfma(acc[r], v, cmk<C2>((T)w.x, (T)w.y));
        }
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r)
    if (r < nrhs) {
      C2* o = out + (long long)r * field + i;
      *o = ACC ? cadd(*o, acc[r]) : acc[r];
    }
}

// ---------------------------------------------------------------- CholQR
// Gram matrix of every (block, chirality) panel: G[(B*2 + chi)][i][j] = <v_i, v_j>
// over the block's sites, all s, the six spin-colour components of chi.
constexpr int GRAM_ROWS = 16;  // fine rows staged per LDS chunk (one row = one 5D site, 6 comps)

__global__ __launch_bounds__(256) void k_gram(const double2* __restrict__ V, double2* __restrict__ G,
                                              BlockArgs a) {
  extern __shared__ double2 lds[];  // [GRAM_ROWS * 6][Nv]
  const int B = blockIdx.x >> 1, chi = blockIdx.x & 1;
  const int Nv = a.Nv;
  const long long V5 = a.V5, field = 12 * V5;
  const int n5 = a.bvol * a.Ls;
  const int npair = Nv * Nv;
  double2 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < n5; j0 += GRAM_ROWS) {
    // stage GRAM_ROWS sites x 6 comps x Nv vectors
    for (int e = threadIdx.x; e < GRAM_ROWS * 6 * Nv; e += 256) {
      const int k = e % Nv, rc = e / Nv, c6 = rc % 6, jj = rc / 6;
      const int j = j0 + jj;
      double2 v = make_double2(0.0, 0.0);
      if (j < n5) {
        const int jl = j / a.Ls, s = j - jl * a.Ls;
        const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
        v = V[k * field + (long long)(chi * 6 + c6) * V5 + i5];
      }
      lds[rc * Nv + k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = threadIdx.x + q * 256;
      if (p < npair) {
        const int i = p / Nv, jc = p % Nv;
        double2 s = acc[q];
        for (int r = 0; r < GRAM_ROWS * 6; ++r) cfmac(s, lds[r * Nv + i], lds[r * Nv + jc]);
        acc[q] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = threadIdx.x + q * 256;
    if (p < npair) G[(long long)blockIdx.x * npair + p] = acc[q];
  }
}

// Cholesky G = R^+ R (R upper, positive real diagonal) and W = R^{-1}, one
// thread per panel.  status[panel] = 1 when a pivot is not positive or a
// column keeps less than 1e-7 of its norm (numerically rank deficient).
__global__ void k_chol_inv(const double2* __restrict__ G, double2* __restrict__ W, int* __restrict__ status,
                           int npanel, int Nv) {
  const int pnl = blockIdx.x * blockDim.x + threadIdx.x;
  if (pnl >= npanel) return;
  const double2* g = G + (long long)pnl * Nv * Nv;
  double2* w = W + (long long)pnl * Nv * Nv;
  // R is built in w's storage row by row first, then inverted in place.
  int bad = 0;
  // R[i][j] for i <= j:  R_ii = sqrt(G_ii - sum_k |R_ki|^2),  R_ij = (G_ij - sum_k conj(R_ki) R_kj) / R_ii
  for (int i = 0; i < Nv; ++i) {
    double d = g[i * Nv + i].x;
    for (int k = 0; k < i; ++k) { double2 r = w[k * Nv + i]; d -= r.x * r.x + r.y * r.y; }
    if (!(d > 0.0) || d < 1e-14 * g[i * Nv + i].x) { bad = 1; d = 1.0; }
    const double rii = sqrt(d);
    w[i * Nv + i] = make_double2(rii, 0.0);
    for (int j = i + 1; j < Nv; ++j) {
      double2 s = g[i * Nv + j];
      for (int k = 0; k < i; ++k) {
        double2 rki = w[k * Nv + i], rkj = w[k * Nv + j];
        s.x -= rki.x * rkj.x + rki.y * rkj.y;
        s.y -= rki.x * rkj.y - rki.y * rkj.x;
      }
      w[i * Nv + j] = make_double2(s.x / rii, s.y / rii);
    }
    for (int j = 0; j < i; ++j) w[i * Nv + j] = make_double2(0.0, 0.0);
  }
  // invert the upper-triangular R in place, column by column from the right:
  // X = R^{-1}: X_jj = 1/R_jj, X_ij = -(sum_{k=i+1..j} R_ik X_kj) / R_ii  (i < j)
  for (int j = Nv - 1; j >= 0; --j) {
    const double xjj = 1.0 / w[j * Nv + j].x;
    // compute column j of X for rows i < j, bottom up, using R entries of rows i
    // (still intact: rows i < j keep R in columns > i ... columns >= j of rows < j
    // hold R until overwritten below, and X_kj for k > i are already final).
    for (int i = j - 1; i >= 0; --i) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) {
        double2 rik = w[i * Nv + k];
        double2 xkj = (k == j) ? make_double2(xjj, 0.0) : w[k * Nv + j];
        s.x += rik.x * xkj.x - rik.y * xkj.y;
        s.y += rik.x * xkj.y + rik.y * xkj.x;
      }
      const double rii = w[i * Nv + i].x;
      // X_ij overwrites R_ij, which no later step of this column reads (rows
      // above i read R_i'k for k > i', including R_i'j of their own row only).
      w[i * Nv + j] = make_double2(-s.x / rii, -s.y / rii);
    }
    w[j * Nv + j] = make_double2(xjj, 0.0);
  }
  status[pnl] = bad;
}

// V[rows of panel] <- V[rows] * W (upper-triangular, Nv x Nv), in place.
__global__ __launch_bounds__(256) void k_apply_rinv(double2* __restrict__ V, const double2* __restrict__ W,
                                                    BlockArgs a) {
  extern __shared__ double2 w[];  // Nv * Nv
  const int B = blockIdx.x >> 1, chi = blockIdx.x & 1;
  const int Nv = a.Nv;
  const long long V5 = a.V5, field = 12 * V5;
  for (int e = threadIdx.x; e < Nv * Nv; e += 256) w[e] = W[(long long)blockIdx.x * Nv * Nv + e];
  __syncthreads();
  const int n5 = a.bvol * a.Ls;
  for (int r = threadIdx.x; r < n5 * 6; r += 256) {
    const int j = r / 6, c6 = r % 6;
    const int jl = j / a.Ls, s = j - jl * a.Ls;
    const long long i5 = (long long)block_site(a, B, jl) * a.Ls + s;
    const long long off = (long long)(chi * 6 + c6) * V5 + i5;
    // fully unrolled with predicates so that row[] stays in registers
    double2 row[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) row[k] = (k < Nv) ? V[k * field + off] : make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k < Nv) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i <= k; ++i) cfma(acc, row[i], w[i * Nv + k]);
        V[k * field + off] = acc;
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- host API

size_t restrict_partial_doubles(const CoarseGeometry& cg, int nrhs) {
  return (size_t)nrhs * cg.Vc * NSPLIT * 2 * cg.n2;
}

template <class C2, class CC2>
void restrict_op(const C2* V, const C2* x, CC2* coarse, double* partial, const Geometry& g,
                 const CoarseGeometry& cg, int nrhs, hipStream_t st) {
  BlockArgs a = make_args(g, cg);
  constexpr bool f64 = sizeof(typename real_of<C2>::type) == 8;
  constexpr int RG = 2, KR = f64 ? 4 : 6;
  if constexpr (!f64) {
    // basis and fields read once; rows per workgroup a multiple of 64
    if (nrhs >= 2 && cg.Nv <= 24 && (cg.bvol * g.Ls) % (64 * NSPLIT) == 0) {
      hipLaunchKernelGGL(k_restrict_lds, dim3(cg.Vc * NSPLIT, ceil_div(nrhs, RX)), dim3(RT), 0, st,
                         reinterpret_cast<const float2*>(V), reinterpret_cast<const float2*>(x), partial, a, nrhs);
      MG_LAUNCH_CHECK();
      long long tot = (long long)nrhs * cg.Vc * cg.n2;
      hipLaunchKernelGGL((k_restrict_finalize<CC2>), dim3(ceil_div(tot, 256)), dim3(256), 0, st, partial,
                         coarse, cg.Vc, cg.n2, nrhs);
      MG_LAUNCH_CHECK();
      return;
    }
  }
  // the FP32 kernel reads s-pairs: Ls even keeps every pair inside one site
  if (nrhs >= 2 && (f64 || g.Ls % 2 == 0)) {
    hipLaunchKernelGGL((k_restrict_mr<C2, RG, KR>), dim3(cg.Vc * NSPLIT, ceil_div(nrhs, RG)), dim3(256), 0, st, V,
                       x, partial, a, nrhs);
  } else {
    hipLaunchKernelGGL((k_restrict<C2>), dim3(cg.Vc * NSPLIT, nrhs), dim3(256), 0, st, V, x, partial, a);
  }
  MG_LAUNCH_CHECK();
  long long tot = (long long)nrhs * cg.Vc * cg.n2;
  hipLaunchKernelGGL((k_restrict_finalize<CC2>), dim3(ceil_div(tot, 256)), dim3(256), 0, st, partial,
                     coarse, cg.Vc, cg.n2, nrhs);
  MG_LAUNCH_CHECK();
}

template <class C2, class CC2>
void prolong_op(const C2* V, const CC2* coarse, C2* fine, bool accumulate, const Geometry& g,
                const CoarseGeometry& cg, int nrhs, hipStream_t st) {
  BlockArgs a = make_args(g, cg);
  constexpr bool f64 = sizeof(typename real_of<C2>::type) == 8;
  constexpr int RG = f64 ? 2 : 4;
  constexpr int RW = f64 ? 8 : 16;
  if (nrhs > RG && nrhs <= RW) {  // basis read once
    dim3 grid(ceil_div(12LL * g.V5, 256));
    if (accumulate)
      hipLaunchKernelGGL((k_prolong_wide<C2, CC2, true, RW>), grid, dim3(256), 0, st, V, coarse, fine, a, nrhs);
    else
      hipLaunchKernelGGL((k_prolong_wide<C2, CC2, false, RW>), grid, dim3(256), 0, st, V, coarse, fine, a, nrhs);
  } else if (nrhs >= 2) {
    dim3 grid(ceil_div(g.V5, 256), ceil_div(nrhs, RG));
    if (accumulate)
      hipLaunchKernelGGL((k_prolong_mr<C2, CC2, true, RG>), grid, dim3(256), 0, st, V, coarse, fine, a, nrhs);
    else
      hipLaunchKernelGGL((k_prolong_mr<C2, CC2, false, RG>), grid, dim3(256), 0, st, V, coarse, fine, a, nrhs);
  } else {
    dim3 grid(ceil_div(g.V5, 256), nrhs);
    if (accumulate)
      hipLaunchKernelGGL((k_prolong<C2, CC2, true>), grid, dim3(256), 0, st, V, coarse, fine, a);
    else
      hipLaunchKernelGGL((k_prolong<C2, CC2, false>), grid, dim3(256), 0, st, V, coarse, fine, a);
  }
  MG_LAUNCH_CHECK();
}

template void restrict_op<double2, double2>(const double2*, const double2*, double2*, double*,
                                            const Geometry&, const CoarseGeometry&, int, hipStream_t);
template void restrict_op<float2, float2>(const float2*, const float2*, float2*, double*, const Geometry&,
                                          const CoarseGeometry&, int, hipStream_t);
template void prolong_op<double2, double2>(const double2*, const double2*, double2*, bool, const Geometry&,
                                           const CoarseGeometry&, int, hipStream_t);
template void prolong_op<float2, float2>(const float2*, const float2*, float2*, bool, const Geometry&,
                                         const CoarseGeometry&, int, hipStream_t);

// Two passes of Cholesky QR on every (block, chirality) panel of the FP64 basis.
// Returns false if any panel is numerically rank deficient.
bool orthonormalise_basis(double2* V, const Geometry& g, const CoarseGeometry& cg, hipStream_t st) {
  if (cg.Nv > 32) fail(MGDWF_ERR_INVALID_ARG, "nvec above 32 is not supported");
  BlockArgs a = make_args(g, cg);
  const int npanel = 2 * cg.Vc;
  const size_t nn = (size_t)cg.Nv * cg.Nv;
  DevBuf G(npanel * nn * sizeof(double2)), W(npanel * nn * sizeof(double2)), stat(npanel * sizeof(int));
  std::vector<int> hs(npanel);
  bool ok = true;
  for (int pass = 0; pass < 2; ++pass) {
    size_t lds = (size_t)GRAM_ROWS * 6 * cg.Nv * sizeof(double2);
    hipLaunchKernelGGL(k_gram, dim3(npanel), dim3(256), lds, st, V, G.as<double2>(), a);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_chol_inv, dim3(ceil_div(npanel, 64)), dim3(64), 0, st, G.as<double2>(),
                       W.as<double2>(), stat.as<int>(), npanel, cg.Nv);
    MG_LAUNCH_CHECK();
    MG_HIP(hipMemcpyAsync(hs.data(), stat.p, npanel * sizeof(int), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    for (int v : hs) if (v) ok = false;
    if (!ok) return false;
    hipLaunchKernelGGL(k_apply_rinv, dim3(npanel), dim3(256), nn * sizeof(double2), st, V,
                       W.as<double2>(), a);
    MG_LAUNCH_CHECK();
  }
  return ok;
}

}  // namespace mgdwf
