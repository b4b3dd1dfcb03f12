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
#include <algorithm>

#include <hip/hip_runtime.h>

#include "mg_internal.h"
#include "blas.h"

namespace mgdwf {

// from transfer.hip
template <class C2, class CC2>
void restrict_op(const C2* V, const C2* x, CC2* coarse, double* partial, const Geometry& g,
                 const CoarseGeometry& cg, int nrhs, hipStream_t st);
// from dslash.hip
void dslash_split(const double2* in, double2* out9, const double2* gauge, const Geometry& g, const int block[4],
                  double M5, double mf, int chi, hipStream_t st, bool dagger = false);

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

CoarseArgs coarse_args(const CoarseGeometry& cg) {
  CoarseArgs a;
  for (int m = 0; m < 4; ++m) a.Lc[m] = cg.Lc[m];
  a.Vc = cg.Vc;
  a.n2 = cg.n2;
  return a;
}

__device__ __forceinline__ int opposite(int d) { return d == 0 ? 0 : (((d - 1) ^ 1) + 1); }

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

// Adjoint stencil in the same form as D_c: (D_c^+ y)(X) = sum_e DcH[X][e] y(X + delta_e)
// with DcH[X][e] = Dc[X + delta_e][opposite(e)]^+.  Column-major blocks on both sides.
__global__ void k_adjoint_blocks(const double2* __restrict__ Dc, double2* __restrict__ DcH, CoarseArgs a) {
  const int blk = blockIdx.x;  // X * 9 + e
  const int X = blk / 9, e = blk % 9;
  const int Y = coarse_neighbour(a, X, e);
  const int n2 = a.n2;
  const double2* src = Dc + ((long long)Y * 9 + opposite(e)) * n2 * n2;
  double2* dst = DcH + (long long)blk * n2 * n2;
  for (int i = threadIdx.x; i < n2 * n2; i += blockDim.x) {
    const int r = i % n2, c = i / n2;           // dst element (r, c), column major
    const double2 v = src[(long long)r * n2 + c]; // src element (c, r)
    dst[i] = make_double2(v.x, -v.y);
  }
}

// y[rhs] = sum_d M[X][d] x[rhs](X + delta_d) for up to NR right-hand sides, each
// block read once for all of them.  Workgroup = one coarse site, 9 wavefronts,
// one per stencil direction d; lane = output row; the nine partial sums are
// added in a fixed order through LDS.
template <class MC2, class VC2, int NR>
__global__ __launch_bounds__(576) void k_capply(const MC2* __restrict__ M, const VC2* __restrict__ x,
                                                VC2* __restrict__ y, CoarseArgs a, int nrhs, int rhs0) {
  using T = typename real_of<VC2>::type;
  __shared__ T red[NR][64][2];
  const int X = blockIdx.x;
  const int n2 = a.n2;
  const int d = threadIdx.x >> 6, row = threadIdx.x & 63;  // one wavefront per stencil direction
  const int nr = min(NR, nrhs - rhs0);
  const long long vs = (long long)a.Vc * n2;  // RHS stride
  VC2 acc[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) acc[j] = cmk<VC2>(0, 0);
  if (row < n2) {
    const int Y = coarse_neighbour(a, X, d);
    const MC2* Md = M + ((long long)X * 9 + d) * n2 * n2;
    const VC2* xv = x + (long long)rhs0 * vs + (long long)Y * n2;
    for (int c = 0; c < n2; ++c) {
      const MC2 m = Md[c * n2 + row];
      const VC2 mv = cmk<VC2>((T)m.x, (T)m.y);
#pragma unroll
      for (int j = 0; j < NR; ++j)
        if (j < nr) cfma(acc[j], mv, xv[j * vs + c]);
    }
  }
  // add the nine directions in a fixed order (bitwise reproducible)
  for (int w = 0; w < 9; ++w) {
    if (d == w)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        if (w == 0) { red[j][row][0] = acc[j].x; red[j][row][1] = acc[j].y; }
        else { red[j][row][0] += acc[j].x; red[j][row][1] += acc[j].y; }
      }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nr * n2; i += blockDim.x) {
    const int j = i / n2, r = i % n2;
    y[(long long)(rhs0 + j) * vs + (long long)X * n2 + r] = cmk<VC2>(red[j][r][0], red[j][r][1]);
  }
}

__global__ void k_dc_to_f32(const double2* __restrict__ in, float2* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// ---------------------------------------------------------------- 16-bit storage
// FP16: the hardware conversion (round to nearest even).  BF16: round to
// nearest even on the upper half of the IEEE single (NaN kept quiet).
__device__ __forceinline__ uint16_t to_f16(float v) {
  _Float16 h = (_Float16)v;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t to_bf16(float v) {
  uint32_t b = __builtin_bit_cast(uint32_t, v);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

template <bool BF>
__device__ __forceinline__ uint16_t to16(float v) { return BF ? to_bf16(v) : to_f16(v); }

// One workgroup per block (X, d): scale = max |Re|, |Im| over the block; store
// Re/scale and Im/scale row major (row r, col c at r * n2 + c).
template <bool BF>
__global__ __launch_bounds__(256) void k_pack_blocks(const double2* __restrict__ M, uint16_t* __restrict__ re,
                                                     uint16_t* __restrict__ im, float* __restrict__ sc, int n2) {
  __shared__ double wmax[4];
  const long long blk = blockIdx.x;
  const double2* src = M + blk * n2 * n2;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n2 * n2; i += 256) mx = fmax(mx, fmax(fabs(src[i].x), fabs(src[i].y)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  const double s = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  if (threadIdx.x == 0) sc[blk] = (float)s;
  for (int i = threadIdx.x; i < n2 * n2; i += 256) {
    const int r = i / n2, c = i % n2;
    const double2 v = src[(long long)c * n2 + r];
    re[blk * n2 * n2 + i] = to16<BF>((float)(v.x * inv));
    im[blk * n2 * n2 + i] = to16<BF>((float)(v.y * inv));
  }
}

// Coarse vectors -> 16-bit with one scale per (site, RHS):
// xp[(rhs * Vc + X) * 2 n2 + k] = Re x_k / s, [.. + n2 + k] = Im x_k / s.
// One wavefront per (RHS, site), lane k < n2 <= 64 handles component k.
template <bool BF>
__global__ __launch_bounds__(256) void k_pack_vec(const float2* __restrict__ x, uint16_t* __restrict__ xp,
                                                  float* __restrict__ xs, int Vc, int n2, int nrhs) {
  const long long i = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int k = threadIdx.x & 63;
  if (i >= (long long)nrhs * Vc) return;  // whole wavefronts leave together
  const float2 v = k < n2 ? x[i * n2 + k] : make_float2(0.f, 0.f);
  float mx = fmaxf(fabsf(v.x), fabsf(v.y));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  const float inv = mx > 0.f ? 1.f / mx : 0.f;
  if (k == 0) xs[i] = mx;
  if (k < n2) {
    uint16_t* o = xp + i * 2 * n2;
    o[k] = to16<BF>(v.x * inv);
    o[n2 + k] = to16<BF>(v.y * inv);
  }
}

typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <bool BF>
__device__ __forceinline__ f4v mfma16(uint2 a, uint2 b, f4v c) {
  if (BF) return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a), __builtin_bit_cast(s4v, b), c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4v, a), __builtin_bit_cast(h4v, b), c, 0, 0, 0);
}

// 16-bit coarse apply on MFMA, FP32 accumulation.  The complex product is the
// real product of [[Re, -Im], [Im, Re]] (2 n2 x 2 n2) with [Re x; Im x]
// (2 n2 x 16 RHS).  16x16x16 tiles: lane l holds A[row l%16][k 4(l/16)..+3],
// B[k 4(l/16)..+3][col l%16] and C[row 4(l/16)..+3][col l%16].  Each
// direction's tile sum is rescaled by (block scale) x (input scale of its RHS)
// before it joins the FP32 accumulator.  Workgroup = one coarse site and a
// chunk of 16 RHS; one wavefront per stencil direction d, the nine partial
// results added in LDS in a fixed order.
template <bool BF>
__global__ __launch_bounds__(576) void k_capply_mfma(const uint16_t* __restrict__ Are, const uint16_t* __restrict__ Aim,
                                                     const float* __restrict__ Asc, const uint16_t* __restrict__ xp,
                                                     const float* __restrict__ xs, float2* __restrict__ y, CoarseArgs a,
                                                     int nrhs) {
  constexpr int MTMAX = 8;  // 2 n2 / 16 <= 8
  __shared__ float red[128][17];
  const int X = blockIdx.x;
  const int rhs0 = blockIdx.y * 16;
  const int n2 = a.n2;
  const int MT = 2 * n2 / 16;
  const int d = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int col = l & 15, kq = l >> 4;
  const int rhs = rhs0 + col;
  const bool valid = rhs < nrhs;
  const int Y = coarse_neighbour(a, X, d);
  const long long blk = (long long)X * 9 + d;
  uint2 bf[MTMAX];
  const uint16_t* xrow = xp + ((long long)(valid ? rhs : 0) * a.Vc + Y) * 2 * n2;
#pragma unroll
  for (int kt = 0; kt < MTMAX; ++kt)
    bf[kt] = (kt < MT && valid) ? *reinterpret_cast<const uint2*>(xrow + kt * 16 + 4 * kq) : make_uint2(0u, 0u);
  f4v t[MTMAX];
#pragma unroll
  for (int m = 0; m < MTMAX; ++m) t[m] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < MTMAX; ++mt) {
    if (mt >= MT) continue;
    const int i = mt * 16 + (l & 15);           // expanded row
    const bool im_row = i >= n2;
    const int rr = im_row ? i - n2 : i;
#pragma unroll
    for (int kt = 0; kt < MTMAX; ++kt) {
      if (kt >= MT) continue;
      const int k = kt * 16 + 4 * kq;             // expanded column of this lane's 4 values
      const bool im_col = k >= n2;
      const int kk = im_col ? k - n2 : k;
      const uint16_t* src = (im_row != im_col) ? Aim : Are;
      uint2 av = *reinterpret_cast<const uint2*>(src + blk * n2 * n2 + (long long)rr * n2 + kk);
      if (!im_row && im_col) { av.x ^= 0x80008000u; av.y ^= 0x80008000u; }  // -Im in the upper right
      t[mt] = mfma16<BF>(av, bf[kt], t[mt]);
    }
  }
  const float s = Asc[blk] * (valid ? xs[(long long)rhs * a.Vc + Y] : 0.f);
  for (int w = 0; w < 9; ++w) {
    if (d == w) {
#pragma unroll
      for (int mt = 0; mt < MTMAX; ++mt)
        if (mt < MT)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float& r = red[mt * 16 + 4 * kq + j][col];
            r = (w == 0 ? 0.f : r) + s * t[mt][j];
          }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < 16 * n2; i += blockDim.x) {
    const int r = i % n2, cl = i / n2;
    if (rhs0 + cl < nrhs) y[((long long)(rhs0 + cl) * a.Vc + X) * n2 + r] = make_float2(red[r][cl], red[n2 + r][cl]);
  }
}

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));

template <bool BF>
__device__ __forceinline__ f4v mfma32(uint4 a, uint4 b, f4v c) {
  if (BF) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a), __builtin_bit_cast(b8v, b), c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0, 0);
}

// k_capply_mfma on the 16x16x32 tiles of gfx950: a lane holds eight
// consecutive k of its A row and of its B column (16-byte loads), so each
// direction takes half the MFMA instructions and half the loads.  Whatever
// order the hardware gives the 32 k-slots, A's and B's slot (lane group,
// element) hold the same k, so the tile sum is the full contraction.  Needs
// 2 n2 divisible by 32 (n2 by 16, as for every 16-bit store).
// y(X) for RHS rhs0 .. rhs0 + 15 into red[row][col] (row < 2 n2: Re rows, then
// Im rows).  Called by all 576 threads of a workgroup; ends with a barrier.
template <bool BF>
__device__ __forceinline__ void apply_site32(const uint16_t* Are, const uint16_t* Aim, const float* Asc,
                                             const uint16_t* xp, const float* xs, const CoarseArgs& a, int nrhs,
                                             int X, int rhs0, float (*red)[17]) {
  // opaque to the optimiser, so a caller that applies in a loop recomputes
  // the operator addresses each time instead of holding them in registers
  int n2 = a.n2;
  asm volatile("" : "+s"(X), "+s"(n2));
  constexpr int MTMAX = 8;  // 2 n2 / 16 <= 8
  constexpr int KTMAX = 4;  // 2 n2 / 32 <= 4
  const int MT = 2 * n2 / 16, KT = 2 * n2 / 32;
  const int d = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int col = l & 15, kq = l >> 4;
  const int rhs = rhs0 + col;
  const bool valid = rhs < nrhs;
  const int Y = coarse_neighbour(a, X, d);
  const long long blk = (long long)X * 9 + d;
  uint4 bf[KTMAX];
  const uint16_t* xrow = xp + ((long long)(valid ? rhs : 0) * a.Vc + Y) * 2 * n2;
#pragma unroll
  for (int kt = 0; kt < KTMAX; ++kt)
    bf[kt] = (kt < KT && valid) ? *reinterpret_cast<const uint4*>(xrow + kt * 32 + 8 * kq) : make_uint4(0u, 0u, 0u, 0u);
  f4v t[MTMAX];
#pragma unroll
  for (int m = 0; m < MTMAX; ++m) t[m] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < MTMAX; ++mt) {
    if (mt >= MT) continue;
    const int i = mt * 16 + (l & 15);           // expanded row
    const bool im_row = i >= n2;
    const int rr = im_row ? i - n2 : i;
#pragma unroll
    for (int kt = 0; kt < KTMAX; ++kt) {
      if (kt >= KT) continue;
      const int k = kt * 32 + 8 * kq;             // expanded column of this lane's 8 values
      const bool im_col = k >= n2;                // n2 % 8 == 0: the 8 stay on one side
      const int kk = im_col ? k - n2 : k;
      const uint16_t* src = (im_row != im_col) ? Aim : Are;
      uint4 av = *reinterpret_cast<const uint4*>(src + blk * n2 * n2 + (long long)rr * n2 + kk);
      if (!im_row && im_col) {  // -Im in the upper right
        av.x ^= 0x80008000u; av.y ^= 0x80008000u; av.z ^= 0x80008000u; av.w ^= 0x80008000u;
      }
      t[mt] = mfma32<BF>(av, bf[kt], t[mt]);
    }
  }
  const float s = Asc[blk] * (valid ? xs[(long long)rhs * a.Vc + Y] : 0.f);
  for (int w = 0; w < 9; ++w) {
    if (d == w) {
#pragma unroll
      for (int mt = 0; mt < MTMAX; ++mt)
        if (mt < MT)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float& r = red[mt * 16 + 4 * kq + j][col];
            r = (w == 0 ? 0.f : r) + s * t[mt][j];
          }
    }
    __syncthreads();
  }
}

template <bool BF>
__global__ __launch_bounds__(576) void k_capply_mfma32(const uint16_t* __restrict__ Are,
                                                       const uint16_t* __restrict__ Aim,
                                                       const float* __restrict__ Asc, const uint16_t* __restrict__ xp,
                                                       const float* __restrict__ xs, float2* __restrict__ y,
                                                       CoarseArgs a, int nrhs) {
  __shared__ float red[128][17];
  const int X = blockIdx.x;
  const int rhs0 = blockIdx.y * 16;
  const int n2 = a.n2;
  apply_site32<BF>(Are, Aim, Asc, xp, xs, a, nrhs, X, rhs0, red);
  for (int i = threadIdx.x; i < 16 * n2; i += blockDim.x) {
    const int r = i % n2, cl = i / n2;
    if (rhs0 + cl < nrhs) y[((long long)(rhs0 + cl) * a.Vc + X) * n2 + r] = make_float2(red[r][cl], red[n2 + r][cl]);
  }
}

// ---------------------------------------------------------------- persistent coarse CGNE
// The coarse solve (CGNE on D_c D_c^+ y = b, x = D_c^+ y, from x = 0) as one
// cooperative launch of at most one workgroup per CU; workgroup w owns the
// coarse sites w, w + G, w + 2G, ... (G workgroups), every RHS (<= 16) at
// once.  Per iteration: q = D_c p at each own site, then x += alpha p and
// r -= alpha q there (alpha = |r|^2 / |p|^2), r packed to 16 bits with its
// per-site |r|^2; grid barrier; |r|^2 summed over all sites (each workgroup
// sums the same partials in the same order, so all take the same decision);
// t = D_c^+ r, p = t + beta p (beta = |r_new|^2 / |r|^2), p packed with its
// |p|^2; grid barrier.  The loop ends when every RHS has |r|^2 <= tol^2 |b|^2
// at one of the tests after every 8th iteration (as in the launched loop), or
// after maxiter iterations; the last iteration skips the D_c^+ apply, whose
// result nobody reads.
//
// The grid barrier is this file's own: an arrival counter and a generation
// word in device memory, agent-scope release/acquire, and a wait bounded in
// wall-clock time.  A wait that runs out sets the error word, and every
// workgroup that sees it leaves the kernel, so a barrier that can never
// complete ends the launch with an error instead of hanging it.
__global__ void k_zero_words(int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

struct GridSync {
  unsigned count;  // arrivals in the current generation
  unsigned gen;    // generation, bumped by the last arrival
  int err;         // set by a wait that ran out of time
  int pad;
};

struct PersistArgs {
  const uint16_t *Are, *Aim, *Hre, *Him;  // 16-bit D_c and D_c^+ (the adjoint stencil)
  const float *Asc, *Hsc;
  const float2* b;
  float2 *x, *r, *p;
  uint16_t *rp, *pp;     // packed r and p: [rhs][X][2 n2]
  float *rs, *ps;        // their per-(rhs, X) scales
  double *part_r, *part_p;  // per-(rhs, X) |.|^2
  long long* count;      // coarse applications are added here (one thread)
  GridSync* gs;          // zeroed before the launch
  long long wait_ticks;  // bound of one barrier wait, in wall-clock ticks
  double tol2;
  int maxiter, nrhs;
  CoarseArgs a;
};

// Every thread of every workgroup calls it; returns false (the same in every
// thread of the workgroup) when the barrier failed and the kernel must end.
__device__ bool grid_barrier(GridSync* gs, unsigned nblocks, long long wait_ticks, int* ok_lds) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g = __hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gs->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            wall_clock64() - t0 > wait_ticks) {
          __hip_atomic_store(&gs->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (__hip_atomic_load(&gs->err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    *ok_lds = ok;
  }
  __syncthreads();
  return *ok_lds != 0;
}

template <bool BF>
__global__ __launch_bounds__(576) void k_cgne_persistent(PersistArgs q) {
  __shared__ float red[128][17];
  __shared__ float2 v[16][64];  // the current site's new r or p, per RHS
  __shared__ double rr0[16], rr[16], pp[16], rn[16];
  __shared__ int ok_lds;
  const CoarseArgs& a = q.a;
  const int n2 = a.n2, nrhs = q.nrhs, Vc = a.Vc;
  const int G = gridDim.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ne = nrhs * n2;
  auto at = [&](int rhs, int X, int k) { return ((long long)rhs * Vc + X) * n2 + k; };
  // v -> 16-bit (one scale per RHS) at site X and |v|^2 per RHS; wave w takes RHS w, w + 9
  auto pack_site = [&](int X, uint16_t* xp, float* xs, double* part) {
    for (int rhs = w; rhs < nrhs; rhs += 9) {
      const float2 val = l < n2 ? v[rhs][l] : make_float2(0.f, 0.f);
      float mx = fmaxf(fabsf(val.x), fabsf(val.y));
      double nn = (double)val.x * val.x + (double)val.y * val.y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        nn += __shfl_xor(nn, off, 64);
      }
      const float inv = mx > 0.f ? 1.f / mx : 0.f;
      const long long i = (long long)rhs * Vc + X;
      if (l == 0) {
        xs[i] = mx;
        part[i] = nn;
      }
      if (l < n2) {
        xp[i * 2 * n2 + l] = to16<BF>(val.x * inv);
        xp[i * 2 * n2 + n2 + l] = to16<BF>(val.y * inv);
      }
    }
    __syncthreads();  // v is rewritten for the next site
  };
  // dst[rhs] = sum over all sites of part[rhs][.], fixed order
  auto reduce_all = [&](const double* part, double* dst) {
    for (int rhs = w; rhs < nrhs; rhs += 9) {
      double s = 0.0;
      for (int Y = l; Y < Vc; Y += 64) s += part[(long long)rhs * Vc + Y];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (l == 0) dst[rhs] = s;
    }
    __syncthreads();
  };
  auto barrier = [&]() { return grid_barrier(q.gs, (unsigned)G, q.wait_ticks, &ok_lds); };
  long long napp = 0;
  // x = 0, r = b, |b|^2
  for (int X = blockIdx.x; X < Vc; X += G) {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int rhs = e / n2, k = e - rhs * n2;
      const float2 bv = q.b[at(rhs, X, k)];
      q.x[at(rhs, X, k)] = make_float2(0.f, 0.f);
      q.r[at(rhs, X, k)] = bv;
      v[rhs][k] = bv;
    }
    __syncthreads();
    pack_site(X, q.rp, q.rs, q.part_r);
  }
  if (!barrier()) return;
  reduce_all(q.part_r, rr0);
  if (threadIdx.x < nrhs) rr[threadIdx.x] = rr0[threadIdx.x];
  // p = D_c^+ r, |p|^2
  for (int X = blockIdx.x; X < Vc; X += G) {
    apply_site32<BF>(q.Hre, q.Him, q.Hsc, q.rp, q.rs, a, nrhs, X, 0, red);
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int rhs = e / n2, k = e - rhs * n2;
      const float2 t = make_float2(red[k][rhs], red[n2 + k][rhs]);
      q.p[at(rhs, X, k)] = t;
      v[rhs][k] = t;
    }
    __syncthreads();
    pack_site(X, q.pp, q.ps, q.part_p);
  }
  ++napp;
  if (!barrier()) return;
  reduce_all(q.part_p, pp);
  for (int it = 0; it < q.maxiter; ++it) {
    // q = D_c p; x += alpha p; r -= alpha q
    for (int X = blockIdx.x; X < Vc; X += G) {
      apply_site32<BF>(q.Are, q.Aim, q.Asc, q.pp, q.ps, a, nrhs, X, 0, red);
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int rhs = e / n2, k = e - rhs * n2;
        const float alpha = (float)(pp[rhs] > 0.0 ? rr[rhs] / pp[rhs] : 0.0);
        const long long i = at(rhs, X, k);
        const float2 pv = q.p[i], xv = q.x[i], rv = q.r[i];
        const float2 qv = make_float2(red[k][rhs], red[n2 + k][rhs]);
        q.x[i] = make_float2(xv.x + alpha * pv.x, xv.y + alpha * pv.y);
        const float2 rn2 = make_float2(rv.x - alpha * qv.x, rv.y - alpha * qv.y);
        q.r[i] = rn2;
        v[rhs][k] = rn2;
      }
      __syncthreads();
      pack_site(X, q.rp, q.rs, q.part_r);
    }
    ++napp;
    if (!barrier()) return;
    reduce_all(q.part_r, rn);
    // the launched loop's schedule: the residual is tested after every 8th
    // iteration (the same decision in every workgroup)
    const int n = it + 1;
    bool done = n % 8 == 0;
    for (int rhs = 0; rhs < nrhs && done; ++rhs)
      if (!(rn[rhs] <= q.tol2 * rr0[rhs])) done = false;
    if (done || n == q.maxiter) break;
    // t = D_c^+ r; p = t + beta p
    for (int X = blockIdx.x; X < Vc; X += G) {
      apply_site32<BF>(q.Hre, q.Him, q.Hsc, q.rp, q.rs, a, nrhs, X, 0, red);
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int rhs = e / n2, k = e - rhs * n2;
        const float beta = (float)(rr[rhs] > 0.0 ? rn[rhs] / rr[rhs] : 0.0);
        const long long i = at(rhs, X, k);
        const float2 pv = q.p[i];
        const float2 t = make_float2(red[k][rhs] + beta * pv.x, red[n2 + k][rhs] + beta * pv.y);
        q.p[i] = t;
        v[rhs][k] = t;
      }
      __syncthreads();
      pack_site(X, q.pp, q.ps, q.part_p);
    }
    ++napp;
    if (threadIdx.x < nrhs) rr[threadIdx.x] = rn[threadIdx.x];
    if (!barrier()) return;
    reduce_all(q.part_p, pp);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *q.count += napp;
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

static void pack_store(CoarseStore& s, const CoarseGeometry& cg, hipStream_t st) {
  const long long nblk = 9LL * cg.Vc, n = nblk * cg.n2 * cg.n2;
  s.m32.alloc(n * sizeof(float2));
  hipLaunchKernelGGL(k_dc_to_f32, dim3(std::min(ceil_div(n, 256), 8192)), dim3(256), 0, st, s.m64.as<double2>(),
                     s.m32.as<float2>(), n);
  MG_LAUNCH_CHECK();
  s.re16.alloc(n * 2); s.im16.alloc(n * 2); s.sc16.alloc(nblk * sizeof(float));
  s.reb.alloc(n * 2); s.imb.alloc(n * 2); s.scb.alloc(nblk * sizeof(float));
  hipLaunchKernelGGL(k_pack_blocks<false>, dim3(nblk), dim3(256), 0, st, s.m64.as<double2>(), s.re16.as<uint16_t>(),
                     s.im16.as<uint16_t>(), s.sc16.as<float>(), cg.n2);
  MG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_pack_blocks<true>, dim3(nblk), dim3(256), 0, st, s.m64.as<double2>(), s.reb.as<uint16_t>(),
                     s.imb.as<uint16_t>(), s.scb.as<float>(), cg.n2);
  MG_LAUNCH_CHECK();
}

// From Dc.m64: the adjoint stencil and the FP32 / FP16 / BF16 copies of both.
void finish_coarse_op(CoarseStore& Dc, CoarseStore& DcH, const CoarseGeometry& cg, hipStream_t st) {
  const long long nblk = 9LL * cg.Vc, n = nblk * cg.n2 * cg.n2;
  DcH.m64.alloc(n * sizeof(double2));
  hipLaunchKernelGGL(k_adjoint_blocks, dim3(nblk), dim3(256), 0, st, Dc.m64.as<double2>(), DcH.m64.as<double2>(),
                     coarse_args(cg));
  MG_LAUNCH_CHECK();
  pack_store(Dc, cg, st);
  pack_store(DcH, cg, st);
}

void coarse_apply64(const CoarseStore& s, const double2* x, double2* y, const CoarseGeometry& cg, int nrhs,
                    hipStream_t st) {
  if (cg.n2 > 64) fail(MGDWF_ERR_INVALID_ARG, "2*nvec above 64 is not supported");
  for (int r0 = 0; r0 < nrhs; r0 += 8) {
    hipLaunchKernelGGL((k_capply<double2, double2, 8>), dim3(cg.Vc), dim3(576), 0, st, s.m64.as<double2>(), x, y,
                       coarse_args(cg), nrhs, r0);
    MG_LAUNCH_CHECK();
  }
}

size_t coarse_pack_bytes(const CoarseGeometry& cg, int nrhs) {
  return (size_t)nrhs * cg.Vc * (2 * cg.n2 * sizeof(uint16_t) + sizeof(float)) + 256;
}

void coarse_apply32(const CoarseStore& s, mgdwf_prec prec, const float2* x, float2* y, const CoarseGeometry& cg,
                    int nrhs, void* pack, int ctile, hipStream_t st) {
  if (cg.n2 > 64) fail(MGDWF_ERR_INVALID_ARG, "2*nvec above 64 is not supported");
  if (prec == MGDWF_F32 || prec == MGDWF_F64) {
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      hipLaunchKernelGGL((k_capply<float2, float2, 16>), dim3(cg.Vc), dim3(576), 0, st, s.m32.as<float2>(), x, y,
                         coarse_args(cg), nrhs, r0);
      MG_LAUNCH_CHECK();
    }
    return;
  }
  if (cg.n2 % 16) fail(MGDWF_ERR_INVALID_ARG, "16-bit coarse operator needs nvec divisible by 8");
  const bool bf = prec == MGDWF_BF16;
  uint16_t* xp = static_cast<uint16_t*>(pack);
  float* xs = reinterpret_cast<float*>(xp + (size_t)nrhs * cg.Vc * 2 * cg.n2);
  const long long nsv = (long long)nrhs * cg.Vc;
  if (bf) hipLaunchKernelGGL(k_pack_vec<true>, dim3(ceil_div(nsv, 4)), dim3(256), 0, st, x, xp, xs, cg.Vc, cg.n2, nrhs);
  else hipLaunchKernelGGL(k_pack_vec<false>, dim3(ceil_div(nsv, 4)), dim3(256), 0, st, x, xp, xs, cg.Vc, cg.n2, nrhs);
  MG_LAUNCH_CHECK();
  dim3 grid(cg.Vc, ceil_div(nrhs, 16));
  if (ctile == 1) {  // 16x16x32 tiles
    if (bf)
      hipLaunchKernelGGL(k_capply_mfma32<true>, grid, dim3(576), 0, st, s.reb.as<uint16_t>(), s.imb.as<uint16_t>(),
                         s.scb.as<float>(), xp, xs, y, coarse_args(cg), nrhs);
    else
      hipLaunchKernelGGL(k_capply_mfma32<false>, grid, dim3(576), 0, st, s.re16.as<uint16_t>(),
                         s.im16.as<uint16_t>(), s.sc16.as<float>(), xp, xs, y, coarse_args(cg), nrhs);
    MG_LAUNCH_CHECK();
    return;
  }
  if (bf)
    hipLaunchKernelGGL(k_capply_mfma<true>, grid, dim3(576), 0, st, s.reb.as<uint16_t>(), s.imb.as<uint16_t>(),
                       s.scb.as<float>(), xp, xs, y, coarse_args(cg), nrhs);
  else
    hipLaunchKernelGGL(k_capply_mfma<false>, grid, dim3(576), 0, st, s.re16.as<uint16_t>(), s.im16.as<uint16_t>(),
                       s.sc16.as<float>(), xp, xs, y, coarse_args(cg), nrhs);
  MG_LAUNCH_CHECK();
}

size_t persistent_cgne_bytes(const CoarseGeometry& cg, int nrhs) {
  const size_t nsv = (size_t)nrhs * cg.Vc;
  return 2 * nsv * 2 * cg.n2 * sizeof(uint16_t) + 2 * nsv * sizeof(float) + 2 * nsv * sizeof(double) +
         sizeof(GridSync) + 7 * 256;
}

// Workgroups of k_cgne_persistent that one CU can hold at once, from the
// kernel's own register and LDS use: 576 threads are 9 wavefronts spread
// over the 4 SIMDs (3 on the fullest), each SIMD holds 512 VGPRs per lane
// (granule 8) and a CU 160 KB of LDS.
static int persistent_fit_per_cu(const void* fn) {
  hipFuncAttributes at{};
  MG_HIP(hipFuncGetAttributes(&at, fn));
  const int vgpr = std::max(8, (at.numRegs + 7) / 8 * 8);
  const int waves_per_simd = 512 / vgpr;
  const int by_vgpr = waves_per_simd / 3;  // the fullest SIMD carries 3 wavefronts of each workgroup
  const int by_lds = at.sharedSizeBytes > 0 ? (int)((160 * 1024) / at.sharedSizeBytes) : 64;
  return std::min(by_vgpr, by_lds);
}

bool coarse_cgne_persistent(const CoarseStore& D, const CoarseStore& DH, mgdwf_prec prec, const float2* b, float2* x,
                            float2* r, float2* p, void* work, long long* count, const CoarseGeometry& cg, int nrhs,
                            double tol, int maxiter, double wait_seconds, int device, hipStream_t st) {
  if (!(prec == MGDWF_F16 || prec == MGDWF_BF16) || cg.n2 % 16 || cg.n2 > 64 || nrhs < 1 || nrhs > 16 ||
      maxiter < 1)
    return false;
  const bool bf = prec == MGDWF_BF16;
  const void* fn = bf ? reinterpret_cast<const void*>(&k_cgne_persistent<true>)
                      : reinterpret_cast<const void*>(&k_cgne_persistent<false>);
  int coop = 0, ncu = 0, per_cu = 0, clock_khz = 0;
  MG_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device));
  MG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
  MG_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device));
  MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 576, 0));
  // At most one workgroup per CU, whatever the occupancy query says: the
  // kernel takes about 140 VGPRs, so a SIMD holds 3 wavefronts and a CU one
  // 9-wavefront workgroup; a grid of two workgroups per CU can never be
  // resident at once and its first grid barrier would wait for ever.
  if (!coop || per_cu < 1 || persistent_fit_per_cu(fn) < 1 || clock_khz <= 0) return false;
  const int G = std::min(cg.Vc, ncu);
  const size_t nsv = (size_t)nrhs * cg.Vc;
  char* w = static_cast<char*>(work);
  auto take = [&](size_t bytes) {
    char* q = w;
    w += (bytes + 255) / 256 * 256;
    return q;
  };
  PersistArgs q;
  q.Are = (bf ? D.reb : D.re16).as<uint16_t>();
  q.Aim = (bf ? D.imb : D.im16).as<uint16_t>();
  q.Asc = (bf ? D.scb : D.sc16).as<float>();
  q.Hre = (bf ? DH.reb : DH.re16).as<uint16_t>();
  q.Him = (bf ? DH.imb : DH.im16).as<uint16_t>();
  q.Hsc = (bf ? DH.scb : DH.sc16).as<float>();
  q.b = b;
  q.x = x;
  q.r = r;
  q.p = p;
  q.rp = reinterpret_cast<uint16_t*>(take(nsv * 2 * cg.n2 * sizeof(uint16_t)));
  q.pp = reinterpret_cast<uint16_t*>(take(nsv * 2 * cg.n2 * sizeof(uint16_t)));
  q.rs = reinterpret_cast<float*>(take(nsv * sizeof(float)));
  q.ps = reinterpret_cast<float*>(take(nsv * sizeof(float)));
  q.part_r = reinterpret_cast<double*>(take(nsv * sizeof(double)));
  q.part_p = reinterpret_cast<double*>(take(nsv * sizeof(double)));
  q.gs = reinterpret_cast<GridSync*>(take(sizeof(GridSync)));
  q.count = count;
  q.wait_ticks = (long long)(std::max(0.0, wait_seconds) * 1e3 * clock_khz);
  q.tol2 = tol * tol;
  q.maxiter = maxiter;
  q.nrhs = nrhs;
  q.a = coarse_args(cg);
  // the barrier words start from zero (a fill kernel, not a memset node, so
  // the sequence stays valid inside a captured graph)
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(q.gs),
                     (int)(sizeof(GridSync) / sizeof(int)));
  MG_LAUNCH_CHECK();
  void* args[] = {&q};
  MG_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(576), args, 0, st));
  return true;
}

int persistent_cgne_error(const void* work, const CoarseGeometry& cg, int nrhs, hipStream_t st) {
  const size_t nsv = (size_t)nrhs * cg.Vc;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t off = 2 * up(nsv * 2 * cg.n2 * sizeof(uint16_t)) + 2 * up(nsv * sizeof(float)) +
                     2 * up(nsv * sizeof(double));
  GridSync h{};
  MG_HIP(hipMemcpyAsync(&h, static_cast<const char*>(work) + off, sizeof h, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  return h.err;
}

}  // namespace mgdwf
