// Host wrappers of the solver vector kernels (vecops.hip).
#pragma once

#include <functional>

#include "mg_internal.h"

namespace mgdwf {

constexpr int NSLOT = 128;       // scalar slots per right-hand side
constexpr int VEC_BLOCKS = 1024; // most workgroups of a grid-stride vector kernel (partials per RHS)
// workgroups (and partial sums per RHS) of a vector kernel over n elements
int vec_blocks(long long n);

void finalize_rhs(const double* partial, int nparts, int ncomp, double* sl, int dst, int nrhs, hipStream_t st);

template <class C2>
void mr_update(C2* x, C2* r, const C2* p, const C2* q, long long n, int nrhs, const double* sl, int num, int den,
               bool first, double* partial, hipStream_t st);
template <class C2>
void cg_dir(C2* p, const C2* r, long long n, int nrhs, const double* sl, int num, int den, double* partial,
            hipStream_t st);
template <class C2>
void res_update(C2* rout, const C2* rin, const C2* q, long long n, int nrhs, const double* sl, int num, int den,
                hipStream_t st);
template <class C2>
void lincomb(C2* x, const C2* const* ps, int nv, long long n, int nrhs, const double* sl, int num, bool acc,
             hipStream_t st);
template <class C2>
void multidot_rhs(const C2* const* avec, int nv, const C2* b, const C2* c, long long n, int nrhs, double* partial,
                  double* sl, int dst, hipStream_t st);
template <class C2>
void orth_update(C2* q, C2* z, const C2* const* qs, const C2* const* zs, int nv, long long n, int nrhs,
                 const double* sl, int dots, int nrm, hipStream_t st);
// x = sum_m coef[rhs * 16 + m] p_m, complex FP64 coefficients on the device
template <class C2>
void lincomb_c(C2* x, const C2* const* ps, int nv, long long n, int nrhs, const double2* coef, hipStream_t st);
// z and zs may be null (q alone is orthogonalised); e may be null (r alone moves)
template <class C2>
void gcr_update(C2* e, C2* r, const C2* z, const C2* q, long long n, int nrhs, const double* sl, int cr, int nq,
                bool first, double* partial, hipStream_t st);
// x = (first ? 0 : x) + alpha rin, rnew = rin - alpha p, alpha = <p, rin>/|p|^2 from
// slots cr (complex) and nq: a minimal-residual step on a Hermitian operator
template <class C2>
void mrh_update(C2* x, C2* rnew, const C2* rin, const C2* p, long long n, int nrhs, const double* sl, int cr, int nq,
                bool first, hipStream_t st);
template <class C2>
void scale_by_rsqrt_slot(C2* y, const C2* x, long long n, int nrhs, const double* sl, int den, hipStream_t st);
template <class A2, class B2>
void convert(const A2* in, B2* out, long long n, hipStream_t st);
template <class A2, class B2>
void add_to(B2* y, const A2* x, long long n, hipStream_t st);
template <class C2>
void zero(C2* y, long long n, hipStream_t st);
template <class C2>
void reflect5(const C2* in, C2* out, const Geometry& g, int nf, hipStream_t st);

// dslash.hip
template <class C2>
int dslash_nblocks(const Geometry& g, int nrhs);
template <class C2>
void dslash_ex(const C2* in, C2* out, const C2* b, const C2* gauge, const Geometry& g, double M5, double mf,
               bool dagger, int mode, int nrhs, double* partial, hipStream_t st);
// FP32 tilings: how many, and (x, y, z tile, t-slices per workgroup at nrhs
// right-hand sides) of entry i if it applies to g, with its MGDWF_TILE_* flags.
int dslash_ftile_count();
bool dslash_ftile_desc(const Geometry& g, int i, int nrhs, int desc[4], int* flags);

// transfer.hip
size_t restrict_partial_doubles(const CoarseGeometry& cg, int nrhs);
template <class C2, class CC2>
void restrict_op(const C2* V, const C2* x, CC2* coarse, double* partial, const Geometry& g,
                 const CoarseGeometry& cg, int nrhs, hipStream_t st);
template <class C2, class CC2>
void prolong_op(const C2* V, const CC2* coarse, C2* fine, bool accumulate, const Geometry& g,
                const CoarseGeometry& cg, int nrhs, hipStream_t st);
bool orthonormalise_basis(double2* V, const Geometry& g, const CoarseGeometry& cg, hipStream_t st);

// coarse.hip
void build_coarse_op(const double2* Vhat, const double2* gauge, double2* Dc, double2* work9, double2* cwork,
                     double* partial, const Geometry& g, const CoarseGeometry& cg, double M5, double mf,
                     hipStream_t st);
void finish_coarse_op(CoarseStore& Dc, CoarseStore& DcH, const CoarseGeometry& cg, hipStream_t st);
void coarse_apply64(const CoarseStore& s, const double2* x, double2* y, const CoarseGeometry& cg, int nrhs,
                    hipStream_t st);
size_t coarse_pack_bytes(const CoarseGeometry& cg, int nrhs);
// ctile: MFMA shape of the 16-bit apply, 0 = 16x16x16, 1 = 16x16x32
void coarse_apply32(const CoarseStore& s, mgdwf_prec prec, const float2* x, float2* y, const CoarseGeometry& cg,
                    int nrhs, void* pack, int ctile, hipStream_t st);
// Coarse CGNE (x = D_c^+ y, D_c D_c^+ y = b, from x = 0, to |r| <= tol |b| tested
// every 8 iterations, or maxiter iterations) as one persistent cooperative
// launch on the 16-bit store, at most one workgroup per CU, each owning
// every G-th coarse site;
// r and p are workspaces of the vector size, work holds persistent_cgne_bytes,
// and the coarse applications it makes are added to *count (device).  Its
// grid barriers wait at most wait_seconds each; persistent_cgne_error (which
// synchronises the stream) is nonzero after a launch whose barrier ran out.
// Returns false, launching nothing, where it does not apply (precision,
// nrhs > 16, no cooperative launch).
size_t persistent_cgne_bytes(const CoarseGeometry& cg, int nrhs);
bool coarse_cgne_persistent(const CoarseStore& D, const CoarseStore& DH, mgdwf_prec prec, const float2* b, float2* x,
                            float2* r, float2* p, void* work, long long* count, const CoarseGeometry& cg, int nrhs,
                            double tol, int maxiter, double wait_seconds, int device, hipStream_t st);
int persistent_cgne_error(const void* work, const CoarseGeometry& cg, int nrhs, hipStream_t st);

// squared.hip: A_c = P^+ D^+ D P, 33 offsets [X][o] of column-major 2Nv x 2Nv
// blocks (o: self, +-mu, then the diagonals +-mu +-nu, mu < nu)
size_t sq_coarse_entries(const CoarseGeometry& cg);
void build_sq_coarse_op(const double2* Vhat, const double2* gauge, double2* Ac, double2* work9, double2* zwork9,
                        double2* cwork, double* partial, const Geometry& g, const CoarseGeometry& cg, double M5,
                        double mf, hipStream_t st);
void sq_to_f32(const double2* Ac, float2* Ac32, const CoarseGeometry& cg, hipStream_t st);
void sq_canonical(const double2* Ac, double2* out, const CoarseGeometry& cg, hipStream_t st);
void sq_apply64(const double2* Ac, const double2* x, double2* y, const CoarseGeometry& cg, int nrhs, hipStream_t st);
void sq_apply32(const float2* Ac32, const float2* x, float2* y, const CoarseGeometry& cg, int nrhs, hipStream_t st);

// level2.hip: a third level under the squared method.  cg: the coarse lattice
// (level 1), c2: the level-2 lattice (Lc = blocks, Vc = blocks, Nv = Nv2,
// block = coarse sites per block).  W: Nv2 coarse vectors [j][Vc][2][Nv].
bool orthonormalise_level2(double2* W, const CoarseGeometry& cg, const CoarseGeometry& c2, int* err_dev,
                           hipStream_t st);
template <class F2>
void restrict2(const F2* W, const F2* in, F2* out, const CoarseGeometry& cg, const CoarseGeometry& c2, int nrhs,
               hipStream_t st);
template <class F2>
void prolong2(const F2* W, const F2* cc, F2* out, bool acc, const CoarseGeometry& cg, const CoarseGeometry& c2,
              int nrhs, hipStream_t st);
// out = a - b
template <class F2>
void sub_into(F2* out, const F2* a, const F2* b, long long n, hipStream_t st);
// Galerkin operator W^+ A W of a Hermitian operator A on the lattice cg into
// the 33-offset form over c2 (Vcc x 33 column-major 2Nv2 blocks), read off per
// source block: apply(in, out, n) applies A to n vectors of cg; probes and
// applied: 2 Nv2 vectors of cg each, rr: 2 Nv2 vectors of c2
void build_galerkin_op(const std::function<void(const double2*, double2*, int)>& apply, const double2* W,
                       double2* Acc, double2* probes, double2* applied, double2* rr, const CoarseGeometry& cg,
                       const CoarseGeometry& c2, hipStream_t st);
// A_cc = R2 A_c P2 into the 33-offset form (Vcc x 33 column-major 2Nv2 blocks);
// probes and applied: 2 Nv2 coarse vectors each, rr: 2 Nv2 level-2 vectors
void build_level2_op(const double2* Ac, const double2* W, double2* Acc, double2* probes, double2* applied,
                     double2* rr, const CoarseGeometry& cg, const CoarseGeometry& c2, hipStream_t st);

}  // namespace mgdwf
