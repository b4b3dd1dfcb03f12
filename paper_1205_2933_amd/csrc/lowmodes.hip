// Low modes of D^+D and their coverage by the coarse space.
//
// Paper, Sec. 2 (the choice of the coarse space, Fig. 1 right): a coarse
// space built from a few low modes, cut into blocks, also holds most of the
// modes just above them.  This file measures that for the library's bases:
// the lowest eigenpairs of N = D^+ D by Lanczos on N^-1 (each step two
// multigrid solves, N^-1 = D^-1 G D^-1 G with G = gamma5 R5, since
// D^+ = G D G), full reorthogonalisation, the Ritz problem of the
// tridiagonal matrix solved on the host by cyclic Jacobi rotations; and the
// fraction |P R e|^2 / |e|^2 of any field inside the coarse space.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "solver.h"

namespace mgdwf {

namespace {

// out = G in, (G psi)(x, s) = gamma5 psi(x, Ls - 1 - s); gamma5 = diag(1, 1, -1, -1)
__global__ void k_gamma5_r5(const double2* __restrict__ in, double2* __restrict__ out, long long V5, int Ls) {
  const long long n = 12 * V5;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long comp = i / V5, i5 = i - comp * V5;
    const long long x4 = i5 / Ls;
    const int s = (int)(i5 - x4 * Ls);
    const double2 v = in[comp * V5 + x4 * Ls + (Ls - 1 - s)];
    out[i] = comp >= 6 ? make_double2(-v.x, -v.y) : v;
  }
}

// out = a x + b y (real a, b)
__global__ void k_axpby(double2* __restrict__ out, const double2* __restrict__ x, const double2* __restrict__ y,
                        double a, double b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = make_double2(a * x[i].x + b * y[i].x, a * x[i].y + b * y[i].y);
}

std::vector<double> slots_of(mgdwf_ctx* c) {
  std::vector<double> h(NSLOT);
  MG_HIP(hipMemcpyAsync(h.data(), c->buf<double>("slots", NSLOT), NSLOT * sizeof(double), hipMemcpyDeviceToHost,
                        c->st));
  MG_HIP(hipStreamSynchronize(c->st));
  return h;
}

constexpr int S_LM = 8;  // slot block of the multi-dot (2 x 16 + 3 entries)

// <v_j, w> for the nv fields v (device pointers) into dots (host, complex as pairs)
void dots_with(mgdwf_ctx* c, const std::vector<double2*>& v, const double2* w, std::vector<double2>& dots) {
  const long long nf = c->fine_len();
  const int nv = (int)v.size();
  double2** tab = c->buf<double2*>("lm_tab", 16);
  MG_HIP(hipMemcpyAsync(tab, v.data(), nv * sizeof(double2*), hipMemcpyHostToDevice, c->st));
  double* partial = c->buf<double>("vpart", (size_t)VEC_BLOCKS * (2 * 16 + 3));
  multidot_rhs<double2>(tab, nv, w, nullptr, nf, 1, partial, c->buf<double>("slots", NSLOT), S_LM, c->st);
  std::vector<double> h = slots_of(c);
  dots.resize(nv);
  for (int j = 0; j < nv; ++j) dots[j] = make_double2(h[S_LM + 2 * j], h[S_LM + 2 * j + 1]);
}

// w += sum_j coef_j v_j (at most 16 fields)
void add_comb(mgdwf_ctx* c, const std::vector<double2*>& v, const std::vector<double2>& coef, double2* w) {
  const long long nf = c->fine_len();
  const int nv = (int)v.size();
  double2** tab = c->buf<double2*>("lm_tab", 16);
  MG_HIP(hipMemcpyAsync(tab, v.data(), nv * sizeof(double2*), hipMemcpyHostToDevice, c->st));
  std::vector<double2> cf(16, make_double2(0.0, 0.0));
  std::copy(coef.begin(), coef.end(), cf.begin());
  double2* cd = c->buf<double2>("lm_coef", 16);
  MG_HIP(hipMemcpyAsync(cd, cf.data(), 16 * sizeof(double2), hipMemcpyHostToDevice, c->st));
  double2* tmp = c->buf<double2>("lm_tmp", nf);
  lincomb_c<double2>(tmp, tab, nv, nf, 1, cd, c->st);
  add_to<double2, double2>(w, tmp, nf, c->st);
  MG_HIP(hipStreamSynchronize(c->st));  // the host tables are reused
}

double norm2(mgdwf_ctx* c, const double2* v) {
  const long long nf = c->fine_len();
  double* partial = c->buf<double>("vpart", (size_t)VEC_BLOCKS * (2 * 16 + 3));
  multidot_rhs<double2>(nullptr, 0, v, nullptr, nf, 1, partial, c->buf<double>("slots", NSLOT), S_LM, c->st);
  return slots_of(c)[S_LM];
}

void scale(mgdwf_ctx* c, double2* out, const double2* x, double a) {
  const long long nf = c->fine_len();
  hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(nf)), dim3(256), 0, c->st, out, x, x, a, 0.0, nf);
  MG_LAUNCH_CHECK();
}

// Eigen-decomposition of a real symmetric n x n matrix (row major) by cyclic
// Jacobi rotations: a holds the eigenvalues on its diagonal on return, z the
// eigenvectors as columns.
void jacobi_eigen(std::vector<double>& a, std::vector<double>& z, int n) {
  z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = cs * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = cs * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
          z[(size_t)k * n + p] = cs * zkp - sn * zkq;
          z[(size_t)k * n + q] = sn * zkp + cs * zkq;
        }
      }
  }
}

}  // namespace

// w = N^-1 v = D^-1 G D^-1 G v with the installed multigrid, solves to tol
static void apply_ninv(mgdwf_ctx* c, const double2* v, double2* w, double tol) {
  const long long nf = c->fine_len();
  double2* g = c->buf<double2>("lm_g", nf);
  double2* y = c->buf<double2>("lm_y", nf);
  const int nb = (int)std::min<long long>(ceil_div(nf, 256), 8192);
  mgdwf_solve_params sp{tol, 2000, 16};  // restarts every 16: fewer stalls with a small basis
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_gamma5_r5, dim3(nb), dim3(256), 0, c->st, pass == 0 ? v : y, g, (long long)c->g.V5, c->g.Ls);
    MG_LAUNCH_CHECK();
    double2* x = pass == 0 ? y : w;
    zero<double2>(x, nf, c->st);
    mgdwf_solve_report rep{};
    try {
      mg_solve(c, g, x, 1, sp, &rep);
    } catch (const Error& e) {
      if (e.code != MGDWF_ERR_NOT_CONVERGED) throw;
      char msg[160];
      snprintf(msg, sizeof msg, "a Lanczos solve missed %.1e: |r|/|b| %.2e after %d iterations%s", tol,
               rep.true_relres, rep.outer_iters, (rep.flags & 2u) ? " (stalled)" : "");
      fail(MGDWF_ERR_NOT_CONVERGED, msg);
    }
  }
}

void low_modes(mgdwf_ctx* c, const double2* v0, int nev, int m, double tol, double* evals, double2* evecs,
               double* resid) {
  const long long nf = c->fine_len();
  double2* V = c->buf<double2>("lm_V", (size_t)(m + 1) * nf);
  double2* w = c->buf<double2>("lm_w", nf);
  c->buf<double>("slots", NSLOT);
  auto vec = [&](int j) { return V + (long long)j * nf; };
  const double n0 = std::sqrt(norm2(c, v0));
  if (!(n0 > 0.0) || !std::isfinite(n0)) fail(MGDWF_ERR_INVALID_ARG, "start vector is zero or not finite");
  scale(c, vec(0), v0, 1.0 / n0);
  std::vector<double> alpha(m, 0.0), beta(m, 0.0);
  int k = 0;
  for (; k < m; ++k) {
    apply_ninv(c, vec(k), w, tol);
    // full reorthogonalisation against v_0 .. v_k, twice; alpha_k from the first pass
    for (int pass = 0; pass < 2; ++pass)
      for (int j0 = 0; j0 <= k; j0 += 16) {
        const int nv = std::min(16, k + 1 - j0);
        std::vector<double2*> vs(nv);
        for (int j = 0; j < nv; ++j) vs[j] = vec(j0 + j);
        std::vector<double2> d;
        dots_with(c, vs, w, d);
        if (pass == 0 && j0 + nv == k + 1) alpha[k] = d[nv - 1].x;
        for (double2& q : d) q = make_double2(-q.x, -q.y);
        add_comb(c, vs, d, w);
      }
    beta[k] = std::sqrt(norm2(c, w));
    if (!(beta[k] > 1e-14 * std::fabs(alpha[k]))) { ++k; break; }  // invariant subspace
    scale(c, vec(k + 1), w, 1.0 / beta[k]);
  }
  const int n = k;
  if (nev > n) fail(MGDWF_ERR_NUMERIC, "Lanczos ended before nev Ritz vectors");
  std::vector<double> T((size_t)n * n, 0.0), S;
  for (int i = 0; i < n; ++i) {
    T[(size_t)i * n + i] = alpha[i];
    if (i + 1 < n) T[(size_t)i * n + i + 1] = T[(size_t)(i + 1) * n + i] = beta[i];
  }
  jacobi_eigen(T, S, n);
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return T[(size_t)a * n + a] > T[(size_t)b * n + b]; });
  double2* y = c->buf<double2>("lm_ritz", nf);
  double2* t = c->buf<double2>("lm_t", nf);
  double2* q = c->buf<double2>("lm_q", nf);
  for (int i = 0; i < nev; ++i) {
    const int col = order[i];
    const double theta = T[(size_t)col * n + col];
    const double lam = 1.0 / theta;  // eigenvalue of N
    evals[i] = lam;
    zero<double2>(y, nf, c->st);
    for (int j0 = 0; j0 < n; j0 += 16) {
      const int nv = std::min(16, n - j0);
      std::vector<double2*> vs(nv);
      std::vector<double2> cf(nv);
      for (int j = 0; j < nv; ++j) {
        vs[j] = vec(j0 + j);
        cf[j] = make_double2(S[(size_t)(j0 + j) * n + col], 0.0);
      }
      add_comb(c, vs, cf, y);
    }
    const double yn = std::sqrt(norm2(c, y));
    scale(c, y, y, 1.0 / yn);
    if (resid) {  // |N y - lambda y| / lambda
      dslash_ex<double2>(y, t, nullptr, c->U64.as<double2>(), c->g, c->M5, c->mf, false, 0, 1, nullptr, c->st);
      dslash_ex<double2>(t, q, nullptr, c->U64.as<double2>(), c->g, c->M5, c->mf, true, 0, 1, nullptr, c->st);
      hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(nf)), dim3(256), 0, c->st, t, q, y, 1.0, -lam, nf);
      MG_LAUNCH_CHECK();
      resid[i] = std::sqrt(norm2(c, t)) / lam;
    }
    if (evecs)
      MG_HIP(hipMemcpyAsync(evecs + (long long)i * nf, y, nf * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
  }
}

// frac[i] = |P R e_i|^2 / |e_i|^2 for n internal FP64 fields e
void coarse_coverage(mgdwf_ctx* c, const double2* e, int n, double* frac) {
  const long long nf = c->fine_len(), nc = c->coarse_len();
  double2* cv = c->buf<double2>("lm_cv", nc);
  double2* pe = c->buf<double2>("lm_pe", nf);
  c->buf<double>("slots", NSLOT);
  for (int i = 0; i < n; ++i) {
    const double2* ei = e + (long long)i * nf;
    fine_restrict<double2>(c, c->V64.as<double2>(), ei, cv, 1);
    fine_prolong<double2>(c, c->V64.as<double2>(), cv, pe, false, 1);
    const double num = norm2(c, pe), den = norm2(c, ei);
    frac[i] = den > 0.0 ? num / den : 0.0;
  }
}

}  // namespace mgdwf
