// Solver entry points used by the C ABI (solver.hip).
#pragma once

#include "mg_internal.h"

struct mgdwf_ctx;

namespace mgdwf {

void mg_solve(mgdwf_ctx* c, double2* b64, double2* x64, int nrhs, const mgdwf_solve_params& sp,
              mgdwf_solve_report* rep);
// z = M b: one application of the two-level V-cycle in the handle's precisions
void vcycle_apply(mgdwf_ctx* c, const double2* b64, double2* z64, int nrhs);
void mg_setup(mgdwf_ctx* c, const mgdwf_mg_params& p, double2* W, mgdwf_setup_report* rep);
// Lowest nev eigenpairs of D^+D by m Lanczos steps on (D^+D)^-1 (two
// multigrid solves to tol per step): eigenvalues ascending into evals (host),
// unit eigenvectors into evecs (nev internal FP64 fields, may be null),
// |N y - lambda y| / lambda into resid (host, may be null).
void low_modes(mgdwf_ctx* c, const double2* v0, int nev, int m, double tol, double* evals, double2* evecs,
               double* resid);
// frac[i] = |P R e_i|^2 / |e_i|^2 for n internal FP64 fields, installed basis
void coarse_coverage(mgdwf_ctx* c, const double2* e, int n, double* frac);
// third level under the squared coarse operator (W0: internal = canonical coarse layout)
void setup_level2(mgdwf_ctx* c, const mgdwf_level2_params& p, const double2* W0, double* null_residual);
void cgne_solve(mgdwf_ctx* c, double2* b, double2* x, const mgdwf_solve_params& sp, mgdwf_solve_report* rep);

}  // namespace mgdwf
