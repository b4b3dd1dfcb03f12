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
void cgne_solve(mgdwf_ctx* c, double2* b, double2* x, const mgdwf_solve_params& sp, mgdwf_solve_report* rep);

}  // namespace mgdwf
