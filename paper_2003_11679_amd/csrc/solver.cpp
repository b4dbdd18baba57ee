// Solver entry points (filled in with the GIBC solve).
#include "problem.h"

namespace sie {
struct SolveState {};
void solver_destroy(SolveState *s) { delete s; }
}  // namespace sie

extern "C" {
sie_status sie_set_planewaves(sie_problem *, int32_t, const double *, const sie_c128 *) { return SIE_ESTATE; }
sie_status sie_solve(sie_problem *, sie_precision, const sie_solver_opts *, sie_report *) { return SIE_ESTATE; }
sie_status sie_get_currents(const sie_problem *, int32_t, sie_c128 *, sie_c128 *) { return SIE_ESTATE; }
sie_status sie_far_field(const sie_problem *, int32_t, int64_t, const double *, sie_c128 *) { return SIE_ESTATE; }
}
