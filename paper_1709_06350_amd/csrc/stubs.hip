// Entry points of forms that are built in later stages.
#include "mr.h"
#include "mr_ctx.h"
namespace mr {
void Ctx::release_adjoint() {}
}
extern "C" {
int mr_adjoint_solve(mr_ctx*, const double*, const double*, const double*, double*, mr_info*) { return mr::fail(MR_EINVAL, "not available"); }
int mr_solve_batched(int, const int*, const double* const*, double* const*, const mr_opts*, mr_info*, void*) { return mr::fail(MR_EINVAL, "not available"); }
}
