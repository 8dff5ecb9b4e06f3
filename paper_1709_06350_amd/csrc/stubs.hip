// Entry points of forms that are built in later stages.
#include "mr.h"
#include "mr_ctx.h"
extern "C" {
int mr_solve_batched(int, const int*, const double* const*, double* const*, const mr_opts*, mr_info*, void*) { return mr::fail(MR_EINVAL, "not available"); }
}
