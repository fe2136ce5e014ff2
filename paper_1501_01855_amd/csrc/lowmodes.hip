// Kernel low modes (placeholder until the eigensolver lands).
#include "context.h"
#include "ops.h"

namespace ovl {

void lowmodes_compute(Context &c, double rho, int n_low, double tol, double *evals, double *lmax)
{
    (void)c; (void)rho; (void)n_low; (void)tol; (void)evals; (void)lmax;
    throw Error{OVL_ERR_UNSUPPORTED, "lowmodes_compute: not built yet"};
}

}  // namespace ovl
