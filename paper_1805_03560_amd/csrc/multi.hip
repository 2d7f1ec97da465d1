// Multi right-hand-side CG: every rhs has its own kappa and its own device scalars.
#include "internal.h"

namespace whmc {

whmc_status cg_solve_multi(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                           const whmc_cg_params* p, whmc_cg_stats* st) {
  const size_t n = (size_t)24 * c->Vh;
  whmc_status worst = WHMC_OK;
  for (int r = 0; r < nrhs; ++r) {
    whmc_status rc = cg_solve(c, x + r * n, b + r * n, kappas + r, 1, p, st ? st + r : nullptr);
    if (rc == WHMC_ENOCONV) worst = rc;
    else if (rc != WHMC_OK) return rc;
  }
  return worst;
}

}  // namespace whmc
