// Interface preconditioner (placeholder until the H_theta kernels land).
#include "internal.h"

namespace edd {

int precond_setup(edd_problem *p) {
  (void)p;
  return EDD_OK;
}

int precond_apply(edd_problem *p, const double *r, double *z,
                  const edd_solve_opts *o, edd_solve_stats *st,
                  bool low_precision) {
  (void)p; (void)r; (void)z; (void)o; (void)st; (void)low_precision;
  return EDD_EINVAL;
}

}  // namespace edd
