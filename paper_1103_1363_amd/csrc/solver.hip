#include "lq_internal.h"
namespace lq {
void solve(lq_ctx*, double*, const double*, int, double, double, double, const lq_solver_params*, lq_solve_report*) {
  throw Error(LQ_EINVAL, "not built yet");
}
void free_work(lq_ctx*) {}
}
