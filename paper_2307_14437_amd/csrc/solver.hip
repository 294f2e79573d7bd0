// Preconditioned conjugate gradients for eq. GoFD-2 (placeholder entry points).
#include "internal.h"

extern "C" int gofd_precond_create(gofd_ctx ctx, gofd_transfer, gofd_fdop, int, gofd_precond*, gofd_precond_info*) {
  return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "not built yet");
}
extern "C" int gofd_precond_free(gofd_precond) { return GOFD_E_UNSUPPORTED; }
extern "C" int gofd_precond_export(gofd_ctx ctx, gofd_precond, int32_t*, int32_t*, double*) {
  return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "not built yet");
}
extern "C" int gofd_solve(gofd_ctx ctx, gofd_transfer, gofd_fdop, gofd_precond, int, const double*, int, double,
                          const gofd_solve_opts*, double*, gofd_solve_info*) {
  return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "not built yet");
}
extern "C" int gofd_solve_batched(gofd_ctx ctx, int, const gofd_transfer*, const gofd_fdop*, const gofd_precond*,
                                  const int*, const double* const*, int, double, const gofd_solve_opts*,
                                  double* const*, gofd_solve_info*) {
  return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "not built yet");
}
extern "C" int gofd_solve_adjoint(gofd_ctx ctx, gofd_transfer, gofd_fdop, gofd_precond, const double*, const double*,
                                  const double*, double, const gofd_solve_opts*, double*, double*, double*,
                                  gofd_solve_info*) {
  return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "not built yet");
}
