// Entry points whose implementation is not in this build yet.
#include "fde_internal.h"

extern "C" {
static int unsupported(const char* what) {
    fde::set_error("%s is not implemented in this build", what);
    return FDE_EUNSUPPORTED;
}
int fde_build_hmatrix(fde_op*, const fde_hparams*, fde_hmat** out) {
    if (out) *out = nullptr;
    return unsupported("fde_build_hmatrix");
}
void fde_hmat_destroy(fde_hmat*) {}
int fde_hmat_counts(const fde_hmat*, int*, int*) { return unsupported("fde_hmat_counts"); }
int fde_hmat_to_dense(fde_hmat*, double*, int) { return unsupported("fde_hmat_to_dense"); }
int fde_hlu_factor(fde_hmat*, const fde_hlu_params*, fde_hlu** out) {
    if (out) *out = nullptr;
    return unsupported("fde_hlu_factor");
}
void fde_hlu_destroy(fde_hlu*) {}
int fde_hlu_to_dense(fde_hlu*, double*, int, int*) { return unsupported("fde_hlu_to_dense"); }
int fde_hlu_max_rank(fde_hlu*, int*) { return unsupported("fde_hlu_max_rank"); }
int fde_hlu_solve(fde_hlu*, int, const double*, int, double*, int) { return unsupported("fde_hlu_solve"); }
int fde_solve(fde_op*, fde_hlu*, int, const double*, int, double*, int, const fde_solve_params*,
              fde_solve_info*) {
    return unsupported("fde_solve");
}
int fde_solve_batched(fde_ctx*, int, fde_op* const*, fde_hlu* const*, const int*, const double* const*,
                      const int*, double* const*, const int*, const fde_solve_params*, fde_solve_info*) {
    return unsupported("fde_solve_batched");
}
}
