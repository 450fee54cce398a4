// Batched left-preconditioned BiCGSTAB (Section 4.2, eq. (precondsys)) on the device.
#pragma once

#include "fde_internal.h"

namespace fde {

struct BicgDev {           // one right-hand side of one operator; group blocks, column c at + c*Nd
    const double* G;       // right-hand side column
    double* X;             // solution column
    double *r, *rh, *p, *s, *v, *t, *W;
    int Nd, c;
};

struct BicgState {
    double gnorm, bnorm, rho, alpha, omega, relres, truerel, pad;
    int iters, conv, status, active;
};

void bc_init(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, int maxit);
void bc_half1(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, double tol);
void bc_half2(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, double tol, int maxit);
// which: 0 r <- G, 1 v <- W, 2 t <- W (systems with mask set: no preconditioner)
void bc_copy(hipStream_t st, int ns, const BicgDev* sys, const int* mask, int which);
void bc_count_active(hipStream_t st, int ns, const BicgState* ss, int* out);
void bc_true_residual(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss);

}  // namespace fde
