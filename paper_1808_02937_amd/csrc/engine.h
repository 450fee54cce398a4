// Continuous FGMRES engine: requests (one operator and preconditioner, a block of right-hand
// sides each) join and leave between steps; every step advances all requests in flight by one
// Arnoldi step in shared launches (Section 4.2's preconditioned iteration, right-preconditioned
// flexible GMRES with the true FP64 residual test).
#pragma once

#include <vector>

#include "hlu.h"

namespace fde {

struct KrylovEngine;

struct EngineDone {
    long long id;
    std::vector<fde_solve_info> info;   // one per right-hand side
};

KrylovEngine* engine_create(Ctx* c, int restart, int maxit, double rtol, int max_systems);
void engine_destroy(KrylovEngine* e);
int engine_free_slots(const KrylovEngine* e);
int engine_groups(const KrylovEngine* e);
// start solving A X = G for nrhs columns (device arrays; X is overwritten); the request's
// arithmetic does not depend on what else is in flight
void engine_add(KrylovEngine* e, Op* op, HLUObj* prec, int nrhs, const double* G, int ldg, double* X, int ldx,
                long long id);
// one Arnoldi step of every request in flight (one host synchronisation); requests that
// finished are appended to done
void engine_step(KrylovEngine* e, std::vector<EngineDone>& done);

}  // namespace fde
