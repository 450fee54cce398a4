// Batched right-preconditioned FGMRES(m) (Section 4.2) on the device.
#pragma once

#include "fde_internal.h"

namespace fde {

constexpr int kMaxRestart = 64;

struct SysDev {            // one right-hand side of one operator
    double* V;             // Krylov basis of the operator group: block i at V + i*bs, column c at + c*Nd
    double* Z;             // preconditioned basis, same layout
    double* W;             // A z_j for the group (Nd x nr)
    double* R;             // A x for the group (Nd x nr)
    const double* G;       // right-hand side column
    double* X;             // solution column
    int64_t bs;            // block stride Nd * nr
    int Nd, c;
};

struct SysState {
    double H[(kMaxRestart + 1) * kMaxRestart];
    double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
    double gnorm, relres, est;
    int active, jend, iters, conv, status, pad;
};

// sel: the slots of the systems a launch works on (block b takes slot sel[b]); nullptr: slots
// 0 .. ns-1. jv: the Arnoldi step of each selected system; nullptr: the scalar j for all.
void fg_gnorm(hipStream_t st, int ns, const SysDev* sys, SysState* ss, const int* sel = nullptr);
void fg_zero_x(hipStream_t st, int ns, const SysDev* sys, const int* sel = nullptr);
void fg_cycle_start(hipStream_t st, int ns, const SysDev* sys, SysState* ss, int first, int maxit,
                    const int* sel = nullptr);
void fg_copy_step(hipStream_t st, int ns, const SysDev* sys, const int* mask, int j, const int* sel = nullptr,
                  const int* jv = nullptr);
void fg_arnoldi(hipStream_t st, int ns, const SysDev* sys, SysState* ss, int j, int m, double rtol, int maxit,
                const int* sel = nullptr, const int* jv = nullptr);
void fg_count_active(hipStream_t st, int ns, const SysState* ss, int* out);
void fg_update(hipStream_t st, int ns, const SysDev* sys, SysState* ss, const int* sel = nullptr);
void fg_check(hipStream_t st, int ns, const SysDev* sys, SysState* ss, double rtol, const int* sel = nullptr);

struct SysStatus {   // what the host reads of a system after a step
    double relres;
    int active, conv, status, iters, jend, pad;
};
void fg_gather_status(hipStream_t st, int n, const SysState* ss, const int* sel, SysStatus* out);
// largest and smallest singular value of the m x m triangle left in ss[0] by m Arnoldi steps (device)
void fg_sigma(hipStream_t st, const SysState* ss, int m, double* out);

}  // namespace fde
