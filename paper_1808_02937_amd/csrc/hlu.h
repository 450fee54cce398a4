// H-LU factor object shared by the H-LU entry points and the Krylov driver.
#pragma once

#include <algorithm>

#include "hinterp.h"

struct fde_hmat : fde::HMat {
    fde::DevBuf<int> d_ranks;
};

namespace fde {

struct HLUObj {
    fde_hmat* hm = nullptr;
    Op* op = nullptr;
    HTree t;
    int prec = FDE_FP32;
    double tol = 1e-3, pivot_floor = 0.0;
    int kmax = 8;
    Program lu, sv;
    size_t esz = 4;               // bytes per factor element
    DevBuf<char> arena, work_lu, scr, sv_rhs, sv_work;
    DevBuf<double> scrd;
    DevBuf<int> ranks, status, h2p;
    DevBuf<unsigned long long> prof;   // op profile (FDE_PROFILE_OPS=1)
    DevBuf<double> flops;              // [0] factorisation, [1] H-solves
    double factor_ms = 0.0;
    DevBuf<LRBlockDev> lr;
    DevBuf<OpRec> ops_lu, ops_sv;
    int64_t scr_t = 0, scr_d = 0;
    int kpmax = 0;
    int64_t sv_nrhs_cap = 0;
    template <class T>
    Inst<T> inst(bool solve, int nrhs, const double* B, int ldb, double* X, int ldx) {
        Inst<T> d{};
        d.ops = solve ? ops_sv.p : ops_lu.p;
        d.nops = (int)(solve ? sv.ops.size() : lu.ops.size());
        d.arena = reinterpret_cast<T*>(arena.p);
        d.work = reinterpret_cast<T*>(solve ? sv_work.p : work_lu.p);
        d.rhs = reinterpret_cast<T*>(sv_rhs.p);
        d.ranks = ranks.p;
        d.lr = lr.p;
        d.scr = reinterpret_cast<T*>(scr.p);
        d.scrd = scrd.p;
        d.mrmax = std::max(t.max_lr_rows, 1);
        d.kpmax = kpmax;
        d.h2p = h2p.p;
        d.Nd = op->Nd;
        d.B = B;
        d.ldb = ldb;
        d.X = X;
        d.ldx = ldx;
        d.bstep = 0;
        d.xstep = 0;
        d.nrhs = nrhs;
        d.tol = tol;
        d.kmax = kmax;
        d.pivot_floor = pivot_floor;
        d.status = status.p;
        d.prof = prof.p;
        d.flops = flops.p + (solve ? 1 : 0);
        return d;
    }
};

}  // namespace fde

struct fde_hlu : fde::HLUObj {};

namespace fde {
void hlu_prepare_solve(HLUObj* f, int nrhs);
void hlu_solve(HLUObj* f, int nrhs, const double* B, int ldb, double* X, int ldx);
}  // namespace fde
