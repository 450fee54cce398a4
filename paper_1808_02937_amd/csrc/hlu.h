// H-LU factor object shared by the H-LU entry points and the Krylov driver.
#pragma once

#include <algorithm>
#include <memory>

#include "hinterp.h"

struct fde_hmat : fde::HMat {
    fde::DevBuf<int> d_ranks;
};

namespace fde {

// Everything about a factorisation that depends only on the structure of the
// H-matrix (mesh, leaf size, admissibility, rank capacity): the level-scheduled
// H-LU program, the H-solve program, the low-rank block table and the index
// map, on the host and on the device. Read-only once made; shared by every
// factorisation of that structure in a context.
struct Plan {
    HTree t;               // t.op is cleared: a plan outlives the operator it was made for
    Program lu, sv;
    int kpmax = 0;
    bool sv_lds = false;   // every H-solve op works on all right-hand-side columns (LDS kernel usable)
    int lu_variant = 0;    // H-LU kernel variant: widest possible recompression 16, 32, or 0 (wider)
    DevBuf<OpRec> ops_lu, ops_sv;
    DevBuf<int> h2p;
    HsTables hs;            // leaf-step H-solve
    DevBuf<HsStep> d_hs_steps;
    DevBuf<HsRec> d_hs_recs;
    std::vector<int> lr_rows;   // larger dimension of each low-rank block (diagnostics)
};

// the plan for a factorisation with rank capacity kmax of an H-matrix (cached per context)
std::shared_ptr<const Plan> get_plan(Ctx* c, const HTree& hmt, int kmax);
// host-only plan (no device copies), for sizing and checking
void make_plan_host(const HTree& hmt, int kmax, Plan& p, bool check);

struct HLUObj {
    fde_hmat* hm = nullptr;
    Op* op = nullptr;
    std::shared_ptr<const Plan> plan;
    const HTree& t() const { return plan->t; }
    int prec = FDE_FP32;          // arithmetic of the factorisation and the H-solves (FP32 or FP64)
    bool bf16uv = false;          // FDE_FP32_BF16UV: after the factorisation U, V are kept in BF16 only
    DevBuf<char> lr16;            // the BF16 U, V (the arena's tail from lr_base; the arena keeps the head)
    int64_t lr_base = 0;
    double tol = 1e-3, pivot_floor = 0.0;
    int kmax = 8;
    size_t esz = 4;               // bytes per factor element
    DevBuf<char> arena, work_lu, scr, sv_rhs, sv_work;
    DevBuf<char> hs_prep;              // leaf-step H-solve: solve-ready diagonal leaves (after each factorisation)
    DevBuf<double> scrd;
    DevBuf<int> ranks, status;
    DevBuf<unsigned long long> prof;   // op profile (FDE_PROFILE_OPS=1)
    DevBuf<double> flops;              // [0] factorisation, [1] H-solves
    DevBuf<double> lu_flops;           // per op of the factorisation (summed when asked for)
    double factor_ms = 0.0;
    int64_t sv_nrhs_cap = 0;
    template <class T>
    Inst<T> inst(bool solve, int nrhs, const double* B, int ldb, double* X, int ldx) {
        Inst<T> d{};
        d.ops = solve ? plan->ops_sv.p : plan->ops_lu.p;
        d.nops = (int)(solve ? plan->sv.ops.size() : plan->lu.ops.size());
        d.arena = reinterpret_cast<T*>(arena.p);
        d.work = reinterpret_cast<T*>(solve ? sv_work.p : work_lu.p);
        d.rhs = reinterpret_cast<T*>(sv_rhs.p);
        d.ranks = ranks.p;
        d.scr = reinterpret_cast<T*>(scr.p);
        d.scrd = scrd.p;
        d.h2p = plan->h2p.p;
        d.Nd = op->Nd;
        d.B = B;
        d.ldb = ldb;
        d.X = X;
        d.ldx = ldx;
        d.bstep = 0;
        d.xstep = 0;
        d.nrhs = nrhs;
        d.nslots = plan->t.nslots;
        d.work_rows = (int)plan->sv.work_elems;
        d.hs_steps = plan->d_hs_steps.p;
        d.hs_recs = plan->d_hs_recs.p;
        d.hs_nleaf = plan->hs.nleaf;
        d.hs_tslots = plan->hs.tslots;
        d.hs_prep = reinterpret_cast<const T*>(hs_prep.p);
        d.tol = tol;
        d.kmax = kmax;
        d.pivot_floor = pivot_floor;
        d.status = status.p;
        d.prof = prof.p;
        d.flops = flops.p + (solve ? 1 : 0);
        d.op_flops = solve ? nullptr : lu_flops.p;
        d.lr16 = bf16uv ? reinterpret_cast<const unsigned short*>(lr16.p) : nullptr;
        d.lr_base = lr_base;
        return d;
    }
};

}  // namespace fde

struct fde_hlu : fde::HLUObj {};

namespace fde {
void hlu_prepare_solve(HLUObj* f, int nrhs);
void hlu_solve(HLUObj* f, int nrhs, const double* B, int ldb, double* X, int ldx);
// columns per workgroup of the leaf-step H-solve for these factors and nrhs columns (0: does not
// fit LDS, the op-list interpreter runs), in a launch of share_cols columns over all its
// instances; *global_rhs: only with the right-hand sides in global memory, in a workspace of
// hsolve_rhs_elems(Nd, nrhs) elements
int hsolve_cols(Ctx* c, const HLUObj* f, int nrhs, size_t* lds_bytes, bool* global_rhs, int share_cols);
// elements of an H-solve right-hand side workspace for nrhs columns (also enough for the op-list
// interpreter, which uses Nd x nrhs of it)
int64_t hsolve_rhs_elems(int Nd, int nrhs);
// LDS bytes of one workgroup of the leaf-step H-solve of f for wc columns
size_t hsolve_lds_for(const HLUObj* f, int wc, bool global_rhs);
// FDE_EUNSUPPORTED when f keeps BF16 low-rank factors and the LDS H-solve does not fit (wc == 0)
void require_lds_for_bf16(const HLUObj* f, int wc);
}  // namespace fde
