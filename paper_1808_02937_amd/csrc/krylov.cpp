// Host driver of the batched Krylov solvers (Section 4.2): right-preconditioned FGMRES(m), and the
// paper's left-preconditioned BiCGSTAB.
//
// The paper preconditions A X = G with the H-LU of A~ and iterates with
// BiCGSTAB (eq. (precondsys)); here the preconditioner is applied on the right
// inside flexible GMRES, because a mixed-precision H-solve is not an exactly
// linear operator, and the iteration stops on the true FP64 residual
// ||G - A X|| / ||G|| (recomputed with the full stiffness apply at the end of
// every cycle), so the FP32 preconditioner never limits the final accuracy.
//
// Every system (one right-hand side of one operator) advances in lock-step:
// each Arnoldi step is one batched H-solve launch, one stiffness apply per
// operator and one fused CGS2/Givens launch; the host reads back one integer
// (how many systems are still in their cycle) per step.
#include <algorithm>
#include <cstring>

#include <list>
#include <memory>

#include "bicgstab.h"
#include "engine.h"
#include "hlu.h"
#include "krylov.h"

namespace fde {

namespace {

struct Group {
    Op* op;
    HLUObj* prec;
    int nr;
    const double* G;
    int ldg;
    double* X;
    int ldx;
    int sys0;
    DevBuf<double> V, Z, W, R;
    DevBuf<char> rhs, work;   // H-solve buffers of this group
};

// The per-operator applies of a Krylov step are independent small kernel chains (a few
// workgroups each). They run concurrently: the groups are spread over the context's stream and up
// to c->nside side streams (3 unless set otherwise), forked after the work queued so far and joined
// back before the next step. Groups of one operator share a stream, since the operator's workspace
// is theirs.
void ensure_side_streams(Ctx* c) {
    if ((int)c->side.size() >= c->nside) return;
    for (int k = (int)c->side.size(); k < c->nside; ++k) {
        hipStream_t s = nullptr;
        FDE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->side.push_back(s);
        hipEvent_t e = nullptr;
        FDE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->side_done.push_back(e);
    }
    if (!c->fork_ev) FDE_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
}

// fn(group, stream) for every group with right-hand sides
template <class F>
void apply_groups(Ctx* c, std::vector<Group>& groups, F fn) {
    int active = 0;
    for (auto& g : groups)
        if (g.nr) ++active;
    if (active <= 1 || c->nside == 0) {
        for (auto& g : groups)
            if (g.nr) fn(g, c->stream);
        return;
    }
    ensure_side_streams(c);
    const int ns = c->nside;
    FDE_HIP(hipEventRecord(c->fork_ev, c->stream));
    for (int k = 0; k < ns; ++k) FDE_HIP(hipStreamWaitEvent(c->side[k], c->fork_ev, 0));
    std::vector<Op*> seen;   // operator -> stream slot (0: the context's stream)
    for (auto& g : groups) {
        if (!g.nr) continue;
        size_t slot = std::find(seen.begin(), seen.end(), g.op) - seen.begin();
        if (slot == seen.size()) seen.push_back(g.op);
        const int k = (int)(slot % (ns + 1));
        fn(g, k == 0 ? c->stream : c->side[k - 1]);
    }
    for (int k = 0; k < ns; ++k) {
        FDE_HIP(hipEventRecord(c->side_done[k], c->side[k]));
        FDE_HIP(hipStreamWaitEvent(c->stream, c->side_done[k], 0));
    }
}

template <class T>
Inst<T> group_inst(Group& g, int m) {
    Inst<T> d = g.prec->inst<T>(true, g.nr, g.V.p, g.op->Nd, g.Z.p, g.op->Nd);
    d.work = reinterpret_cast<T*>(g.work.p);
    d.rhs = reinterpret_cast<T*>(g.rhs.p);
    d.bstep = (int64_t)g.op->Nd * g.nr;
    d.flops = g.prec->flops.p + 1;
    d.xstep = (int64_t)g.op->Nd * g.nr;
    (void)m;
    return d;
}

// Left-preconditioned BiCGSTAB of every system in lock step: per step two applies of A per
// operator (on the side streams), two H-solves per group and two fused update kernels; the host
// reads back the number of systems still iterating once per step.
void run_bicgstab(Ctx* c, std::vector<Group>& groups, int ns, int maxit, double rtol, fde_solve_info* info,
                  int* rc_out) {
    hipStream_t st = c->stream;
    struct BGroup {
        DevBuf<double> r, rh, p, s, v, t, W;
    };
    std::vector<BGroup> bg(groups.size());
    std::vector<BicgDev> sys;
    std::vector<int> mask;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group& g = groups[gi];
        if (!g.nr) continue;
        BGroup& b = bg[gi];
        const size_t bs = (size_t)g.op->Nd * g.nr;
        for (DevBuf<double>* d : {&b.r, &b.rh, &b.p, &b.s, &b.v, &b.t, &b.W}) d->alloc(c, bs);
        for (int k = 0; k < g.nr; ++k) {
            BicgDev d{};
            d.G = g.G + (int64_t)k * g.ldg;
            d.X = g.X + (int64_t)k * g.ldx;
            d.r = b.r.p;
            d.rh = b.rh.p;
            d.p = b.p.p;
            d.s = b.s.p;
            d.v = b.v.p;
            d.t = b.t.p;
            d.W = b.W.p;
            d.Nd = g.op->Nd;
            d.c = k;
            sys.push_back(d);
            mask.push_back(g.prec ? 0 : 1);
        }
        const size_t need = g.op->apply_ws_doubles(g.nr);
        if (g.op->ws.n < need) g.op->ws.alloc(c, need);
    }
    DevBuf<BicgDev> d_sys;
    DevBuf<BicgState> d_ss;
    DevBuf<int> d_mask, d_count;
    d_sys.alloc(c, sys.size());
    d_ss.alloc(c, ns);
    d_mask.alloc(c, ns);
    d_count.alloc(c, 1);
    upload(c, d_sys.p, sys.data(), sys.size() * sizeof(BicgDev));
    upload(c, d_mask.p, mask.data(), ns * sizeof(int));
    const bool any_copy = std::any_of(mask.begin(), mask.end(), [](int v) { return v != 0; });
    // M applied to the blocks of every group with a preconditioner: dst <- A~^{-1} src
    auto precond = [&](int which) {
        if (any_copy) bc_copy(st, ns, d_sys.p, d_mask.p, which);
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Group& g = groups[gi];
            if (!g.nr || !g.prec) continue;
            BGroup& b = bg[gi];
            const int Nd = g.op->Nd;
            if (which == 0)
                hlu_solve(g.prec, g.nr, g.G, g.ldg, b.r.p, Nd);
            else
                hlu_solve(g.prec, g.nr, b.W.p, Nd, which == 1 ? b.v.p : b.t.p, Nd);
        }
    };
    auto apply_into_W = [&](int which) {   // W <- A p (0), A s (1), A x (2)
        apply_groups(c, groups, [&](Group& g, hipStream_t s) {
            BGroup& b = bg[&g - groups.data()];
            const double* src = which == 0 ? b.p.p : (which == 1 ? b.s.p : nullptr);
            if (which == 2)
                stiffness_apply(g.op, g.nr, g.X, g.ldx, b.W.p, g.op->Nd, 0.0, 0.0, false, s);
            else
                stiffness_apply(g.op, g.nr, src, g.op->Nd, b.W.p, g.op->Nd, 0.0, 0.0, false, s);
        });
    };
    precond(0);
    bc_init(st, ns, d_sys.p, d_ss.p, maxit);
    for (int it = 0; it < maxit; ++it) {
        apply_into_W(0);
        precond(1);
        bc_half1(st, ns, d_sys.p, d_ss.p, rtol);
        apply_into_W(1);
        precond(2);
        bc_half2(st, ns, d_sys.p, d_ss.p, rtol, maxit);
        int active = 0;
        bc_count_active(st, ns, d_ss.p, d_count.p);
        FDE_HIP(hipMemcpyAsync(&active, d_count.p, sizeof(int), hipMemcpyDeviceToHost, st));
        FDE_HIP(hipStreamSynchronize(st));
        if (active == 0) break;
    }
    apply_into_W(2);
    bc_true_residual(st, ns, d_sys.p, d_ss.p);
    std::vector<BicgState> hs(ns);
    FDE_HIP(hipMemcpyAsync(hs.data(), d_ss.p, ns * sizeof(BicgState), hipMemcpyDeviceToHost, st));
    FDE_HIP(hipStreamSynchronize(st));
    int rc = FDE_OK;
    for (int k = 0; k < ns; ++k) {
        info[k].iters = hs[k].iters;
        info[k].relres = hs[k].truerel;
        info[k].status = hs[k].conv ? FDE_OK
                                    : (hs[k].status == -3 ? FDE_EBREAKDOWN : (hs[k].status ? FDE_EDEVICE : FDE_ENOCONV));
        if (!hs[k].conv) rc = hs[k].status == -3 ? FDE_EBREAKDOWN : FDE_ENOCONV;
    }
    *rc_out = rc;
}

void run(Ctx* c, int n, fde_op* const* ops, fde_hlu* const* precs, const int* nrhs, const double* const* G,
         const int* ldg, double* const* X, const int* ldx, const fde_solve_params* prm, fde_solve_info* info,
         int* rc_out) {
    const int m = prm ? prm->restart : 30;
    const int maxit = prm ? prm->maxit : 500;
    const double rtol = prm ? prm->rtol : 1e-10;
    const int method = prm ? prm->method : FDE_FGMRES;
    if (method != FDE_FGMRES && method != FDE_BICGSTAB) fail(FDE_EINVAL, "unknown Krylov method %d", method);
    if (method == FDE_FGMRES && (m < 1 || m > kMaxRestart))
        fail(FDE_EINVAL, "restart must be in [1, %d] (got %d)", kMaxRestart, m);
    if (maxit < 1) fail(FDE_EINVAL, "maxit must be >= 1");
    if (!(rtol > 0.0)) fail(FDE_EINVAL, "rtol must be > 0");
    hipStream_t st = c->stream;
    std::vector<Group> groups(n);
    int ns = 0;
    for (int i = 0; i < n; ++i) {
        Op* op = ops[i];
        if (!op || op->ctx != c) fail(FDE_EINVAL, "system %d: operator missing or from another context", i);
        if (nrhs[i] < 0 || (nrhs[i] > 0 && (!G[i] || !X[i])) || ldg[i] < op->Nd || ldx[i] < op->Nd)
            fail(FDE_EINVAL, "system %d: bad right-hand side arguments", i);
        HLUObj* f = precs ? precs[i] : nullptr;
        if (f && f->op != op) fail(FDE_EINVAL, "system %d: preconditioner built for another operator", i);
        Group& g = groups[i];
        g.op = op;
        g.prec = f;
        g.nr = nrhs[i];
        g.G = G[i];
        g.ldg = ldg[i];
        g.X = X[i];
        g.ldx = ldx[i];
        g.sys0 = ns;
        ns += g.nr;
    }
    if (ns == 0) {
        *rc_out = FDE_OK;
        return;
    }
    if (method == FDE_BICGSTAB) {
        run_bicgstab(c, groups, ns, maxit, rtol, info, rc_out);
        return;
    }
    std::vector<SysDev> sys;
    std::vector<int> mask(ns, 0);
    std::vector<Inst<float>> i32;
    std::vector<Inst<double>> i64;
    struct HsLaunch {
        bool lds = true, bf16 = false, gx = false;
        int wc = 1, nchunk = 1;
        size_t bytes = 0;
        std::vector<std::pair<const HLUObj*, int>> members;   // factors and their chunk widths
    } hs32, hs64;
    int prec_cols = 0;   // columns of every preconditioned group: the H-solve launches' width
    for (auto& g : groups)
        if (g.prec) prec_cols += g.nr;
    for (auto& g : groups) {
        if (g.nr == 0) continue;
        const int64_t bs = (int64_t)g.op->Nd * g.nr;
        g.V.alloc(c, (m + 1) * bs);
        g.Z.alloc(c, m * bs);
        g.W.alloc(c, bs);
        g.R.alloc(c, bs);
        FDE_HIP(hipMemsetAsync(g.V.p, 0, g.V.bytes(), st));
        FDE_HIP(hipMemsetAsync(g.Z.p, 0, g.Z.bytes(), st));
        for (int k = 0; k < g.nr; ++k) {
            SysDev s{};
            s.V = g.V.p;
            s.Z = g.Z.p;
            s.W = g.W.p;
            s.R = g.R.p;
            s.G = g.G + (int64_t)k * g.ldg;
            s.X = g.X + (int64_t)k * g.ldx;
            s.bs = bs;
            s.Nd = g.op->Nd;
            s.c = k;
            sys.push_back(s);
            mask[g.sys0 + k] = g.prec ? 0 : 1;
        }
        if (g.prec) {
            // leaf-step H-solve workspace: whole chunks of columns (where the right-hand sides
            // stay in global memory the last chunk is written in full)
            g.rhs.alloc(c, hsolve_rhs_elems(g.op->Nd, g.nr) * g.prec->esz);
            g.work.alloc(c, std::max<int64_t>(g.prec->plan->sv.work_elems, 1) * g.nr * g.prec->esz);
            // leaf-step H-solve: each system with its own chunk width (as when solved alone); a
            // launch per precision sized for the largest, with the right-hand sides in global
            // memory for all if one needs it; any system that does not fit at all sends its
            // precision to the op-list interpreter
            HsLaunch& h = g.prec->prec == FDE_FP64 ? hs64 : hs32;
            size_t b = 0;
            bool gx = false;
            const int w = hsolve_cols(c, g.prec, g.nr, &b, &gx, prec_cols);
            require_lds_for_bf16(g.prec, w);
            h.bf16 = h.bf16 || g.prec->bf16uv;
            if (w == 0) {
                h.lds = false;
            } else {
                h.wc = std::max(h.wc, w);
                h.nchunk = std::max(h.nchunk, (g.nr + w - 1) / w);
                h.gx = h.gx || gx;
                h.members.push_back({g.prec, w});
                h.bytes = std::max(h.bytes, b);
            }
            if (g.prec->prec == FDE_FP64) {
                i64.push_back(group_inst<double>(g, m));
                i64.back().hs_wc = w;
            } else {
                i32.push_back(group_inst<float>(g, m));
                i32.back().hs_wc = w;
            }
        }
    }
    for (HsLaunch* h : {&hs32, &hs64})
        if (h->gx) {   // one launch: every member's chunk with its right-hand sides in global memory
            h->bytes = 0;
            for (auto& m : h->members) h->bytes = std::max(h->bytes, hsolve_lds_for(m.first, m.second, true));
        }
    DevBuf<SysDev> d_sys;
    DevBuf<SysState> d_ss;
    DevBuf<int> d_mask, d_count;
    DevBuf<Inst<float>> d_i32;
    DevBuf<Inst<double>> d_i64;
    d_sys.alloc(c, sys.size());
    d_ss.alloc(c, ns);
    d_mask.alloc(c, ns);
    d_count.alloc(c, 1);
    upload(c, d_sys.p, sys.data(), sys.size() * sizeof(SysDev));
    upload(c, d_mask.p, mask.data(), ns * sizeof(int));
    if (!i32.empty()) {
        d_i32.alloc(c, i32.size());
        upload(c, d_i32.p, i32.data(), i32.size() * sizeof(Inst<float>));
    }
    if (!i64.empty()) {
        d_i64.alloc(c, i64.size());
        upload(c, d_i64.p, i64.data(), i64.size() * sizeof(Inst<double>));
    }
    const bool any_copy = std::any_of(mask.begin(), mask.end(), [](int v) { return v != 0; });
    // apply workspaces come from the context's cache, ordered on its stream: reserve them here,
    // before any apply runs on a side stream
    for (auto& g : groups)
        if (g.nr) {
            const size_t need = g.op->apply_ws_doubles(g.nr);
            if (g.op->ws.n < need) g.op->ws.alloc(c, need);
        }
    fg_gnorm(st, ns, d_sys.p, d_ss.p);
    fg_zero_x(st, ns, d_sys.p);
    std::vector<SysState> hs(ns);
    bool first = true;
    for (;;) {
        fg_cycle_start(st, ns, d_sys.p, d_ss.p, first ? 1 : 0, maxit);
        first = false;
        for (int j = 0; j < m; ++j) {
            if (any_copy) fg_copy_step(st, ns, d_sys.p, d_mask.p, j);
            if (!i32.empty()) {
                if (hs32.lds)
                    launch_hsolve<float>(st, (int)i32.size(), hs32.nchunk, hs32.wc, d_i32.p, j, hs32.bytes, hs32.bf16,
                                         hs32.gx);
                else
                    launch_interp<float>(st, (int)i32.size(), d_i32.p, j);
            }
            if (!i64.empty()) {
                if (hs64.lds)
                    launch_hsolve<double>(st, (int)i64.size(), hs64.nchunk, hs64.wc, d_i64.p, j, hs64.bytes, false,
                                          hs64.gx);
                else
                    launch_interp<double>(st, (int)i64.size(), d_i64.p, j);
            }
            apply_groups(c, groups, [&](Group& g, hipStream_t s) {
                stiffness_apply(g.op, g.nr, g.Z.p + (int64_t)j * g.op->Nd * g.nr, g.op->Nd, g.W.p, g.op->Nd, 0.0, 0.0,
                                false, s);
            });
            fg_arnoldi(st, ns, d_sys.p, d_ss.p, j, m, rtol, maxit);
            int active = 0;
            fg_count_active(st, ns, d_ss.p, d_count.p);
            FDE_HIP(hipMemcpyAsync(&active, d_count.p, sizeof(int), hipMemcpyDeviceToHost, st));
            FDE_HIP(hipStreamSynchronize(st));
            if (active == 0) break;
        }
        fg_update(st, ns, d_sys.p, d_ss.p);
        apply_groups(c, groups, [&](Group& g, hipStream_t s) {
            stiffness_apply(g.op, g.nr, g.X, g.ldx, g.R.p, g.op->Nd, 0.0, 0.0, false, s);
        });
        fg_check(st, ns, d_sys.p, d_ss.p, rtol);
        FDE_HIP(hipMemcpyAsync(hs.data(), d_ss.p, ns * sizeof(SysState), hipMemcpyDeviceToHost, st));
        FDE_HIP(hipStreamSynchronize(st));
        bool more = false;
        for (const auto& s : hs)
            if (!s.conv && s.status == 0 && s.iters < maxit) more = true;
        if (!more) break;
    }
    int rc = FDE_OK;
    for (int k = 0; k < ns; ++k) {
        info[k].iters = hs[k].iters;
        info[k].relres = hs[k].relres;
        info[k].status = hs[k].conv ? FDE_OK : (hs[k].status ? FDE_EINVAL : FDE_ENOCONV);
        if (!hs[k].conv) rc = FDE_ENOCONV;
    }
    *rc_out = rc;
}

}  // namespace

// ------------------------------------------------------------------ continuous engine
//
// Every request owns its Krylov blocks and nrhs system slots in the engine's fixed device arrays
// (SysDev, SysState), and keeps its own Arnoldi step j. A step launches, over the requests
// running a cycle: the copy of unpreconditioned blocks, one H-solve launch per precision (each
// request's instance points at its own block j), the applies (side streams), and one Arnoldi
// launch whose blocks read their slot and step from index arrays. Requests whose cycle ended get
// the update, the true residual and the check, read back at the next step; they then finish or
// start a new cycle. The kernels act per system, so a request's bits do not depend on the others.

struct EGroup {
    long long id = 0;
    Op* op = nullptr;
    HLUObj* prec = nullptr;
    int nr = 0;
    const double* G = nullptr;
    int ldg = 0;
    double* X = nullptr;
    int ldx = 0;
    std::vector<int> slots;
    DevBuf<int> d_slots;
    int j = 0;
    enum Phase { START, RUN, CHECK } phase = START;
    bool finished = false;
    DevBuf<double> V, Z, W, R;
    DevBuf<char> rhs, work;
    int hs_wc = 0;            // leaf-step H-solve columns per workgroup (0: interpreter)
    size_t hs_bytes = 0;
    bool hs_gx = false;       // its right-hand sides only fit in global memory
};

struct KrylovEngine {
    Ctx* c = nullptr;
    int m = 30, maxit = 500;
    double rtol = 1e-10;
    int cap = 0;
    DevBuf<SysDev> d_sys;
    DevBuf<SysState> d_ss;
    DevBuf<int> d_mask, d_sel, d_jv, d_sel_all, d_start;
    DevBuf<SysStatus> d_stat;
    DevBuf<Inst<float>> d_i32;
    DevBuf<Inst<double>> d_i64;
    std::vector<int> free_slots;
    std::list<std::unique_ptr<EGroup>> groups;
};

KrylovEngine* engine_create(Ctx* c, int restart, int maxit, double rtol, int max_systems) {
    if (restart < 1 || restart > kMaxRestart) fail(FDE_EINVAL, "restart must be in [1, %d]", kMaxRestart);
    if (maxit < 1 || !(rtol > 0.0) || max_systems < 1) fail(FDE_EINVAL, "bad engine parameters");
    auto e = std::make_unique<KrylovEngine>();
    e->c = c;
    e->m = restart;
    e->maxit = maxit;
    e->rtol = rtol;
    e->cap = max_systems;
    e->d_sys.alloc(c, max_systems);
    e->d_ss.alloc(c, max_systems);
    e->d_mask.alloc(c, max_systems);
    for (DevBuf<int>* b : {&e->d_sel, &e->d_jv, &e->d_sel_all, &e->d_start}) b->alloc(c, max_systems);
    e->d_stat.alloc(c, max_systems);
    e->d_i32.alloc(c, max_systems);
    e->d_i64.alloc(c, max_systems);
    for (int k = max_systems - 1; k >= 0; --k) e->free_slots.push_back(k);
    return e.release();
}

void engine_destroy(KrylovEngine* e) {
    if (!e) return;
    (void)hipStreamSynchronize(e->c->stream);
    delete e;
}

int engine_free_slots(const KrylovEngine* e) { return (int)e->free_slots.size(); }
int engine_groups(const KrylovEngine* e) { return (int)e->groups.size(); }

void engine_add(KrylovEngine* e, Op* op, HLUObj* prec, int nrhs, const double* G, int ldg, double* X, int ldx,
                long long id) {
    Ctx* c = e->c;
    hipStream_t st = c->stream;
    if (nrhs < 1 || nrhs > (int)e->free_slots.size()) fail(FDE_EINVAL, "engine: %d columns, %zu free slots", nrhs,
                                                            e->free_slots.size());
    if (!op || op->ctx != c || (prec && prec->op != op)) fail(FDE_EINVAL, "engine: operator or preconditioner");
    if (!G || !X || ldg < op->Nd || ldx < op->Nd) fail(FDE_EINVAL, "engine: bad right-hand side arguments");
    auto g = std::make_unique<EGroup>();
    g->id = id;
    g->op = op;
    g->prec = prec;
    g->nr = nrhs;
    g->G = G;
    g->ldg = ldg;
    g->X = X;
    g->ldx = ldx;
    const int64_t bs = (int64_t)op->Nd * nrhs;
    g->V.alloc(c, (e->m + 1) * bs);
    g->Z.alloc(c, e->m * bs);
    g->W.alloc(c, bs);
    g->R.alloc(c, bs);
    FDE_HIP(hipMemsetAsync(g->V.p, 0, g->V.bytes(), st));
    FDE_HIP(hipMemsetAsync(g->Z.p, 0, g->Z.bytes(), st));
    FDE_HIP(hipMemsetAsync(g->R.p, 0, g->R.bytes(), st));   // A x_0 = 0: the first cycle starts from G
    if (prec) {
        g->rhs.alloc(c, hsolve_rhs_elems(op->Nd, nrhs) * prec->esz);
        g->work.alloc(c, std::max<int64_t>(prec->plan->sv.work_elems, 1) * nrhs * prec->esz);
        g->hs_wc = hsolve_cols(c, prec, nrhs, &g->hs_bytes, &g->hs_gx, nrhs);
        require_lds_for_bf16(prec, g->hs_wc);
    }
    const size_t need = op->apply_ws_doubles(nrhs);
    if (op->ws.n < need) op->ws.alloc(c, need);
    for (int k = 0; k < nrhs; ++k) {
        const int slot = e->free_slots.back();
        e->free_slots.pop_back();
        g->slots.push_back(slot);
        SysDev d{};
        d.V = g->V.p;
        d.Z = g->Z.p;
        d.W = g->W.p;
        d.R = g->R.p;
        d.G = G + (int64_t)k * ldg;
        d.X = X + (int64_t)k * ldx;
        d.bs = bs;
        d.Nd = op->Nd;
        d.c = k;
        upload(c, e->d_sys.p + slot, &d, sizeof d);
        const int mk = prec ? 0 : 1;
        upload(c, e->d_mask.p + slot, &mk, sizeof mk);
    }
    g->d_slots.alloc(c, nrhs);
    upload(c, g->d_slots.p, g->slots.data(), nrhs * sizeof(int));
    fg_gnorm(st, nrhs, e->d_sys.p, e->d_ss.p, g->d_slots.p);
    fg_zero_x(st, nrhs, e->d_sys.p, g->d_slots.p);
    e->groups.push_back(std::move(g));
}

namespace {

// H-solves of block j of every running group with a preconditioner of precision T, one launch
template <class T>
void engine_hsolve(KrylovEngine* e, std::vector<EGroup*>& run, DevBuf<Inst<T>>& d_inst, int prec_code) {
    std::vector<Inst<T>> insts;
    bool lds = true, bf16 = false, gx = false;
    int wc = 1, nchunk = 1;
    size_t bytes = 0;
    for (EGroup* g : run) {
        if (!g->prec || g->prec->prec != prec_code) continue;
        const int64_t bs = (int64_t)g->op->Nd * g->nr;
        Inst<T> d = g->prec->inst<T>(true, g->nr, g->V.p + g->j * bs, g->op->Nd, g->Z.p + g->j * bs, g->op->Nd);
        d.work = reinterpret_cast<T*>(g->work.p);
        d.rhs = reinterpret_cast<T*>(g->rhs.p);
        d.flops = g->prec->flops.p + 1;
        d.hs_wc = g->hs_wc;
        insts.push_back(d);
        bf16 = bf16 || g->prec->bf16uv;
        if (g->hs_wc == 0) {
            lds = false;
        } else {
            wc = std::max(wc, g->hs_wc);
            nchunk = std::max(nchunk, (g->nr + g->hs_wc - 1) / g->hs_wc);
            bytes = std::max(bytes, g->hs_bytes);
            gx = gx || g->hs_gx;
        }
    }
    if (insts.empty()) return;
    if (lds && gx) {   // one launch: every chunk with its right-hand sides in global memory
        bytes = 0;
        for (EGroup* g : run)
            if (g->prec && g->prec->prec == prec_code) bytes = std::max(bytes, hsolve_lds_for(g->prec, g->hs_wc, true));
    }
    upload(e->c, d_inst.p, insts.data(), insts.size() * sizeof(Inst<T>));
    if (lds)
        launch_hsolve<T>(e->c->stream, (int)insts.size(), nchunk, wc, d_inst.p, 0, bytes, bf16, gx);
    else
        launch_interp<T>(e->c->stream, (int)insts.size(), d_inst.p, 0);
}

// fn(group, stream) over groups, each operator's groups on one of the context's streams
template <class F>
void engine_apply(Ctx* c, std::vector<EGroup*>& gs, F fn) {
    if (gs.size() <= 1 || c->nside == 0) {
        for (EGroup* g : gs) fn(*g, c->stream);
        return;
    }
    ensure_side_streams(c);
    const int ns = c->nside;
    FDE_HIP(hipEventRecord(c->fork_ev, c->stream));
    for (int k = 0; k < ns; ++k) FDE_HIP(hipStreamWaitEvent(c->side[k], c->fork_ev, 0));
    std::vector<Op*> seen;
    for (EGroup* g : gs) {
        size_t slot = std::find(seen.begin(), seen.end(), g->op) - seen.begin();
        if (slot == seen.size()) seen.push_back(g->op);
        const int k = (int)(slot % (ns + 1));
        fn(*g, k == 0 ? c->stream : c->side[k - 1]);
    }
    for (int k = 0; k < ns; ++k) {
        FDE_HIP(hipEventRecord(c->side_done[k], c->side[k]));
        FDE_HIP(hipStreamWaitEvent(c->stream, c->side_done[k], 0));
    }
}

}  // namespace

void engine_step(KrylovEngine* e, std::vector<EngineDone>& done) {
    Ctx* c = e->c;
    hipStream_t st = c->stream;
    if (e->groups.empty()) return;
    // new requests start their first cycle
    std::vector<int> start;
    for (auto& g : e->groups)
        if (g->phase == EGroup::START) {
            start.insert(start.end(), g->slots.begin(), g->slots.end());
            g->phase = EGroup::RUN;
            g->j = 0;
        }
    if (!start.empty()) {
        upload(c, e->d_start.p, start.data(), start.size() * sizeof(int));
        fg_cycle_start(st, (int)start.size(), e->d_sys.p, e->d_ss.p, 0, e->maxit, e->d_start.p);
    }
    // one Arnoldi step of every running request
    std::vector<EGroup*> run;
    std::vector<int> sel, jv;
    for (auto& g : e->groups)
        if (g->phase == EGroup::RUN) {
            run.push_back(g.get());
            for (int s : g->slots) {
                sel.push_back(s);
                jv.push_back(g->j);
            }
        }
    if (!run.empty()) {
        upload(c, e->d_sel.p, sel.data(), sel.size() * sizeof(int));
        upload(c, e->d_jv.p, jv.data(), jv.size() * sizeof(int));
        fg_copy_step(st, (int)sel.size(), e->d_sys.p, e->d_mask.p, 0, e->d_sel.p, e->d_jv.p);
        engine_hsolve<float>(e, run, e->d_i32, FDE_FP32);
        engine_hsolve<double>(e, run, e->d_i64, FDE_FP64);
        engine_apply(c, run, [&](EGroup& g, hipStream_t s) {
            const int64_t bs = (int64_t)g.op->Nd * g.nr;
            stiffness_apply(g.op, g.nr, g.Z.p + g.j * bs, g.op->Nd, g.W.p, g.op->Nd, 0.0, 0.0, false, s);
        });
        fg_arnoldi(st, (int)sel.size(), e->d_sys.p, e->d_ss.p, 0, e->m, e->rtol, e->maxit, e->d_sel.p, e->d_jv.p);
    }
    // status of the running requests and of those whose check was queued in the step before
    std::vector<EGroup*> seen;
    std::vector<int> all;
    for (auto& g : e->groups)
        if (g->phase == EGroup::RUN || g->phase == EGroup::CHECK) {
            seen.push_back(g.get());
            all.insert(all.end(), g->slots.begin(), g->slots.end());
        }
    std::vector<SysStatus> hst(all.size());
    if (!all.empty()) {
        upload(c, e->d_sel_all.p, all.data(), all.size() * sizeof(int));
        fg_gather_status(st, (int)all.size(), e->d_ss.p, e->d_sel_all.p, e->d_stat.p);
        FDE_HIP(hipMemcpyAsync(hst.data(), e->d_stat.p, all.size() * sizeof(SysStatus), hipMemcpyDeviceToHost, st));
    }
    FDE_HIP(hipStreamSynchronize(st));
    size_t k = 0;
    std::vector<EGroup*> cycle_end, restart;
    for (EGroup* g : seen) {
        const SysStatus* s = hst.data() + k;
        k += g->slots.size();
        if (g->phase == EGroup::CHECK) {
            bool more = false;
            for (int i = 0; i < g->nr; ++i)
                if (!s[i].conv && s[i].status == 0 && s[i].iters < e->maxit) more = true;
            if (more) {
                restart.push_back(g);
                continue;
            }
            EngineDone d;
            d.id = g->id;
            for (int i = 0; i < g->nr; ++i)
                d.info.push_back(fde_solve_info{s[i].iters, s[i].relres,
                                                s[i].conv ? FDE_OK : (s[i].status ? FDE_EINVAL : FDE_ENOCONV)});
            done.push_back(std::move(d));
            g->finished = true;
            continue;
        }
        // running: the step was taken; the cycle ends once no system of the request is active
        g->j += 1;
        bool any = false;
        for (int i = 0; i < g->nr; ++i) any = any || s[i].active;
        if (!any) cycle_end.push_back(g);
    }
    // finished requests leave (their slots are free for the next admission)
    for (auto it = e->groups.begin(); it != e->groups.end();) {
        if ((*it)->finished) {
            for (int s : (*it)->slots) e->free_slots.push_back(s);
            it = e->groups.erase(it);
        } else {
            ++it;
        }
    }
    // cycle ends: x += Z y, the true residual G - A x, the convergence check (read at the next step)
    for (EGroup* g : cycle_end) {
        fg_update(st, g->nr, e->d_sys.p, e->d_ss.p, g->d_slots.p);
        g->phase = EGroup::CHECK;
    }
    engine_apply(c, cycle_end, [&](EGroup& g, hipStream_t s) {
        stiffness_apply(g.op, g.nr, g.X, g.ldx, g.R.p, g.op->Nd, 0.0, 0.0, false, s);
    });
    for (EGroup* g : cycle_end) fg_check(st, g->nr, e->d_sys.p, e->d_ss.p, e->rtol, g->d_slots.p);
    // checked and not converged: a new cycle from the true residual
    for (EGroup* g : restart) {
        fg_cycle_start(st, g->nr, e->d_sys.p, e->d_ss.p, 0, e->maxit, g->d_slots.p);
        g->phase = EGroup::RUN;
        g->j = 0;
    }
}

// ------------------------------------------------------------------ singular value estimates
//
// m steps of Arnoldi (classical Gram-Schmidt twice, the FGMRES kernels) on an operator B from a
// seeded start vector; the singular values of the resulting (m+1) x m Hessenberg matrix bound
// those of B from inside [sigma_min(B), sigma_max(B)] and reach them as the Krylov space fills
// (exactly once m = Nd). B is one of: A; A^{-1} (each product a right-preconditioned FGMRES solve
// to 1e-13 with the given H-LU); A~^{-1} as the H-LU solve (exact when the factors are); A~^{-1} A.
void sigma_estimate(Op* op, HLUObj* f, int kind, int m, const double* v0_host, double* smax, double* smin) {
    Ctx* c = op->ctx;
    hipStream_t st = c->stream;
    const int Nd = op->Nd;
    if (m < 1 || m > kMaxRestart || m > Nd) fail(FDE_EINVAL, "steps must be in [1, min(%d, Nd)]", kMaxRestart);
    if (kind != FDE_SIGMA_A && !f) fail(FDE_EINVAL, "this estimate needs the H-LU factors");
    if (f && f->op != op) fail(FDE_EINVAL, "factors built for another operator");
    DevBuf<double> V, Z, W, R, G, X;
    V.alloc(c, (int64_t)(m + 1) * Nd);
    Z.alloc(c, (int64_t)m * Nd);
    W.alloc(c, Nd);
    R.alloc(c, Nd);
    G.alloc(c, Nd);
    X.alloc(c, Nd);
    FDE_HIP(hipMemsetAsync(V.p, 0, V.bytes(), st));
    FDE_HIP(hipMemsetAsync(R.p, 0, R.bytes(), st));
    upload(c, G.p, v0_host, sizeof(double) * Nd);
    SysDev d{};
    d.V = V.p;
    d.Z = Z.p;
    d.W = W.p;
    d.R = R.p;
    d.G = G.p;
    d.X = X.p;
    d.bs = Nd;
    d.Nd = Nd;
    d.c = 0;
    DevBuf<SysDev> d_sys;
    DevBuf<SysState> d_ss;
    DevBuf<double> d_out;
    d_sys.alloc(c, 1);
    d_ss.alloc(c, 1);
    d_out.alloc(c, 2);
    upload(c, d_sys.p, &d, sizeof d);
    fg_gnorm(st, 1, d_sys.p, d_ss.p);
    fg_cycle_start(st, 1, d_sys.p, d_ss.p, 1, m + 1);   // v_0 = G / |G|
    const size_t need = op->apply_ws_doubles(1);
    if (op->ws.n < need) op->ws.alloc(c, need);
    DevBuf<double> T;
    T.alloc(c, Nd);
    fde_solve_params sp{FDE_FGMRES, 30, 1000, 1e-13};
    for (int j = 0; j < m; ++j) {
        double* vj = V.p + (int64_t)j * Nd;
        switch (kind) {
            case FDE_SIGMA_A:
                stiffness_apply(op, 1, vj, Nd, W.p, Nd, 0.0, 0.0, false);
                break;
            case FDE_SIGMA_AINV: {
                fde_op* ops[1] = {static_cast<fde_op*>(op)};
                fde_hlu* precs[1] = {static_cast<fde_hlu*>(f)};
                int nr = 1, ld = Nd;
                const double* Gs[1] = {vj};
                double* Xs[1] = {W.p};
                fde_solve_info info{};
                int rc = FDE_OK;
                run(c, 1, ops, precs, &nr, Gs, &ld, Xs, &ld, &sp, &info, &rc);
                if (rc != FDE_OK) fail(rc, "sigma estimate: an inner solve did not converge");
                break;
            }
            case FDE_SIGMA_ATILDE_INV:
                hlu_solve(f, 1, vj, Nd, W.p, Nd);
                break;
            case FDE_SIGMA_PRECOND:
                stiffness_apply(op, 1, vj, Nd, T.p, Nd, 0.0, 0.0, false);
                hlu_solve(f, 1, T.p, Nd, W.p, Nd);
                break;
            default:
                fail(FDE_EINVAL, "unknown estimate kind %d", kind);
        }
        // rtol < 0: no residual test (on a well-conditioned operator the GMRES residual estimate
        // can reach zero long before the space is full)
        fg_arnoldi(st, 1, d_sys.p, d_ss.p, j, m, -1.0, m + 1);
    }
    fg_sigma(st, d_ss.p, m, d_out.p);
    double out[2];
    FDE_HIP(hipMemcpyAsync(out, d_out.p, sizeof out, hipMemcpyDeviceToHost, st));
    FDE_HIP(hipStreamSynchronize(st));
    *smax = out[0];
    *smin = out[1];
}

// run() with the systems of operators that have a degree per element taken to the extended
// unknowns: their right-hand sides scattered (zero on the outside unknowns, which then stay zero
// in every Krylov vector), their solutions gathered back
void run_public(Ctx* c, int n, fde_op* const* ops, fde_hlu* const* precs, const int* nrhs, const double* const* G,
                const int* ldg, double* const* X, const int* ldx, const fde_solve_params* prm, fde_solve_info* info,
                int* rc_out) {
    bool any = false;
    for (int i = 0; i < n; ++i) any = any || (ops[i] && ops[i]->hp);
    if (!any) {
        run(c, n, ops, precs, nrhs, G, ldg, X, ldx, prm, info, rc_out);
        return;
    }
    std::vector<const double*> g(G, G + n);
    std::vector<double*> x(X, X + n);
    std::vector<int> lg(ldg, ldg + n), lx(ldx, ldx + n);
    std::vector<DevBuf<double>> ge(n), xe(n);
    for (int i = 0; i < n; ++i) {
        Op* op = ops[i];
        if (!op || !op->hp || nrhs[i] <= 0) continue;
        if (op->ctx != c) fail(FDE_EINVAL, "system %d: operator from another context", i);
        if (!G[i] || !X[i] || ldg[i] < op->hp_nd || ldx[i] < op->hp_nd)
            fail(FDE_EINVAL, "system %d: bad right-hand side arguments", i);
        ge[i].alloc(c, (size_t)op->Nd * nrhs[i]);
        xe[i].alloc(c, (size_t)op->Nd * nrhs[i]);
        hp_scatter(op, nrhs[i], G[i], ldg[i], ge[i].p, op->Nd, c->stream);
        g[i] = ge[i].p;
        x[i] = xe[i].p;
        lg[i] = lx[i] = op->Nd;
    }
    run(c, n, ops, precs, nrhs, g.data(), lg.data(), x.data(), lx.data(), prm, info, rc_out);
    for (int i = 0; i < n; ++i)
        if (ops[i]->hp && nrhs[i] > 0) hp_gather(ops[i], nrhs[i], xe[i].p, ops[i]->Nd, X[i], ldx[i], c->stream);
    FDE_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace fde

using namespace fde;

extern "C" {

int fde_solve(fde_op* op, fde_hlu* prec, int nrhs, const double* G, int ldg, double* X, int ldx,
              const fde_solve_params* prm, fde_solve_info* info) {
    int rc = FDE_OK;
    try {
        if (!op || !info) fail(FDE_EINVAL, "null operator or info");
        fde_op* ops[1] = {op};
        fde_hlu* precs[1] = {prec};
        const double* Gs[1] = {G};
        double* Xs[1] = {X};
        run_public(op->ctx, 1, ops, precs, &nrhs, Gs, &ldg, Xs, &ldx, prm, info, &rc);
    } catch (const Error& e) {
        set_error("%s", e.msg.c_str());
        return e.code;
    } catch (...) {
        set_error("unexpected internal error");
        return FDE_EDEVICE;
    }
    if (rc == FDE_ENOCONV) set_error("the Krylov solver did not reach rtol within maxit for at least one right-hand side");
    if (rc == FDE_EBREAKDOWN) set_error("BiCGSTAB broke down (a vanishing inner product) for at least one right-hand side");
    return rc;
}

int fde_sigma_estimate(fde_op* op, fde_hlu* f, int kind, int steps, unsigned long long seed, double* smax,
                       double* smin) {
    FDE_API_BEGIN
    if (!op || !smax || !smin) fail(FDE_EINVAL, "null argument");
    if (op->hp) fail(FDE_EUNSUPPORTED, "fde_sigma_estimate: one degree per operator only");
    // a seeded start vector with entries uniform in [-1, 1) (splitmix64), the same on every device
    std::vector<double> v0(op->Nd);
    unsigned long long x = seed;
    for (double& v : v0) {
        x += 0x9E3779B97F4A7C15ull;
        unsigned long long z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    sigma_estimate(op, f, kind, steps, v0.data(), smax, smin);
    FDE_API_END
}

int fde_solve_batched(fde_ctx* ctx, int n, fde_op* const* ops, fde_hlu* const* precs, const int* nrhs,
                      const double* const* G, const int* ldg, double* const* X, const int* ldx,
                      const fde_solve_params* prm, fde_solve_info* info) {
    int rc = FDE_OK;
    try {
        if (!ctx || n < 0 || (n > 0 && (!ops || !nrhs || !G || !ldg || !X || !ldx || !info)))
            fail(FDE_EINVAL, "bad arguments");
        std::vector<fde_op*> o(ops, ops + n);
        std::vector<fde_hlu*> p(n, nullptr);
        if (precs) std::copy(precs, precs + n, p.begin());
        run_public(ctx, n, (fde_op* const*)o.data(), (fde_hlu* const*)p.data(), nrhs, G, ldg, X, ldx, prm, info, &rc);
    } catch (const Error& e) {
        set_error("%s", e.msg.c_str());
        return e.code;
    } catch (...) {
        set_error("unexpected internal error");
        return FDE_EDEVICE;
    }
    if (rc == FDE_ENOCONV) set_error("the Krylov solver did not reach rtol within maxit for at least one right-hand side");
    if (rc == FDE_EBREAKDOWN) set_error("BiCGSTAB broke down (a vanishing inner product) for at least one right-hand side");
    return rc;
}

}  // extern "C"
