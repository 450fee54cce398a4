// C entry points of the H-matrix (Section 3) and the H-LU / H-solves (Section 4.1).
#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>

#include "hbuild.h"
#include "hlu.h"

using namespace fde;




namespace {

std::vector<LeafDev> leaf_table(const HTree& t) {
    std::vector<LeafDev> v;
    for (int b : t.dense_blocks) {
        const Block& B = t.bl[b];
        LeafDev l{};
        l.off = B.off;
        l.r0 = t.cl[B.tau].d0;
        l.c0 = t.cl[B.sigma].d0;
        l.m = t.cl[B.tau].size();
        l.n = t.cl[B.sigma].size();
        l.lowrank = 0;
        l.slot = -1;
        v.push_back(l);
    }
    for (int b : t.lr_blocks) {
        const Block& B = t.bl[b];
        LeafDev l{};
        l.uoff = B.uoff;
        l.voff = B.voff;
        l.r0 = t.cl[B.tau].d0;
        l.c0 = t.cl[B.sigma].d0;
        l.m = t.cl[B.tau].size();
        l.n = t.cl[B.sigma].size();
        l.lowrank = 1;
        l.slot = B.slot;
        v.push_back(l);
    }
    return v;
}

template <class V>
void upload_vec(Ctx* c, DevBuf<V>& buf, const std::vector<V>& v) {
    buf.alloc(c, v.size());
    upload(c, buf.p, v.data(), v.size() * sizeof(V));
}

void tree_params(HTree& t, Op* op, const fde_hparams* prm) {
    const int R = prm ? prm->R : 8;
    const double lam = prm ? prm->lambda : 1.0;
    const int leaf = prm ? prm->leaf_elems : 8;
    if (R < 1 || R > 64) fail(FDE_EINVAL, "R must be in [1, 64] (got %d)", R);
    if (!(lam > 0.0) || !std::isfinite(lam)) fail(FDE_EINVAL, "lambda must be > 0 (got %g)", lam);
    if (leaf < 2) fail(FDE_EINVAL, "leaf_elems must be >= 2 (got %d)", leaf);
    t.op = op;
    t.R = R;
    t.leaf = leaf;
    t.lambda = lam;
    t.kmax = R;
}

int rank_capacity(const HTree& t, const fde_hlu_params* prm) {
    const int cap = prm && prm->rank_cap > 0 ? prm->rank_cap : t.R;
    return std::max(cap, t.R);
}

void build_hmat(fde_hmat* hm, Op* op, const fde_hparams* prm) {
    Ctx* c = op->ctx;
    HTree& t = hm->t;
    tree_params(t, op, prm);
    const int R = t.R;
    build_trees(&t);
    hm->d_arena.alloc(c, t.arena_elems);
    upload_vec(c, hm->d_h2p, t.h2p);
    // dense near blocks: exact entries of A
    std::vector<DenseBlkDev> dbl;
    int max_elems = 0;
    for (int b : t.dense_blocks) {
        const Block& B = t.bl[b];
        dbl.push_back(DenseBlkDev{B.off, t.cl[B.tau].d0, t.cl[B.sigma].d0, t.cl[B.tau].size(), t.cl[B.sigma].size()});
        max_elems = std::max(max_elems, dbl.back().m * dbl.back().n);
    }
    DevBuf<DenseBlkDev> d_dbl;
    upload_vec(c, d_dbl, dbl);
    launch_hbuild_dense(op, (int)dbl.size(), max_elems, d_dbl.p, hm->d_h2p.p, hm->d_arena.p);
    // low-rank factors from the Taylor expansion (Lemma; Section 3.2)
    // Gauss-Legendre nodes per element for a singular side (cluster id, expansion centre c0): the
    // integrand (x - c0)^(1-alpha-nu) L_m(x) is analytic inside the Bernstein ellipse of parameter
    // rho = (2q+1) + sqrt((2q+1)^2 - 1), q = dist(c0, cluster) / (widest element there), so n nodes
    // err like rho^-(2n - P); half of log rho is used (the negative powers grow towards the
    // singularity) for 1e-20, within [P/2 + 4, P + 24]
    const int P = op->P;
    std::vector<double> hmax_cl(t.cl.size(), -1.0);
    auto singular_nodes = [&](int id, double c0) {
        const Cluster& X = t.cl[id];
        if (hmax_cl[id] < 0.0) {
            double hm = 0.0;
            for (int e = std::max(X.e0 - 1, 0); e < std::min(X.e1 + 1, op->N); ++e) hm = std::max(hm, op->h[e]);
            hmax_cl[id] = hm;
        }
        const int n_max = P + 24, n_min = P / 2 + 4;
        const double delta = std::max({X.lo - c0, c0 - X.hi, 0.0});
        if (!(delta > 0.0) || !(hmax_cl[id] > 0.0)) return n_max;
        const double a = 2.0 * delta / hmax_cl[id] + 1.0, lr = std::log(a + std::sqrt(a * a - 1.0));
        const int n = (int)std::ceil((P + 1 + 2.0 * 20.0 * std::log(10.0) / lr) / 2.0) + 2;
        return std::min(n_max, std::max(n_min, n));
    };
    std::vector<FacSideDev> sides;
    hm->init_rank.assign(t.lr_blocks.size(), R);
    for (size_t k = 0; k < t.lr_blocks.size(); ++k) {
        const Block& B = t.bl[t.lr_blocks[k]];
        const Cluster& Tc = t.cl[B.lower ? B.tau : B.sigma];   // t-cluster (right)
        const Cluster& Sc = t.cl[B.lower ? B.sigma : B.tau];   // s-cluster (left)
        const double rT = 0.5 * (Tc.hi - Tc.lo), rS = 0.5 * (Sc.hi - Sc.lo);
        FacSideDev ts{}, ss{};
        if (rS <= rT) {   // expand in s about the centre of the s-cluster
            const double s0 = 0.5 * (Sc.lo + Sc.hi);
            ts = FacSideDev{0, Tc.d0, Tc.size(), 1, 0, s0, rS, 1.0, op->gamma0};
            ss = FacSideDev{0, Sc.d0, Sc.size(), 0, 0, s0, rS, 1.0, 1.0};
        } else {          // expand in t about the centre of the t-cluster
            const double t0 = 0.5 * (Tc.lo + Tc.hi);
            ts = FacSideDev{0, Tc.d0, Tc.size(), 0, 0, t0, rT, 1.0, 1.0};
            ss = FacSideDev{0, Sc.d0, Sc.size(), 1, 1, t0, rT, -1.0, op->gamma0};
        }
        // nodes per element: the regular side's integrand is a polynomial of degree R - 1 + P (exact);
        // the singular side's is analytic on each element away from the expansion centre
        const int t_id = B.lower ? B.tau : B.sigma, s_id = B.lower ? B.sigma : B.tau;
        ts.nq = ts.sing ? singular_nodes(t_id, ts.c) : (R + P) / 2 + 2;
        ss.nq = ss.sing ? singular_nodes(s_id, ss.c) : (R + P) / 2 + 2;
        FacSideDev u = B.lower ? ts : ss, v = B.lower ? ss : ts;
        const double w = B.lower ? op->theta : 1.0 - op->theta;
        u.mult *= w;
        u.off = B.uoff;
        v.off = B.voff;
        if (w == 0.0) {
            hm->init_rank[k] = 0;
            v.mult = 0.0;
        }
        sides.push_back(u);
        sides.push_back(v);
    }
    DevBuf<FacSideDev> d_sides;
    upload_vec(c, d_sides, sides);
    launch_hbuild_factors(op, R, sides, d_sides.p, hm->d_arena.p);
    upload_vec(c, hm->d_ranks, hm->init_rank);
    if (op->hp) {   // a degree per element: the outside unknowns decoupled in every leaf
        std::vector<LeafDev> lv = leaf_table(t);
        DevBuf<LeafDev> d_lv;
        upload_vec(c, d_lv, lv);
        hp_mask_leaves(op, (int)lv.size(), d_lv.p, hm->d_ranks.p, hm->d_h2p.p, hm->d_arena.p, c->stream);
    }
}

void report_profile(HLUObj* f, const char* what) {
    if (!f->prof.p) return;
    unsigned long long h[kProfSlots];
    FDE_HIP(hipMemcpy(h, f->prof.p, sizeof h, hipMemcpyDeviceToHost));
    print_op_profile(what, h, f->op->ctx->device);
    FDE_HIP(hipMemset(f->prof.p, 0, sizeof h));
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        FDE_HIP(hipEventCreate(&a));
        FDE_HIP(hipEventCreate(&b));
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    float ms() {
        float t = 0.f;
        FDE_HIP(hipEventElapsedTime(&t, a, b));
        return t;
    }
};

bool serial_requested() {
    const char* e = getenv("FDE_HLU_SERIAL");
    return e && e[0] == '1';
}

// The ops of a batch of factorisations in level order (level l of every instance, then level
// l + 1), with level offsets. It depends only on the plans, so the last one is kept in the context.
struct BatchTasks {
    std::vector<std::shared_ptr<const Plan>> plans;
    DevBuf<LevelTask> tasks;
    std::vector<int> loff;
};

const BatchTasks& batch_tasks(Ctx* c, const std::vector<HLUObj*>& fs) {
    auto* cached = static_cast<BatchTasks*>(c->lu_tasks.get());
    if (cached && cached->plans.size() == fs.size()) {
        bool same = true;
        for (size_t i = 0; i < fs.size() && same; ++i) same = cached->plans[i] == fs[i]->plan;
        if (same) return *cached;
    }
    auto bt = std::make_shared<BatchTasks>();
    for (HLUObj* f : fs) bt->plans.push_back(f->plan);
    size_t nlev = 0, ntot = 0;
    for (HLUObj* f : fs) {
        nlev = std::max(nlev, f->plan->lu.level_off.size() - 1);
        ntot += f->plan->lu.ops.size();
    }
    std::vector<LevelTask> tasks;
    tasks.reserve(ntot);
    bt->loff.assign(1, 0);
    for (size_t l = 0; l < nlev; ++l) {
        for (size_t i = 0; i < fs.size(); ++i) {
            const Plan& P = *fs[i]->plan;
            const std::vector<int>& lo = P.lu.level_off;
            if (l + 1 >= lo.size()) continue;
            for (int pc = lo[l]; pc < lo[l + 1]; ++pc)
                tasks.push_back(LevelTask{P.ops_lu.p + pc, (int)i, pc});
        }
        bt->loff.push_back((int)tasks.size());
    }
    upload_vec(c, bt->tasks, tasks);
    c->lu_tasks = bt;
    return *bt;
}

// Factorise a batch of H-LUs of one precision. Level-scheduled: launch l runs level l of
// every factorisation (one workgroup per op); FDE_HLU_SERIAL=1 runs each op list in one
// workgroup instead (the same ops in the same level order, one at a time).
template <class T>
void factor_batch_run(Ctx* c, std::vector<HLUObj*>& fs, const char* what) {
    std::vector<Inst<T>> ins;
    for (HLUObj* f : fs) ins.push_back(f->inst<T>(false, 0, nullptr, 0, nullptr, 0));
    DevBuf<Inst<T>> d_ins;
    upload_vec(c, d_ins, ins);
    const bool serial = serial_requested();
    int variant = 16;
    for (HLUObj* f : fs) {
        const int v = f->plan->lu_variant;
        if (v == 0 || variant == 0) variant = 0;
        else variant = std::max(variant, v);
    }
    static const std::vector<int> no_levels(1, 0);
    const BatchTasks* bt = serial ? nullptr : &batch_tasks(c, fs);
    const std::vector<int>& loff = bt ? bt->loff : no_levels;
    const LevelTask* d_tasks = bt ? bt->tasks.p : nullptr;
    EventPair ev;
    const char* pl = getenv("FDE_PROFILE_LEVELS");
    const bool prof_levels = pl && pl[0] == '1' && !serial;
    std::vector<hipEvent_t> lev_ev;
    if (prof_levels) {
        lev_ev.resize(loff.size());
        for (auto& e : lev_ev) FDE_HIP(hipEventCreate(&e));
    }
    FDE_HIP(hipEventRecord(ev.a, c->stream));
    if (serial) {
        launch_interp<T>(c->stream, (int)ins.size(), d_ins.p, 0, variant);
    } else {
        for (size_t l = 0; l + 1 < loff.size(); ++l) {
            if (prof_levels) FDE_HIP(hipEventRecord(lev_ev[l], c->stream));
            launch_level<T>(c->stream, loff[l + 1] - loff[l], d_ins.p, d_tasks + loff[l], variant);
        }
        if (prof_levels) FDE_HIP(hipEventRecord(lev_ev.back(), c->stream));
    }
    FDE_HIP(hipEventRecord(ev.b, c->stream));
    // the H-solve's diagonal leaves in solve-ready form, from the factors just computed
    for (HLUObj* f : fs)
        if (f->plan->sv_lds)
            launch_hs_prepare<T>(c->stream, reinterpret_cast<const T*>(f->arena.p), f->plan->d_hs_steps.p,
                                 f->plan->hs.nleaf, reinterpret_cast<T*>(f->hs_prep.p));
    if (prof_levels) {
        // per level: time, tasks and the op mix of the first factorisation; the slowest levels
        FDE_HIP(hipEventSynchronize(lev_ev.back()));
        struct Row {
            float ms;
            size_t l;
        };
        std::vector<Row> rows;
        float tot = 0.f;
        for (size_t l = 0; l + 1 < loff.size(); ++l) {
            float ms = 0.f;
            FDE_HIP(hipEventElapsedTime(&ms, lev_ev[l], lev_ev[l + 1]));
            rows.push_back({ms, l});
            tot += ms;
        }
        std::sort(rows.begin(), rows.end(), [](const Row& a, const Row& b) { return a.ms > b.ms; });
        const auto& lo = fs[0]->plan->lu.level_off;
        fprintf(stderr, "[fde levels] %zu levels, %.3f ms; slowest:\n", rows.size(), tot);
        for (size_t r = 0; r < std::min<size_t>(rows.size(), 12); ++r) {
            const size_t l = rows[r].l;
            int cnt[kOpCodes] = {0};
            int maxm = 0;
            if (l + 1 < lo.size())
                for (int pc = lo[l]; pc < lo[l + 1]; ++pc) {
                    const OpRec& o = fs[0]->plan->lu.ops[pc];
                    cnt[o.code]++;
                    if (o.code == OP_LRSUB) maxm = std::max(maxm, fs[0]->plan->lr_rows[o.blk]);
                }
            fprintf(stderr, "  level %zu: %.3f ms, %d tasks; getrf %d trsm %d gemm %d lrsub %d (largest %d rows) zero %d\n",
                    l, rows[r].ms, loff[l + 1] - loff[l], cnt[OP_GETRF], cnt[OP_TRSM], cnt[OP_GEMM], cnt[OP_LRSUB],
                    maxm, cnt[OP_ZERO]);
        }
        float bucket[4] = {0, 0, 0, 0};
        int bn[4] = {0, 0, 0, 0};
        for (const Row& r : rows) {
            const int b = r.ms < 0.05f ? 0 : r.ms < 0.2f ? 1 : r.ms < 1.f ? 2 : 3;
            bucket[b] += r.ms;
            bn[b]++;
        }
        fprintf(stderr, "  levels <50us: %d (%.2f ms), <200us: %d (%.2f ms), <1ms: %d (%.2f ms), >=1ms: %d (%.2f ms)\n",
                bn[0], bucket[0], bn[1], bucket[1], bn[2], bucket[2], bn[3], bucket[3]);
        // levels by their heaviest op: recompression by block rows, else the first op code present
        struct Agg {
            int n = 0;
            float ms = 0.f;
            int tasks = 0;
        };
        std::map<std::string, Agg> kinds;
        for (const Row& r : rows) {
            const size_t l = r.l;
            int maxm = -1, has[kOpCodes] = {0};
            for (int pc = lo[l]; pc < lo[l + 1]; ++pc) {
                const OpRec& o = fs[0]->plan->lu.ops[pc];
                has[o.code] = 1;
                if (o.code == OP_LRSUB) maxm = std::max(maxm, fs[0]->plan->lr_rows[o.blk]);
            }
            std::string k;
            if (maxm >= 0) k = "lrsub<=" + std::to_string(maxm);
            else if (has[OP_GETRF]) k = "getrf";
            else if (has[OP_TRSM]) k = "trsm";
            else if (has[OP_GEMM]) k = "gemm";
            else k = "other";
            Agg& a = kinds[k];
            a.n++;
            a.ms += r.ms;
            a.tasks += loff[l + 1] - loff[l];
        }
        for (auto& kv : kinds)
            fprintf(stderr, "  levels led by %s: %d levels, %.2f ms (%.1f us each), %.0f tasks each\n", kv.first.c_str(),
                    kv.second.n, kv.second.ms, 1e3 * kv.second.ms / kv.second.n, (double)kv.second.tasks / kv.second.n);
        for (auto& e : lev_ev) (void)hipEventDestroy(e);
    }
    std::vector<int> st(2 * fs.size());
    for (size_t i = 0; i < fs.size(); ++i)
        FDE_HIP(hipMemcpyAsync(&st[2 * i], fs[i]->status.p, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    FDE_HIP(hipStreamSynchronize(c->stream));
    const float ms = ev.ms();
    for (HLUObj* f : fs) f->factor_ms = ms;
    for (size_t i = 0; i < fs.size(); ++i) {
        if (st[2 * i] == FDE_EBREAKDOWN)
            fail(FDE_EBREAKDOWN, "H-LU breakdown in H-matrix %zu: leaf pivot below the floor (op %d)", i, st[2 * i + 1]);
        if (st[2 * i] != 0) fail(FDE_EDEVICE, "H-LU status %d in H-matrix %zu", st[2 * i], i);
    }
    for (HLUObj* f : fs) report_profile(f, what);
}

void factor_prepare(HLUObj* f, fde_hmat* hm, const fde_hlu_params* prm) {
    Op* op = hm->t.op;
    Ctx* c = op->ctx;
    f->hm = hm;
    f->op = op;
    f->tol = prm ? prm->tol : 1e-3;
    f->prec = prm ? prm->precision : FDE_FP32;
    f->pivot_floor = prm ? prm->pivot_floor : 1e-14;
    if (!(f->tol >= 0.0) || !std::isfinite(f->tol)) fail(FDE_EINVAL, "tol must be >= 0");
    if (f->prec != FDE_FP32 && f->prec != FDE_FP64 && f->prec != FDE_FP32_BF16UV)
        fail(FDE_EINVAL, "precision must be FDE_FP32, FDE_FP64 or FDE_FP32_BF16UV");
    f->bf16uv = f->prec == FDE_FP32_BF16UV;
    if (f->bf16uv) f->prec = FDE_FP32;   // the factorisation itself runs in FP32
    if (!(f->pivot_floor >= 0.0)) fail(FDE_EINVAL, "pivot_floor must be >= 0");
    f->kmax = rank_capacity(hm->t, prm);
    f->esz = f->prec == FDE_FP64 ? 8 : 4;
    f->plan = get_plan(c, hm->t, f->kmax);
    const Plan& P = *f->plan;
    f->arena.alloc(c, P.t.arena_elems * f->esz);
    f->work_lu.alloc(c, std::max<int64_t>(P.lu.work_elems, 1) * f->esz);
    f->scr.alloc(c, P.lu.scr_t * f->esz);
    f->scrd.alloc(c, P.lu.scr_d);
    if (P.sv_lds) f->hs_prep.alloc(c, (int64_t)2 * P.hs.nleaf * kHsPrepStride * f->esz);
    f->status.alloc(c, 2);
    FDE_HIP(hipMemsetAsync(f->status.p, 0, 2 * sizeof(int), c->stream));
    f->flops.alloc(c, 2);
    FDE_HIP(hipMemsetAsync(f->flops.p, 0, 2 * sizeof(double), c->stream));
    f->lu_flops.alloc(c, std::max<size_t>(f->plan->lu.ops.size(), 1));
    FDE_HIP(hipMemsetAsync(f->lu_flops.p, 0, f->lu_flops.bytes(), c->stream));
    if (profile_ops_enabled()) {
        f->prof.alloc(c, kProfSlots);
        FDE_HIP(hipMemsetAsync(f->prof.p, 0, kProfSlots * sizeof(unsigned long long), c->stream));
    }
    upload_vec(c, f->ranks, hm->init_rank);
    // copy A~ into the factor layout, converting to the factor precision
    std::vector<SegDev> segs;
    for (int b : P.t.dense_blocks) {
        const Block &S = hm->t.bl[b], &D = P.t.bl[b];
        segs.push_back(SegDev{S.off, D.off, (int64_t)P.t.cl[S.tau].size() * P.t.cl[S.sigma].size()});
    }
    for (int b : P.t.lr_blocks) {
        const Block &S = hm->t.bl[b], &D = P.t.bl[b];
        const int R = hm->t.R;
        segs.push_back(SegDev{S.uoff, D.uoff, (int64_t)P.t.cl[S.tau].size() * R});
        segs.push_back(SegDev{S.voff, D.voff, (int64_t)P.t.cl[S.sigma].size() * R});
    }
    // runs contiguous on both sides are merged (with a rank capacity of R the whole arena is one
    // run), then cut into pieces of at most 8192 entries, one workgroup each
    {
        std::vector<SegDev> runs;
        for (const SegDev& g : segs) {
            if (!runs.empty() && runs.back().src + runs.back().len == g.src && runs.back().dst + runs.back().len == g.dst)
                runs.back().len += g.len;
            else
                runs.push_back(g);
        }
        constexpr int64_t kPiece = 8192;
        segs.clear();
        for (const SegDev& g : runs)
            for (int64_t o = 0; o < g.len; o += kPiece)
                segs.push_back(SegDev{g.src + o, g.dst + o, std::min(kPiece, g.len - o)});
    }
    DevBuf<SegDev> d_segs;
    upload_vec(c, d_segs, segs);
    if (f->prec == FDE_FP64)
        launch_segcopy<double, double>(c->stream, (int)segs.size(), d_segs.p, hm->d_arena.p,
                                       reinterpret_cast<double*>(f->arena.p));
    else
        launch_segcopy<double, float>(c->stream, (int)segs.size(), d_segs.p, hm->d_arena.p,
                                      reinterpret_cast<float*>(f->arena.p));
}

// FDE_FP32_BF16UV: the low-rank factors (the arena's tail, from the first U on) rounded to BF16;
// the FP32 arena keeps the dense head only. Called once the factorisation and the solve-ready
// leaves are queued.
void keep_uv_in_bf16(HLUObj* f) {
    if (!f->bf16uv) return;
    Ctx* c = f->op->ctx;
    const HTree& t = f->t();
    int64_t base = t.arena_elems;
    for (int b : t.lr_blocks) base = std::min<int64_t>(base, t.bl[b].uoff);
    const int64_t n = t.arena_elems - base;
    f->lr_base = base;
    // rounded up to whole 32-bit words: the H-solve reads the word holding each element
    f->lr16.alloc(c, (std::max<int64_t>(n, 1) + 1) / 2 * 2 * sizeof(unsigned short));
    launch_to_bf16(c->stream, reinterpret_cast<const float*>(f->arena.p) + base, n,
                   reinterpret_cast<unsigned short*>(f->lr16.p));
    DevBuf<char> head;
    head.alloc(c, std::max<int64_t>(base, 1) * sizeof(float));
    if (base > 0) FDE_HIP(hipMemcpyAsync(head.p, f->arena.p, base * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    std::swap(f->arena.p, head.p);
    std::swap(f->arena.n, head.n);
    // head now holds the full FP32 arena; it goes back to the stream-ordered cache
}

void factor(HLUObj* f, fde_hmat* hm, const fde_hlu_params* prm) {
    factor_prepare(f, hm, prm);
    std::vector<HLUObj*> one{f};
    if (f->prec == FDE_FP64)
        factor_batch_run<double>(f->op->ctx, one, "H-LU");
    else
        factor_batch_run<float>(f->op->ctx, one, "H-LU");
    keep_uv_in_bf16(f);
}

// cache key: everything the programs depend on -- the mesh and the H-matrix and rank parameters
std::string plan_key(const HTree& t, int kmax) {
    const Op* op = t.op;
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    const int ints[5] = {op->N, op->P, t.leaf, t.R, kmax};
    put(ints, sizeof ints);
    put(&t.lambda, sizeof t.lambda);
    put(op->x.data(), op->x.size() * sizeof(double));
    return k;
}

}  // namespace

namespace fde {

void make_plan_host(const HTree& hmt, int kmax, Plan& p, bool check) {
    p.t = hmt;
    assign_storage(&p.t, kmax);
    gen_hlu(p.t, p.lu);
    Program original;
    if (check) original = p.lu;
    schedule_levels(p.t, p.lu, check);
    if (check) check_schedule(p.t, original, p.lu);
    gen_hsolve(p.t, p.sv);
    gen_hsolve_steps(p.t, p.hs);
    validate_hsolve_steps(p.t, p.hs);
    // the LDS H-solve: pipelined steps, leaves of at most 64 rows, at most 64 records a step
    p.sv_lds = p.hs.ok && p.hs.maxrow <= kHsolveMaxRow && p.hs.maxrec <= 64;
    p.kpmax = lrsub_kprime_max(p.t, p.lu);
    int widest = 0;
    for (const OpRec& o : p.lu.ops)
        if (o.code == OP_LRSUB) widest = std::max(widest, p.t.kmax + (o.dim[2] >= 0 ? o.dim[2] : p.t.kmax));
    p.lu_variant = widest <= 16 ? 16 : widest <= 32 ? 32 : 0;
    // Recompressions wider than 32 would run the Gram-Schmidt / Jacobi path of the general kernel
    // variant. That path once faulted the GPU in exact mode with no cause shown, so it is refused.
    if (p.lu_variant == 0)
        fail(FDE_EUNSUPPORTED, "H-LU needs recompression of width %d > 32 (rank capacity above 16)", widest);
    if (p.kpmax > kMaxKp) fail(FDE_EUNSUPPORTED, "H-LU needs recompression of width %d > %d", p.kpmax, kMaxKp);
    validate_program(p.t, p.lu, p.t.arena_elems, p.lu.work_elems, 1, false);
    validate_program(p.t, p.sv, p.t.arena_elems, p.sv.work_elems, 1, true);
    validate_program(p.t, p.sv, p.t.arena_elems, p.sv.work_elems, 64, true);
}

std::shared_ptr<const Plan> get_plan(Ctx* c, const HTree& hmt, int kmax) {
    constexpr size_t kCached = 8;
    const std::string key = plan_key(hmt, kmax);
    for (size_t i = 0; i < c->plans.size(); ++i)
        if (c->plans[i].first == key) {
            auto hit = c->plans[i];
            c->plans.erase(c->plans.begin() + i);
            c->plans.insert(c->plans.begin(), hit);
            return hit.second;
        }
    std::shared_ptr<Plan> p;
    auto pre = c->host_plans.find(key);   // host part built ahead (prefetch_plans)
    if (pre != c->host_plans.end()) {
        p = std::static_pointer_cast<Plan>(pre->second);
        c->host_plans.erase(pre);
    } else {
        p = std::make_shared<Plan>();
        make_plan_host(hmt, kmax, *p, false);
    }
    upload_vec(c, p->h2p, p->t.h2p);
    std::vector<LRBlockDev> lrt;
    for (int b : p->t.lr_blocks) {
        const Block& B = p->t.bl[b];
        lrt.push_back(LRBlockDev{B.uoff, B.voff, (int)p->t.cl[B.tau].size(), (int)p->t.cl[B.sigma].size(), B.slot, -1});
    }
    // the device copy of a program carries the record of the block each LRSUB / LRMV works on
    auto device_ops = [&](const Program& pr) {
        std::vector<OpRec> v = pr.ops;
        for (OpRec& o : v)
            if ((o.code == OP_LRSUB || o.code == OP_LRMV) && o.blk >= 0) o.lb = lrt[o.blk];
        return v;
    };
    upload_vec(c, p->ops_lu, device_ops(p->lu));
    upload_vec(c, p->ops_sv, device_ops(p->sv));
    upload_vec(c, p->d_hs_steps, p->hs.steps);
    upload_vec(c, p->d_hs_recs, p->hs.recs);
    for (const LRBlockDev& b : lrt) p->lr_rows.push_back(std::max(b.m, b.n));
    p->t.op = nullptr;
    c->plans.insert(c->plans.begin(), {key, p});
    if (c->plans.size() > kCached) c->plans.pop_back();
    return p;
}

// Host parts of the plans a batch will need and the context does not hold, built on up to 16 host
// threads at once (each plan is independent host work: op lists, level schedule, H-solve tables);
// get_plan then only uploads them.
void prefetch_plans(Ctx* c, const std::vector<std::pair<const HTree*, int>>& items) {
    std::vector<std::pair<std::string, std::pair<const HTree*, int>>> todo;
    for (const auto& it : items) {
        std::string key = plan_key(*it.first, it.second);
        bool have = c->host_plans.count(key) > 0;
        for (const auto& kv : c->plans) have = have || kv.first == key;
        for (const auto& t : todo) have = have || t.first == key;
        if (!have) todo.push_back({std::move(key), it});
    }
    if (todo.size() < 2) return;   // one plan: get_plan builds it
    std::vector<std::shared_ptr<Plan>> built(todo.size());
    std::vector<std::string> errs(todo.size());
    std::vector<int> codes(todo.size(), FDE_OK);
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t i; (i = next.fetch_add(1)) < todo.size();) {
            try {
                auto p = std::make_shared<Plan>();
                make_plan_host(*todo[i].second.first, todo[i].second.second, *p, false);
                built[i] = p;
            } catch (const Error& e) {
                codes[i] = e.code;
                errs[i] = e.msg;
            } catch (...) {
                codes[i] = FDE_EDEVICE;
                errs[i] = "plan construction failed";
            }
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({todo.size(), (size_t)hw, size_t(16)});
    std::vector<std::thread> pool;
    for (size_t k = 1; k < nt; ++k) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    for (size_t i = 0; i < todo.size(); ++i) {
        if (codes[i] != FDE_OK) fail(codes[i], "%s", errs[i].c_str());
        c->host_plans[todo[i].first] = built[i];
    }
}

void hlu_prepare_solve(HLUObj* f, int nrhs) {
    if (nrhs > f->sv_nrhs_cap) {
        Ctx* c = f->op->ctx;
        const int64_t cap = std::max<int64_t>(nrhs, 1);
        f->sv_rhs.alloc(c, hsolve_rhs_elems(f->op->Nd, (int)cap) * f->esz);
        f->sv_work.alloc(c, std::max<int64_t>(f->plan->sv.work_elems, 1) * cap * f->esz);
        f->sv_nrhs_cap = cap;
    }
}

// solves on factors whose U, V are BF16 need the LDS H-solve (the op-list interpreter reads FP32)
void require_lds_for_bf16(const HLUObj* f, int wc) {
    if (f->bf16uv && wc == 0)
        fail(FDE_EUNSUPPORTED, "BF16 low-rank factors: the leaf-step H-solve does not fit LDS (Nd = %d)", f->op->Nd);
}

int hsolve_cols(Ctx* c, const HLUObj* f, int nrhs, size_t* lds_bytes, bool* global_rhs, int share_cols) {
    *global_rhs = false;
    if (!f->plan->sv_lds || nrhs <= 0) return 0;
    if (!c->lds_limit) c->lds_limit = device_lds_limit(c->device);
    if (!c->num_cu) c->num_cu = device_cu_count(c->device);
    // FDE_HSOLVE_VARIANT in the environment (checks of one variant against another): "global"
    // keeps the right-hand sides in global memory even where they fit LDS, "ops" runs the op-list
    // interpreter; FDE_HSOLVE_COLS=w asks for chunks of w columns (1, 2, 4 or 8; narrowed where
    // LDS requires)
    const char* env = std::getenv("FDE_HSOLVE_VARIANT");
    if (env && std::strcmp(env, "ops") == 0) return 0;
    const bool force = env && std::strcmp(env, "global") == 0;
    // chunk width (columns per workgroup; 1, 2, 4 or 8, one kernel each). A workgroup walks the
    // whole chain of leaf steps for its chunk, so narrow chunks side by side finish first as long
    // as the launch (this instance's share of share_cols columns) fills no more than the compute
    // units; past that, wider chunks share each factor load among their columns
    const int64_t target = std::max<int64_t>(1, (int64_t)c->num_cu * nrhs / std::max(share_cols, nrhs));
    int wc0 = 1;
    while (wc0 < kHsolveMaxCols && (nrhs + wc0 - 1) / wc0 > target) wc0 *= 2;
    if (const char* ew = std::getenv("FDE_HSOLVE_COLS")) {
        const int w = std::atoi(ew);
        if (w == 1 || w == 2 || w == 4 || w == 8) wc0 = w;
    }
    for (const bool gx : {false, true}) {
        if (!gx && force) continue;
        auto need = [&](int w) { return hsolve_lds_for(f, w, gx); };
        int wc = wc0;
        while (wc > 1 && need(wc) > c->lds_limit) wc /= 2;
        if (need(wc) > c->lds_limit) continue;
        *lds_bytes = need(wc);
        *global_rhs = gx;
        return wc;
    }
    return 0;
}

size_t hsolve_lds_for(const HLUObj* f, int wc, bool global_rhs) {
    const Plan& P = *f->plan;
    return hsolve_lds_bytes(f->op->Nd, P.hs.tslots, f->kmax, P.t.nslots, wc, f->esz, global_rhs);
}

int64_t hsolve_rhs_elems(int Nd, int nrhs) {
    // whole chunks of kHsolveMaxCols columns, and a row of slack: the solve reads up to a chunk of
    // entries past the last column it needs (and discards them)
    const int64_t cols = ((int64_t)std::max(nrhs, 1) + kHsolveMaxCols - 1) / kHsolveMaxCols * kHsolveMaxCols;
    return (int64_t)Nd * cols + kHsolveMaxRow;
}

void hlu_solve(HLUObj* f, int nrhs, const double* B, int ldb, double* X, int ldx) {
    Ctx* c = f->op->ctx;
    hipStream_t st = c->stream;
    size_t lds = 0;
    bool gx = false;
    const int wc = hsolve_cols(c, f, nrhs, &lds, &gx, nrhs);
    require_lds_for_bf16(f, wc);
    if (wc > 0) {
        // one workgroup per chunk of wc columns; right-hand sides in LDS, or in sv_rhs (whole chunks)
        const int nchunk = (nrhs + wc - 1) / wc;
        if (gx) hlu_prepare_solve(f, nrhs);
        if (f->prec == FDE_FP64) {
            Inst<double> d = f->inst<double>(true, nrhs, B, ldb, X, ldx);
            d.hs_wc = wc;
            launch_hsolve_one<double>(st, d, nchunk, wc, lds, false, gx);
        } else {
            Inst<float> d = f->inst<float>(true, nrhs, B, ldb, X, ldx);
            d.hs_wc = wc;
            launch_hsolve_one<float>(st, d, nchunk, wc, lds, f->bf16uv, gx);
        }
        return;
    }
    hlu_prepare_solve(f, nrhs);
    if (f->prec == FDE_FP64)
        launch_interp_one<double>(st, f->inst<double>(true, nrhs, B, ldb, X, ldx));
    else
        launch_interp_one<float>(st, f->inst<float>(true, nrhs, B, ldb, X, ldx));
}

}  // namespace fde



extern "C" {

int fde_build_hmatrix(fde_op* op, const fde_hparams* prm, fde_hmat** out) {
    FDE_API_BEGIN
    if (!op || !out) fail(FDE_EINVAL, "null argument");
    *out = nullptr;
    fde_hmat* hm = new fde_hmat();
    try {
        build_hmat(hm, op, prm);
    } catch (...) {
        delete hm;
        throw;
    }
    *out = hm;
    FDE_API_END
}

void fde_hmat_destroy(fde_hmat* hm) {
    if (!hm) return;
    delete hm;   // its blocks return to the context's stream-ordered cache
}

int fde_hmat_counts(const fde_hmat* hm, int* nd, int* nr) {
    FDE_API_BEGIN
    if (!hm) fail(FDE_EINVAL, "null H-matrix");
    if (nd) *nd = (int)hm->t.dense_blocks.size();
    if (nr) *nr = (int)hm->t.lr_blocks.size();
    FDE_API_END
}

int fde_hmat_to_dense(fde_hmat* hm, double* out, int ld) {
    FDE_API_BEGIN
    if (!hm || !out || ld < hm->t.op->pub_nd()) fail(FDE_EINVAL, "bad arguments");
    Op* op = hm->t.op;
    Ctx* c = op->ctx;
    std::vector<LeafDev> lv = leaf_table(hm->t);
    DevBuf<LeafDev> d_lv;
    upload_vec(c, d_lv, lv);
    DevBuf<double> ext;   // a degree per element: the extended matrix, then the space's part
    if (op->hp) ext.alloc(c, (size_t)op->Nd * op->Nd);
    launch_to_dense<double>(c->stream, (int)lv.size(), d_lv.p, hm->d_arena.p, hm->d_ranks.p, hm->d_h2p.p,
                            op->hp ? ext.p : out, op->hp ? op->Nd : ld);
    if (op->hp) hp_gather_matrix(op, ext.p, op->Nd, out, ld, c->stream);
    FDE_HIP(hipStreamSynchronize(c->stream));
    FDE_API_END
}

int fde_hlu_plan(const double* nodes, int N, int P, const fde_hparams* hp, int rank_cap, int check,
                 fde_hlu_plan_info* out) {
    FDE_API_BEGIN
    if (!nodes || !out) fail(FDE_EINVAL, "null argument");
    if (N < 1) fail(FDE_EINVAL, "N must be >= 1 (got %d)", N);
    if (P < 2 || P > 32) fail(FDE_EINVAL, "P must be in [2, 32] (got %d)", P);
    for (int e = 0; e < N; ++e)
        if (!std::isfinite(nodes[e]) || !std::isfinite(nodes[e + 1]) || !(nodes[e + 1] > nodes[e]))
            fail(FDE_EINVAL, "mesh must be finite and strictly increasing (at node %d)", e);
    Op op;   // host fields only
    op.N = N;
    op.P = P;
    op.Nd = N * P - 1;
    op.x.assign(nodes, nodes + N + 1);
    HTree t;
    tree_params(t, &op, hp);
    build_trees(&t);
    fde_hlu_params hl{};
    hl.rank_cap = rank_cap;
    Plan p;
    make_plan_host(t, rank_capacity(t, &hl), p, check != 0);
    fde_hlu_plan_info& r = *out;
    r = fde_hlu_plan_info{};
    r.ops = (long long)p.lu.ops.size();
    r.levels = (int)p.lu.level_off.size() - 1;
    for (int l = 0; l < r.levels; ++l) r.max_width = std::max(r.max_width, p.lu.level_off[l + 1] - p.lu.level_off[l]);
    r.solve_ops = (long long)p.sv.ops.size();
    r.arena_elems = p.t.arena_elems;
    r.work_elems = std::max<int64_t>(p.lu.work_elems, 1);
    r.scratch_elems = p.lu.scr_t;
    r.scratch_f64 = p.lu.scr_d;
    const long long fixed = 8 * r.scratch_f64 + 4 * (long long)p.t.nslots + 8 + 16;   // + status, flop counters
    r.bytes_fp32 = 4 * (r.arena_elems + r.work_elems + r.scratch_elems) + fixed;
    r.bytes_fp64 = 8 * (r.arena_elems + r.work_elems + r.scratch_elems) + fixed;
    r.lr_blocks = p.t.nslots;
    r.hsolve_steps = p.sv_lds ? 2 * p.hs.nleaf : 0;
    r.hsolve_tslots = p.hs.tslots;
    if (p.sv_lds) {
        const int kmax = rank_capacity(t, &hl);
        r.hsolve_lds_fp32 = (long long)hsolve_lds_bytes(op.Nd, p.hs.tslots, kmax, p.t.nslots, 1, 4, false);
        r.hsolve_lds_fp32_global_rhs = (long long)hsolve_lds_bytes(op.Nd, p.hs.tslots, kmax, p.t.nslots, 1, 4, true);
    }
    FDE_API_END
}

int fde_hlu_factor(fde_hmat* hm, const fde_hlu_params* prm, fde_hlu** out) {
    FDE_API_BEGIN
    if (!hm || !out) fail(FDE_EINVAL, "null argument");
    *out = nullptr;
    fde_hlu* f = new fde_hlu();
    try {
        factor(f, hm, prm);
    } catch (...) {
        delete f;
        throw;
    }
    *out = f;
    FDE_API_END
}

int fde_hlu_factor_batched(int n, fde_hmat* const* hms, const fde_hlu_params* prm, fde_hlu** out) {
    FDE_API_BEGIN
    if (n < 0 || (n > 0 && (!hms || !out))) fail(FDE_EINVAL, "bad arguments");
    for (int i = 0; i < n; ++i) out[i] = nullptr;
    if (n == 0) return FDE_OK;
    std::vector<HLUObj*> fs;
    Ctx* c = nullptr;
    try {
        for (int i = 0; i < n; ++i) {
            if (!hms[i]) fail(FDE_EINVAL, "H-matrix %d is NULL", i);
            if (!c) c = hms[i]->t.op->ctx;
            if (hms[i]->t.op->ctx != c) fail(FDE_EINVAL, "H-matrices from different contexts");
        }
        {
            std::vector<std::pair<const HTree*, int>> items;
            for (int i = 0; i < n; ++i) items.push_back({&hms[i]->t, rank_capacity(hms[i]->t, prm)});
            prefetch_plans(c, items);
        }
        for (int i = 0; i < n; ++i) {
            fde_hlu* f = new fde_hlu();
            fs.push_back(f);
            factor_prepare(f, hms[i], prm);
        }
        std::vector<HLUObj*> f32, f64;
        for (HLUObj* f : fs) (f->prec == FDE_FP64 ? f64 : f32).push_back(f);
        if (!f32.empty()) factor_batch_run<float>(c, f32, "H-LU (batched)");
        if (!f64.empty()) factor_batch_run<double>(c, f64, "H-LU (batched)");
        for (HLUObj* f : fs) keep_uv_in_bf16(f);
    } catch (...) {
        for (HLUObj* f : fs) delete static_cast<fde_hlu*>(f);
        throw;
    }
    for (int i = 0; i < n; ++i) out[i] = static_cast<fde_hlu*>(fs[i]);
    FDE_API_END
}

void fde_hlu_destroy(fde_hlu* f) {
    if (!f) return;
    if (f->prof.p) {   // op profile (FDE_PROFILE_OPS=1): read after the queued solves
        (void)hipDeviceSynchronize();
        try {
            report_profile(f, "H-solves");
        } catch (...) {
        }
    }
    delete f;
}

int fde_hlu_to_dense(fde_hlu* f, double* out, int ld, int* h2p) {
    FDE_API_BEGIN
    if (!f || !out || ld < f->op->Nd) fail(FDE_EINVAL, "bad arguments");
    if (f->op->hp) fail(FDE_EUNSUPPORTED, "fde_hlu_to_dense: one degree per operator only");
    Ctx* c = f->op->ctx;
    std::vector<LeafDev> lv = leaf_table(f->t());
    DevBuf<LeafDev> d_lv;
    upload_vec(c, d_lv, lv);
    if (f->prec == FDE_FP64) {
        launch_to_dense<double>(c->stream, (int)lv.size(), d_lv.p, reinterpret_cast<double*>(f->arena.p), f->ranks.p,
                                nullptr, out, ld);
    } else if (f->bf16uv) {   // the FP32 head and the BF16 tail widened into a full FP32 arena
        DevBuf<float> full;
        full.alloc(c, std::max<int64_t>(f->t().arena_elems, 1));
        if (f->lr_base > 0)
            FDE_HIP(hipMemcpyAsync(full.p, f->arena.p, f->lr_base * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        launch_from_bf16(c->stream, reinterpret_cast<const unsigned short*>(f->lr16.p),
                         f->t().arena_elems - f->lr_base, full.p + f->lr_base);
        launch_to_dense<float>(c->stream, (int)lv.size(), d_lv.p, full.p, f->ranks.p, nullptr, out, ld);
        FDE_HIP(hipStreamSynchronize(c->stream));
    } else {
        launch_to_dense<float>(c->stream, (int)lv.size(), d_lv.p, reinterpret_cast<float*>(f->arena.p), f->ranks.p,
                               nullptr, out, ld);
    }
    FDE_HIP(hipStreamSynchronize(c->stream));
    if (h2p) std::memcpy(h2p, f->t().h2p.data(), f->t().h2p.size() * sizeof(int));
    FDE_API_END
}

int fde_hlu_stats(fde_hlu* f, double* factor_flops, double* factor_ms, double* solve_flops) {
    FDE_API_BEGIN
    if (!f) fail(FDE_EINVAL, "null factor");
    double fl[2] = {0.0, 0.0};
    std::vector<double> per_op(f->lu_flops.n);
    FDE_HIP(hipMemcpyAsync(fl, f->flops.p, sizeof fl, hipMemcpyDeviceToHost, f->op->ctx->stream));
    if (!per_op.empty())
        FDE_HIP(hipMemcpyAsync(per_op.data(), f->lu_flops.p, f->lu_flops.bytes(), hipMemcpyDeviceToHost,
                               f->op->ctx->stream));
    FDE_HIP(hipStreamSynchronize(f->op->ctx->stream));
    for (double v : per_op) fl[0] += v;
    if (factor_flops) *factor_flops = fl[0];
    if (factor_ms) *factor_ms = f->factor_ms;
    if (solve_flops) *solve_flops = fl[1];
    FDE_API_END
}

int fde_hlu_max_rank(fde_hlu* f, int* mr) {
    FDE_API_BEGIN
    if (!f || !mr) fail(FDE_EINVAL, "bad arguments");
    std::vector<int> r(f->t().lr_blocks.size());
    if (!r.empty()) {
        FDE_HIP(hipMemcpyAsync(r.data(), f->ranks.p, r.size() * sizeof(int), hipMemcpyDeviceToHost, f->op->ctx->stream));
        FDE_HIP(hipStreamSynchronize(f->op->ctx->stream));
    }
    *mr = r.empty() ? 0 : *std::max_element(r.begin(), r.end());
    FDE_API_END
}

int fde_hlu_solve_variant(fde_hlu* f, int nrhs, int* variant, int* cols, long long* lds_bytes) {
    FDE_API_BEGIN
    if (!f || nrhs < 1) fail(FDE_EINVAL, "bad arguments");
    size_t lds = 0;
    bool gx = false;
    const int wc = hsolve_cols(f->op->ctx, f, nrhs, &lds, &gx, nrhs);
    if (variant) *variant = wc == 0 ? FDE_HSOLVE_OPS : gx ? FDE_HSOLVE_GLOBAL_RHS : FDE_HSOLVE_LDS;
    if (cols) *cols = wc;
    if (lds_bytes) *lds_bytes = wc ? (long long)lds : 0;
    FDE_API_END
}

int fde_hlu_solve(fde_hlu* f, int nrhs, const double* B, int ldb, double* X, int ldx) {
    FDE_API_BEGIN
    if (!f || nrhs < 0 || (nrhs && (!B || !X)) || ldb < f->op->pub_nd() || ldx < f->op->pub_nd())
        fail(FDE_EINVAL, "bad arguments");
    if (nrhs == 0) return FDE_OK;
    Op* op = f->op;
    if (!op->hp) {
        hlu_solve(f, nrhs, B, ldb, X, ldx);
        return FDE_OK;
    }
    // a degree per element: the columns on the extended unknowns and back
    DevBuf<double> be, xe;
    be.alloc(op->ctx, (size_t)op->Nd * nrhs);
    xe.alloc(op->ctx, (size_t)op->Nd * nrhs);
    hp_scatter(op, nrhs, B, ldb, be.p, op->Nd, op->ctx->stream);
    hlu_solve(f, nrhs, be.p, op->Nd, xe.p, op->Nd);
    hp_gather(op, nrhs, xe.p, op->Nd, X, ldx, op->ctx->stream);
    FDE_API_END
}

}  // extern "C"
