// Solver cache, batched serving and continuous serving (many problems, many right-hand sides).
//
// A server owns, for every problem it has admitted, the operator and the H-LU
// factors of its H-matrix (the H-matrix itself is freed once factored). A
// batch of requests is served in three moves: the problems without cached
// factors are admitted against the HBM budget (least recently used entries
// that the batch does not need are evicted first), their operators and
// H-matrices are built and all of them are factored together in one
// level-scheduled H-LU; then every right-hand side of the batch is solved by
// one batched FGMRES. Admission uses an estimate made before any allocation:
// the operator's storage by its mesh class, the H-matrix and the factors from
// the host plan of the H-LU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "hlu.h"

using namespace fde;

struct fde_server {
    fde_ctx* ctx = nullptr;
    fde_hparams hp{};
    fde_hlu_params lp{};
    fde_solve_params sp{};
    size_t budget = 0;
    struct Entry {
        fde_op* op = nullptr;
        fde_hlu* lu = nullptr;
        size_t bytes = 0;        // device bytes of the operator and the factors
        uint64_t stamp = 0;
        int users = 0;           // requests in flight on these factors (never evicted meanwhile)
    };
    std::unordered_map<std::string, Entry> cache;
    size_t cached_bytes = 0;
    uint64_t clock = 0;
    long long hits = 0, misses = 0, evictions = 0;
    // continuous serving: submitted requests wait in arrival order, are admitted as engine slots
    // and memory allow, and advance one Krylov step per fde_server_step together with the rest
    struct Req {
        std::vector<double> nodes;
        fde_problem prob{};
        std::string key;
        int nrhs = 0;
        const double* G = nullptr;
        int ldg = 0;
        double* X = nullptr;
        int ldx = 0;
        enum State { QUEUED, RUNNING, DONE } state = QUEUED;
        std::vector<fde_solve_info> info;
        int cached = 0;
        int rc = FDE_OK;
    };
    std::deque<long long> queue;
    std::unordered_map<long long, Req> reqs;
    long long next_ticket = 1;
    int running = 0;
    KrylovEngine* eng = nullptr;
    int max_systems = 256;
};

namespace {

std::string problem_key(const fde_problem& p) {
    std::string k;
    auto put = [&](const void* q, size_t n) { k.append(static_cast<const char*>(q), n); };
    put(&p.N, sizeof p.N);
    put(&p.P, sizeof p.P);
    put(&p.alpha, sizeof p.alpha);
    put(&p.theta, sizeof p.theta);
    put(&p.rho, sizeof p.rho);
    put(p.nodes, sizeof(double) * (p.N + 1));
    return k;
}

// device bytes an operator and its factors hold (their own buffers; shared plans not counted)
size_t entry_bytes(const fde_op* op, const fde_hlu* f) {
    size_t b = op->d_x.bytes() + op->d_h.bytes() + op->d_hpow.bytes() + op->d_rules.bytes() + op->d_lmass.bytes() +
               op->d_mom.bytes() + op->d_gen.bytes() + op->d_sym.bytes() + op->d_tw.bytes() + op->d_lq_x.bytes() +
               op->d_lq_xi.bytes() + op->d_lq_w.bytes() + op->d_lq_f.bytes() + op->d_lq_da.bytes() +
               op->d_lq_db.bytes() + op->d_lq_off.bytes() + op->ws.bytes();
    if (f)
        b += f->arena.bytes() + f->work_lu.bytes() + f->scr.bytes() + f->sv_rhs.bytes() + f->sv_work.bytes() +
             f->hs_prep.bytes() + f->scrd.bytes() + f->ranks.bytes() + f->status.bytes() + f->prof.bytes() +
             f->flops.bytes() + f->lu_flops.bytes() + f->lr16.bytes();
    return b;
}

void drop(fde_server* s, std::unordered_map<std::string, fde_server::Entry>::iterator it) {
    fde_hlu_destroy(it->second.lu);
    fde_op_destroy(it->second.op);
    s->cached_bytes -= std::min(s->cached_bytes, it->second.bytes);
    s->cache.erase(it);
    ++s->evictions;
}

// device bytes an entry for this problem will hold (operator, transient H-matrix, factors)
size_t estimate(fde_server* s, const fde_problem& p) {
    fde_hlu_plan_info pi{};
    check_rc(fde_hlu_plan(p.nodes, p.N, p.P, &s->hp, s->lp.rank_cap, 0, &pi));
    const size_t fac = (size_t)(s->lp.precision == FDE_FP64 ? pi.bytes_fp64 : pi.bytes_fp32);   // BF16 U, V: less
    const size_t hmat = 8 * (size_t)pi.arena_elems;   // FP64 H-matrix, freed after the factorisation
    return op_device_bytes(p.nodes, p.N, p.P, 16) + hmat + fac;
}

// operators, H-matrices and one batched H-LU for problems probs[idx[..]]; on a failure each is
// built alone so that only the failing ones are lost. rc[a] is the status of problem idx[a].
void build_problems(fde_server* s, const fde_problem* probs, const std::vector<int>& idx, std::vector<fde_op*>& ops,
                    std::vector<fde_hlu*>& lus, std::vector<int>& rc) {
    const size_t n = idx.size();
    ops.assign(n, nullptr);
    lus.assign(n, nullptr);
    rc.assign(n, FDE_OK);
    std::vector<fde_hmat*> hms(n, nullptr);
    int all = FDE_OK;
    for (size_t a = 0; a < n; ++a) {
        const fde_problem& p = probs[idx[a]];
        rc[a] = fde_op_create(s->ctx, p.nodes, p.N, p.P, p.alpha, p.theta, p.rho, FDE_APPLY_AUTO, &ops[a]);
        if (rc[a] == FDE_OK) rc[a] = fde_build_hmatrix(ops[a], &s->hp, &hms[a]);
        if (rc[a] != FDE_OK) all = rc[a];
    }
    if (all == FDE_OK && n > 0) all = fde_hlu_factor_batched((int)n, hms.data(), &s->lp, lus.data());
    if (all != FDE_OK)
        for (size_t a = 0; a < n; ++a)
            if (rc[a] == FDE_OK) {
                lus[a] = nullptr;
                rc[a] = fde_hlu_factor(hms[a], &s->lp, &lus[a]);
            }
    for (fde_hmat* h : hms) fde_hmat_destroy(h);
    for (size_t a = 0; a < n; ++a)
        if (rc[a] != FDE_OK) {
            fde_hlu_destroy(lus[a]);
            fde_op_destroy(ops[a]);
            ops[a] = nullptr;
            lus[a] = nullptr;
        }
}

// evict least recently used entries that no request uses and `keep` does not name, until
// `extra` more bytes fit the budget; true if they fit
bool make_room(fde_server* s, size_t extra, const std::vector<std::string>& keep) {
    if (!s->budget) return true;
    while (s->cached_bytes + extra > s->budget) {
        auto victim = s->cache.end();
        for (auto it = s->cache.begin(); it != s->cache.end(); ++it) {
            if (it->second.users > 0 || it->second.stamp == s->clock) continue;
            if (std::find(keep.begin(), keep.end(), it->first) != keep.end()) continue;
            if (victim == s->cache.end() || it->second.stamp < victim->second.stamp) victim = it;
        }
        if (victim == s->cache.end()) return false;
        drop(s, victim);
    }
    return true;
}

}  // namespace

extern "C" {

int fde_server_create(fde_ctx* ctx, const fde_hparams* hp, const fde_hlu_params* lp, const fde_solve_params* sp,
                      size_t budget_bytes, fde_server** out) {
    FDE_API_BEGIN
    if (!ctx || !out) fail(FDE_EINVAL, "null argument");
    *out = nullptr;
    auto* s = new fde_server();
    s->ctx = ctx;
    s->hp = hp ? *hp : fde_hparams{8, 1.0, 8};
    s->lp = lp ? *lp : fde_hlu_params{1e-3, 0, FDE_FP32, 1e-14};
    s->sp = sp ? *sp : fde_solve_params{FDE_FGMRES, 30, 500, 1e-10};
    s->budget = budget_bytes;
    *out = s;
    FDE_API_END
}

void fde_server_destroy(fde_server* s) {
    if (!s) return;
    engine_destroy(s->eng);
    for (auto& kv : s->cache) {
        fde_hlu_destroy(kv.second.lu);
        fde_op_destroy(kv.second.op);
    }
    delete s;
}

int fde_server_solve(fde_server* s, int n, const fde_problem* probs, const int* nrhs, const double* const* G,
                     const int* ldg, double* const* X, const int* ldx, fde_solve_info* info, int* cached) {
    FDE_API_BEGIN
    if (!s || n < 0 || (n > 0 && (!probs || !nrhs || !G || !ldg || !X || !ldx || !info))) fail(FDE_EINVAL, "bad arguments");
    if (n == 0) return FDE_OK;
    ++s->clock;
    std::vector<std::string> keys(n);
    std::vector<int> missing;              // first request index of every key without factors
    std::unordered_map<std::string, int> first;
    for (int i = 0; i < n; ++i) {
        if (!probs[i].nodes || nrhs[i] < 0) fail(FDE_EINVAL, "request %d: bad problem", i);
        keys[i] = problem_key(probs[i]);
        const bool hit = s->cache.count(keys[i]) > 0;
        if (cached) cached[i] = hit ? 1 : 0;
        if (hit) {
            s->cache[keys[i]].stamp = s->clock;
            ++s->hits;
        } else if (!first.count(keys[i])) {
            first[keys[i]] = i;
            missing.push_back(i);
            ++s->misses;
        } else {
            ++s->hits;   // a repeat inside the batch shares the factors built for it
        }
    }
    // admission: make room for every missing problem, evicting least recently used entries
    // that this batch does not use; a problem that cannot fit is answered with FDE_ENOMEM
    std::vector<int> admitted;
    std::vector<char> rejected(n, 0);
    size_t need = 0;
    for (int i : missing) {
        const size_t e = estimate(s, probs[i]);
        if (!make_room(s, need + e, keys)) {
            for (int r = 0; r < n; ++r)
                if (keys[r] == keys[i]) rejected[r] = 1;
            continue;
        }
        need += e;
        admitted.push_back(i);
    }
    // build the admitted problems: operators and H-matrices, then one batched factorisation; a
    // problem whose build fails is answered with that failure, the others are served
    std::vector<fde_op*> ops;
    std::vector<fde_hlu*> lus;
    std::vector<int> brc;
    build_problems(s, probs, admitted, ops, lus, brc);
    std::vector<int> failed(n, FDE_OK);
    for (size_t a = 0; a < admitted.size(); ++a) {
        if (brc[a] != FDE_OK) {
            for (int r = 0; r < n; ++r)
                if (keys[r] == keys[admitted[a]]) failed[r] = brc[a];
            continue;
        }
        fde_server::Entry e;
        e.op = ops[a];
        e.lu = lus[a];
        e.bytes = entry_bytes(ops[a], lus[a]);
        e.stamp = s->clock;
        s->cache[keys[admitted[a]]] = e;
        s->cached_bytes += e.bytes;
    }
    // one batched solve of every right-hand side whose problem has factors
    std::vector<fde_op*> sops;
    std::vector<fde_hlu*> sprec;
    std::vector<int> snr, sldg, sldx;
    std::vector<const double*> sG;
    std::vector<double*> sX;
    std::vector<int> first_info;   // info offset of each request
    int ns = 0;
    for (int i = 0; i < n; ++i) {
        first_info.push_back(ns);
        ns += nrhs[i];
    }
    std::vector<int> served;
    for (int i = 0; i < n; ++i) {
        if (rejected[i] || failed[i] != FDE_OK || nrhs[i] == 0) continue;
        const auto& e = s->cache.at(keys[i]);
        sops.push_back(e.op);
        sprec.push_back(e.lu);
        snr.push_back(nrhs[i]);
        sG.push_back(G[i]);
        sldg.push_back(ldg[i]);
        sX.push_back(X[i]);
        sldx.push_back(ldx[i]);
        served.push_back(i);
    }
    std::vector<fde_solve_info> sinfo;
    for (int i : served) sinfo.resize(sinfo.size() + nrhs[i]);
    int src = FDE_OK;
    if (!served.empty())
        src = fde_solve_batched(s->ctx, (int)served.size(), sops.data(), sprec.data(), snr.data(), sG.data(),
                                sldg.data(), sX.data(), sldx.data(), &s->sp, sinfo.data());
    if (src != FDE_OK && src != FDE_ENOCONV) return src;
    size_t k = 0;
    for (int i : served)
        for (int j = 0; j < nrhs[i]; ++j) info[first_info[i] + j] = sinfo[k++];
    bool any_rejected = false;
    for (int i = 0; i < n; ++i)
        if (rejected[i]) {
            any_rejected = true;
            for (int j = 0; j < nrhs[i]; ++j) info[first_info[i] + j] = fde_solve_info{0, 0.0, FDE_ENOMEM};
        }
    int first_fail = FDE_OK;
    for (int i = 0; i < n; ++i)
        if (failed[i] != FDE_OK) {
            for (int j = 0; j < nrhs[i]; ++j) info[first_info[i] + j] = fde_solve_info{0, 0.0, failed[i]};
            if (first_fail == FDE_OK) first_fail = failed[i];
        }
    if (any_rejected) fail(FDE_ENOMEM, "a problem does not fit the server's HBM budget");
    if (first_fail != FDE_OK) fail(first_fail, "building a problem failed; the other requests were served");
    if (src == FDE_ENOCONV) {
        set_error("FGMRES did not reach rtol within maxit for at least one right-hand side");
        return FDE_ENOCONV;
    }
    FDE_API_END
}

int fde_server_submit(fde_server* s, const fde_problem* prob, int nrhs, const double* G, int ldg, double* X, int ldx,
                      long long* ticket) {
    FDE_API_BEGIN
    if (!s || !prob || !prob->nodes || prob->N < 1 || nrhs < 0 || !ticket || (nrhs > 0 && (!G || !X)))
        fail(FDE_EINVAL, "bad arguments");
    const int Nd = prob->N * prob->P - 1;
    if (nrhs > 0 && (ldg < Nd || ldx < Nd)) fail(FDE_EINVAL, "leading dimensions below Nd = %d", Nd);
    if (nrhs > s->max_systems) fail(FDE_EINVAL, "a request of %d columns exceeds the %d systems in flight", nrhs,
                                    s->max_systems);
    fde_server::Req r;
    r.nodes.assign(prob->nodes, prob->nodes + prob->N + 1);
    r.prob = *prob;
    r.prob.nodes = r.nodes.data();
    r.key = problem_key(r.prob);
    r.nrhs = nrhs;
    r.G = G;
    r.ldg = ldg;
    r.X = X;
    r.ldx = ldx;
    const long long t = s->next_ticket++;
    auto it = s->reqs.emplace(t, std::move(r)).first;
    it->second.prob.nodes = it->second.nodes.data();
    s->queue.push_back(t);
    *ticket = t;
    FDE_API_END
}

int fde_server_step(fde_server* s, int* in_flight) {
    FDE_API_BEGIN
    if (!s) fail(FDE_EINVAL, "null server");
    Ctx* c = s->ctx;
    if (!s->eng) s->eng = engine_create(c, s->sp.restart, s->sp.maxit, s->sp.rtol, s->max_systems);
    ++s->clock;
    // admission in arrival order, while slots and memory allow
    std::vector<long long> admit;
    std::vector<long long> to_build;            // first request of every key built now
    std::vector<std::string> keys_now;
    int slots = engine_free_slots(s->eng);
    size_t reserve = 0;
    while (!s->queue.empty()) {
        fde_server::Req& r = s->reqs.at(s->queue.front());
        if (r.nrhs == 0) {
            r.state = fde_server::Req::DONE;
            s->queue.pop_front();
            continue;
        }
        if (r.nrhs > slots) break;
        const bool have = s->cache.count(r.key) > 0;
        const bool building = std::find(keys_now.begin(), keys_now.end(), r.key) != keys_now.end();
        if (!have && !building) {
            size_t est = 0;
            try {
                est = estimate(s, r.prob);
            } catch (const Error& e) {   // an invalid problem fails alone
                r.rc = e.code;
                r.state = fde_server::Req::DONE;
                s->queue.pop_front();
                continue;
            }
            std::vector<std::string> keep = keys_now;
            for (long long t : admit) keep.push_back(s->reqs.at(t).key);
            if (!make_room(s, reserve + est, keep)) {
                if (s->running == 0 && admit.empty()) {   // nothing will free memory: it cannot fit
                    r.rc = FDE_ENOMEM;
                    r.state = fde_server::Req::DONE;
                    s->queue.pop_front();
                    continue;
                }
                break;   // wait for running requests to release their factors
            }
            reserve += est;
            keys_now.push_back(r.key);
            to_build.push_back(s->queue.front());
            ++s->misses;
        } else {
            ++s->hits;
            r.cached = have ? 1 : 0;
        }
        slots -= r.nrhs;
        admit.push_back(s->queue.front());
        s->queue.pop_front();
    }
    if (!to_build.empty()) {
        std::vector<fde_problem> probs;
        std::vector<int> idx;
        for (long long t : to_build) {
            idx.push_back((int)probs.size());
            probs.push_back(s->reqs.at(t).prob);
        }
        std::vector<fde_op*> ops;
        std::vector<fde_hlu*> lus;
        std::vector<int> brc;
        build_problems(s, probs.data(), idx, ops, lus, brc);
        for (size_t a = 0; a < to_build.size(); ++a) {
            const std::string& key = s->reqs.at(to_build[a]).key;
            if (brc[a] != FDE_OK) {
                for (long long t : admit)
                    if (s->reqs.at(t).key == key) {
                        s->reqs.at(t).rc = brc[a];
                        s->reqs.at(t).state = fde_server::Req::DONE;
                    }
                continue;
            }
            fde_server::Entry e;
            e.op = ops[a];
            e.lu = lus[a];
            e.bytes = entry_bytes(ops[a], lus[a]);
            e.stamp = s->clock;
            s->cache[key] = e;
            s->cached_bytes += e.bytes;
        }
    }
    for (long long t : admit) {
        fde_server::Req& r = s->reqs.at(t);
        if (r.state == fde_server::Req::DONE) continue;
        fde_server::Entry& e = s->cache.at(r.key);
        e.stamp = s->clock;
        ++e.users;
        engine_add(s->eng, e.op, e.lu, r.nrhs, r.G, r.ldg, r.X, r.ldx, t);
        r.state = fde_server::Req::RUNNING;
        ++s->running;
    }
    std::vector<EngineDone> done;
    if (engine_groups(s->eng) > 0) engine_step(s->eng, done);
    for (EngineDone& d : done) {
        fde_server::Req& r = s->reqs.at(d.id);
        r.info = std::move(d.info);
        r.state = fde_server::Req::DONE;
        --s->running;
        auto it = s->cache.find(r.key);
        if (it != s->cache.end() && it->second.users > 0) --it->second.users;
    }
    if (in_flight) *in_flight = (int)s->queue.size() + s->running;
    FDE_API_END
}

int fde_server_poll(fde_server* s, long long ticket, int* done, fde_solve_info* info, int* cached) {
    FDE_API_BEGIN
    if (!s || !done) fail(FDE_EINVAL, "null argument");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) fail(FDE_EINVAL, "unknown ticket %lld (never submitted, or already collected)", ticket);
    fde_server::Req& r = it->second;
    *done = r.state == fde_server::Req::DONE ? 1 : 0;
    if (!*done) return FDE_OK;
    if (cached) *cached = r.cached;
    int rc = r.rc;
    for (int j = 0; j < r.nrhs; ++j) {
        const fde_solve_info si = r.rc != FDE_OK ? fde_solve_info{0, 0.0, r.rc} : r.info[j];
        if (info) info[j] = si;
        if (rc == FDE_OK && si.status != FDE_OK) rc = si.status;
    }
    s->reqs.erase(it);
    if (rc != FDE_OK) fail(rc, "request %lld finished with status %d", ticket, rc);
    FDE_API_END
}

int fde_server_stats(const fde_server* s, int* entries, size_t* bytes, long long* hits, long long* misses,
                     long long* evictions) {
    FDE_API_BEGIN
    if (!s) fail(FDE_EINVAL, "null server");
    if (entries) *entries = (int)s->cache.size();
    if (bytes) *bytes = s->cached_bytes;
    if (hits) *hits = s->hits;
    if (misses) *misses = s->misses;
    if (evictions) *evictions = s->evictions;
    FDE_API_END
}

}  // extern "C"
