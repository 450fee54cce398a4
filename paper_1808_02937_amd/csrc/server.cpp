// Solver cache and batched serving (many problems, many right-hand sides).
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
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

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
        size_t bytes = 0;        // device bytes measured when built
        uint64_t stamp = 0;
    };
    std::unordered_map<std::string, Entry> cache;
    size_t cached_bytes = 0;
    uint64_t clock = 0;
    long long hits = 0, misses = 0, evictions = 0;
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
    const size_t fac = (size_t)(s->lp.precision == FDE_FP64 ? pi.bytes_fp64 : pi.bytes_fp32);
    const size_t hmat = 8 * (size_t)pi.arena_elems;   // FP64 H-matrix, freed after the factorisation
    return op_device_bytes(p.nodes, p.N, p.P, 16) + hmat + fac;
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
        if (s->budget) {
            while (s->cached_bytes + need + e > s->budget) {
                auto victim = s->cache.end();
                for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
                    if (it->second.stamp != s->clock && (victim == s->cache.end() || it->second.stamp < victim->second.stamp))
                        victim = it;
                if (victim == s->cache.end()) break;
                drop(s, victim);
            }
            if (s->cached_bytes + need + e > s->budget) {
                for (int r = 0; r < n; ++r)
                    if (keys[r] == keys[i]) rejected[r] = 1;
                continue;
            }
        }
        need += e;
        admitted.push_back(i);
    }
    // build the admitted problems: operators and H-matrices, then one batched factorisation
    std::vector<fde_op*> ops(admitted.size(), nullptr);
    std::vector<fde_hmat*> hms(admitted.size(), nullptr);
    std::vector<fde_hlu*> lus(admitted.size(), nullptr);
    const size_t before = s->ctx->in_use;
    int rc = FDE_OK;
    for (size_t a = 0; a < admitted.size() && rc == FDE_OK; ++a) {
        const fde_problem& p = probs[admitted[a]];
        rc = fde_op_create(s->ctx, p.nodes, p.N, p.P, p.alpha, p.theta, p.rho, FDE_APPLY_AUTO, &ops[a]);
        if (rc == FDE_OK) rc = fde_build_hmatrix(ops[a], &s->hp, &hms[a]);
    }
    if (rc == FDE_OK && !admitted.empty())
        rc = fde_hlu_factor_batched((int)admitted.size(), hms.data(), &s->lp, lus.data());
    for (fde_hmat* h : hms) fde_hmat_destroy(h);
    if (rc != FDE_OK) {
        for (fde_hlu* f : lus) fde_hlu_destroy(f);
        for (fde_op* o : ops) fde_op_destroy(o);
        return rc;   // the message of the failing call is kept
    }
    const size_t built = s->ctx->in_use > before ? s->ctx->in_use - before : 0;
    for (size_t a = 0; a < admitted.size(); ++a) {
        fde_server::Entry e;
        e.op = ops[a];
        e.lu = lus[a];
        e.bytes = built / std::max<size_t>(admitted.size(), 1);
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
        if (rejected[i] || nrhs[i] == 0) continue;
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
    if (any_rejected) fail(FDE_ENOMEM, "a problem does not fit the server's HBM budget");
    if (src == FDE_ENOCONV) {
        set_error("FGMRES did not reach rtol within maxit for at least one right-hand side");
        return FDE_ENOCONV;
    }
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
