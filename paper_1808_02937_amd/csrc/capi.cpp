// C entry points: context, operator, load vector, stiffness apply, utilities.
// Every entry point catches the library's internal failures and returns a
// status code; the message is kept per thread for fde_last_error().
#include <mutex>
#include <map>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "fde_internal.h"

namespace fde {

namespace {
thread_local std::string g_last_error;
}

void set_error(const char* fmt, ...) {
    char buf[2048];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void fail(int code, const char* fmt, ...) {
    char buf[2048];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, buf};
}

const char* last_error_cstr() { return g_last_error.c_str(); }

namespace {

// block sizes: multiples of 256 bytes up to 64 KiB, then of 1/8 of the power of two below
size_t block_size(size_t bytes) {
    if (bytes <= 65536) return (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    size_t p = 65536;
    while (p * 2 <= bytes) p *= 2;
    const size_t g = p / 8;
    return (bytes + g - 1) / g * g;
}

void release_pool(Ctx* c) {
    if (c->pool.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->pool) (void)hipFree(kv.second);
    c->pool.clear();
    c->pooled = 0;
}

constexpr size_t kPoolCap = size_t(8) << 30;   // cached bytes kept at most

}  // namespace

constexpr size_t kStageBytes = size_t(32) << 20;   // pinned staging ring

// wait for the oldest staged copy and recycle its event
void retire_oldest(Ctx* c) {
    Ctx::Staged s = c->staged.front();
    c->staged.pop_front();
    (void)hipEventSynchronize(s.ev);
    c->spare_events.push_back(s.ev);
}

Ctx::~Ctx() {
    (void)hipStreamSynchronize(stream);
    plans.clear();   // members holding blocks give them back before the cache is released
    lu_tasks.reset();
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : side_done) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    gl.reset();
    while (!staged.empty()) retire_oldest(this);
    for (hipEvent_t e : spare_events) (void)hipEventDestroy(e);
    if (stage) (void)hipHostFree(stage);
    release_pool(this);
}

void* dev_alloc(Ctx* c, size_t bytes) {
    const size_t sz = block_size(bytes);
    // a cached block of this size class or at most twice as large
    auto it = c->pool.lower_bound(sz);
    if (it != c->pool.end() && it->first <= 2 * sz) {
        void* p = it->second;
        const size_t have = it->first;
        if (!(c->budget && c->in_use + have > c->budget)) {
            c->pool.erase(it);
            c->pooled -= have;
            c->in_use += have;
            c->live[p] = have;
            return p;
        }
    }
    if (c->budget && c->in_use + sz > c->budget)
        fail(FDE_ENOMEM, "HBM budget exceeded: %zu bytes in use + %zu requested > budget %zu", c->in_use, sz,
             c->budget);
    if (c->budget && c->in_use + c->pooled + sz > c->budget) release_pool(c);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess && !c->pool.empty()) {   // the device is full of cached blocks: return them, retry
        (void)hipGetLastError();
        release_pool(c);
        e = hipMalloc(&p, sz);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(FDE_ENOMEM, "hipMalloc(%zu) failed: %s", sz, hipGetErrorString(e));
    }
    c->in_use += sz;
    c->live[p] = sz;
    return p;
}

void dev_free(Ctx* c, void* p, size_t bytes) {
    if (!p) return;
    auto it = c->live.find(p);
    const size_t sz = it != c->live.end() ? it->second : block_size(bytes);
    if (it != c->live.end()) c->live.erase(it);
    c->in_use = sz > c->in_use ? 0 : c->in_use - sz;
    c->pool.emplace(sz, p);
    c->pooled += sz;
    if (c->pooled > kPoolCap) release_pool(c);
}

void upload(Ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (bytes > kStageBytes / 4) {   // large tables: a direct copy (it waits for the stream)
        FDE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
        return;
    }
    if (!c->stage) FDE_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->stage), kStageBytes, hipHostMallocDefault));
    // copies that have completed free their regions
    while (!c->staged.empty() && hipEventQuery(c->staged.front().ev) == hipSuccess) retire_oldest(c);
    const size_t need = (bytes + 255) / 256 * 256;
    size_t start = c->stage_head + need <= kStageBytes ? c->stage_head : 0;
    for (;;) {
        bool busy = false;
        for (const Ctx::Staged& s : c->staged)
            if (start < s.end && s.start < start + need) busy = true;
        if (!busy) break;
        retire_oldest(c);
    }
    std::memcpy(c->stage + start, src, bytes);
    FDE_HIP(hipMemcpyAsync(dst, c->stage + start, bytes, hipMemcpyHostToDevice, c->stream));
    hipEvent_t ev;
    if (!c->spare_events.empty()) {
        ev = c->spare_events.back();
        c->spare_events.pop_back();
    } else {
        FDE_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    FDE_HIP(hipEventRecord(ev, c->stream));
    c->staged.push_back(Ctx::Staged{start, start + need, ev});
    c->stage_head = start + need;
}

namespace {

double nodes_for(double len, double dist, int P) {
    const double a = 1.0 + 2.0 * dist / len;
    const double rho = a + std::sqrt(a * a - 1.0);
    return std::ceil(0.5 * (P + 36.8 / std::log(rho))) + 1;
}

// Quadrature panels of the load vector on element e. Elements touching a or b
// carry geometric panels toward that end and a Gauss-Jacobi end panel, so an
// endpoint singularity f ~ d^{-alpha} (the behaviour of -D^2 I^{2-alpha} of a
// function with nonzero slope at the end) is integrated to ~1e-16; elements
// near an end are graded toward it as in the far-field moments; the rest use
// one Gauss-Legendre panel. Gauss-Legendre panels are expanded into nodes on the
// device; the Gauss-Jacobi end panels (their weights carry the singular factor)
// are given node by node (x, xi, w, d_a, d_b).
void element_load_panels(const Op* op, int e, std::vector<LoadPanel>& pans, std::vector<double>& ex, int& nodes) {
    const double a = op->x.front(), b = op->x.back();
    const double xl = op->x[e], xr = op->x[e + 1], he = xr - xl;
    const int P = op->P;
    const int nbase = std::max(24, P + 12);
    const double da_l = xl - a, db_r = b - xr;
    auto add_panel = [&](double lo, double hi, int n, int side) {
        // lo, hi: distances from the element end on `side` (0: x_e, 1: x_{e+1})
        n = std::min(std::max(n, 1), kMaxGL);
        pans.push_back(LoadPanel{lo, hi, e, side, n, nodes, -1, 0});
        nodes += n;
    };
    const bool touch_a = (e == 0), touch_b = (e == op->N - 1);
    if (touch_a || touch_b) {
        // panels [s^{l+1} T, s^l T] down to 1e-12 T, then [0, delta] with the Gauss-Jacobi rule
        // for the weight d^{1-alpha} (exact for f ~ d^{-alpha} x polynomial, times a test
        // function vanishing at the end)
        const double s = 0.3;
        auto graded = [&](double top, int side, double far_dist) {
            double hi = top;
            for (int l = 0; hi > 1e-12 * top; ++l) {
                const double lo = hi * s;
                int n = 16;
                if (l == 0) n = std::max(n, (int)nodes_for(hi - lo, far_dist, P));
                add_panel(lo, hi, n, side);
                hi = lo;
            }
            const int nj = 16;
            std::vector<double> gx(nj), gw(nj);
            gauss_jacobi(nj, 0.0, 1.0 - op->alpha, gx.data(), gw.data());
            const double delta = hi;
            const int ex0 = (int)(ex.size() / 5);
            for (int i = 0; i < nj; ++i) {
                const double u = 0.5 * delta * (1.0 + gx[i]);
                // int_0^delta F du = (delta/2)^{2-alpha} int (1+t)^{1-alpha} F u^{alpha-1} dt
                const double w = std::pow(0.5 * delta, 2.0 - op->alpha) * gw[i] * std::pow(u, op->alpha - 1.0);
                const double xv = side == 0 ? xl + u : xr - u;
                const double xi = side == 0 ? 2.0 * u / he - 1.0 : 1.0 - 2.0 * u / he;
                const double da = side == 0 ? da_l + u : da_l + (he - u);
                const double db = side == 0 ? db_r + (he - u) : db_r + u;
                ex.insert(ex.end(), {xv, xi, w, da, db});
            }
            pans.push_back(LoadPanel{0.0, delta, e, side, nj, nodes, ex0, 0});
            nodes += nj;
        };
        if (touch_a && touch_b) {
            graded(0.5 * he, 0, 0.5 * he);
            graded(0.5 * he, 1, 0.5 * he);
        } else if (touch_a) {
            graded(he, 0, b - xr + 1e-300);
        } else {
            graded(he, 1, xl - a + 1e-300);
        }
        return;
    }
    const double da = xl - a, db = b - xr;
    const int side = da <= db ? 0 : 1;
    const double g = std::min(da, db), gother = std::max(da, db);
    if (g >= he) {
        int n = (int)std::max<double>(nbase, nodes_for(he, g, P));
        n = std::max(n, (int)nodes_for(he, gother, P));
        add_panel(0.0, he, n, side);
        return;
    }
    for (int j = 0;; ++j) {
        const double lo = g * (std::exp2((double)j) - 1.0);
        double hi = g * (std::exp2((double)(j + 1)) - 1.0);
        const bool last = hi >= he;
        if (last) hi = he;
        add_panel(lo, hi, (int)std::max<double>(nbase, nodes_for(hi - lo, g + lo, P)), side);
        if (last) break;
    }
}

// the load-vector rule on the device: panels on the host (a few per element), nodes expanded by
// a kernel; the host copies of x, d_a, d_b are fetched only when asked for (host_load_rule)
void build_load_rule(Op* op) {
    Ctx* c = op->ctx;
    std::vector<LoadPanel> pans;
    std::vector<double> ex;
    pans.reserve((size_t)op->N + 64);
    op->lq_off.assign(op->N + 1, 0);
    int nodes = 0;
    for (int e = 0; e < op->N; ++e) {
        op->lq_off[e] = nodes;
        element_load_panels(op, e, pans, ex, nodes);
    }
    op->lq_off[op->N] = nodes;
    op->lq_n = nodes;
    op->lq_x.clear();
    op->lq_da.clear();
    op->lq_db.clear();
    for (auto* d : {&op->d_lq_x, &op->d_lq_xi, &op->d_lq_w, &op->d_lq_da, &op->d_lq_db, &op->d_lq_f})
        d->alloc(c, (size_t)nodes);
    op->d_lq_off.alloc(c, op->lq_off.size());
    upload(c, op->d_lq_off.p, op->lq_off.data(), op->lq_off.size() * sizeof(int));
    DevBuf<LoadPanel> d_pans;
    DevBuf<double> d_ex;
    d_pans.alloc(c, pans.size());
    upload(c, d_pans.p, pans.data(), pans.size() * sizeof(LoadPanel));
    d_ex.alloc(c, std::max<size_t>(ex.size(), 1));
    if (!ex.empty()) upload(c, d_ex.p, ex.data(), ex.size() * sizeof(double));
    launch_load_rule(op, (int)pans.size(), d_pans.p, d_ex.p);
}

// host copies of the load-vector nodes and their distances to a and b
void host_load_rule(Op* op) {
    const size_t n = (size_t)op->lq_n;
    if (op->lq_x.size() == n) return;
    Ctx* c = op->ctx;
    op->lq_x.resize(n);
    op->lq_da.resize(n);
    op->lq_db.resize(n);
    FDE_HIP(hipMemcpyAsync(op->lq_x.data(), op->d_lq_x.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FDE_HIP(hipMemcpyAsync(op->lq_da.data(), op->d_lq_da.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FDE_HIP(hipMemcpyAsync(op->lq_db.data(), op->d_lq_db.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FDE_HIP(hipStreamSynchronize(c->stream));
}

// (P+1)^2 mass of the reference basis [phi_L, phi_R, psi_1..psi_{P-1}] on [-1,1]
void local_mass(int P, std::vector<double>& M) {
    const int n = P + 3;
    std::vector<double> gx(n), gw(n);
    gauss_jacobi(n, 0.0, 0.0, gx.data(), gw.data());
    const int P1 = P + 1;
    M.assign(P1 * P1, 0.0);
    std::vector<double> B(P1), L(P + 2);
    for (int q = 0; q < n; ++q) {
        const double t = gx[q];
        L[0] = 1.0;
        L[1] = t;
        for (int k = 1; k + 1 < P + 2; ++k) L[k + 1] = ((2 * k + 1) * t * L[k] - k * L[k - 1]) / (k + 1);
        B[0] = 0.5 * (1.0 - t);
        B[1] = 0.5 * (1.0 + t);
        for (int p = 1; p < P; ++p) B[1 + p] = L[p - 1] - L[p + 1];
        for (int i = 0; i < P1; ++i)
            for (int j = 0; j < P1; ++j) M[i * P1 + j] += gw[q] * B[i] * B[j];
    }
}

void init_ctx_tables(Ctx* c) {
    const size_t cnt = (size_t)kMaxGL * (kMaxGL + 1);
    c->gl.alloc(c, cnt);
    upload(c, c->gl.p, gauss_legendre_table(), cnt * sizeof(double));
    FDE_HIP(hipStreamSynchronize(c->stream));
}

// constant ratio h_{e+1}/h_e (uniform: ratio 1)?
bool mesh_ratio(const double* x, int N, double* ratio) {
    bool geo = true;
    double r = 1.0;
    if (N > 1) {
        r = (x[2] - x[1]) / (x[1] - x[0]);
        for (int e = 1; e + 1 < N && geo; ++e) {
            const double q = (x[e + 2] - x[e + 1]) / (x[e + 1] - x[e]);
            if (std::fabs(q - r) > 1e-12 * std::max(1.0, r)) geo = false;
        }
    }
    *ratio = r;
    return geo;
}

void build_op(Op* op, const double* nodes, int N, int P, double alpha, double theta, double rho,
              int mode) {
    if (N < 1) fail(FDE_EINVAL, "N must be >= 1 (got %d)", N);
    if (P < 2 || P > 32) fail(FDE_EINVAL, "P must be in [2, 32] (got %d)", P);
    if (!(alpha > 1.0 && alpha < 2.0)) fail(FDE_EINVAL, "alpha must be in (1,2) (got %g)", alpha);
    if (!(theta >= 0.0 && theta <= 1.0)) fail(FDE_EINVAL, "theta must be in [0,1] (got %g)", theta);
    if (!(rho >= 0.0) || !std::isfinite(rho)) fail(FDE_EINVAL, "rho must be finite and >= 0 (got %g)", rho);
    if (!nodes) fail(FDE_EINVAL, "nodes is NULL");
    if (mode < FDE_APPLY_AUTO || mode > FDE_APPLY_TOEPLITZ) fail(FDE_EINVAL, "bad apply mode %d", mode);
    op->N = N;
    op->P = P;
    op->Nd = N * P - 1;
    op->alpha = alpha;
    op->theta = theta;
    op->rho = rho;
    op->gamma0 = 1.0 / std::tgamma(2.0 - alpha);
    op->x.assign(nodes, nodes + N + 1);
    op->h.resize(N);
    for (int e = 0; e < N; ++e) {
        if (!std::isfinite(op->x[e]) || !std::isfinite(op->x[e + 1]) || !(op->x[e + 1] > op->x[e]))
            fail(FDE_EINVAL, "mesh must be finite and strictly increasing (at node %d)", e);
        op->h[e] = op->x[e + 1] - op->x[e];
    }
    // constant ratio h_{e+1}/h_e ?
    bool geo = true;
    double r = 1.0;
    if (N > 1) {
        r = op->h[1] / op->h[0];
        for (int e = 1; e + 1 < N && geo; ++e) {
            const double q = op->h[e + 1] / op->h[e];
            if (std::fabs(q - r) > 1e-12 * std::max(1.0, r)) geo = false;
        }
    }
    bool uni = geo && std::fabs(r - 1.0) <= 1e-12;
    if (uni) r = 1.0;
    if (mode == FDE_APPLY_TOEPLITZ && !geo)
        fail(FDE_EINVAL, "Toeplitz apply needs a uniform or constant-ratio mesh");
    // one workgroup holds a half-length complex sequence (16 bytes x L/2) in LDS
    const bool fits = 2 * N <= 8192;
    if (mode == FDE_APPLY_TOEPLITZ && !fits)
        fail(FDE_EUNSUPPORTED, "Toeplitz apply supports N <= 4096 (got %d)", N);
    op->toeplitz = geo && fits && mode != FDE_APPLY_DENSE;
    op->uniform = uni;
    op->ratio = r;
    Ctx* c = op->ctx;
    op->d_x.alloc(c, N + 1);
    op->d_h.alloc(c, N);
    upload(c, op->d_x.p, op->x.data(), (N + 1) * sizeof(double));
    upload(c, op->d_h.p, op->h.data(), N * sizeof(double));
    {
        // the scale of the Toeplitz moments, K^{ef} = (h_e/2)^(2-alpha) (h_f/2) G_{e-f}: one pow per element
        std::vector<double> hp(N);
        for (int e = 0; e < N; ++e) hp[e] = std::pow(0.5 * op->h[e], 2.0 - alpha);
        op->d_hpow.alloc(c, N);
        upload(c, op->d_hpow.p, hp.data(), N * sizeof(double));
    }
    std::vector<double> rules(2 * (P + 1) + 2 * P);
    gauss_jacobi(P + 1, 0.0, 2.0 - alpha, rules.data(), rules.data() + P + 1);
    gauss_jacobi(P, 0.0, 1.0 - alpha, rules.data() + 2 * (P + 1), rules.data() + 2 * (P + 1) + P);
    op->d_rules.alloc(c, rules.size());
    upload(c, op->d_rules.p, rules.data(), rules.size() * sizeof(double));
    std::vector<double> lm;
    local_mass(P, lm);
    op->d_lmass.alloc(c, lm.size());
    upload(c, op->d_lmass.p, lm.data(), lm.size() * sizeof(double));
    if (op->toeplitz) {
        int L = 1;
        while (L < 2 * N) L *= 2;
        if (L < 4) L = 4;
        op->L = L;
        const int M = L / 2;
        // exp(-2 pi i j / L): j / L is exact (L a power of two), cos and sin in FP64; the host table
        // is kept per L for the process (operators of one size share it)
        static std::mutex tw_mu;
        static std::map<int, std::vector<double2>> tw_memo;
        std::vector<double2> tw;
        {
            std::lock_guard<std::mutex> lk(tw_mu);
            auto it = tw_memo.find(L);
            if (it != tw_memo.end()) tw = it->second;
        }
        if (tw.empty()) {
            tw.resize(M + 1);
            for (int j = 0; j <= M; ++j) {
                const double ang = -2.0 * 3.14159265358979323846 * ((double)j / L);
                tw[j] = make_double2(std::cos(ang), std::sin(ang));
            }
            std::lock_guard<std::mutex> lk(tw_mu);
            tw_memo.emplace(L, tw);
        }
        op->d_tw.alloc(c, M + 1);
        upload(c, op->d_tw.p, tw.data(), tw.size() * sizeof(double2));
        op->d_gen.alloc(c, (size_t)N * P * P);
        op->d_sym.alloc(c, (size_t)P * P * (M + 1));
        launch_generators(op);
        build_symbol(op);
    } else {
        op->d_mom.alloc(c, (size_t)tri(N) * P * P);
        launch_pair_moments_dense(op);
    }
    build_load_rule(op);
}

}  // namespace

size_t op_device_bytes(const double* x, int N, int P, int nrhs) {
    double r;
    const bool geo = mesh_ratio(x, N, &r);
    const bool toeplitz = geo && 2 * N <= 8192;
    size_t b = 8 * ((size_t)2 * N + 1) + 8 * (4 * (size_t)P + 2) + 8 * (size_t)(P + 1) * (P + 1);
    const size_t nq = (size_t)N * 48 + 256;   // load-vector nodes (graded panels near the ends)
    b += nq * 8 * 5 + (size_t)(N + 1) * 4;
    const size_t cz = 2 * (size_t)nrhs * N * P;
    if (toeplitz) {
        int L = 4;
        while (L < 2 * N) L *= 2;
        const size_t M = L / 2;
        b += 16 * (M + 1) + 8 * (size_t)N * P * P + 16 * (size_t)P * P * (M + 1);
        b += 8 * (cz + 8 * (size_t)nrhs * P * (M + 1));
    } else {
        b += 8 * (size_t)tri(N) * P * P;
        b += 8 * (cz + (size_t)nrhs * tri(N / 8 + 1) * 2 * 8 * P);   // apply partial sums (upper bound)
    }
    return b;
}

}  // namespace fde

using namespace fde;



extern "C" {

const char* fde_last_error(void) { return fde::last_error_cstr(); }
const char* fde_version(void) { return "fde-hsolve 0.1 (gfx950)"; }

int fde_gauss_jacobi(int n, double a, double b, double* x, double* w) {
    FDE_API_BEGIN
    if (!x || !w) fail(FDE_EINVAL, "null output");
    fde::gauss_jacobi(n, a, b, x, w);
    FDE_API_END
}

int fde_ctx_create(int device, void* hip_stream, size_t budget, fde_ctx** out) {
    FDE_API_BEGIN
    if (!out) fail(FDE_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    FDE_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(FDE_EINVAL, "device %d out of range (%d devices)", device, ndev);
    FDE_HIP(hipSetDevice(device));
    fde_ctx* c = new fde_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->budget = budget;
    try {
        init_ctx_tables(c);
        init_apply_scratch(device);
    } catch (...) {
        delete c;
        throw;
    }
    *out = c;
    FDE_API_END
}

void fde_ctx_destroy(fde_ctx* c) {
    if (!c) return;
    try {
        (void)hipStreamSynchronize(c->stream);
    } catch (...) {
    }
    delete c;
}

int fde_ctx_set_stream(fde_ctx* c, void* s) {
    FDE_API_BEGIN
    if (!c) fail(FDE_EINVAL, "null context");
    // cached blocks may still be in use by work queued on the old stream
    FDE_HIP(hipStreamSynchronize(c->stream));
    c->stream = static_cast<hipStream_t>(s);
    FDE_API_END
}

int fde_ctx_set_apply_streams(fde_ctx* c, int n) {
    FDE_API_BEGIN
    if (!c || n < 0 || n > 3) fail(FDE_EINVAL, "need a context and 0 <= n <= 3 (got %d)", n);
    FDE_HIP(hipStreamSynchronize(c->stream));
    c->nside = n;
    FDE_API_END
}

size_t fde_ctx_bytes_in_use(const fde_ctx* c) { return c ? c->in_use : 0; }

int fde_op_create(fde_ctx* c, const double* nodes, int N, int P, double alpha, double theta, double rho,
                  int mode, fde_op** out) {
    FDE_API_BEGIN
    if (!c || !out) fail(FDE_EINVAL, "null context or output");
    *out = nullptr;
    FDE_HIP(hipSetDevice(c->device));
    fde_op* op = new fde_op();
    op->ctx = c;
    try {
        build_op(op, nodes, N, P, alpha, theta, rho, mode);
    } catch (...) {
        delete op;
        throw;
    }
    *out = op;
    FDE_API_END
}

int fde_op_create_hp(fde_ctx* c, const double* nodes, int N, const int* P, double alpha, double theta, double rho,
                     int mode, fde_op** out) {
    FDE_API_BEGIN
    if (!c || !out || !P) fail(FDE_EINVAL, "null argument");
    *out = nullptr;
    if (N < 1) fail(FDE_EINVAL, "N must be >= 1 (got %d)", N);
    int Pmax = 0;
    for (int e = 0; e < N; ++e) {
        if (P[e] < 1 || P[e] > 32) fail(FDE_EINVAL, "element %d: degree must be in [1, 32] (got %d)", e, P[e]);
        Pmax = std::max(Pmax, P[e]);
    }
    if (Pmax < 2) fail(FDE_EINVAL, "the largest degree must be >= 2");
    FDE_HIP(hipSetDevice(c->device));
    fde_op* op = new fde_op();
    op->ctx = c;
    try {
        build_op(op, nodes, N, Pmax, alpha, theta, rho, mode);
        // the space's unknowns among the extended ones: bubbles p < P_e of element e, the hats
        op->hp = true;
        op->hp_P.assign(P, P + N);
        std::vector<int> map;
        std::vector<double> keep(op->Nd, 0.0);
        for (int e = 0; e < N; ++e)
            for (int p = 1; p < P[e]; ++p) map.push_back(e * (Pmax - 1) + p - 1);
        for (int j = 1; j < N; ++j) map.push_back(N * (Pmax - 1) + j - 1);
        for (int i : map) keep[i] = 1.0;
        op->hp_nd = (int)map.size();
        if (op->hp_nd < 1) fail(FDE_EINVAL, "the space has no unknowns");
        op->d_hp_map.alloc(c, map.size());
        upload(c, op->d_hp_map.p, map.data(), map.size() * sizeof(int));
        op->d_hp_keep.alloc(c, keep.size());
        upload(c, op->d_hp_keep.p, keep.data(), keep.size() * sizeof(double));
    } catch (...) {
        delete op;
        throw;
    }
    *out = op;
    FDE_API_END
}

void fde_op_destroy(fde_op* op) {
    if (!op) return;
    delete op;   // its blocks return to the context's stream-ordered cache
}

int fde_op_ndof(const fde_op* op) { return op ? op->pub_nd() : -1; }
int fde_op_is_toeplitz(const fde_op* op) { return op ? (op->toeplitz ? 1 : 0) : -1; }

int fde_op_pair_moments(fde_op* op, int npairs, const int* e, const int* f, double* out) {
    FDE_API_BEGIN
    if (!op || npairs < 0 || (npairs && (!e || !f || !out))) fail(FDE_EINVAL, "bad arguments");
    for (int i = 0; i < npairs; ++i)
        if (e[i] < 0 || e[i] >= op->N || f[i] < 0 || f[i] > e[i])
            fail(FDE_EINVAL, "pair %d: need 0 <= f <= e < N (e=%d f=%d)", i, e[i], f[i]);
    if (npairs == 0) return FDE_OK;
    Ctx* c = op->ctx;
    DevBuf<int> de, df;
    DevBuf<double> dout;
    de.alloc(c, npairs);
    df.alloc(c, npairs);
    dout.alloc(c, (size_t)npairs * op->P * op->P);
    upload(c, de.p, e, npairs * sizeof(int));
    upload(c, df.p, f, npairs * sizeof(int));
    launch_pair_moments_list(op, npairs, de.p, df.p, dout.p);
    FDE_HIP(hipMemcpyAsync(out, dout.p, dout.bytes(), hipMemcpyDeviceToHost, c->stream));
    FDE_HIP(hipStreamSynchronize(c->stream));
    FDE_API_END
}

int fde_op_dense(fde_op* op, double* A, int lda) {
    FDE_API_BEGIN
    if (!op || !A || lda < op->pub_nd()) fail(FDE_EINVAL, "bad arguments");
    if (op->Nd > 65535) fail(FDE_EUNSUPPORTED, "fde_op_dense is meant for Nd <= 65535 (got %d)", op->Nd);
    if (!op->hp) {
        launch_dense_matrix(op, A, lda);
        return FDE_OK;
    }
    DevBuf<double> Ae;   // the extended matrix, then the space's rows and columns
    Ae.alloc(op->ctx, (size_t)op->Nd * op->Nd);
    launch_dense_matrix(op, Ae.p, op->Nd);
    hp_gather_matrix(op, Ae.p, op->Nd, A, lda, op->ctx->stream);
    FDE_HIP(hipStreamSynchronize(op->ctx->stream));
    FDE_API_END
}

int fde_load_nodes(fde_op* op, int* nq, double* x, double* da, double* db) {
    FDE_API_BEGIN
    if (!op || !nq) fail(FDE_EINVAL, "bad arguments");
    host_load_rule(op);
    const size_t n = op->lq_x.size();
    *nq = (int)n;
    if (x) std::memcpy(x, op->lq_x.data(), n * sizeof(double));
    if (da) std::memcpy(da, op->lq_da.data(), n * sizeof(double));
    if (db) std::memcpy(db, op->lq_db.data(), n * sizeof(double));
    FDE_API_END
}

namespace {


// G from the values in d_lq_f, then the lifting of the boundary values (a degree per element:
// over the extended unknowns, then the space's entries)
void assemble_load(Op* op, double c1, double c2, double* G) {
    Ctx* c = op->ctx;
    DevBuf<double> ge;
    double* Ge = G;
    if (op->hp) {
        ge.alloc(c, op->Nd);
        Ge = ge.p;
    }
    launch_load_vector(op, Ge);
    if (c1 != 0.0 || c2 != 0.0) {
        // lifting: G -= A [0; c1, c2] through the boundary hats
        DevBuf<double> t;
        t.alloc(c, op->Nd);
        stiffness_apply(op, 1, nullptr, op->Nd, t.p, op->Nd, c1, c2, true);
        axpy_cols(c->stream, op->Nd, 1, -1.0, t.p, op->Nd, Ge, op->Nd);
    }
    if (op->hp) hp_gather(op, 1, Ge, op->Nd, G, op->hp_nd, c->stream);
}

}  // namespace

int fde_load_vector_powers(fde_op* op, int nterms, const double* coef, const double* expo, const int* side,
                           double c1, double c2, double* G) {
    FDE_API_BEGIN
    if (!op || !G || nterms < 0 || nterms > 64 || (nterms > 0 && (!coef || !expo || !side)))
        fail(FDE_EINVAL, "bad arguments");
    if (!std::isfinite(c1) || !std::isfinite(c2)) fail(FDE_EINVAL, "boundary values must be finite");
    for (int k = 0; k < nterms; ++k) {
        if (!std::isfinite(coef[k]) || !std::isfinite(expo[k])) fail(FDE_EINVAL, "term %d is not finite", k);
        if (side[k] != 0 && side[k] != 1) fail(FDE_EINVAL, "term %d: side must be 0 or 1", k);
    }
    Ctx* c = op->ctx;
    DevBuf<double> d_ce;
    DevBuf<int> d_s;
    const int nt = std::max(nterms, 1);
    d_ce.alloc(c, 2 * nt);
    d_s.alloc(c, nt);
    if (nterms > 0) {
        upload(c, d_ce.p, coef, nterms * sizeof(double));
        upload(c, d_ce.p + nt, expo, nterms * sizeof(double));
        upload(c, d_s.p, side, nterms * sizeof(int));
    }
    launch_eval_powers(op, nterms, d_ce.p, d_ce.p + nt, d_s.p);
    assemble_load(op, c1, c2, G);
    FDE_API_END
}

int fde_load_vector(fde_op* op, const double* f, double c1, double c2, double* G) {
    FDE_API_BEGIN
    if (!op || !f || !G) fail(FDE_EINVAL, "bad arguments");
    if (!std::isfinite(c1) || !std::isfinite(c2)) fail(FDE_EINVAL, "boundary values must be finite");
    Ctx* c = op->ctx;
    const size_t nq = (size_t)op->lq_n;
    for (size_t q = 0; q < nq; ++q)
        if (!std::isfinite(f[q])) {
            host_load_rule(op);
            fail(FDE_EINVAL, "f is not finite at node %zu (x = %.17g)", q, op->lq_x[q]);
        }
    upload(c, op->d_lq_f.p, f, nq * sizeof(double));
    assemble_load(op, c1, c2, G);
    FDE_API_END
}

int fde_load_vector_fn(fde_op* op, fde_fn fn, void* user, double c1, double c2, double* G) {
    FDE_API_BEGIN
    if (!op || !fn) fail(FDE_EINVAL, "bad arguments");
    host_load_rule(op);
    std::vector<double> fv(op->lq_x.size());
    for (size_t q = 0; q < fv.size(); ++q) fv[q] = fn(op->lq_x[q], user);
    const int rc = fde_load_vector(op, fv.data(), c1, c2, G);
    if (rc != FDE_OK) return rc;
    FDE_API_END
}

int fde_stiffness_apply(fde_op* op, int nrhs, const double* X, int ldx, double* Y, int ldy) {
    FDE_API_BEGIN
    if (!op || nrhs < 0 || (nrhs && (!X || !Y)) || ldx < op->pub_nd() || ldy < op->pub_nd())
        fail(FDE_EINVAL, "bad arguments");
    if (nrhs == 0) return FDE_OK;
    if (!op->hp) {
        stiffness_apply(op, nrhs, X, ldx, Y, ldy, 0.0, 0.0, false);
        return FDE_OK;
    }
    // a degree per element: the columns on the extended unknowns and back
    Ctx* c = op->ctx;
    DevBuf<double> xe, ye;
    xe.alloc(c, (size_t)op->Nd * nrhs);
    ye.alloc(c, (size_t)op->Nd * nrhs);
    hp_scatter(op, nrhs, X, ldx, xe.p, op->Nd, c->stream);
    stiffness_apply(op, nrhs, xe.p, op->Nd, ye.p, op->Nd, 0.0, 0.0, false);
    hp_gather(op, nrhs, ye.p, op->Nd, Y, ldy, c->stream);
    FDE_API_END
}

int fde_stiffness_apply_timed(fde_op* op, int nrhs, const double* X, int ldx, double* Y, int ldy, double* core_ms) {
    FDE_API_BEGIN
    if (op && op->hp) fail(FDE_EUNSUPPORTED, "fde_stiffness_apply_timed: one degree per operator only");
    if (!op || nrhs <= 0 || !X || !Y || !core_ms || ldx < op->Nd || ldy < op->Nd) fail(FDE_EINVAL, "bad arguments");
    hipEvent_t ev[2] = {nullptr, nullptr};
    FDE_HIP(hipEventCreate(&ev[0]));
    try {
        FDE_HIP(hipEventCreate(&ev[1]));
        stiffness_apply(op, nrhs, X, ldx, Y, ldy, 0.0, 0.0, false, nullptr, nullptr, ev);
        FDE_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.0f;
        FDE_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        *core_ms = ms;
    } catch (...) {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        throw;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    FDE_API_END
}

int fde_stiffness_apply_noalloc(fde_op* op, int nrhs, const double* X, int ldx, double* Y, int ldy) {
    FDE_API_BEGIN
    if (op && op->hp) fail(FDE_EUNSUPPORTED, "fde_stiffness_apply_noalloc: one degree per operator only");
    if (!op || nrhs < 0 || (nrhs && (!X || !Y)) || ldx < op->Nd || ldy < op->Nd)
        fail(FDE_EINVAL, "bad arguments");
    if (nrhs == 0) return FDE_OK;
    const size_t need = op->apply_ws_doubles(nrhs);
    if (need > kApplyScratchDoubles)
        fail(FDE_EINVAL, "fde_stiffness_apply_noalloc: %d columns of this operator need %zu doubles of workspace, "
             "the fixed scratch holds %zu (use fde_stiffness_apply, or fewer columns per call)", nrhs, need,
             kApplyScratchDoubles);
    stiffness_apply(op, nrhs, X, ldx, Y, ldy, 0.0, 0.0, false, nullptr, apply_scratch(op->ctx->device));
    FDE_API_END
}

}  // extern "C"
