// Gauss-Jacobi rules, written for this library (no external quadrature code).
//
// The paper leaves the quadrature of the singular stiffness entries to the
// literature; the library builds every rule it uses here: Gauss-Legendre
// (a = b = 0) and Gauss-Jacobi rules for the weights (1+x)^{2-alpha} and
// (1+x)^{1-alpha} of the Duffy-transformed singular integrals.
//
// Method: the nodes are the eigenvalues of the symmetric Jacobi matrix of the
// orthonormal Jacobi polynomials (three-term recurrence), located one by one
// by Sturm-sequence bisection and polished by Newton steps on the degree-n
// orthonormal polynomial; the weights are the Christoffel numbers
// w_i = 1 / sum_{k<n} p_k(x_i)^2 of the orthonormal polynomials.
#include <algorithm>
#include <tuple>
#include <mutex>
#include <map>
#include <cmath>
#include <vector>

#include "fde_internal.h"

namespace fde {

namespace {

struct Recurrence {
    std::vector<double> alpha;  // diagonal, k = 0..n-1
    std::vector<double> sbeta;  // sqrt(beta_k), k = 1..n (index k)
    double mu0;
};

Recurrence jacobi_recurrence(int n, double a, double b) {
    Recurrence r;
    r.alpha.resize(n);
    r.sbeta.assign(n + 1, 0.0);
    const double ab = a + b;
    for (int k = 0; k < n; ++k) {
        const double k2 = 2.0 * k + ab;
        if (k == 0)
            r.alpha[k] = (b - a) / (ab + 2.0);
        else
            r.alpha[k] = (b * b - a * a) / (k2 * (k2 + 2.0));
    }
    for (int k = 1; k <= n; ++k) {
        const double k2 = 2.0 * k + ab;
        double beta;
        if (k == 1)
            beta = 4.0 * (1.0 + a) * (1.0 + b) / ((2.0 + ab) * (2.0 + ab) * (3.0 + ab));
        else
            beta = 4.0 * k * (k + a) * (k + b) * (k + ab) / (k2 * k2 * (k2 + 1.0) * (k2 - 1.0));
        r.sbeta[k] = std::sqrt(beta);
    }
    r.mu0 = std::exp((ab + 1.0) * std::log(2.0) + std::lgamma(a + 1.0) + std::lgamma(b + 1.0) -
                     std::lgamma(ab + 2.0));
    return r;
}

// number of eigenvalues of the n x n Jacobi matrix below x (Sturm count)
int sturm_count(const Recurrence& r, int n, double x) {
    int cnt = 0;
    double q = r.alpha[0] - x;
    if (q < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
        if (q == 0.0) q = 1e-300;
        q = (r.alpha[k] - x) - r.sbeta[k] * r.sbeta[k] / q;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// orthonormal p_0..p_n at x; returns p_n and its derivative, and sum_{k<n} p_k^2
void orthonormal(const Recurrence& r, int n, double x, double* pn, double* dpn, double* sum2) {
    double pm = 0.0, p = 1.0 / std::sqrt(r.mu0);
    double dpm = 0.0, dp = 0.0;
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        s += p * p;
        const double pk1 = ((x - r.alpha[k]) * p - r.sbeta[k] * pm) / r.sbeta[k + 1];
        const double dpk1 = (p + (x - r.alpha[k]) * dp - r.sbeta[k] * dpm) / r.sbeta[k + 1];
        pm = p;
        p = pk1;
        dpm = dp;
        dp = dpk1;
    }
    *pn = p;
    *dpn = dp;
    *sum2 = s;
}

}  // namespace

namespace {
void gauss_jacobi_compute(int n, double a, double b, double* x, double* w);
}  // namespace

void gauss_jacobi(int n, double a, double b, double* x, double* w) {
    if (n < 1 || !(a > -1.0) || !(b > -1.0))
        fail(FDE_EINVAL, "gauss_jacobi: need n >= 1, a > -1, b > -1 (n=%d a=%g b=%g)", n, a, b);
    // rules are memoised per (n, a, b) for the process: every operator of a given P and alpha asks
    // for the same few, and the bisection below costs tens of microseconds per rule
    static std::mutex mu;
    static std::map<std::tuple<int, double, double>, std::vector<double>> memo;
    const auto key = std::make_tuple(n, a, b);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) {
            std::copy(it->second.begin(), it->second.begin() + n, x);
            std::copy(it->second.begin() + n, it->second.end(), w);
            return;
        }
    }
    gauss_jacobi_compute(n, a, b, x, w);
    std::vector<double> v(x, x + n);
    v.insert(v.end(), w, w + n);
    std::lock_guard<std::mutex> lk(mu);
    memo.emplace(key, std::move(v));
}

namespace {

void gauss_jacobi_compute(int n, double a, double b, double* x, double* w) {
    Recurrence r = jacobi_recurrence(n, a, b);
    for (int i = 0; i < n; ++i) {
        // the i-th smallest eigenvalue lies in [lo, hi] with count(lo) <= i < count(hi)
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (sturm_count(r, n, mid) > i)
                hi = mid;
            else
                lo = mid;
        }
        double xi = 0.5 * (lo + hi);
        for (int it = 0; it < 3; ++it) {
            double pn, dpn, s;
            orthonormal(r, n, xi, &pn, &dpn, &s);
            if (dpn == 0.0) break;
            const double dx = pn / dpn;
            if (!(std::fabs(dx) < 1e-12)) break;
            xi -= dx;
        }
        double pn, dpn, s;
        orthonormal(r, n, xi, &pn, &dpn, &s);
        x[i] = xi;
        w[i] = 1.0 / s;
    }
}

}  // namespace

const double* gauss_legendre_table() {
    // built once per process (thread-safe static initialisation); the rules are
    // used by every panel of every load-vector quadrature and by the device table
    static const std::vector<double> table = [] {
        const int tot = kMaxGL * (kMaxGL + 1) / 2;
        std::vector<double> t(2 * tot);
        for (int n = 1; n <= kMaxGL; ++n) {
            const int off = n * (n - 1) / 2;
            gauss_jacobi(n, 0.0, 0.0, t.data() + off, t.data() + tot + off);
        }
        return t;
    }();
    return table.data();
}

}  // namespace fde
