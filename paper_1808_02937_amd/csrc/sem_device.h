// Device helpers shared by the assembly and H-matrix kernels: Legendre values,
// the derivative map D of each unknown, and one entry of A = rho M + S.
#pragma once

#include "fde_internal.h"

namespace fde {

__device__ inline double legendre_at(int n, double x) {
    if (n == 0) return 1.0;
    double pm = 1.0, p = x;
    for (int k = 1; k < n; ++k) {
        const double pn = ((2 * k + 1) * x * p - k * pm) / (k + 1);
        pm = p;
        p = pn;
    }
    return p;
}

// Elements supporting unknown i (paper order), the Legendre index of its
// derivative there and the coefficient: bubble (e,p): -(2p+1) 2/h_e on L_p;
// hat j: +1/h_{j-1} on element j-1, -1/h_j on element j (both L_0).
__device__ inline void dof_elems(int i, int N, int P, const double* h, int* ne, int* el, int* md,
                                 double* cf) {
    const int nb = N * (P - 1);
    if (i < nb) {
        const int e = i / (P - 1), p = i % (P - 1) + 1;
        *ne = 1;
        el[0] = e;
        md[0] = p;
        cf[0] = -(2.0 * p + 1.0) * 2.0 / h[e];
    } else {
        const int j = i - nb + 1;
        *ne = 2;
        el[0] = j - 1;
        md[0] = 0;
        cf[0] = 1.0 / h[j - 1];
        el[1] = j;
        md[1] = 0;
        cf[1] = -1.0 / h[j];
    }
}

struct SemDev {
    int N, P, toep;
    double alpha, theta, rho;
    const double* h;
    const double* mom;    // dense: packed lower-triangular pairs
    const double* gen;    // Toeplitz generators
    const double* lmass;  // (P+1)^2 reference mass
    const double* hpow;   // Toeplitz: (h_e / 2)^(2 - alpha) per element
};

// K^{ef}_{mn}, f <= e
__device__ inline double moment(const SemDev& s, int e, int f, int m, int n) {
    const int P = s.P;
    if (!s.toep) return s.mom[(tri(e) + f) * P * P + m * P + n];
    const double sc = s.hpow[e] * 0.5 * s.h[f];
    return sc * s.gen[(int64_t)(e - f) * P * P + m * P + n];
}

// local index of unknown i on element e in [phi_L, phi_R, psi_1..psi_{P-1}]
__device__ inline int local_index(int i, int e, int N, int P) {
    const int nb = N * (P - 1);
    if (i < nb) return 1 + (i % (P - 1)) + 1;
    return (e == i - nb) ? 1 : 0;   // hat j = i-nb+1: right hat of element j-1, left hat of element j
}

// A[i][j] = rho M + theta D^T K D + (1-theta) D^T K^T D  (paper order)
__device__ inline double sem_entry(const SemDev& s, int i, int j) {
    const int N = s.N, P = s.P;
    int ni, ei[2], mi[2], nj, ej[2], mj[2];
    double ci[2], cj[2];
    dof_elems(i, N, P, s.h, &ni, ei, mi, ci);
    dof_elems(j, N, P, s.h, &nj, ej, mj, cj);
    double v = 0.0;
    for (int a = 0; a < ni; ++a)
        for (int b = 0; b < nj; ++b) {
            const int e = ei[a], f = ej[b];
            if (f <= e) v += s.theta * ci[a] * cj[b] * moment(s, e, f, mi[a], mj[b]);
            if (e <= f) v += (1.0 - s.theta) * ci[a] * cj[b] * moment(s, f, e, mj[b], mi[a]);
        }
    if (s.rho != 0.0) {
        for (int a = 0; a < ni; ++a)
            for (int b = 0; b < nj; ++b) {
                if (ej[b] != ei[a]) continue;
                const int e = ei[a];
                v += s.rho * 0.5 * s.h[e] * s.lmass[local_index(i, e, N, P) * (P + 1) + local_index(j, e, N, P)];
            }
    }
    return v;
}

inline SemDev sem_dev(const Op* op) {
    SemDev s;
    s.N = op->N;
    s.P = op->P;
    s.toep = op->toeplitz ? 1 : 0;
    s.alpha = op->alpha;
    s.theta = op->theta;
    s.rho = op->rho;
    s.h = op->d_h.p;
    s.mom = op->d_mom.p;
    s.gen = op->d_gen.p;
    s.lmass = op->d_lmass.p;
    s.hpow = op->d_hpow.p;
    return s;
}

}  // namespace fde
