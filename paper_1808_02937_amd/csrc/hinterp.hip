// Interpreter of H-arithmetic programs: one 256-thread workgroup runs the op
// list of one instance (one operator's H-LU or H-solve); a launch serves many
// instances of different sizes at once.
//
// Ops: GETRF (dense LU without pivoting, Section 4.1 takes L_H unit lower and
// no pivoting; a pivot below the floor is a breakdown), TRSM, GEMM, ZERO, and
// LRSUB -- C <- trunc(U_C V_C^T - X Y^T): thin QR of [U_C, -X] and [V_C, Y] by
// classical Gram-Schmidt with one reorthogonalisation, the small core
// R_u R_v^T decomposed by one-sided (Hestenes) Jacobi in FP64, and the
// singular values above tol * sigma_1 kept, at most kmax of them (the
// truncation to a prescribed tolerance of Section 4.1). LOAD/STORE move FP64
// vectors in the paper's order to and from the internal order.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "hinterp.h"

namespace fde {

namespace {

constexpr int kT = kInterpThreads;
constexpr int kW = kT / 64;

struct Shared {
    double part[1024];
    double red[kW][32];
    double dots[kMaxKp];
    int order[kMaxKp];
    int flag;
    int stop;
    int r;
    int sweeps;
    double lrsub_flops;
};

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double group_sum(double v, int G) {
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double block_sum(double v, Shared& sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh.red[wave][0] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kW; ++w) s += sh.red[w][0];
    __syncthreads();
    return s;
}
__device__ inline double block_max(double v, Shared& sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) sh.red[wave][0] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kW; ++w) s = fmax(s, sh.red[w][0]);
    __syncthreads();
    return s;
}

template <class T>
__device__ inline T* vptr(const Inst<T>& d, const View& v) {
    switch (v.base) {
        case B_ARENA: return d.arena + v.off;
        case B_WORK: return d.work + v.off;
        case B_RHS: return d.rhs + v.off;
        default: return d.work + v.off * d.nrhs;
    }
}

template <class T>
__device__ inline int dimval(const Inst<T>& d, int code) {
    return code >= 0 ? code : (code == -1 ? d.nrhs : d.ranks[-2 - code]);
}

// ------------------------------------------------------------------ GEMM / ZERO
template <class T>
__device__ void op_gemm(const Inst<T>& d, const OpRec& o) {
    const int m = dimval(d, o.dim[0]), n = dimval(d, o.dim[1]), k = dimval(d, o.dim[2]);
    T* C = vptr(d, o.v[0]);
    const T* A = vptr(d, o.v[1]);
    const T* B = vptr(d, o.v[2]);
    const T alpha = (T)o.alpha, beta = (T)o.beta;
    const int64_t mn = (int64_t)m * n;
    const int ars = o.v[1].rs, acs = o.v[1].cs, brs = o.v[2].rs, bcs = o.v[2].cs;
    const int crs = o.v[0].rs, ccs = o.v[0].cs;
    if (mn <= 0) return;
    if (mn * 4 >= kT || k < 64) {
        // one thread per output
        for (int64_t idx = threadIdx.x; idx < mn; idx += kT) {
            const int i = (int)(idx % m), j = (int)(idx / m);
            const T* a = A + (int64_t)i * ars;
            const T* b = B + (int64_t)j * bcs;
            T s = 0;
            for (int l = 0; l < k; ++l) s += a[(int64_t)l * acs] * b[(int64_t)l * brs];
            T* c = C + (int64_t)i * crs + (int64_t)j * ccs;
            *c = (beta == T(0) ? T(0) : beta * *c) + alpha * s;
        }
        return;
    }
    // few outputs, long inner dimension: a group of G lanes per output, reduced by shuffles
    int G = 64;
    while (G > 1 && (int64_t)G * mn > kT) G >>= 1;
    const int ngroups = kT / G, gid = threadIdx.x / G, gl = threadIdx.x % G;
    for (int64_t idx = gid; idx < mn; idx += ngroups) {
        const int i = (int)(idx % m), j = (int)(idx / m);
        const T* a = A + (int64_t)i * ars;
        const T* b = B + (int64_t)j * bcs;
        double s = 0.0;
        for (int l = gl; l < k; l += G) s += (double)a[(int64_t)l * acs] * (double)b[(int64_t)l * brs];
        s = group_sum(s, G);
        if (gl == 0) {
            T* c = C + (int64_t)i * crs + (int64_t)j * ccs;
            *c = (beta == T(0) ? T(0) : beta * *c) + alpha * (T)s;
        }
    }
}

template <class T>
__device__ void op_zero(const Inst<T>& d, const OpRec& o) {
    const int m = dimval(d, o.dim[0]), n = dimval(d, o.dim[1]);
    T* C = vptr(d, o.v[0]);
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * n; idx += kT) {
        const int i = (int)(idx % m), j = (int)(idx / m);
        C[(int64_t)i * o.v[0].rs + (int64_t)j * o.v[0].cs] = T(0);
    }
}

// ------------------------------------------------------------------ TRSM
template <class T>
__device__ void op_trsm(const Inst<T>& d, const OpRec& o) {
    const int n = dimval(d, o.dim[0]), w = dimval(d, o.dim[1]);
    if (n <= 0 || w <= 0) return;
    T* X = vptr(d, o.v[0]);
    const T* Tm = vptr(d, o.v[1]);
    const int xrs = o.v[0].rs, xcs = o.v[0].cs, trs = o.v[1].rs, tcs = o.v[1].cs;
    const bool lower = o.flags & 1, unit = o.flags & 2;
    auto Tat = [&](int i, int j) -> T { return Tm[(int64_t)i * trs + (int64_t)j * tcs]; };
    if (w <= kW && n <= 256) {
        // one wavefront per column: lane l holds rows l, l+64, l+128, l+192; no barriers
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (wave < w) {
            T* x = X + (int64_t)wave * xcs;
            T xr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = lane + 64 * r;
                xr[r] = row < n ? x[(int64_t)row * xrs] : T(0);
            }
            for (int s = 0; s < n; ++s) {
                const int i = lower ? s : n - 1 - s;
                const int slot = i >> 6, src = i & 63;
                T own = xr[0];
#pragma unroll
                for (int r = 1; r < 4; ++r)
                    if (slot == r) own = xr[r];
                T xi = __shfl(own, src, 64);
                if (!unit) xi /= Tat(i, i);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = lane + 64 * r;
                    if (row == i) xr[r] = xi;
                    if (row < n && (lower ? row > i : row < i)) xr[r] -= Tat(row, i) * xi;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = lane + 64 * r;
                if (row < n) x[(int64_t)row * xrs] = xr[r];
            }
        }
        return;
    }
    if (w >= 64) {
        for (int j = threadIdx.x; j < w; j += kT) {
            T* x = X + (int64_t)j * xcs;
            if (lower) {
                for (int i = 0; i < n; ++i) {
                    T xi = x[(int64_t)i * xrs];
                    if (!unit) xi /= Tat(i, i);
                    x[(int64_t)i * xrs] = xi;
                    for (int l = i + 1; l < n; ++l) x[(int64_t)l * xrs] -= Tat(l, i) * xi;
                }
            } else {
                for (int i = n - 1; i >= 0; --i) {
                    T xi = x[(int64_t)i * xrs];
                    if (!unit) xi /= Tat(i, i);
                    x[(int64_t)i * xrs] = xi;
                    for (int l = 0; l < i; ++l) x[(int64_t)l * xrs] -= Tat(l, i) * xi;
                }
            }
        }
        return;
    }
    for (int s = 0; s < n; ++s) {
        const int i = lower ? s : n - 1 - s;
        if (!unit) {
            if (threadIdx.x < w) X[(int64_t)i * xrs + (int64_t)threadIdx.x * xcs] /= Tat(i, i);
            __syncthreads();
        }
        const int lo = lower ? i + 1 : 0, cnt = lower ? n - i - 1 : i;
        for (int idx = threadIdx.x; idx < cnt * w; idx += kT) {
            const int l = lo + idx % cnt, j = idx / cnt;
            X[(int64_t)l * xrs + (int64_t)j * xcs] -= Tat(l, i) * X[(int64_t)i * xrs + (int64_t)j * xcs];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ GETRF
template <class T>
__device__ bool op_getrf(const Inst<T>& d, const OpRec& o, Shared& sh, int pc) {
    const int n = o.dim[0];
    T* A = vptr(d, o.v[0]);
    const int rs = o.v[0].rs, cs = o.v[0].cs;
    auto at = [&](int i, int j) -> T& { return A[(int64_t)i * rs + (int64_t)j * cs]; };
    double amax = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += kT) amax = fmax(amax, fabs((double)at(idx % n, idx / n)));
    amax = block_max(amax, sh);
    for (int k = 0; k < n; ++k) {
        const T akk = at(k, k);
        if (!(fabs((double)akk) > d.pivot_floor * amax) || !(fabs((double)akk) > 0.0)) {
            if (threadIdx.x == 0) {
                d.status[0] = FDE_EBREAKDOWN;
                d.status[1] = pc;
            }
            return false;
        }
        for (int i = k + 1 + threadIdx.x; i < n; i += kT) at(i, k) /= akk;
        __syncthreads();
        const int r = n - k - 1;
        for (int idx = threadIdx.x; idx < r * r; idx += kT) {
            const int i = k + 1 + idx % r, j = k + 1 + idx / r;
            at(i, j) -= at(i, k) * at(k, j);
        }
        __syncthreads();
    }
    return true;
}

// ------------------------------------------------------------------ LRSUB
// thin QR of Q (rows x kp, ld rows) in place, R (kp x kp, ld kp)
template <class T>
__device__ void qr_cgs2(T* Q, int rows, int kp, T* R, Shared& sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double eps = sizeof(T) == 4 ? 1.2e-7 : 2.3e-16;
    for (int j = 0; j < kp; ++j) {
        T* qj = Q + (int64_t)j * rows;
        double nn = 0.0;
        for (int i = threadIdx.x; i < rows; i += kT) nn += (double)qj[i] * (double)qj[i];
        const double nrm0 = sqrt(block_sum(nn, sh));
        for (int pass = 0; pass < 2; ++pass) {
            for (int c0 = 0; c0 < j; c0 += 32) {
                const int cn = min(32, j - c0);
                double part[32];
#pragma unroll
                for (int c = 0; c < 32; ++c) part[c] = 0.0;
                for (int i = threadIdx.x; i < rows; i += kT) {
                    const double qv = (double)qj[i];
#pragma unroll
                    for (int c = 0; c < 32; ++c)
                        if (c < cn) part[c] += (double)Q[(int64_t)(c0 + c) * rows + i] * qv;
                }
#pragma unroll
                for (int c = 0; c < 32; ++c) {
                    const double v = wave_sum(part[c]);
                    if (c < cn && lane == 0) sh.red[wave][c] = v;
                }
                __syncthreads();
                if (threadIdx.x < cn) {
                    double s = 0.0;
                    for (int w = 0; w < kW; ++w) s += sh.red[w][threadIdx.x];
                    sh.dots[c0 + threadIdx.x] = s;
                }
                __syncthreads();
            }
            for (int i = threadIdx.x; i < rows; i += kT) {
                double s = 0.0;
                for (int c = 0; c < j; ++c) s += sh.dots[c] * (double)Q[(int64_t)c * rows + i];
                qj[i] = (T)((double)qj[i] - s);
            }
            for (int c = threadIdx.x; c < j; c += kT)
                R[c + (int64_t)j * kp] = (T)((pass == 0 ? 0.0 : (double)R[c + (int64_t)j * kp]) + sh.dots[c]);
            __syncthreads();
        }
        nn = 0.0;
        for (int i = threadIdx.x; i < rows; i += kT) nn += (double)qj[i] * (double)qj[i];
        const double nrm = sqrt(block_sum(nn, sh));
        const bool keep = nrm > 8.0 * eps * nrm0 && nrm > 1e-300;
        const double inv = keep ? 1.0 / nrm : 0.0;
        for (int i = threadIdx.x; i < rows; i += kT) qj[i] = (T)((double)qj[i] * inv);
        if (threadIdx.x == 0) R[j + (int64_t)j * kp] = (T)(keep ? nrm : 0.0);
        for (int c = j + 1 + threadIdx.x; c < kp; c += kT) R[c + (int64_t)j * kp] = T(0);
        __syncthreads();
    }
}

// one-sided Jacobi on the columns of M (kp x kp, FP64); W accumulates the rotations
__device__ void jacobi_svd(double* M, double* W, int kp, Shared& sh) {
    const int n2 = kp + (kp & 1);
    const int npairs = n2 / 2;
    int G = 64;
    while (G > 1 && G * npairs > kT) G >>= 1;
    const int ngroups = kT / G;
    const int gid = threadIdx.x / G, gl = threadIdx.x % G;
    if (threadIdx.x == 0) sh.sweeps = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) {
            sh.flag = 0;
            sh.sweeps = sweep + 1;
        }
        __syncthreads();
        for (int round = 0; round < n2 - 1; ++round) {
            for (int pi = gid; pi < npairs; pi += ngroups) {
                int p, q;
                if (pi == 0) {
                    p = round;
                    q = n2 - 1;
                } else {
                    p = (round + pi) % (n2 - 1);
                    q = (round - pi + n2 - 1) % (n2 - 1);
                }
                if (p >= kp || q >= kp) continue;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = gl; i < kp; i += G) {
                    const double mp = M[i + (int64_t)p * kp], mq = M[i + (int64_t)q * kp];
                    a += mp * mp;
                    b += mq * mq;
                    g += mp * mq;
                }
                a = group_sum(a, G);
                b = group_sum(b, G);
                g = group_sum(g, G);
                if (g != 0.0 && fabs(g) > 1e-15 * sqrt(a * b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    for (int i = gl; i < kp; i += G) {
                        const double mp = M[i + (int64_t)p * kp], mq = M[i + (int64_t)q * kp];
                        M[i + (int64_t)p * kp] = c * mp - s * mq;
                        M[i + (int64_t)q * kp] = s * mp + c * mq;
                        const double wp = W[i + (int64_t)p * kp], wq = W[i + (int64_t)q * kp];
                        W[i + (int64_t)p * kp] = c * wp - s * wq;
                        W[i + (int64_t)q * kp] = s * wp + c * wq;
                    }
                    if (gl == 0) sh.flag = 1;
                }
            }
            __syncthreads();
        }
        const int rot = sh.flag;
        __syncthreads();
        if (!rot) break;
    }
}

// ----- fast recompression for k' <= 32: FP64 Gram matrices + wavefront one-sided Jacobi

// one-sided (Hestenes) Jacobi run by one wavefront: lane j holds column j of M (kp x kp, column-major
// in global scratch); on return M holds the rotated columns, W the accumulated rotations and
// nrm[j] = ||rotated column j||. Both lanes of a pair form the same dot products in the same order.
template <int KP>
__device__ void wave_jacobi(double* M, double* W, double* nrm, int kp) {
    const int lane = threadIdx.x & 63;
    double col[KP], w[KP];
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        col[i] = (lane < kp && i < kp) ? M[i + lane * kp] : 0.0;
        w[i] = (i == lane) ? 1.0 : 0.0;
    }
    const int n2 = kp + (kp & 1);
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool rotated = false;
        for (int r = 0; r < n2 - 1; ++r) {
            int partner;
            if (lane >= n2)
                partner = lane;
            else if (lane == n2 - 1)
                partner = r;
            else if (lane == r)
                partner = n2 - 1;
            else
                partner = (((2 * r - lane) % (n2 - 1)) + (n2 - 1)) % (n2 - 1);
            double a = 0.0, g = 0.0;
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const double pv = __shfl(col[i], partner, 64);
                a += col[i] * col[i];
                g += (lane < partner) ? col[i] * pv : pv * col[i];
            }
            const double b = __shfl(a, partner, 64);
            const bool valid = lane < kp && partner < kp && partner != lane;
            const bool prole = lane < partner;
            const double ap = prole ? a : b, aq = prole ? b : a;
            const bool rot = valid && g != 0.0 && fabs(g) > 1e-15 * sqrt(ap * aq);
            double c = 1.0, s = 0.0;
            if (rot) {
                const double zeta = (aq - ap) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                c = 1.0 / sqrt(1.0 + t * t);
                s = c * t;
                rotated = true;
            }
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const double pv = __shfl(col[i], partner, 64);
                const double pw = __shfl(w[i], partner, 64);
                if (rot) {
                    col[i] = prole ? c * col[i] - s * pv : s * pv + c * col[i];
                    w[i] = prole ? c * w[i] - s * pw : s * pw + c * w[i];
                }
            }
        }
        if (!__any(rotated)) break;
    }
    if (lane < kp) {
        double nn = 0.0;
#pragma unroll
        for (int i = 0; i < KP; ++i)
            if (i < kp) {
                M[i + lane * kp] = col[i];
                W[i + lane * kp] = w[i];
                nn += col[i] * col[i];
            }
        nrm[lane] = sqrt(nn);
    }
}

template <class T>
struct Cat {   // the columns of [A, sb * B]: rows i, A m x ka, B m x kb
    const T* A;
    int ars, acs, ka;
    const T* B;
    int brs, bcs, kb;
    double sb;
    __device__ double at(int i, int c) const {
        return c < ka ? (double)A[(int64_t)i * ars + (int64_t)c * acs]
                      : sb * (double)B[(int64_t)i * brs + (int64_t)(c - ka) * bcs];
    }
};

// G (kp x kp, FP64, global scratch) = Cat^T Cat; threads split (entry, row slice); part in LDS
template <class T>
__device__ void gram(const Cat<T>& U, int m, int kp, double* G, double* part) {
    const int nent = kp * (kp + 1) / 2;
    int S = kT / nent;
    if (S < 1) S = 1;
    if (S > 64) S = 64;
    for (int t = threadIdx.x; t < nent * S; t += kT) {
        const int e = t % nent, sl = t / nent;
        int q = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (q * (q + 1) / 2 > e) --q;
        while ((q + 1) * (q + 2) / 2 <= e) ++q;
        const int p = e - q * (q + 1) / 2;   // p <= q
        const int r0 = (int)((int64_t)m * sl / S), r1 = (int)((int64_t)m * (sl + 1) / S);
        double acc = 0.0;
        for (int i = r0; i < r1; ++i) acc += U.at(i, p) * U.at(i, q);
        part[t] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nent; e += kT) {
        double acc = 0.0;
        for (int sl = 0; sl < S; ++sl) acc += part[sl * nent + e];
        int q = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (q * (q + 1) / 2 > e) --q;
        while ((q + 1) * (q + 2) / 2 <= e) ++q;
        const int p = e - q * (q + 1) / 2;
        G[p + q * kp] = acc;
        G[q + p * kp] = acc;
    }
    __syncthreads();
}

// From the eigen-decomposition G = W diag(lam) W^T (rotated columns in G, norms lam):
// R = diag(sqrt lam) W^T and F = W diag(lam^{+1/2}) (pseudo-inverse square root)
__device__ void side_factors(const double* W, const double* lam, int kp, double* R, double* F) {
    double lmax = 0.0;
    for (int j = 0; j < kp; ++j) lmax = fmax(lmax, lam[j]);
    const double floor_ = kp * 2.3e-16 * lmax;
    for (int idx = threadIdx.x; idx < kp * kp; idx += kT) {
        const int i = idx % kp, j = idx / kp;
        const double li = lam[i];
        const bool keep = li > floor_ && li > 0.0;
        R[i + j * kp] = keep ? sqrt(li) * W[j + i * kp] : 0.0;         // R[i][j] = sqrt(lam_i) W[j][i]
        const double lj = lam[j];
        F[i + j * kp] = (lj > floor_ && lj > 0.0) ? W[i + j * kp] / sqrt(lj) : 0.0;
    }
}

// C = A B (kp x kp, column-major, FP64 scratch)
__device__ void small_mm(const double* A, const double* B, double* C, int kp) {
    for (int idx = threadIdx.x; idx < kp * kp; idx += kT) {
        const int i = idx % kp, j = idx / kp;
        double s = 0.0;
        for (int l = 0; l < kp; ++l) s += A[i + l * kp] * B[l + j * kp];
        C[i + j * kp] = s;
    }
}

template <class T>
__device__ void op_lrsub_fast(const Inst<T>& d, const OpRec& o, Shared& sh, const LRBlockDev& L, int kc, int kx) {
    T* U = d.arena + L.uoff;
    T* V = d.arena + L.voff;
    const int m = L.m, n = L.n, kp = kc + kx;
    const int wave = threadIdx.x >> 6;
    const T* Xp = vptr(d, o.v[0]);
    const T* Yp = vptr(d, o.v[1]);
    const Cat<T> Uc{U, 1, m, kc, Xp, o.v[0].rs, o.v[0].cs, kx, -1.0};
    const Cat<T> Vc{V, 1, n, kc, Yp, o.v[1].rs, o.v[1].cs, kx, 1.0};
    const int K2 = kp * kp;
    double* base = d.scrd + o.sofs_d;
    double *Gu = base, *Gv = Gu + K2, *Wu = Gv + K2, *Wv = Wu + K2, *Ru = Wv + K2, *Rv = Ru + K2;
    double *Fu = Rv + K2, *Fv = Fu + K2, *Mc = Fv + K2, *Wm = Mc + K2, *T1 = Wm + K2, *T2 = T1 + K2;
    double *lu = T2 + K2, *lv = lu + 32, *sg = lv + 32;
    double* Qs = sg + 32;   // FP64 copy of the orthogonalised rows for the second pass (max rows x kp)
    double* part = sh.part;
    gram(Uc, m, kp, Gu, part);
    gram(Vc, n, kp, Gv, part);
    if (wave == 0) {
        if (kp <= 16) wave_jacobi<16>(Gu, Wu, lu, kp); else wave_jacobi<32>(Gu, Wu, lu, kp);
    } else if (wave == 1) {
        if (kp <= 16) wave_jacobi<16>(Gv, Wv, lv, kp); else wave_jacobi<32>(Gv, Wv, lv, kp);
    }
    __syncthreads();
    side_factors(Wu, lu, kp, Ru, Fu);
    side_factors(Wv, lv, kp, Rv, Fv);
    __syncthreads();
    if (sizeof(T) == 8) {
        // second pass: Q1 = U' F, G2 = Q1^T Q1 = W2 diag(l2) W2^T, R <- R2 R1, F <- F1 F2
        for (int side = 0; side < 2; ++side) {
            const Cat<T>& C = side == 0 ? Uc : Vc;
            const int rows = side == 0 ? m : n;
            double* F = side == 0 ? Fu : Fv;
            double* R = side == 0 ? Ru : Rv;
            for (int i = threadIdx.x; i < rows; i += kT) {
                double row[32];
#pragma unroll
                for (int l = 0; l < 32; ++l) row[l] = l < kp ? C.at(i, l) : 0.0;
                for (int c = 0; c < kp; ++c) {
                    double s = 0.0;
#pragma unroll
                    for (int l = 0; l < 32; ++l)
                        if (l < kp) s += row[l] * F[l + c * kp];
                    Qs[(int64_t)i + (int64_t)c * rows] = s;
                }
            }
            __syncthreads();
            const Cat<double> Q{Qs, 1, rows, kp, nullptr, 0, 0, 0, 0.0};
            gram(Q, rows, kp, Gu, part);
            if (wave == 0) {
                if (kp <= 16) wave_jacobi<16>(Gu, Wu, lu, kp); else wave_jacobi<32>(Gu, Wu, lu, kp);
            }
            __syncthreads();
            side_factors(Wu, lu, kp, T1, T2);   // T1 = R2, T2 = F2
            __syncthreads();
            small_mm(T1, R, Mc, kp);             // R2 R1
            __syncthreads();
            for (int idx = threadIdx.x; idx < K2; idx += kT) R[idx] = Mc[idx];
            __syncthreads();
            small_mm(F, T2, Mc, kp);             // F1 F2
            __syncthreads();
            for (int idx = threadIdx.x; idx < K2; idx += kT) F[idx] = Mc[idx];
            __syncthreads();
        }
    }
    // core M = R_u R_v^T and its SVD
    for (int idx = threadIdx.x; idx < K2; idx += kT) {
        const int i = idx % kp, j = idx / kp;
        double s = 0.0;
        for (int l = 0; l < kp; ++l) s += Ru[i + l * kp] * Rv[j + l * kp];
        Mc[idx] = s;
    }
    __syncthreads();
    if (wave == 0) {
        if (kp <= 16) wave_jacobi<16>(Mc, Wm, sg, kp); else wave_jacobi<32>(Mc, Wm, sg, kp);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kp; j += kT) {
        int r = 0;
        const double sj = sg[j];
        for (int i = 0; i < kp; ++i) r += (sg[i] > sj || (sg[i] == sj && i < j)) ? 1 : 0;
        sh.order[r] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double smax = sg[sh.order[0]];
        int r = 0;
        if (smax > 0.0)
            while (r < kp && sg[sh.order[r]] > d.tol * smax) ++r;
        if (r > d.kmax) r = d.kmax;
        sh.r = r;
        d.ranks[L.slot] = r;
        const double K = kp;
        sh.lrsub_flops = 2.0 * (m + n) * K * (K + 1.0) * (sizeof(T) == 8 ? 2.0 : 1.0) + 2.0 * (m + n) * K * r;
    }
    __syncthreads();
    const int r = sh.r;
    // Cu[:, c] = F_u * (M W)[:, order c] ; Cv[:, c] = F_v * W_m[:, order c]   (kp x r, into T1 / T2)
    for (int idx = threadIdx.x; idx < kp * r; idx += kT) {
        const int i = idx % kp, c = idx / kp, jc = sh.order[c];
        double su = 0.0, sv = 0.0;
        for (int l = 0; l < kp; ++l) {
            su += Fu[i + l * kp] * Mc[l + jc * kp];
            sv += Fv[i + l * kp] * Wm[l + jc * kp];
        }
        T1[i + c * kp] = su;
        T2[i + c * kp] = sv;
    }
    __syncthreads();
    // row-local, in place: U[i, :r] = U'[i, :] Cu, V[j, :r] = V'[j, :] Cv
    for (int i = threadIdx.x; i < m + n; i += kT) {
        const bool isu = i < m;
        const int row = isu ? i : i - m;
        const Cat<T>& C = isu ? Uc : Vc;
        const double* Cm = isu ? T1 : T2;
        T* out = isu ? U : V;
        const int ld = isu ? m : n;
        double rv[32];
#pragma unroll
        for (int l = 0; l < 32; ++l) rv[l] = l < kp ? C.at(row, l) : 0.0;
        for (int c = 0; c < r; ++c) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 32; ++l)
                if (l < kp) s += rv[l] * Cm[l + c * kp];
            out[row + (int64_t)c * ld] = (T)s;
        }
    }
    __syncthreads();
}

template <class T>
__device__ void op_lrsub(const Inst<T>& d, const OpRec& o, Shared& sh) {
    const int kx = dimval(d, o.dim[2]);
    if (threadIdx.x == 0) sh.lrsub_flops = 0.0;
    if (kx <= 0) return;
    const LRBlockDev L = d.lr[o.blk];
    // k' <= 32: Gram-based recompression (accurate to ~kappa^2 eps in the kept directions)
    if (d.ranks[L.slot] + kx <= 32) {
        op_lrsub_fast(d, o, sh, L, d.ranks[L.slot], kx);
        return;
    }
    T* U = d.arena + L.uoff;
    T* V = d.arena + L.voff;
    const int m = L.m, n = L.n, kc = d.ranks[L.slot], kp = kc + kx;
    const T* Xp = vptr(d, o.v[0]);
    const T* Yp = vptr(d, o.v[1]);
    const int xrs = o.v[0].rs, xcs = o.v[0].cs, yrs = o.v[1].rs, ycs = o.v[1].cs;
    // private scratch of this op: [U, -X], [V, Y], R_u, R_v; FP64 core, rotations, singular values
    T* Up = d.scr + o.sofs_t;
    T* Vp = Up + (int64_t)m * kp;
    T* Ru = Vp + (int64_t)n * kp;
    T* Rv = Ru + (int64_t)kp * kp;
    double* Md = d.scrd + o.sofs_d;
    double* Wd = Md + (int64_t)kp * kp;
    double* sig = Wd + (int64_t)kp * kp;
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * kp; idx += kT) {
        const int i = (int)(idx % m), c = (int)(idx / m);
        Up[idx] = c < kc ? U[i + (int64_t)c * m] : -Xp[(int64_t)i * xrs + (int64_t)(c - kc) * xcs];
    }
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * kp; idx += kT) {
        const int j = (int)(idx % n), c = (int)(idx / n);
        Vp[idx] = c < kc ? V[j + (int64_t)c * n] : Yp[(int64_t)j * yrs + (int64_t)(c - kc) * ycs];
    }
    __syncthreads();
    qr_cgs2(Up, m, kp, Ru, sh);
    qr_cgs2(Vp, n, kp, Rv, sh);
    for (int idx = threadIdx.x; idx < kp * kp; idx += kT) {
        const int i = idx % kp, j = idx / kp;
        double s = 0.0;
        for (int l = max(i, j); l < kp; ++l) s += (double)Ru[i + (int64_t)l * kp] * (double)Rv[j + (int64_t)l * kp];
        Md[idx] = s;
        Wd[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_svd(Md, Wd, kp, sh);
    if (threadIdx.x == 0) {
        const double K = kp;
        sh.lrsub_flops = 4.0 * (m + n) * K * K + 2.0 * K * K * K / 3.0 + sh.sweeps * K * (K - 1.0) / 2.0 * 12.0 * K;
    }
    for (int j = threadIdx.x; j < kp; j += kT) {
        double s = 0.0;
        for (int i = 0; i < kp; ++i) s += Md[i + (int64_t)j * kp] * Md[i + (int64_t)j * kp];
        sig[j] = sqrt(s);
    }
    __syncthreads();
    // rank of each singular value in descending order (ties by index)
    for (int j = threadIdx.x; j < kp; j += kT) {
        int r = 0;
        const double sj = sig[j];
        for (int i = 0; i < kp; ++i) r += (sig[i] > sj || (sig[i] == sj && i < j)) ? 1 : 0;
        sh.order[r] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double smax = sig[sh.order[0]];
        int r = 0;
        if (smax > 0.0)
            while (r < kp && sig[sh.order[r]] > d.tol * smax) ++r;
        if (r > d.kmax) r = d.kmax;
        sh.r = r;
        d.ranks[L.slot] = r;
        sh.lrsub_flops += 2.0 * (m + n) * (double)kp * r;
    }
    __syncthreads();
    const int r = sh.r;
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * r; idx += kT) {
        const int i = (int)(idx % m), c = (int)(idx / m);
        const int jc = sh.order[c];
        double s = 0.0;
        for (int l = 0; l < kp; ++l) s += (double)Up[i + (int64_t)l * m] * Md[l + (int64_t)jc * kp];
        U[i + (int64_t)c * m] = (T)s;
    }
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * r; idx += kT) {
        const int j = (int)(idx % n), c = (int)(idx / n);
        const int jc = sh.order[c];
        double s = 0.0;
        for (int l = 0; l < kp; ++l) s += (double)Vp[j + (int64_t)l * n] * Wd[l + (int64_t)jc * kp];
        V[j + (int64_t)c * n] = (T)s;
    }
    __syncthreads();
}

// floating-point operations of one op at its actual dimensions (evaluated before the op runs;
// the recompression adds the part that depends on the rank it finds)
template <class T>
__device__ double op_flops(const Inst<T>& d, const OpRec& o) {
    switch (o.code) {
        case OP_GEMM:
            return 2.0 * dimval(d, o.dim[0]) * dimval(d, o.dim[1]) * dimval(d, o.dim[2]);
        case OP_TRSM: {
            const double n = dimval(d, o.dim[0]);
            return n * n * dimval(d, o.dim[1]);
        }
        case OP_GETRF: {
            const double n = o.dim[0];
            return 2.0 * n * n * n / 3.0;
        }
        default: return 0.0;
    }
}

// one op; false when a leaf pivot broke down (the status is set)
template <class T>
__device__ bool run_op(const Inst<T>& d, int pc, Shared& sh, int step) {
    const OpRec o = d.ops[pc];
    unsigned long long t0 = 0;
    if (d.prof && threadIdx.x == 0) t0 = wall_clock64();
    double fl = 0.0;
    if (threadIdx.x == 0) fl = op_flops(d, o);
    bool ok = true;
    switch (o.code) {
        case OP_GEMM: op_gemm(d, o); break;
        case OP_ZERO: op_zero(d, o); break;
        case OP_TRSM: op_trsm(d, o); break;
        case OP_LRSUB: op_lrsub(d, o, sh); break;
        case OP_GETRF: ok = op_getrf(d, o, sh, pc); break;
        case OP_LOAD: {
            const double* Bs = d.B + (int64_t)step * d.bstep;
            for (int64_t idx = threadIdx.x; idx < (int64_t)d.Nd * d.nrhs; idx += kT) {
                const int h = (int)(idx % d.Nd), j = (int)(idx / d.Nd);
                d.rhs[idx] = (T)Bs[(int64_t)j * d.ldb + d.h2p[h]];
            }
            break;
        }
        case OP_STORE: {
            double* Xs = d.X + (int64_t)step * d.xstep;
            for (int64_t idx = threadIdx.x; idx < (int64_t)d.Nd * d.nrhs; idx += kT) {
                const int h = (int)(idx % d.Nd), j = (int)(idx / d.Nd);
                Xs[(int64_t)j * d.ldx + d.h2p[h]] = (double)d.rhs[idx];
            }
            break;
        }
        default: break;
    }
    if (!ok) return false;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (o.code == OP_LRSUB) fl += sh.lrsub_flops;
        atomicAdd(d.flops, fl);
    }
    if (d.prof && threadIdx.x == 0) {
        atomicAdd(&d.prof[2 * o.code], (unsigned long long)(wall_clock64() - t0));
        atomicAdd(&d.prof[2 * o.code + 1], 1ull);
    }
    return true;
}

template <class T>
__device__ void run_program(const Inst<T>& d, Shared& sh, int step) {
    for (int pc = 0; pc < d.nops; ++pc)
        if (!run_op(d, pc, sh, step)) return;
}

template <class T>
__global__ void __launch_bounds__(kT) k_interp(const Inst<T>* __restrict__ insts, int step) {
    __shared__ Shared sh;
    run_program(insts[blockIdx.x], sh, step);
}

template <class T>
__global__ void __launch_bounds__(kT) k_interp_one(const Inst<T> d) {
    __shared__ Shared sh;
    run_program(d, sh, 0);
}

// one level: the ops of a level are independent, earlier levels have completed (kernel order)
template <class T>
__global__ void __launch_bounds__(kT) k_level(const Inst<T>* __restrict__ insts, const int2* __restrict__ tasks) {
    __shared__ Shared sh;
    const int2 tk = tasks[blockIdx.x];
    const Inst<T>& d = insts[tk.x];
    // after a breakdown in an earlier level the rest of that factorisation is skipped; the
    // status is read once and shared so that every thread takes the same branch
    if (threadIdx.x == 0) sh.stop = d.status[0];
    __syncthreads();
    if (sh.stop != 0) return;
    run_op(d, tk.y, sh, 0);
}

}  // namespace

bool profile_ops_enabled() {
    const char* e = getenv("FDE_PROFILE_OPS");
    return e && e[0] == '1';
}

void print_op_profile(const char* what, const unsigned long long* p, int device) {
    int rate_khz = 0;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device);
    const double ms_per_tick = rate_khz > 0 ? 1.0 / rate_khz : 0.0;
    static const char* names[8] = {"-", "GETRF", "TRSM", "GEMM", "LRSUB", "ZERO", "LOAD", "STORE"};
    fprintf(stderr, "[fde ops] %s:", what);
    for (int c = 1; c < 8; ++c)
        if (p[2 * c + 1]) fprintf(stderr, " %s %llu x %.3f ms = %.2f ms;", names[c], p[2 * c + 1],
                                  p[2 * c] * ms_per_tick / p[2 * c + 1], p[2 * c] * ms_per_tick);
    fprintf(stderr, "\n");
}

template <class T>
void launch_interp(hipStream_t st, int ninst, const Inst<T>* d_insts, int step) {
    if (ninst <= 0) return;
    hipLaunchKernelGGL((k_interp<T>), dim3(ninst), dim3(kT), 0, st, d_insts, step);
    FDE_LAUNCH_CHECK();
}
template void launch_interp<float>(hipStream_t, int, const Inst<float>*, int);
template void launch_interp<double>(hipStream_t, int, const Inst<double>*, int);

template <class T>
void launch_interp_one(hipStream_t st, const Inst<T>& d) {
    hipLaunchKernelGGL((k_interp_one<T>), dim3(1), dim3(kT), 0, st, d);
    FDE_LAUNCH_CHECK();
}
template void launch_interp_one<float>(hipStream_t, const Inst<float>&);
template void launch_interp_one<double>(hipStream_t, const Inst<double>&);

template <class T>
void launch_level(hipStream_t st, int ntasks, const Inst<T>* d_insts, const int2* d_tasks) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL((k_level<T>), dim3(ntasks), dim3(kT), 0, st, d_insts, d_tasks);
    FDE_LAUNCH_CHECK();
}
template void launch_level<float>(hipStream_t, int, const Inst<float>*, const int2*);
template void launch_level<double>(hipStream_t, int, const Inst<double>*, const int2*);

}  // namespace fde
