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
    double red[kW][32];
    double dots[kMaxKp];
    int order[kMaxKp];
    int flag;
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

template <class T>
__device__ void op_lrsub(const Inst<T>& d, const OpRec& o, Shared& sh) {
    const int kx = dimval(d, o.dim[2]);
    if (threadIdx.x == 0) sh.lrsub_flops = 0.0;
    if (kx <= 0) return;
    const LRBlockDev L = d.lr[o.blk];
    T* U = d.arena + L.uoff;
    T* V = d.arena + L.voff;
    const int m = L.m, n = L.n, kc = d.ranks[L.slot], kp = kc + kx;
    const T* Xp = vptr(d, o.v[0]);
    const T* Yp = vptr(d, o.v[1]);
    const int xrs = o.v[0].rs, xcs = o.v[0].cs, yrs = o.v[1].rs, ycs = o.v[1].cs;
    T* Up = d.scr;
    T* Vp = Up + d.mrmax * d.kpmax;
    T* Ru = Vp + d.mrmax * d.kpmax;
    T* Rv = Ru + (int64_t)d.kpmax * d.kpmax;
    double* Md = d.scrd;
    double* Wd = Md + (int64_t)d.kpmax * d.kpmax;
    double* sig = Wd + (int64_t)d.kpmax * d.kpmax;
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

template <class T>
__device__ void run_program(const Inst<T>& d, Shared& sh, int step) {
    const int nops = d.nops;
    const double* Bs = d.B + (int64_t)step * d.bstep;
    double* Xs = d.X + (int64_t)step * d.xstep;
    for (int pc = 0; pc < nops; ++pc) {
        const OpRec o = d.ops[pc];
        unsigned long long t0 = 0;
        if (d.prof && threadIdx.x == 0) t0 = wall_clock64();
        double fl = 0.0;
        if (threadIdx.x == 0) fl = op_flops(d, o);
        switch (o.code) {
            case OP_GEMM: op_gemm(d, o); break;
            case OP_ZERO: op_zero(d, o); break;
            case OP_TRSM: op_trsm(d, o); break;
            case OP_LRSUB: op_lrsub(d, o, sh); break;
            case OP_GETRF:
                if (!op_getrf(d, o, sh, pc)) return;
                break;
            case OP_LOAD:
                for (int64_t idx = threadIdx.x; idx < (int64_t)d.Nd * d.nrhs; idx += kT) {
                    const int h = (int)(idx % d.Nd), j = (int)(idx / d.Nd);
                    d.rhs[idx] = (T)Bs[(int64_t)j * d.ldb + d.h2p[h]];
                }
                break;
            case OP_STORE:
                for (int64_t idx = threadIdx.x; idx < (int64_t)d.Nd * d.nrhs; idx += kT) {
                    const int h = (int)(idx % d.Nd), j = (int)(idx / d.Nd);
                    Xs[(int64_t)j * d.ldx + d.h2p[h]] = (double)d.rhs[idx];
                }
                break;
            default: break;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (o.code == OP_LRSUB) fl += sh.lrsub_flops;
            atomicAdd(d.flops, fl);
        }
        if (d.prof && threadIdx.x == 0) {
            atomicAdd(&d.prof[2 * o.code], (unsigned long long)(wall_clock64() - t0));
            atomicAdd(&d.prof[2 * o.code + 1], 1ull);
        }
    }
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

}  // namespace fde
