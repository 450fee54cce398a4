// Device execution of H-arithmetic programs (H-LU and H-substitutions).
//
// k_level runs one level of level-scheduled programs: workgroup b executes one op
// of one instance, and the ops of a level touch disjoint memory. k_interp runs a
// whole op list per workgroup, one instance each (the serial order, and
// H-solves whose right-hand sides do not fit in LDS); a launch of either kernel
// serves many instances of different sizes at once.
//
// Ops: GETRF (dense LU without pivoting, Section 4.1 takes L_H unit lower and
// no pivoting; a pivot below the floor is a breakdown), TRSM, GEMM, ZERO, and
// LRSUB -- C <- trunc(U_C V_C^T - X Y^T). Up to the variant's width KS the
// recompression works on Gram matrices (pivoted Cholesky in FP32; shifted
// Cholesky QR3 in FP64, the core R_u R_v^T decomposed by one-sided Jacobi in
// registers); wider sums (the general variant, which the host no longer selects)
// take a thin QR of [U_C, -X] and [V_C, Y] by classical Gram-Schmidt with one
// reorthogonalisation and a one-sided Jacobi SVD of the core in FP64. Either way
// the singular values above tol * sigma_1 are kept, at most kmax of them (the
// truncation to a prescribed tolerance of Section 4.1). LOAD/STORE move FP64
// vectors in the paper's order to and from the internal order; LRMV applies a
// low-rank block to a vector.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "hinterp.h"
#include "tri_wave.h"

namespace fde {

namespace {

constexpr int kT = kInterpThreads;
constexpr int kW = kT / 64;

constexpr int kGT = 64;            // GEMM output tile (rows and columns)
constexpr int kGK = 32;            // GEMM k chunk
template <class T>
struct GemmLds {
    T A[kGT][kGK + 1];             // A tile, row-major (padded)
    T B[kGK][kGT + 1];             // B tile, row-major (padded)
};
constexpr int kLU = 64;            // GETRF leaves factored in registers up to this size

// small recompression (k' <= KS): staged rows, Gram matrices, Cholesky factors
template <int KS, bool F64>
struct LrsLds {
    static constexpr int K = KS;                     // widest k'
    static constexpr int CH = KS <= 16 ? 64 : 32;    // rows per staged chunk
    static constexpr int LD = KS + 1;                // row stride of staged rows (odd: no bank conflicts along a column)
    double A[2][CH * LD];   // staged rows of both sides (row-major, stride LD); later C_u, C_v (ld K)
    double G[2][KS * KS];   // Gram matrices; then the core M and rotations Z; then C_u, C_v
    double R[2][KS * KS];   // Cholesky factors R[a][j] (row a, original column j)
    double R2[F64 ? 2 : 1][F64 ? KS * KS : 1];   // FP64: the second pass's factor while the third runs
    double sig[KS];
    int perm[2][KS], perm2[2][KS];
    int q[2], q2[2], q3[2];
};

// LDS of one interpreter workgroup. KS: widest recompression of the small path; GENERAL: the
// variant also carries the Gram-Schmidt path for wider ones (and its larger register file)
template <class T, int KS, bool GENERAL>
struct Shared {
    static constexpr int kSmall = KS;
    static constexpr bool kGeneral = GENERAL;
    union {
        LrsLds<KS, sizeof(T) == 8> ls;
        GemmLds<T> gm;
    };
    OpRec op;        // level kernel: this workgroup's op, rank-dependent sizes resolved
    Inst<T> inst;    // level kernel: its instance
    double red[kW][32];
    double dots[GENERAL ? kMaxKp : 1];
    int order[GENERAL ? kMaxKp : KS];
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

template <class SH>
__device__ inline double block_sum(double v, SH& sh) {
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
template <class SH>
__device__ inline double block_max(double v, SH& sh) {
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
// C = beta C + alpha A B. Products of at least 16 rows go through LDS tiles (64 x 64 outputs, k
// in chunks of 32; each thread a 4 x 4 register tile, masked at the edges) when they have at
// least 16 columns, or more outputs than threads and k >= 16 (one thread per output would walk
// its outputs one after another, a memory latency each); thin products use G lanes per output,
// consecutive lanes along k, reduced by shuffles, or one thread per output.
template <class T, class SH>
__device__ __attribute__((noinline)) void op_gemm(const Inst<T>& d, const OpRec& o, SH& sh) {
    const int m = dimval(d, o.dim[0]), n = dimval(d, o.dim[1]), k = dimval(d, o.dim[2]);
    T* C = vptr(d, o.v[0]);
    const T* A = vptr(d, o.v[1]);
    const T* B = vptr(d, o.v[2]);
    const T alpha = (T)o.alpha, beta = (T)o.beta;
    const int ars = o.v[1].rs, acs = o.v[1].cs, brs = o.v[2].rs, bcs = o.v[2].cs;
    const int crs = o.v[0].rs, ccs = o.v[0].cs;
    if (m <= 0 || n <= 0) return;
    const int t = threadIdx.x;
    if (m >= 16 && (n >= 16 || (k >= 16 && (int64_t)m * n > kT))) {
        // The loads of an operand's stage are issued before any is used (addresses of elements
        // outside the operand are clamped to its first entry), and the 16 entries of C a thread
        // updates are read together after the products: a tile costs a few memory latencies
        // rather than one per element.
        GemmLds<T>& L = sh.gm;
        constexpr int kEl = kGT * kGK / kT;   // tile elements per thread and operand
        const int ti = t % 16, tj = t / 16;   // rows 4 ti .. 4 ti + 3, columns 4 tj .. 4 tj + 3 of a tile
        for (int i0 = 0; i0 < m; i0 += kGT)
            for (int j0 = 0; j0 < n; j0 += kGT) {
                T acc[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[e] = T(0);
                for (int l0 = 0; l0 < k; l0 += kGK) {
                    // stage: consecutive threads along whichever index is contiguous in memory
                    int tid = t;   // opaque: element addresses are formed here, not held across the loops
                    asm volatile("" : "+v"(tid));
                    {
                        T v[kEl];
#pragma unroll
                        for (int e = 0; e < kEl; ++e) {
                            const int idx = tid + e * kT;
                            const int i = ars == 1 ? idx % kGT : idx / kGK, l = ars == 1 ? idx / kGT : idx % kGK;
                            const bool ok = i0 + i < m && l0 + l < k;
                            v[e] = gmem(A)[ok ? (int64_t)(i0 + i) * ars + (int64_t)(l0 + l) * acs : 0];
                        }
#pragma unroll
                        for (int e = 0; e < kEl; ++e) {
                            const int idx = tid + e * kT;
                            const int i = ars == 1 ? idx % kGT : idx / kGK, l = ars == 1 ? idx / kGT : idx % kGK;
                            L.A[i][l] = (i0 + i < m && l0 + l < k) ? v[e] : T(0);
                        }
                    }
                    {
                        T v[kEl];
#pragma unroll
                        for (int e = 0; e < kEl; ++e) {
                            const int idx = tid + e * kT;
                            const int l = brs == 1 ? idx % kGK : idx / kGT, j = brs == 1 ? idx / kGK : idx % kGT;
                            const bool ok = l0 + l < k && j0 + j < n;
                            v[e] = gmem(B)[ok ? (int64_t)(l0 + l) * brs + (int64_t)(j0 + j) * bcs : 0];
                        }
#pragma unroll
                        for (int e = 0; e < kEl; ++e) {
                            const int idx = tid + e * kT;
                            const int l = brs == 1 ? idx % kGK : idx / kGT, j = brs == 1 ? idx / kGK : idx % kGT;
                            L.B[l][j] = (l0 + l < k && j0 + j < n) ? v[e] : T(0);
                        }
                    }
                    __syncthreads();
                    const int kl = min(kGK, k - l0);
                    for (int l = 0; l < kl; ++l) {
                        T av[4], bv[4];
#pragma unroll
                        for (int a = 0; a < 4; ++a) av[a] = L.A[4 * ti + a][l];
#pragma unroll
                        for (int b = 0; b < 4; ++b) bv[b] = L.B[l][4 * tj + b];
#pragma unroll
                        for (int a = 0; a < 4; ++a)
#pragma unroll
                            for (int b = 0; b < 4; ++b) acc[4 * a + b] += av[a] * bv[b];
                    }
                    __syncthreads();
                }
                int tid = t;
                asm volatile("" : "+v"(tid));
                const int ri = tid % 16, rj = tid / 16;
                T cv[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int gi = i0 + 4 * ri + e / 4, gj = j0 + 4 * rj + e % 4;
                    const bool ok = beta != T(0) && gi < m && gj < n;
                    cv[e] = gmem(C)[ok ? (int64_t)gi * crs + (int64_t)gj * ccs : 0];
                }
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int gi = i0 + 4 * ri + e / 4, gj = j0 + 4 * rj + e % 4;
                    if (gi < m && gj < n)
                        C[(int64_t)gi * crs + (int64_t)gj * ccs] = (beta == T(0) ? T(0) : beta * cv[e]) + alpha * acc[e];
                }
            }
        return;
    }
    const int64_t mn = (int64_t)m * n;
    int G = 1;
    while (2 * G * mn <= kT && 2 * G <= 64) G <<= 1;
    if (G >= 2 && k >= 2 * G) {
        const int ngroups = kT / G, gid = t / G, gl = t % G;
        for (int64_t idx = gid; idx < mn; idx += ngroups) {
            const int i = (int)(idx % m), j = (int)(idx / m);
            const T* a = A + (int64_t)i * ars;
            const T* b = B + (int64_t)j * bcs;
            double s = 0.0;
#pragma unroll 4
            for (int l = gl; l < k; l += G) s += (double)a[(int64_t)l * acs] * (double)b[(int64_t)l * brs];
            for (int o2 = G / 2; o2 > 0; o2 >>= 1) s += __shfl_xor(s, o2, 64);
            if (gl == 0) {
                T* c = C + (int64_t)i * crs + (int64_t)j * ccs;
                *c = (beta == T(0) ? T(0) : beta * *c) + alpha * (T)s;
            }
        }
        return;
    }
    for (int64_t idx = t; idx < mn; idx += kT) {
        const int i = (int)(idx % m), j = (int)(idx / m);
        const T* a = A + (int64_t)i * ars;
        const T* b = B + (int64_t)j * bcs;
        T s = 0;
#pragma unroll 8
        for (int l = 0; l < k; ++l) s += a[(int64_t)l * acs] * b[(int64_t)l * brs];
        T* c = C + (int64_t)i * crs + (int64_t)j * ccs;
        *c = (beta == T(0) ? T(0) : beta * *c) + alpha * s;
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
template <class T, class SH>
__device__ __attribute__((noinline)) void op_trsm(const Inst<T>& d, const OpRec& o, SH& sh) {
    const int n = dimval(d, o.dim[0]), w = dimval(d, o.dim[1]);
    if (n <= 0 || w <= 0) return;
    T* X = vptr(d, o.v[0]);
    const T* Tm = vptr(d, o.v[1]);
    const int xrs = o.v[0].rs, xcs = o.v[0].cs, trs = o.v[1].rs, tcs = o.v[1].cs;
    const bool lower = o.flags & 1, unit = o.flags & 2;
    auto Tat = [&](int i, int j) -> T { return Tm[(int64_t)i * trs + (int64_t)j * tcs]; };
    if (n <= 64) {
        if (tcs == 1 && trs != 1) {
            // a triangle read row-wise (the transposed view of a column-major block): every lane
            // would load its own row, 64 cache lines per load instruction. Staged through LDS
            // instead, consecutive threads along each row, padded row stride 65 (no bank conflicts).
            static_assert(sizeof(GemmLds<T>) >= 64 * 65 * sizeof(T), "TRSM triangle stage");
            T* st = reinterpret_cast<T*>(&sh.gm);
            __syncthreads();   // the previous op's use of this LDS is over
            for (int idx = threadIdx.x; idx < 64 * 64; idx += kT) {
                const int i = idx >> 6, c = idx & 63;
                if (i < n && c < n) st[i * 65 + c] = Tm[(int64_t)i * trs + c];
            }
            __syncthreads();
            tri_wave(static_cast<const T*>(st), 65, 1, n, lower, unit, X, xrs, xcs, w, (int)(threadIdx.x >> 6), kW);
            __syncthreads();
            return;
        }
        tri_wave(Tm, trs, tcs, n, lower, unit, X, xrs, xcs, w, (int)(threadIdx.x >> 6), kW);
        return;
    }
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
// LU without pivoting of a dense leaf (unit lower L), right-looking. Leaves up to kLU = 64 rows:
// lane i of every wavefront holds row i, wavefront w its columns 16 w .. 16 w + 15, in registers;
// the step loop is unrolled. At step k the wavefront holding column k forms the multipliers,
// updates its own columns past k (the pivot row broadcast entry by entry with readlane) and puts
// the multipliers and its pivot verdict in LDS; after one barrier the wavefronts to its right
// update their columns. Each entry sees the same operations as in a one-wavefront sweep. The
// slot alternates with the step's parity, so a slot is rewritten only after every wavefront has
// passed the next barrier; every step has its barrier (a counted loop, fully unrolled), and a
// failed pivot stops the updates in every wavefront at the same step. Larger leaves: in place,
// two barriers per step.
template <class T, class SH>
__device__ __attribute__((noinline)) bool op_getrf(const Inst<T>& d, const OpRec& o, SH& sh, int pc) {
    const int n = o.dim[0];
    T* A = vptr(d, o.v[0]);
    const int rs = o.v[0].rs, cs = o.v[0].cs;
    auto at = [&](int i, int j) -> T& { return A[(int64_t)i * rs + (int64_t)j * cs]; };
    if (n <= kLU) {
        static_assert(kLU == 16 * kW, "four wavefronts of 16 columns");
        static_assert(sizeof(GemmLds<T>) >= 2 * 65 * sizeof(T), "GETRF step slots");
        T* slots = reinterpret_cast<T*>(&sh.gm);   // [2][65]: the step's multipliers, then its verdict
        const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
        const int ri = min(i, n - 1);
        T a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = A[(int64_t)ri * rs + (int64_t)min(16 * w + c, n - 1) * cs];
        double amax = 0.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (i >= n || 16 * w + c >= n) a[c] = T(0);
            amax = fmax(amax, fabs((double)a[c]));
        }
        amax = wave_max(amax);
        if (i == 0) sh.red[w][0] = amax;
        __syncthreads();
        amax = fmax(fmax(sh.red[0][0], sh.red[1][0]), fmax(sh.red[2][0], sh.red[3][0]));
        int fail_at = -1;
#pragma unroll
        for (int k = 0; k < kLU; ++k) {
            const bool live = k < n && fail_at < 0;   // the same in every thread
            const int kw = k >> 4, kc = k & 15;
            T* sl = slots + (k & 1) * 65;
            if (live && w == kw) {
                const T akk = lane_bcast(a[kc], k);
                const bool bad = !(fabs((double)akk) > d.pivot_floor * amax) || !(fabs((double)akk) > 0.0);
                if (!bad) {
                    // an opaque copy of the row index: the per-step row masks are formed here rather
                    // than hoisted and held in registers across the elimination
                    int ii = i;
                    asm volatile("" : "+v"(ii));
                    const T l = ii > k ? a[kc] / akk : T(0);
                    if (ii > k) a[kc] = l;
                    sl[i] = l;
#pragma unroll
                    for (int c = kc + 1; c < 16; ++c) a[c] -= l * lane_bcast(a[c], k);
                }
                if (i == 0) sl[64] = bad ? T(1) : T(0);
            }
            __syncthreads();
            if (live) {
                if (sl[64] != T(0)) {
                    fail_at = k;
                } else if (w > kw) {
                    const T l = sl[i];
#pragma unroll
                    for (int c = 0; c < 16; ++c) a[c] -= l * lane_bcast(a[c], k);
                }
            }
        }
        if (fail_at < 0 && i < n)
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (16 * w + c < n) A[(int64_t)i * rs + (int64_t)(16 * w + c) * cs] = a[c];
        if (threadIdx.x == 0) sh.flag = fail_at;
        __syncthreads();
        if (sh.flag >= 0) {
            if (threadIdx.x == 0) {
                d.status[0] = FDE_EBREAKDOWN;
                d.status[1] = pc;
            }
            return false;
        }
        return true;
    }
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
template <class T, class SH>
__device__ void qr_cgs2(T* Q, int rows, int kp, T* R, SH& sh) {
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
template <class SH>
__device__ void jacobi_svd(double* M, double* W, int kp, SH& sh) {
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

// ----- small recompression (k' <= kSK): Cholesky QR of both sides, one small SVD
//
// With A_u = [U_C, -X] (m x k') and A_v = [V_C, Y] (n x k'), U_C V_C^T - X Y^T = A_u A_v^T.
// The Gram matrices A^T A (FP64) are factorised by pivoted Cholesky, P^T G P = R^T R with R
// upper trapezoidal (rank q: pivots below a relative floor are dropped), so that
// A P = Q R with orthonormal Q = (A P)[:, :q] R11^{-1}. Then A_u A_v^T = Q_u M Q_v^T with the
// small core M = (R_u P_u^T)(R_v P_v^T)^T, whose SVD M = W S Z^T (one-sided Jacobi) is truncated
// to the singular values above tol * s_1 (at most kmax): U_C <- A_u C_u, V_C <- A_v C_v with
// C_u = P_u R11_u^{-1} (W S)_r and C_v = P_v R11_v^{-1} Z_r.
// FP64 factors need more than that single pass: the pivot floor loses directions below about
// 1e-7 of a side's largest column and the solves with an ill-conditioned R11 amplify rounding,
// which caps the agreement with a Householder QR + SVD near 1e-9. They take a shifted Cholesky
// QR3 instead (A = Q R with R a general q x k' matrix) and the inverse-free coefficients
// C_u = R_v^T Z_r, C_v = R_u^T W_r S_r^{-1}.

// one side's column c at row i of [F, sgn * G] (F: current factor, ld rows; G: update view)
template <class T>
struct Side {
    const T* F;
    int ldf, kc;
    const T* G;
    int grs, gcs;
    double sgn;
    int rows;
    __device__ double at(int i, int c) const {
        return c < kc ? (double)F[i + (int64_t)c * ldf] : sgn * (double)G[(int64_t)i * grs + (int64_t)(c - kc) * gcs];
    }
};

// Rows [c0, c0 + kCH) of both sides, staged through registers: element t of a thread is side
// s = t / (kEl / 2), column c and chunk row rr, consecutive threads along rr (coalesced down the
// factor columns). All loads of a chunk are issued before any is used (addresses of elements
// outside the block are clamped to the factor's first entry), so a chunk costs one memory latency,
// and the next chunk is loaded while the current one is used.
template <class LS>
struct RowChunk {
    static constexpr int kEl = 2 * LS::CH * LS::K / kT;
    static_assert(kEl * kT == 2 * LS::CH * LS::K, "a chunk is a whole number of elements per thread");
};
template <class T, class LS>
__device__ __attribute__((always_inline)) inline void load_rows(const Side<T>& su, const Side<T>& sv, int c0, int kp,
                                                                T* v) {
    constexpr int kSK = LS::K, kCH = LS::CH, kEl = RowChunk<LS>::kEl;
    // opaque thread index: the per-element addresses are formed here, not hoisted out of the
    // caller's chunk loop and held in registers across it
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int t = 0; t < kEl; ++t) {
        const Side<T>& sd = t < kEl / 2 ? su : sv;
        const int rem = (tid + t * kT) % (kCH * kSK);
        const int c = rem / kCH, i = c0 + rem % kCH;
        const bool ok = i < sd.rows && c < kp;
        const T* p = c < sd.kc ? sd.F + i + (int64_t)c * sd.ldf
                               : sd.G + (int64_t)i * sd.grs + (int64_t)(c - sd.kc) * sd.gcs;
        v[t] = gmem(ok ? p : sd.F)[0];
    }
}
template <class T, class LS>
__device__ __attribute__((always_inline)) inline void store_rows(const Side<T>& su, const Side<T>& sv, int c0, int kp,
                                                                 const T* v, LS& S) {
    constexpr int kSK = LS::K, kCH = LS::CH, kLD = LS::LD, kEl = RowChunk<LS>::kEl;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int t = 0; t < kEl; ++t) {
        const Side<T>& sd = t < kEl / 2 ? su : sv;
        const int rem = (tid + t * kT) % (kCH * kSK);
        const int c = rem / kCH, rr = rem % kCH, i = c0 + rr;
        const bool ok = i < sd.rows && c < kp;
        S.A[t < kEl / 2 ? 0 : 1][rr * kLD + c] = ok ? (c < sd.kc ? (double)v[t] : sd.sgn * (double)v[t]) : 0.0;
    }
}

// largest dv over lanes 0 .. kSK-1 (kSK = 16 or 32) and its lane index pj, ties to the smaller
// index; wave-uniform on return. Each row of 16 lanes is reduced by DPP rotations, the rows'
// winners are read with readlane.
template <int kSK>
__device__ inline void argmax_rows(double& dv, int& pj) {
    static_assert(kSK == 16 || kSK == 32, "pivot search covers one or two rows of 16 lanes");
    auto take = [&](double ov, int op) {
        if (ov > dv || (ov == dv && op < pj)) {
            dv = ov;
            pj = op;
        }
    };
    take(dpp_move<dpp_row_ror(8)>(dv), dpp_move<dpp_row_ror(8)>(pj));
    take(dpp_move<dpp_row_ror(4)>(dv), dpp_move<dpp_row_ror(4)>(pj));
    take(dpp_move<dpp_row_ror(2)>(dv), dpp_move<dpp_row_ror(2)>(pj));
    take(dpp_move<dpp_row_ror(1)>(dv), dpp_move<dpp_row_ror(1)>(pj));
    const double v0 = lane_bcast(dv, 0);
    const int p0 = __builtin_amdgcn_readlane(pj, 0);
    if (kSK == 32) {
        const double v1 = lane_bcast(dv, 16);
        const int p1 = __builtin_amdgcn_readlane(pj, 16);
        const bool second = v1 > v0 || (v1 == v0 && p1 < p0);
        dv = second ? v1 : v0;
        pj = second ? p1 : p0;
    } else {
        dv = v0;
        pj = p0;
    }
}

// Gram matrices G_s = A_s^T A_s of the staged rows of both sides on the FP64 matrix cores, in
// 16 x 16 tiles accumulated in registers over the caller's chunk loop. Tile (ti, tj) of side s
// takes one v_mfma_f64_16x16x4 per four staged rows: lane l brings row 4 kk + l / 16 at column
// 16 ti + l % 16 (A operand: entry (l % 16, l / 16) of the 16 x 4 factor) and at column
// 16 tj + l % 16 (B operand: entry (l / 16, l % 16) of the 4 x 16 factor); register v of lane l
// holds entry (4 v + l / 16, l % 16) of the 16 x 16 result. The waves take the tiles of both sides
// round robin. Rows beyond the block and columns beyond k' are staged as zeros, so every entry of
// G outside k' x k' comes out 0.
typedef double v4d __attribute__((ext_vector_type(4)));
template <class LS>
struct GramTiles {
    static constexpr int T = LS::K / 16, kJobs = 2 * T * T, kPerWave = (kJobs + kW - 1) / kW;
    static_assert(LS::K % 16 == 0 && LS::CH % 4 == 0, "Gram tiles of 16 x 16, four rows per instruction");
    v4d acc[kPerWave];
};
template <class LS>
__device__ inline void gram_tiles_clear(GramTiles<LS>& g) {
#pragma unroll
    for (int u = 0; u < GramTiles<LS>::kPerWave; ++u) g.acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
}
template <class LS>
__device__ inline void gram_tiles_accumulate(const LS& S, GramTiles<LS>& g) {
    using G = GramTiles<LS>;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < G::kPerWave; ++u) {
        const int jb = wave + u * kW;
        if (jb < G::kJobs) {
            const int sd = jb / (G::T * G::T), ti = (jb % (G::T * G::T)) / G::T, tj = jb % G::T;
            const double* A = S.A[sd] + (lane >> 4) * LS::LD + (lane & 15);
#pragma unroll 4
            for (int kk = 0; kk < LS::CH / 4; ++kk) {
                const double a = A[4 * kk * LS::LD + 16 * ti], b = A[4 * kk * LS::LD + 16 * tj];
                g.acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g.acc[u], 0, 0, 0);
            }
        }
    }
}
template <class LS>
__device__ inline void gram_tiles_store(LS& S, const GramTiles<LS>& g) {
    using G = GramTiles<LS>;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < G::kPerWave; ++u) {
        const int jb = wave + u * kW;
        if (jb < G::kJobs) {
            const int sd = jb / (G::T * G::T), ti = (jb % (G::T * G::T)) / G::T, tj = jb % G::T;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                S.G[sd][(16 * ti + 4 * v + (lane >> 4)) * LS::K + 16 * tj + (lane & 15)] = g.acc[u][v];
        }
    }
}

// Cholesky of the k x k Gram G (LDS, ld kSK) by one wavefront, lane j = index j, in registers:
// lane j holds column j and its current diagonal; the pivot is wave-uniform and the new column of
// L is broadcast with readlane for the Schur update. With pivoting the largest remaining diagonal
// is taken next and the factorisation stops when it falls to floor_rel times the largest initial
// diagonal; without it the order is 0, 1, ... On return R[a][j] (a < q, LDS) holds row a of R in
// original column j, perm[a] the a-th pivot and *q the rank.
template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;
// LDS view of a pointer into the workgroup's shared memory (accesses become LDS instructions in a
// function that is not inlined into the kernel)
template <class T>
__device__ inline lds_ptr<T> lmem(T* p) {
    return (lds_ptr<T>)p;
}

template <int kSK>
__device__ __attribute__((noinline)) void wave_cholesky(lds_ptr<const double> G, lds_ptr<double> R, lds_ptr<int> perm,
                                                        lds_ptr<int> q_out, int k, bool pivot, double floor_rel) {
    const int j = threadIdx.x & 63;
    const bool in = j < k;
    double g[kSK];
#pragma unroll
    for (int i = 0; i < kSK; ++i) g[i] = (in && i < k) ? G[i * kSK + j] : 0.0;
    double dj = in ? G[j * kSK + j] : 0.0;
    bool rem = in;
    double d0 = dj;
    int p0 = j;
    argmax_rows<kSK>(d0, p0);
    for (int a = 0; a < k; ++a)
        if (in) R[a * kSK + j] = 0.0;
    int q = k;
    bool done = false;
#pragma unroll
    for (int a = 0; a < kSK; ++a) {
        if (a < k && !done) {
            double dv = pivot ? (rem ? dj : -1.0) : (j == a ? dj : -1.0);
            int pj = j;
            argmax_rows<kSK>(dv, pj);
            const int p = __builtin_amdgcn_readfirstlane(pj);
            if (!(dv > floor_rel * d0) || !(dv > 0.0)) {
                q = a;
                done = true;
            } else {
                const double lp = sqrt(dv), inv = 1.0 / lp;
                if (j == p) rem = false;
                double gp = 0.0;
#pragma unroll
                for (int i = 0; i < kSK; ++i)
                    if (i == p) gp = g[i];
                const double lj = in ? (j == p ? lp : (rem ? gp * inv : 0.0)) : 0.0;
                if (in) R[a * kSK + j] = lj;
                if (j == 0) perm[a] = p;
                if (rem) {   // lj is 0 on lanes k .. kSK-1: their entries of g stay untouched
#pragma unroll
                    for (int i = 0; i < kSK; ++i) g[i] -= lane_bcast(lj, i) * lj;
                    dj -= lj * lj;
                }
            }
        }
    }
    if (j == 0) *q_out = q;
}

// sum over the kLpc consecutive lanes that hold one column (kLpc = 1, 2 or 4); every lane of the
// group gets the same bits (the butterfly adds the same pairs in the same order)
template <int kLpc, class W>
__device__ inline W column_sum(W v) {
    static_assert(kLpc == 1 || kLpc == 2 || kLpc == 4, "a column spans at most one quad");
    if (kLpc >= 2) v += dpp_move<kDppXor1>(v);
    if (kLpc >= 4) v += dpp_move<kDppXor2>(v);
    return v;
}

// Jacobi rotation (c, s) = (cs, cs * t) that zeroes the off-diagonal g of the 2 x 2 Gram
// [[ap, g], [g, aq]] (the smaller root t of t^2 + 2 zeta t - 1 = 0). FP32 uses the hardware
// reciprocal and square-root approximations: both columns take the same (cs, sn), so M Z stays
// the product of the original M with the accumulated Z whatever their last-bit error.
__device__ inline void jacobi_rotation(float ap, float aq, float g, float& cs, float& sn) {
    const float zeta = (aq - ap) * __builtin_amdgcn_rcpf(g + g);
    const float t0 = __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(fmaf(zeta, zeta, 1.0f)));
    const float t = zeta >= 0.0f ? t0 : -t0;
    cs = __builtin_amdgcn_rsqf(fmaf(t, t, 1.0f));
    sn = cs * t;
}
__device__ inline void jacobi_rotation(double ap, double aq, double g, double& cs, double& sn) {
    const double zeta = (aq - ap) / (g + g);
    const double t0 = 1.0 / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
    const double t = zeta >= 0.0 ? t0 : -t0;
    cs = 1.0 / sqrt(fma(t, t, 1.0));
    sn = cs * t;
}

// one-sided Jacobi on the columns of M (rows x cols, column-major ld kSK, LDS) by one wavefront,
// in registers: column c is held by kLpc = 64 / kSK lanes, each with kSK / kLpc interleaved rows
// of M and of the rotations Z. In each round of the round-robin order a lane fetches its partner
// column's rows (one shuffle per row), the pair's dot products are summed over the column's
// lanes, and both columns of the pair apply the same rotation. A pair counts as orthogonal when
// g^2 <= conv^2 ap aq. On return M holds the rotated columns, Z (cols x cols, LDS) the rotations
// and nrm[c] the norm of rotated column c.
template <int kSK, class W>
__device__ void wave_jacobi_lds(double* M, double* Z, double* nrm, int rows, int cols, double conv) {
    constexpr int kLpc = 64 / kSK, kNr = kSK / kLpc;
    const int lane = threadIdx.x & 63;
    const int c = lane / kLpc, sub = lane % kLpc;
    W m[kNr], z[kNr];
#pragma unroll
    for (int u = 0; u < kNr; ++u) {
        const int row = sub + u * kLpc;
        m[u] = (c < cols && row < rows) ? (W)M[row + c * kSK] : W(0);
        z[u] = (c < cols && row == c) ? W(1) : W(0);
    }
    const W conv2 = (W)(conv * conv);
    const int n2 = cols + (cols & 1), nm1 = n2 - 1;
    // round-robin: in round r column c < n2 - 1 meets (2 r - c) mod (n2 - 1), or n2 - 1 when that
    // is c itself; column n2 - 1 meets r. pr tracks (2 r - c) mod (n2 - 1) from round to round.
    const int pr0 = c < nm1 ? (nm1 - c) % nm1 : 0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        bool rotated = false;
        int pr = pr0;
        for (int round = 0; round < nm1; ++round) {
            const int partner = c >= n2 ? c : (c == nm1 ? round : (c == round ? nm1 : pr));
            pr += 2;
            if (pr >= nm1) pr -= nm1;
            if (pr >= nm1) pr -= nm1;
            const bool valid = c < cols && partner < cols && partner != c;
            const int src = (valid ? partner : c) * kLpc + sub;
            W pm[kNr], pz[kNr];
#pragma unroll
            for (int u = 0; u < kNr; ++u) {
                pm[u] = __shfl(m[u], src, 64);
                pz[u] = __shfl(z[u], src, 64);
            }
            W a = 0, b = 0, g = 0;
#pragma unroll
            for (int u = 0; u < kNr; ++u) {
                a += m[u] * m[u];
                b += pm[u] * pm[u];
                g += m[u] * pm[u];
            }
            a = column_sum<kLpc>(a);
            b = column_sum<kLpc>(b);
            g = column_sum<kLpc>(g);
            const bool lower = c < partner;
            const W ap = lower ? a : b, aq = lower ? b : a;
            if (valid && g * g > conv2 * (ap * aq)) {
                W cs, sn;
                jacobi_rotation(ap, aq, g, cs, sn);
                if (sn != W(0)) {
#pragma unroll
                    for (int u = 0; u < kNr; ++u) {
                        m[u] = lower ? cs * m[u] - sn * pm[u] : sn * pm[u] + cs * m[u];
                        z[u] = lower ? cs * z[u] - sn * pz[u] : sn * pz[u] + cs * z[u];
                    }
                    rotated = true;
                }
            }
        }
        if (!__any(rotated)) break;
    }
    double nn = 0.0;
#pragma unroll
    for (int u = 0; u < kNr; ++u) {
        const int row = sub + u * kLpc;
        if (c < cols && row < rows) M[row + c * kSK] = (double)m[u];
        if (c < cols && row < cols) Z[row + c * kSK] = (double)z[u];
        nn += (double)m[u] * (double)m[u];
    }
    nn = column_sum<kLpc>(nn);
    if (c < cols && sub == 0) nrm[c] = sqrt(nn);
}

// value of lane n (0..15, unrolled loop index) of the calling lane's 16-lane row
__device__ __attribute__((always_inline)) inline double row_bcast16(double v, int n) {
    switch (n) {
#define FDE_ROWB(k) \
    case k: return dpp_move<dpp_row_newbcast(k)>(v);
        FDE_ROWB(0) FDE_ROWB(1) FDE_ROWB(2) FDE_ROWB(3) FDE_ROWB(4) FDE_ROWB(5) FDE_ROWB(6) FDE_ROWB(7)
        FDE_ROWB(8) FDE_ROWB(9) FDE_ROWB(10) FDE_ROWB(11) FDE_ROWB(12) FDE_ROWB(13) FDE_ROWB(14) FDE_ROWB(15)
#undef FDE_ROWB
        default: return v;
    }
}

// rows [c0, c0 + CH) of U_C = A_u C_u and V_C = A_v C_v from the staged rows (A) and C_u, C_v (G);
// zeros staged beyond k' and zero rows of C beyond k' make the sums run over all K columns
template <class T, class LS>
__device__ __attribute__((noinline)) void products_chunk(lds_ptr<LS> Sp, int c0, int r, int m, int n, T* U, T* V) {
    auto& S = *Sp;
    constexpr int kSK = LS::K, kCH = LS::CH, kLD = LS::LD;
    for (int idx = threadIdx.x; idx < 2 * kCH * r; idx += kT) {
        const int s = idx / (kCH * r), rem = idx % (kCH * r), rr = rem % kCH, c = rem / kCH, i = c0 + rr;
        if (i >= (s == 0 ? m : n)) continue;
        double v = 0.0;
#pragma unroll 4
        for (int l = 0; l < kSK; ++l) v += S.A[s][rr * kLD + l] * S.G[s][l * kSK + c];
        T* out = s == 0 ? U : V;
        out[i + (int64_t)c * (s == 0 ? m : n)] = (T)v;
    }
}

// C_u = P_u R11_u^{-1} (M Z)_order and C_v = P_v R11_v^{-1} Z_order of the small recompression
// with k' <= 16, by back substitution in the pivot order, into G[side] (row l, column c); called by
// every thread of the workgroup (it holds barriers)
template <class LS>
__device__ __attribute__((noinline)) void solve_factors16(lds_ptr<LS> Sp, lds_ptr<const int> order, int r) {
    auto& S = *Sp;   // LDS-qualified: its accesses are LDS instructions
    constexpr int kSK = LS::K;
    static_assert(kSK == 16, "rows of R11 held in registers, one per lane of a 16-lane column group");
    const int wave = threadIdx.x >> 6;
    // waves 2 s and 2 s + 1 solve side s, four columns at a time: lane l holds row a = l % 16 of
    // R11 (pivot order) and of column c = 4 (wave % 2) + l / 16 (+ 8 per round); the solved
    // entry of row b is broadcast to its column's 16 lanes (one DPP row) with row_newbcast. Rows
    // and steps beyond q carry zeros, so all 16 steps run without branches.
    const int lane = threadIdx.x & 63, sd = wave >> 1, cl = lane >> 4, a = lane & 15;
    const int q = S.q[sd];
    const bool row = a < q;
    double rr[16];
#pragma unroll
    for (int bb = 0; bb < 16; ++bb) rr[bb] = (row && bb < q) ? S.R[sd][a * kSK + S.perm[sd][bb]] : 0.0;
    const double dinv = row ? 1.0 / S.R[sd][a * kSK + S.perm[sd][a]] : 0.0;
    const int pa = row ? S.perm[sd][a] : 0;
    constexpr int kRounds = (16 + 7) / 8;   // r <= kSK columns, 8 per round
    double y[kRounds];
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
        const int c = 8 * u + 4 * (wave & 1) + cl;
        y[u] = (row && c < r) ? S.G[sd][order[c] * kSK + a] : 0.0;
    }
    __syncthreads();   // M and Z read: G becomes C
    for (int idx = threadIdx.x; idx < 2 * kSK * kSK; idx += kT) S.G[idx / (kSK * kSK)][idx % (kSK * kSK)] = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
        if (8 * u < r) {
            double v = y[u];
#pragma unroll
            for (int bb = 15; bb >= 0; --bb) {
                if (a == bb) v *= dinv;
                const double yb = row_bcast16(v, bb);
                if (a < bb) v -= rr[bb] * yb;
            }
            const int c = 8 * u + 4 * (wave & 1) + cl;
            if (row && c < r) S.G[sd][pa * kSK + c] = v;
        }
    }
    __syncthreads();
}

// row <- y with y R[:, perm[:q]] = row[perm[:q]] (forward substitution over the pivot order; R row b
// in original column j at R[b * kSK + j]); entries beyond q become zero. One thread per staged row.
template <int kSK>
__device__ inline void subst_row(double* row, const double* R, const int* perm, int q) {
    double y[kSK];
#pragma unroll
    for (int b = 0; b < kSK; ++b) y[b] = 0.0;
    for (int b = 0; b < q; ++b) {
        const int pb = perm[b];
        double v = row[pb];
#pragma unroll
        for (int c = 0; c < kSK; ++c)
            if (c < b) v -= y[c] * R[c * kSK + pb];
        v /= R[b * kSK + pb];
#pragma unroll
        for (int c = 0; c < kSK; ++c)
            if (c == b) y[c] = v;
    }
#pragma unroll
    for (int b = 0; b < kSK; ++b) row[b] = b < q ? y[b] : 0.0;
}

template <class T, class SH>
__device__ __attribute__((noinline)) void op_lrsub_small(const Inst<T>& d, const OpRec& o, SH& sh, const LRBlockDev& L, int kc, int kx) {
    auto& S = sh.ls;
    constexpr int kSK = SH::kSmall;
    using LS = typename std::remove_reference<decltype(S)>::type;
    constexpr int kCH = LS::CH, kLD = LS::LD, kEl = RowChunk<LS>::kEl;
    T* U = d.arena + L.uoff;
    T* V = d.arena + L.voff;
    const int m = L.m, n = L.n, kp = kc + kx;
    const int wave = threadIdx.x >> 6;
    const bool f64 = sizeof(T) == 8;
    const T* Xp = vptr(d, o.v[0]);
    const T* Yp = vptr(d, o.v[1]);
    const Side<T> su{U, m, kc, Xp, o.v[0].rs, o.v[0].cs, -1.0, m};
    const Side<T> sv{V, n, kc, Yp, o.v[1].rs, o.v[1].cs, 1.0, n};
    const int rmax = max(m, n);
    unsigned long long* const prof = d.prof;   // read once: later stores may alias the instance
    const double tol = d.tol;
    const int kmax = d.kmax;
    unsigned long long tph = (prof && threadIdx.x == 0) ? wall_clock64() : 0ull;
    auto phase = [&](int k) {   // op profile: time of each phase (thread 0)
        if (prof && threadIdx.x == 0) {
            const unsigned long long t = wall_clock64();
            atomicAdd(&prof[2 * kOpCodes + k], t - tph);
            tph = t;
        }
    };
    T rows[kEl];   // the chunk in flight
    // Gram matrices
    GramTiles<LS> gt;
    gram_tiles_clear(gt);
    load_rows<T, LS>(su, sv, 0, kp, rows);
    for (int c0 = 0; c0 < rmax; c0 += kCH) {
        store_rows<T, LS>(su, sv, c0, kp, rows, S);
        __syncthreads();
        if (c0 + kCH < rmax) load_rows<T, LS>(su, sv, c0 + kCH, kp, rows);
        gram_tiles_accumulate(S, gt);
        __syncthreads();
    }
    gram_tiles_store(S, gt);
    __syncthreads();
    phase(0);
    if constexpr (sizeof(T) == 4) {
        // one pass: pivoted Cholesky of the Gram matrices, pivots below 1e-12 of the largest dropped
        if (wave < 2)
            wave_cholesky<kSK>(lmem<const double>(S.G[wave]), lmem(S.R[wave]), lmem(S.perm[wave]), lmem(&S.q[wave]), kp,
                               true, 1e-12);
        __syncthreads();
        phase(1);
    } else {
        // Shifted Cholesky QR3, so that directions far below the largest column survive (exact up to
        // rounding for any conditioning; tol = 0 gives the exact LU). Pass 1: G1 + s I = R1^T R1
        // without pivoting, s = 11 (rows k' + k'(k'+1)) eps tr(G1): Q1 = A R1^{-1} has condition
        // at most about 1/sqrt(s). Pass 2: pivoted Cholesky QR of Q1 (dependent columns dropped at
        // 1e-15), Q1 P2 = Q2 R2. Pass 3: Cholesky QR of Q2, Q2 = Q3 R3. Then A = Q3 R with
        // R = R3 (R2 P2^T) R1.
        if (wave < 2) {
            const int lane = threadIdx.x & 63;
            const double dg = lane < kp ? S.G[wave][lane * kSK + lane] : 0.0;
            const double tr = wave_sum(dg);
            const double rows_s = wave == 0 ? (double)m : (double)n;
            const double shift = 11.0 * (rows_s * kp + kp * (kp + 1.0)) * 2.220446049250313e-16 * tr;
            if (lane < kp) S.G[wave][lane * kSK + lane] = dg + shift;
        }
        __syncthreads();
        if (wave < 2)
            wave_cholesky<kSK>(lmem<const double>(S.G[wave]), lmem(S.R[wave]), lmem(S.perm[wave]), lmem(&S.q[wave]), kp,
                               false, 0.0);
        __syncthreads();
        phase(1);
        for (int pass = 2; pass <= 3; ++pass) {
            // rows of Q1 = A R1^{-1} (pass 2), of Q2 = (Q1 P2)[:, :q2] R2_11^{-1} (pass 3), and their Gram
            GramTiles<LS> g2;
            gram_tiles_clear(g2);
            load_rows<T, LS>(su, sv, 0, kp, rows);
            for (int c0 = 0; c0 < rmax; c0 += kCH) {
                store_rows<T, LS>(su, sv, c0, kp, rows, S);
                __syncthreads();
                if (c0 + kCH < rmax) load_rows<T, LS>(su, sv, c0 + kCH, kp, rows);
                for (int idx = threadIdx.x; idx < 2 * kCH; idx += kT) {
                    const int sd = idx / kCH, rr = idx % kCH;
                    double* row = &S.A[sd][rr * kLD];
                    subst_row<kSK>(row, S.R[sd], S.perm[sd], S.q[sd]);
                    if (pass == 3) subst_row<kSK>(row, S.R2[sd], S.perm2[sd], S.q2[sd]);
                }
                __syncthreads();
                gram_tiles_accumulate(S, g2);
                __syncthreads();
            }
            gram_tiles_store(S, g2);
            __syncthreads();
            if (wave < 2) {
                if (pass == 2)
                    wave_cholesky<kSK>(lmem<const double>(S.G[wave]), lmem(S.R2[wave]), lmem(S.perm2[wave]),
                                       lmem(&S.q2[wave]), S.q[wave], true, 1e-15);
                else   // R3 (row a, column b) into A[wave]: the staged rows are no longer needed
                    wave_cholesky<kSK>(lmem<const double>(S.G[wave]), lmem(S.A[wave]), lmem(S.perm[wave] + 0),
                                       lmem(&S.q3[wave]), S.q2[wave], false, 1e-30);
            }
            __syncthreads();
            if (pass == 2) continue;
            // R1's pivot order is the natural one (no pivoting), so perm may be overwritten above.
            // T = (R2 P2^T) R1 (q2 x k') into G, then R = R3 T (q3 x k') into R
            for (int idx = threadIdx.x; idx < 2 * kSK * kp; idx += kT) {
                const int sd = idx / (kSK * kp), rem = idx % (kSK * kp), a = rem / kp, j = rem % kp;
                double v = 0.0;
                if (a < S.q2[sd])
                    for (int b = 0; b < S.q[sd]; ++b) v += S.R2[sd][a * kSK + b] * S.R[sd][b * kSK + j];
                S.G[sd][a * kSK + j] = v;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < 2 * kSK * kp; idx += kT) {
                const int sd = idx / (kSK * kp), rem = idx % (kSK * kp), a = rem / kp, j = rem % kp;
                double v = 0.0;
                if (a < S.q3[sd])
                    for (int c = a; c < S.q2[sd]; ++c) v += S.A[sd][a * kSK + c] * S.G[sd][c * kSK + j];
                S.R[sd][a * kSK + j] = v;
            }
            if (threadIdx.x < 2) S.q[threadIdx.x] = S.q3[threadIdx.x];
            __syncthreads();
        }
    }
    phase(2);
    const int qu = S.q[0], qv = S.q[1];
    // core M = (R_u P_u^T)(R_v P_v^T)^T (qu x qv, column-major ld kSK) in G[0]; Z in G[1]
    for (int idx = threadIdx.x; idx < qu * qv; idx += kT) {
        const int a = idx % qu, b = idx / qu;
        double v = 0.0;
        for (int j = 0; j < kp; ++j) v += S.R[0][a * kSK + j] * S.R[1][b * kSK + j];
        S.G[0][a + b * kSK] = v;
    }
    __syncthreads();
    // the SVD of the small core runs in the factor precision (the Gram matrices and their
    // Cholesky factors stay FP64)
    if (wave == 0 && qu > 0 && qv > 0) wave_jacobi_lds<kSK, T>(S.G[0], S.G[1], S.sig, qu, qv, f64 ? 1e-15 : 1e-6);
    __syncthreads();
    phase(3);
    for (int j = threadIdx.x; j < qv; j += kT) {
        int rank = 0;
        const double sj = S.sig[j];
        for (int i = 0; i < qv; ++i) rank += (S.sig[i] > sj || (S.sig[i] == sj && i < j)) ? 1 : 0;
        sh.order[rank] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        if (qu > 0 && qv > 0) {
            const double smax = S.sig[sh.order[0]];
            // singular values below 1e-30 sigma_1 are rounding noise and dropped even at tol = 0 (the
            // FP64 factors divide by sigma_r^2)
            if (smax > 0.0)
                while (r < qv && S.sig[sh.order[r]] > tol * smax && S.sig[sh.order[r]] > 1e-30 * smax) ++r;
        }
        if (r > kmax) r = kmax;
        sh.r = r;
        const double K = kp;
        sh.lrsub_flops = (m + n) * K * (K + 1.0) * (f64 ? 5.0 : 1.0) + 2.0 * (m + n) * K * r +
                         2.0 * K * K * K * (f64 ? 3.0 : 1.0) / 3.0 + 2.0 * K * K * K;
    }
    __syncthreads();
    const int r = sh.r;
    if constexpr (sizeof(T) == 8) {
        // C_u = R_v^T Z_r and C_v = R_u^T (M Z)_r S_r^{-2}: then A_u C_u = Q_u M Z_r = Q_u W_r S_r and
        // A_v C_v = Q_v M^T W_r S_r^{-1} = Q_v Z_r, with no inverse of R (row l, column c; into A, then G)
        for (int idx = threadIdx.x; idx < 2 * kSK * kSK; idx += kT) S.A[idx / (kSK * kSK)][idx % (kSK * kSK)] = 0.0;
        __syncthreads();
        for (int idx = threadIdx.x; idx < 2 * kp * r; idx += kT) {
            const int sd = idx / (kp * r), rem = idx % (kp * r), l = rem % kp, c = rem / kp, oc = sh.order[c];
            double v = 0.0;
            if (sd == 0) {
                for (int b = 0; b < qv; ++b) v += S.R[1][b * kSK + l] * S.G[1][b + oc * kSK];
            } else {
                for (int a = 0; a < qu; ++a) v += S.R[0][a * kSK + l] * S.G[0][a + oc * kSK];
                const double sg = S.sig[oc];
                v /= sg * sg;
            }
            S.A[sd][l * kSK + c] = v;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < 2 * kSK * kSK; idx += kT) {
            const int sd = idx / (kSK * kSK), e = idx % (kSK * kSK);
            S.G[sd][e] = S.A[sd][e];
        }
        __syncthreads();
    } else if constexpr (kSK == 16) {
        // C_u (kp x r) = P_u R11_u^{-1} (M Z)_order and C_v = P_v R11_v^{-1} Z_order, by back
        // substitution in the pivot order, into G[side] (row l, column c; M and Z are read first)
        solve_factors16(lmem(&S), lmem<const int>(sh.order), r);
    } else {
        // one lane per (side, output column), into A[side], then moved to G
        for (int idx = threadIdx.x; idx < 2 * kSK * kSK; idx += kT) S.A[idx / (kSK * kSK)][idx % (kSK * kSK)] = 0.0;
        __syncthreads();
        if (threadIdx.x < 2 * r) {
            const int sd = threadIdx.x / r, c = threadIdx.x % r, jc = sh.order[c];
            const int q = S.q[sd];
            const double* rhs = &S.G[sd][jc * kSK];   // column jc (length q)
            double* C = S.A[sd];
            for (int a = q - 1; a >= 0; --a) {
                const int pa = S.perm[sd][a];
                double v = rhs[a];
                for (int bb = a + 1; bb < q; ++bb) v -= S.R[sd][a * kSK + S.perm[sd][bb]] * C[S.perm[sd][bb] * kSK + c];
                C[pa * kSK + c] = v / S.R[sd][a * kSK + pa];
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < 2 * kSK * kSK; idx += kT) {
            const int sd = idx / (kSK * kSK), e = idx % (kSK * kSK);
            S.G[sd][e] = S.A[sd][e];
        }
        __syncthreads();
    }
    phase(4);
    // U_C <- A_u C_u, V_C <- A_v C_v, chunk by chunk (a chunk is staged before its rows are written).
    // With the small path's LDS-only factors and a single chunk, the rows staged for the Gram
    // matrices are still in place (FP64 factors overwrite them in the second pass).
    const bool staged = kSK == 16 && !f64 && rmax <= kCH;
    if (staged) {
        products_chunk<T>(lmem(&S), 0, r, m, n, U, V);
    } else {
        load_rows<T, LS>(su, sv, 0, kp, rows);
        for (int c0 = 0; c0 < rmax; c0 += kCH) {
            store_rows<T, LS>(su, sv, c0, kp, rows, S);
            __syncthreads();
            if (c0 + kCH < rmax) load_rows<T, LS>(su, sv, c0 + kCH, kp, rows);
            products_chunk<T>(lmem(&S), c0, r, m, n, U, V);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) d.ranks[L.slot] = r;
    phase(5);
}

template <class T, class SH>
__device__ __attribute__((noinline)) void op_lrsub(const Inst<T>& d, const OpRec& o, SH& sh) {
    const int kx = dimval(d, o.dim[2]);
    if (threadIdx.x == 0) sh.lrsub_flops = 0.0;
    if (kx <= 0) return;
    const LRBlockDev L = o.lb;
    const int kc0 = L.rank >= 0 ? L.rank : d.ranks[L.slot];
    if (kc0 + kx <= SH::kSmall) {
        op_lrsub_small(d, o, sh, L, kc0, kx);
        return;
    }
    if constexpr (!SH::kGeneral) {
        // the host picks this variant only for programs whose widths fit the small path
        if (threadIdx.x == 0) {
            d.status[0] = FDE_EDEVICE;
            d.status[1] = -1;
        }
        return;
    } else {
    T* U = d.arena + L.uoff;
    T* V = d.arena + L.voff;
    const int m = L.m, n = L.n, kc = kc0, kp = kc + kx;
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

// op pc (record o); false when a leaf pivot broke down (the status is set). d and o are
// referenced where they live (global memory, or the level kernel's LDS copies): the op functions
// are separate (not inlined) functions, and a local copy handed to them by reference would be
// written to every lane's scratch memory for each op
template <class T, class SH>
__device__ bool run_op(const Inst<T>& d, const OpRec& o, int pc, SH& sh, int step) {
    unsigned long long t0 = 0;
    if (d.prof && threadIdx.x == 0) t0 = wall_clock64();
    double fl = 0.0;
    if (threadIdx.x == 0) fl = op_flops(d, o);
    bool ok = true;
    switch (o.code) {
        case OP_GEMM: op_gemm(d, o, sh); break;
        case OP_ZERO: op_zero(d, o); break;
        case OP_TRSM: op_trsm(d, o, sh); break;
        case OP_LRSUB: op_lrsub(d, o, sh); break;
        case OP_GETRF: ok = op_getrf(d, o, sh, pc); break;
        case OP_LRMV: {
            // t = V^T X, then Y += alpha U t
            const LRBlockDev L = o.lb;
            const int rc = -2 - L.slot;
            OpRec g1{};
            g1.code = OP_GEMM;
            g1.v[0] = o.v[2];
            g1.v[1] = View{B_ARENA, L.n, 1, L.voff};
            g1.v[2] = o.v[1];
            g1.dim[0] = rc;
            g1.dim[1] = o.dim[1];
            g1.dim[2] = L.n;
            g1.alpha = 1.f;
            g1.beta = 0.f;
            op_gemm(d, g1, sh);
            __syncthreads();
            OpRec g2 = g1;
            g2.v[0] = o.v[0];
            g2.v[1] = View{B_ARENA, 1, L.m, L.uoff};
            g2.v[2] = o.v[2];
            g2.dim[0] = L.m;
            g2.dim[2] = rc;
            g2.alpha = o.alpha;
            g2.beta = 1.f;
            op_gemm(d, g2, sh);
            if (threadIdx.x == 0) fl = op_flops(d, g1) + op_flops(d, g2);
            break;
        }
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
        // a factorisation runs every op once: its own slot, no counter shared by the whole level
        if (d.op_flops) d.op_flops[pc] = fl;
        else atomicAdd(d.flops, fl);
    }
    if (d.prof && threadIdx.x == 0) {
        atomicAdd(&d.prof[2 * o.code], (unsigned long long)(wall_clock64() - t0));
        atomicAdd(&d.prof[2 * o.code + 1], 1ull);
    }
    return true;
}

template <class T, class SH>
__device__ void run_program(const Inst<T>& d, SH& sh, int step) {
    for (int pc = 0; pc < d.nops; ++pc)
        if (!run_op(d, d.ops[pc], pc, sh, step)) return;
}

template <class T, int KS, bool GENERAL>
__global__ void __launch_bounds__(kT) k_interp(const Inst<T>* __restrict__ insts, int step) {
    __shared__ Shared<T, KS, GENERAL> sh;
    const Inst<T>& d = insts[blockIdx.x];
    run_program(d, sh, step);
}

template <class T>
__global__ void __launch_bounds__(kT) k_interp_one(const Inst<T> d) {
    __shared__ Shared<T, 32, true> sh;
    run_program(d, sh, 0);
}

// one level: the ops of a level are independent, earlier levels have completed (kernel order)
// thread t < 4 of a workgroup whose op and instance sit in LDS: dimension t (< 3) of the op, or
// (t == 3) the rank of its low-rank block, resolved from the rank slots
template <class SH>
__device__ inline void resolve_dims(SH& sh, int t) {
    const bool lrb = sh.op.code == OP_LRSUB || sh.op.code == OP_LRMV;
    const int code = t < 3 ? sh.op.dim[t] : (lrb ? -2 - sh.op.lb.slot : 0);
    const int v = code >= 0 ? code : (code == -1 ? sh.inst.nrhs : gmem(sh.inst.ranks)[-2 - code]);
    if (t < 3)
        sh.op.dim[t] = v;
    else if (lrb)
        sh.op.lb.rank = v;
}

template <class T, int KS, bool GENERAL>
__global__ void __launch_bounds__(kT) k_level(const Inst<T>* __restrict__ insts, const LevelTask* __restrict__ tasks) {
    __shared__ Shared<T, KS, GENERAL> sh;
    const LevelTask tk = tasks[blockIdx.x];
    // one round of loads, in parallel: the op record and the instance (one word per thread)
    constexpr int kOpW = sizeof(OpRec) / 4, kInstW = sizeof(Inst<T>) / 4;
    static_assert(sizeof(OpRec) % 4 == 0 && sizeof(Inst<T>) % 4 == 0 && kOpW + kInstW < kT, "op and instance copies");
    const int t = threadIdx.x;
    if (t < kOpW)
        reinterpret_cast<int*>(&sh.op)[t] = gmem(reinterpret_cast<const int*>(tk.op))[t];
    else if (t < kOpW + kInstW)
        reinterpret_cast<int*>(&sh.inst)[t - kOpW] = gmem(reinterpret_cast<const int*>(insts + tk.inst))[t - kOpW];
    __syncthreads();
    // after a breakdown in an earlier level the rest of that factorisation is skipped (the status
    // is shared so that every thread takes the same branch); sizes given by ranks, and the rank of
    // the op's low-rank block, are read once (ranks change only between levels: the ops of a level
    // are independent)
    if (t == 4) sh.stop = gmem(sh.inst.status)[0];
    if (t < 4) resolve_dims(sh, t);
    __syncthreads();
    if (sh.stop != 0) return;
    run_op(sh.inst, sh.op, tk.pc, sh, 0);
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
    static const char* names[kOpCodes] = {"-", "GETRF", "TRSM", "GEMM", "LRSUB", "ZERO", "LOAD", "STORE", "LRMV"};
    fprintf(stderr, "[fde ops] %s:", what);
    for (int c = 1; c < kOpCodes; ++c)
        if (p[2 * c + 1]) fprintf(stderr, " %s %llu x %.3f ms = %.2f ms;", names[c], p[2 * c + 1],
                                  p[2 * c] * ms_per_tick / p[2 * c + 1], p[2 * c] * ms_per_tick);
    static const char* phases[kProfPhases] = {"gram", "cholesky", "second pass", "core svd", "factors", "products",
                                              "phase 1", "phase 2 after the solve", "phase 2 solve",
                                              "phase 2 helpers"};
    const unsigned long long nl = p[2 * OP_LRSUB + 1];
    if (nl && p[2 * kOpCodes + 1]) {
        fprintf(stderr, "\n[fde ops]   small recompression phases (ms per op):");
        for (int k = 0; k < 6; ++k) fprintf(stderr, " %s %.4f;", phases[k], p[2 * kOpCodes + k] * ms_per_tick / nl);
    }
    const unsigned long long ns = p[2 * OP_TRSM + 1];
    if (p[2 * kOpCodes + 6] && ns) {
        fprintf(stderr, "\n[fde ops]   leaf-step H-solve phases (ms per step):");
        for (int k = 6; k < 10; ++k) fprintf(stderr, " %s %.4f;", phases[k], p[2 * kOpCodes + k] * ms_per_tick / ns);
    }
    fprintf(stderr, "\n");
}

template <class T>
void launch_interp(hipStream_t st, int ninst, const Inst<T>* d_insts, int step, int variant) {
    if (ninst <= 0) return;
    if (variant == 16)
        hipLaunchKernelGGL((k_interp<T, 16, false>), dim3(ninst), dim3(kT), 0, st, d_insts, step);
    else if (variant == 32)
        hipLaunchKernelGGL((k_interp<T, 32, false>), dim3(ninst), dim3(kT), 0, st, d_insts, step);
    else
        hipLaunchKernelGGL((k_interp<T, 32, true>), dim3(ninst), dim3(kT), 0, st, d_insts, step);
    FDE_LAUNCH_CHECK();
}
template void launch_interp<float>(hipStream_t, int, const Inst<float>*, int, int);
template void launch_interp<double>(hipStream_t, int, const Inst<double>*, int, int);

template <class T>
void launch_interp_one(hipStream_t st, const Inst<T>& d) {
    hipLaunchKernelGGL((k_interp_one<T>), dim3(1), dim3(kT), 0, st, d);
    FDE_LAUNCH_CHECK();
}
template void launch_interp_one<float>(hipStream_t, const Inst<float>&);
template void launch_interp_one<double>(hipStream_t, const Inst<double>&);

template <class T>
void launch_level(hipStream_t st, int ntasks, const Inst<T>* d_insts, const LevelTask* d_tasks, int variant) {
    if (ntasks <= 0) return;
    if (variant == 16)
        hipLaunchKernelGGL((k_level<T, 16, false>), dim3(ntasks), dim3(kT), 0, st, d_insts, d_tasks);
    else if (variant == 32)
        hipLaunchKernelGGL((k_level<T, 32, false>), dim3(ntasks), dim3(kT), 0, st, d_insts, d_tasks);
    else
        hipLaunchKernelGGL((k_level<T, 32, true>), dim3(ntasks), dim3(kT), 0, st, d_insts, d_tasks);
    FDE_LAUNCH_CHECK();
}
template void launch_level<float>(hipStream_t, int, const Inst<float>*, const LevelTask*, int);
template void launch_level<double>(hipStream_t, int, const Inst<double>*, const LevelTask*, int);

}  // namespace fde
