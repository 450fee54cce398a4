// Forward and backward H-substitution (Section 4.1) with the right-hand sides
// resident in LDS.
//
// The H-solve program is a chain of small ops -- triangular solves with the
// dense diagonal leaves and products with dense or low-rank off-diagonal
// blocks -- most of which depend on the previous one through the solution
// vector. One workgroup runs the whole chain for a chunk of right-hand-side
// columns: the chunk (Nd x wc), the temporaries and the current ranks sit in
// LDS for the whole solve, so every op reads only its factor block from HBM
// (coalesced along the stored dimension) and the vector entries from LDS. The
// next op record is fetched while the current op runs.
#include "hinterp.h"
#include "tri_wave.h"

namespace fde {

namespace {

constexpr int kHT = 512;
constexpr int kHW = kHT / 64;

template <class T>
struct Lds {
    T* X;      // Nd x wc, ld Nd
    T* W;      // temporaries: offset off * wc, ld rows
    T* red;    // kHT * wc partial sums
    int* rk;   // ranks
    int wc;
};

template <class T>
__device__ inline T* lptr(const Lds<T>& L, const View& v) {
    return v.base == B_RHS ? L.X + v.off : L.W + v.off * L.wc;
}

template <class T>
__device__ inline int hdim(const Lds<T>& L, int code) {
    return code >= 0 ? code : (code == -1 ? L.wc : L.rk[-2 - code]);
}

template <class T>
__device__ inline T group_sum(T v, int G) {
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// C (LDS) = beta C + alpha A (HBM factor) B (LDS)
template <class T>
__device__ void hs_gemm(const Inst<T>& d, const Lds<T>& L, const OpRec& o) {
    const int m = hdim(L, o.dim[0]), n = hdim(L, o.dim[1]), k = hdim(L, o.dim[2]);
    if (m <= 0 || n <= 0) return;
    T* C = lptr(L, o.v[0]);
    const T* B = lptr(L, o.v[2]);
    const T* A = d.arena + o.v[1].off;
    const int ars = o.v[1].rs, acs = o.v[1].cs, brs = o.v[2].rs, bcs = o.v[2].cs;
    const int crs = o.v[0].rs, ccs = o.v[0].cs;
    const T alpha = (T)o.alpha, beta = (T)o.beta;
    const int t = threadIdx.x;
    auto put = [&](int i, int j, T s) {
        T* c = C + (int64_t)i * crs + (int64_t)j * ccs;
        *c = (beta == T(0) ? T(0) : beta * *c) + alpha * s;
    };
    if (k <= 0) {
        for (int idx = t; idx < m * n; idx += kHT) put(idx % m, idx / m, T(0));
        return;
    }
    if (acs == 1 && ars != 1) {
        // A stored transposed (a factor read as V^T or U^T): G lanes per output, consecutive lanes
        // along the contiguous dimension k, reduced by shuffles
        int G = 64;
        while (G > 1 && G * m * n > kHT) G >>= 1;
        const int ng = kHT / G, gid = t / G, gl = t % G;
        for (int idx = gid; idx < m * n; idx += ng) {
            const int i = idx % m, j = idx / m;
            const T* a = A + (int64_t)i * ars;
            const T* b = B + (int64_t)j * bcs;
            T s = 0;
            for (int l = gl; l < k; l += G) s += a[l] * b[(int64_t)l * brs];
            s = group_sum(s, G);
            if (gl == 0) put(i, j, s);
        }
        return;
    }
    if (2 * m >= kHT || k <= 8) {
        // one thread per row, all columns of the chunk
        for (int i = t; i < m; i += kHT) {
            T s[kHsolveMaxCols];
#pragma unroll
            for (int j = 0; j < kHsolveMaxCols; ++j) s[j] = 0;
#pragma unroll 8
            for (int l = 0; l < k; ++l) {
                const T a = A[(int64_t)i * ars + (int64_t)l * acs];
#pragma unroll
                for (int j = 0; j < kHsolveMaxCols; ++j)
                    if (j < n) s[j] += a * B[(int64_t)l * brs + (int64_t)j * bcs];
            }
#pragma unroll
            for (int j = 0; j < kHsolveMaxCols; ++j)
                if (j < n) put(i, j, s[j]);
        }
        return;
    }
    // few rows, longer k: S slices of k per row, partial sums through LDS
    int S = 1;
    while (2 * S * m <= kHT && 2 * S <= k) S <<= 1;
    const int i = t % m, sl = t / m;
    if (sl < S) {
        T s[kHsolveMaxCols];
#pragma unroll
        for (int j = 0; j < kHsolveMaxCols; ++j) s[j] = 0;
#pragma unroll 8
        for (int l = sl; l < k; l += S) {
            const T a = A[(int64_t)i * ars + (int64_t)l * acs];
#pragma unroll
            for (int j = 0; j < kHsolveMaxCols; ++j)
                if (j < n) s[j] += a * B[(int64_t)l * brs + (int64_t)j * bcs];
        }
#pragma unroll
        for (int j = 0; j < kHsolveMaxCols; ++j)
            if (j < n) L.red[(sl * m + i) * n + j] = s[j];
    }
    __syncthreads();
    for (int idx = t; idx < m * n; idx += kHT) {
        const int ii = idx % m, j = idx / m;
        T s = 0;
        for (int q = 0; q < S; ++q) s += L.red[(q * m + ii) * n + j];
        put(ii, j, s);
    }
}

// X (LDS, n x w) <- T^{-1} X with T a dense factor leaf (HBM)
template <class T>
__device__ void hs_trsm(const Inst<T>& d, const Lds<T>& L, const OpRec& o) {
    const int n = hdim(L, o.dim[0]), w = hdim(L, o.dim[1]);
    if (n <= 0 || w <= 0) return;
    T* X = lptr(L, o.v[0]);
    const T* Tm = d.arena + o.v[1].off;
    const int xrs = o.v[0].rs, xcs = o.v[0].cs, trs = o.v[1].rs, tcs = o.v[1].cs;
    const bool lower = o.flags & 1, unit = o.flags & 2;
    if (n <= 64) {
        tri_wave(Tm, trs, tcs, n, lower, unit, X, xrs, xcs, w, (int)(threadIdx.x >> 6), kHW);
        return;
    }
    // larger leaves: column-oriented substitution, one barrier per step
    for (int st = 0; st < n; ++st) {
        const int i = lower ? st : n - 1 - st;
        if (!unit) {
            if ((int)threadIdx.x < w) X[(int64_t)i * xrs + (int64_t)threadIdx.x * xcs] /= Tm[(int64_t)i * trs + (int64_t)i * tcs];
            __syncthreads();
        }
        const int lo = lower ? i + 1 : 0, cnt = lower ? n - i - 1 : i;
        for (int idx = threadIdx.x; idx < cnt * w; idx += kHT) {
            const int l = lo + idx % cnt, j = idx / cnt;
            X[(int64_t)l * xrs + (int64_t)j * xcs] -= Tm[(int64_t)l * trs + (int64_t)i * tcs] * X[(int64_t)i * xrs + (int64_t)j * xcs];
        }
        __syncthreads();
    }
}

// Y (LDS, m x w) += alpha U (V^T X) for a low-rank factor block: t = V^T X into the temporary,
// then Y += alpha U t. The rows of U a thread will need are loaded before the first phase, so
// their latency overlaps the V^T X reduction.
constexpr int kLrmvPre = 16;
template <class T>
__device__ void hs_lrmv(const Inst<T>& d, const Lds<T>& L, const OpRec& o) {
    const LRBlockDev B = d.lr[o.blk];
    const int m = B.m, n = B.n, r = L.rk[B.slot], w = hdim(L, o.dim[1]);
    if (r <= 0 || w <= 0) return;
    T* Y = lptr(L, o.v[0]);
    const T* X = lptr(L, o.v[1]);
    T* t = lptr(L, o.v[2]);
    const int yrs = o.v[0].rs, ycs = o.v[0].cs, xrs = o.v[1].rs, xcs = o.v[1].cs, trs = o.v[2].rs, tcs = o.v[2].cs;
    const T* U = d.arena + B.uoff;
    const T* V = d.arena + B.voff;
    const T alpha = (T)o.alpha;
    const int tid = threadIdx.x;
    const bool pre = m <= kHT && r <= kLrmvPre;
    T u[kLrmvPre];
    if (pre) {
        // unconditional loads (clamped row and column) so that they are all in flight together
        const int row = min(tid, m - 1);
#pragma unroll
        for (int c = 0; c < kLrmvPre; ++c) u[c] = U[row + (int64_t)min(c, r - 1) * m];
#pragma unroll
        for (int c = 0; c < kLrmvPre; ++c) u[c] = c < r ? u[c] : T(0);
    }
    // t(c, j) = sum_l V(l, c) X(l, j): G lanes per output, consecutive lanes along l (contiguous in V)
    int G = 64;
    while (G > 1 && G * r * w > kHT) G >>= 1;
    const int ng = kHT / G, gid = tid / G, gl = tid % G;
    for (int idx = gid; idx < r * w; idx += ng) {
        const int c = idx % r, j = idx / r;
        const T* v = V + (int64_t)c * n;
        const T* x = X + (int64_t)j * xcs;
        T s = 0;
        for (int l = gl; l < n; l += G) s += v[l] * x[(int64_t)l * xrs];
        s = group_sum(s, G);
        if (gl == 0) t[(int64_t)c * trs + (int64_t)j * tcs] = s;
    }
    __syncthreads();
    if (pre) {
        if (tid < m)
            for (int j = 0; j < w; ++j) {
                T s = 0;
#pragma unroll
                for (int c = 0; c < kLrmvPre; ++c)
                    if (c < r) s += u[c] * t[(int64_t)c * trs + (int64_t)j * tcs];
                Y[(int64_t)tid * yrs + (int64_t)j * ycs] += alpha * s;
            }
        return;
    }
    for (int i = tid; i < m; i += kHT)
        for (int j = 0; j < w; ++j) {
            T s = 0;
            for (int c = 0; c < r; ++c) s += U[i + (int64_t)c * m] * t[(int64_t)c * trs + (int64_t)j * tcs];
            Y[(int64_t)i * yrs + (int64_t)j * ycs] += alpha * s;
        }
}

template <class T>
__device__ void hsolve_body(const Inst<T>& d, int c0, int wc, int step, char* smem) {
    const int Nd = d.Nd;
    wc = min(wc, d.nrhs - c0);
    if (wc <= 0) return;
    Lds<T> L;
    L.X = reinterpret_cast<T*>(smem);
    L.W = L.X + (int64_t)Nd * wc;
    L.red = L.W + (int64_t)d.work_rows * wc;
    L.rk = reinterpret_cast<int*>(L.red + kHT * wc);
    L.wc = wc;
    for (int s = threadIdx.x; s < d.nslots; s += kHT) L.rk[s] = d.ranks[s];
    const double* Bs = d.B + (int64_t)step * d.bstep + (int64_t)c0 * d.ldb;
    double* Xs = d.X + (int64_t)step * d.xstep + (int64_t)c0 * d.ldx;
    double flops = 0.0;
    __syncthreads();
    OpRec nxt = d.ops[0];
    for (int pc = 0; pc < d.nops; ++pc) {
        const OpRec o = nxt;
        if (pc + 1 < d.nops) nxt = d.ops[pc + 1];
        unsigned long long t0 = 0;
        if (d.prof && threadIdx.x == 0) t0 = wall_clock64();
        switch (o.code) {
            case OP_LOAD:
                for (int idx = threadIdx.x; idx < Nd * wc; idx += kHT) {
                    const int h = idx % Nd, j = idx / Nd;
                    L.X[idx] = (T)Bs[(int64_t)j * d.ldb + d.h2p[h]];
                }
                break;
            case OP_STORE:
                for (int idx = threadIdx.x; idx < Nd * wc; idx += kHT) {
                    const int h = idx % Nd, j = idx / Nd;
                    Xs[(int64_t)j * d.ldx + d.h2p[h]] = (double)L.X[idx];
                }
                break;
            case OP_GEMM:
                hs_gemm(d, L, o);
                if (threadIdx.x == 0) flops += 2.0 * hdim(L, o.dim[0]) * hdim(L, o.dim[1]) * hdim(L, o.dim[2]);
                break;
            case OP_LRMV:
                hs_lrmv(d, L, o);
                if (threadIdx.x == 0) {
                    const LRBlockDev B = d.lr[o.blk];
                    flops += 2.0 * (B.m + B.n) * L.rk[B.slot] * hdim(L, o.dim[1]);
                }
                break;
            case OP_TRSM:
                hs_trsm(d, L, o);
                if (threadIdx.x == 0) {
                    const double n = hdim(L, o.dim[0]);
                    flops += n * n * hdim(L, o.dim[1]);
                }
                break;
            default: break;
        }
        __syncthreads();
        if (d.prof && threadIdx.x == 0) {
            atomicAdd(&d.prof[2 * o.code], (unsigned long long)(wall_clock64() - t0));
            atomicAdd(&d.prof[2 * o.code + 1], 1ull);
        }
    }
    if (threadIdx.x == 0) atomicAdd(d.flops, flops);
}

template <class T>
__global__ void __launch_bounds__(kHT) k_hsolve(const Inst<T>* __restrict__ insts, int nchunk, int wc, int step) {
    extern __shared__ __align__(16) char smem[];
    const int i = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
    const Inst<T> d = insts[i];
    hsolve_body(d, c * wc, wc, step, smem);
}

template <class T>
__global__ void __launch_bounds__(kHT) k_hsolve_one(const Inst<T> d, int wc) {
    extern __shared__ __align__(16) char smem[];
    hsolve_body(d, blockIdx.x * wc, wc, 0, smem);
}

template <class K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        FDE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)bytes));
}

}  // namespace

size_t hsolve_lds_bytes(int Nd, int work_rows, int nslots, int wc, size_t esz) {
    return ((size_t)Nd + work_rows + kHT) * wc * esz + (size_t)nslots * sizeof(int) + 16;
}

size_t device_lds_limit(int device) {
    int v = 0;
    FDE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    return (size_t)v;
}

template <class T>
void launch_hsolve(hipStream_t st, int ninst, int nchunk, int wc, const Inst<T>* d_insts, int step, size_t lds) {
    if (ninst <= 0 || nchunk <= 0) return;
    allow_lds(k_hsolve<T>, lds);
    hipLaunchKernelGGL((k_hsolve<T>), dim3(ninst * nchunk), dim3(kHT), lds, st, d_insts, nchunk, wc, step);
    FDE_LAUNCH_CHECK();
}
template void launch_hsolve<float>(hipStream_t, int, int, int, const Inst<float>*, int, size_t);
template void launch_hsolve<double>(hipStream_t, int, int, int, const Inst<double>*, int, size_t);

template <class T>
void launch_hsolve_one(hipStream_t st, const Inst<T>& d, int nchunk, int wc, size_t lds) {
    if (nchunk <= 0) return;
    allow_lds(k_hsolve_one<T>, lds);
    hipLaunchKernelGGL((k_hsolve_one<T>), dim3(nchunk), dim3(kHT), lds, st, d, wc);
    FDE_LAUNCH_CHECK();
}
template void launch_hsolve_one<float>(hipStream_t, const Inst<float>&, int, int, size_t);
template void launch_hsolve_one<double>(hipStream_t, const Inst<double>&, int, int, size_t);

}  // namespace fde
