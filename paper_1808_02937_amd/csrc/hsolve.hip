// Forward and backward H-substitution (Section 4.1) by leaf steps, with the
// right-hand sides resident in LDS.
//
// One workgroup (512 threads) solves a chunk of wc right-hand-side columns of
// one instance. The chunk (Nd x wc), the short vectors t_B = V_B^T x_sigma of
// the low-rank blocks in flight and the ranks stay in LDS for the whole solve;
// only factor blocks are read from HBM. The step of leaf i (host tables, see
// gen_hsolve_steps):
//   A. the eight wavefronts split the contributions to the leaf's rows (chunks
//      of dense off-diagonal blocks times solved entries, rows of U_B times t_B)
//      and leave partial sums in LDS; the wavefronts that will solve also load
//      their row of the diagonal leaf meanwhile;
//   B. wavefront j sums the partials of column j and solves with the diagonal
//      leaf in registers (row-scaled unit triangular substitution, readlane);
//   C. for every low-rank block whose column cluster is now solved, each
//      wavefront forms one entry of t_B = V_B^T x_sigma (a coalesced dot
//      product reduced by shuffles).
#include "hinterp.h"
#include "tri_wave.h"

namespace fde {

namespace {

constexpr int kHT = 512;
constexpr int kHW = kHT / 64;

template <class T>
__device__ inline T wave_sum_t(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// one contribution item with its factor values (a chunk of a dense block or kHsChunk columns of
// U_B rows; a low-rank item of rank above kHsChunk takes the rest synchronously)
// items per wavefront and step whose values are prefetched (register budget)
template <class T>
struct kIpwOf {
    static constexpr int value = 2;
};
struct ItemRef {
    int64_t off;
    int ld, col0, ncol, slot, tslot;
    bool live;
};

__device__ inline ItemRef load_item(const HsItem* items, int it, int it1) {
    ItemRef r{};
    r.live = it < it1;
    if (r.live) {
        const HsItem m = items[it];
        r.off = m.off;
        r.ld = m.ld;
        r.col0 = m.col0;
        r.ncol = m.ncol;
        r.slot = m.slot;
        r.tslot = m.tslot;
    }
    return r;
}

template <class T>
__device__ void hsteps_body(const Inst<T>& d, int c0, int wc, int step, char* smem) {
    const int Nd = d.Nd, L = d.hs_nleaf, kmax = d.kmax;
    wc = min(wc, d.nrhs - c0);
    if (wc <= 0) return;
    T* X = reinterpret_cast<T*>(smem);                 // Nd x wc, ld Nd
    T* tb = X + (int64_t)Nd * wc;                       // tslots x kmax x wc
    T* part = tb + (int64_t)d.hs_tslots * kmax * wc;    // kHW x 64 x wc partial sums
    int* rk = reinterpret_cast<int*>(part + kHT * wc);
    // the wavefront index is uniform across the wavefront: item records then load as scalars
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int s = threadIdx.x; s < d.nslots; s += kHT) rk[s] = d.ranks[s];
    const double* Bs = d.B + (int64_t)step * d.bstep + (int64_t)c0 * d.ldb;
    double* Xs = d.X + (int64_t)step * d.xstep + (int64_t)c0 * d.ldx;
    for (int idx = threadIdx.x; idx < Nd * wc; idx += kHT) {
        const int h = idx % Nd, j = idx / Nd;
        X[idx] = (T)Bs[(int64_t)j * d.ldb + d.h2p[h]];
    }
    double flops = 0.0;
    const int nsteps = 2 * L;
    constexpr int kIpw = kIpwOf<T>::value;
    // pipeline state: factor values of this step's first items (per wavefront), the item records
    // of the next step, and the diagonal row of this step
    HsStep st = d.hs_steps[0];
    ItemRef cur[kIpw], nxt[kIpw];
    T av[kIpw][kHsChunk];
    T tr[64];
    T diag = T(1);
    auto load_values = [&](const ItemRef* r, int n) {
        const int li = min(lane, n - 1);
#pragma unroll
        for (int k = 0; k < kIpw; ++k)
#pragma unroll
            for (int c = 0; c < kHsChunk; ++c) {
                const int cc = r[k].ncol > 0 ? min(c, r[k].ncol - 1) : c;
                av[k][c] = r[k].live ? d.arena[r[k].off + li + (int64_t)cc * r[k].ld] : T(0);
            }
    };
    auto load_diag = [&](const HsStep& sx) {
        const int n = sx.nrow, li = min(lane, n - 1);
        const T* Tm = d.arena + sx.diag;
#pragma unroll
        for (int c = 0; c < 64; ++c) tr[c] = Tm[li + (int64_t)min(c, n - 1) * n];
        diag = Tm[li + (int64_t)li * n];
    };
#pragma unroll
    for (int k = 0; k < kIpw; ++k) cur[k] = load_item(d.hs_items, st.it0 + wave + k * kHW, st.it1);
    load_values(cur, st.nrow);
    if (wave < wc) load_diag(st);
    HsStep stn = st;
    if (nsteps > 1) {
        stn = d.hs_steps[1];
#pragma unroll
        for (int k = 0; k < kIpw; ++k) nxt[k] = load_item(d.hs_items, stn.it0 + wave + k * kHW, stn.it1);
    }
    __syncthreads();
    unsigned long long tph = (d.prof && threadIdx.x == 0) ? wall_clock64() : 0ull;
    auto phase = [&](int k) {   // op profile: step phases (thread 0); TRSM counts the steps
        if (d.prof && threadIdx.x == 0) {
            const unsigned long long t = wall_clock64();
            atomicAdd(&d.prof[2 * kOpCodes + k], t - tph);
            if (k == 7) atomicAdd(&d.prof[2 * OP_TRSM + 1], 1ull);
            tph = t;
        }
    };
    for (int s = 0; s < nsteps; ++s) {
        const bool fwd = s < L;
        const int n = st.nrow;
        const int li = min(lane, n - 1);
        // A: partial sums of the contributions to the leaf's rows (row = lane)
        T acc[kHsolveMaxCols];
#pragma unroll
        for (int j = 0; j < kHsolveMaxCols; ++j) acc[j] = T(0);
#pragma unroll
        for (int k = 0; k < kIpw; ++k) {
            if (!cur[k].live) continue;
            const ItemRef& m = cur[k];
            if (m.ncol > 0) {
                if (lane == 0) flops += 2.0 * n * m.ncol * wc;
#pragma unroll
                for (int c = 0; c < kHsChunk; ++c)
                    if (c < m.ncol)
#pragma unroll
                        for (int j = 0; j < kHsolveMaxCols; ++j)
                            if (j < wc) acc[j] += av[k][c] * X[m.col0 + c + (int64_t)j * Nd];
            } else {
                const int r = rk[m.slot];
                if (lane == 0) flops += 2.0 * n * r * wc;
                const T* t = tb + (int64_t)m.tslot * kmax * wc;
#pragma unroll
                for (int c = 0; c < kHsChunk; ++c)
                    if (c < r)
#pragma unroll
                        for (int j = 0; j < kHsolveMaxCols; ++j)
                            if (j < wc) acc[j] += av[k][c] * t[c * wc + j];
                for (int c = kHsChunk; c < r; ++c) {   // ranks above kHsChunk: the rest directly
                    const T a = d.arena[m.off + li + (int64_t)c * m.ld];
                    for (int j = 0; j < wc; ++j) acc[j] += a * t[c * wc + j];
                }
            }
        }
        // items beyond the prefetched ones (steps with more than kIpw items per wavefront)
        for (int it = st.it0 + wave + kIpw * kHW; it < st.it1; it += kHW) {
            const HsItem m = d.hs_items[it];
            const T* A = d.arena + m.off + li;
            const int cols = m.ncol > 0 ? m.ncol : rk[m.slot];
            if (lane == 0) flops += 2.0 * n * cols * wc;
            const T* t = m.ncol > 0 ? nullptr : tb + (int64_t)m.tslot * kmax * wc;
            for (int c0u = 0; c0u < cols; c0u += kHsChunk) {
                T a[kHsChunk];   // eight loads in flight together (clamped columns)
#pragma unroll
                for (int c = 0; c < kHsChunk; ++c) a[c] = A[(int64_t)min(c0u + c, cols - 1) * m.ld];
#pragma unroll
                for (int c = 0; c < kHsChunk; ++c)
                    if (c0u + c < cols)
                        for (int j = 0; j < wc; ++j)
                            acc[j] += a[c] * (m.ncol > 0 ? X[m.col0 + c0u + c + (int64_t)j * Nd] : t[(c0u + c) * wc + j]);
            }
        }
#pragma unroll
        for (int j = 0; j < kHsolveMaxCols; ++j)
            if (j < wc) part[(wave * 64 + lane) * wc + j] = acc[j];
        // prefetch: factor values of the next step's items, the records of the step after
        HsStep st2 = stn;
        if (s + 1 < nsteps) {
            load_values(nxt, stn.nrow);
#pragma unroll
            for (int k = 0; k < kIpw; ++k) cur[k] = nxt[k];
            if (s + 2 < nsteps) {
                st2 = d.hs_steps[s + 2];
#pragma unroll
                for (int k = 0; k < kIpw; ++k) nxt[k] = load_item(d.hs_items, st2.it0 + wave + k * kHW, st2.it1);
            }
        }
        __syncthreads();
        phase(6);
        // B: wavefront j sums the partials of column j and solves with the diagonal leaf
        if (wave < wc) {
            const int j = wave;
            const bool act = lane < n;
            T y = act ? X[st.row0 + lane + (int64_t)j * Nd] : T(0);
#pragma unroll
            for (int w = 0; w < kHW; ++w) y -= part[(w * 64 + lane) * wc + j];
            const T dinv = (!fwd && act) ? T(1) / diag : T(1);
            if (lane == 0) flops += (double)n * n;
#pragma unroll
            for (int c = 0; c < 64; ++c) tr[c] = (c < n && act) ? tr[c] * dinv : T(0);
            T x = act ? y * dinv : T(0);
            if (fwd) {
#pragma unroll
                for (int c = 0; c < 64; ++c)
                    if (c < n) {
                        const T xs = lane_bcast(x, c);
                        if (lane > c) x -= tr[c] * xs;
                    }
            } else {
#pragma unroll
                for (int c = 63; c >= 0; --c)
                    if (c < n) {
                        const T xs = lane_bcast(x, c);
                        if (lane < c) x -= tr[c] * xs;
                    }
            }
            if (act) X[st.row0 + lane + (int64_t)j * Nd] = x;
            if (s + 1 < nsteps) load_diag(stn);   // the next step's diagonal row, in flight during C and A
        }
        __syncthreads();
        phase(7);
        // C: t_B = V_B^T x_sigma for the blocks whose column cluster is now solved; the (block,
        // column) pairs are spread over the wavefronts
        if (st.tc1 > st.tc0) {
            const int npair = (st.tc1 - st.tc0) * kmax;
            for (int pq = wave; pq < npair; pq += kHW) {
                const HsTcomp tcm = d.hs_tc[st.tc0 + pq / kmax];
                const int c = pq % kmax;
                const int r = rk[tcm.slot];
                T* t = tb + (int64_t)tcm.tslot * kmax * wc;
                if (lane == 0 && c == 0) flops += 2.0 * tcm.ld * r * wc;
                const T* v = d.arena + tcm.voff + (int64_t)c * tcm.ld;
                for (int j = 0; j < wc; ++j) {
                    T sum = 0;
                    if (c < r) {
#pragma unroll 4
                        for (int k = lane; k < tcm.ld; k += 64) sum += v[k] * X[tcm.col0 + k + (int64_t)j * Nd];
                    }
                    sum = wave_sum_t(sum);
                    if (lane == 0) t[c * wc + j] = sum;
                }
            }
            __syncthreads();
        }
        phase(8);
        st = stn;
        stn = st2;
    }
    for (int idx = threadIdx.x; idx < Nd * wc; idx += kHT) {
        const int h = idx % Nd, j = idx / Nd;
        Xs[(int64_t)j * d.ldx + d.h2p[h]] = (double)X[idx];
    }
    if (lane == 0) atomicAdd(d.flops, flops);
}

template <class T>
__global__ void __launch_bounds__(kHT) k_hsolve(const Inst<T>* __restrict__ insts, int nchunk, int wc, int step) {
    extern __shared__ __align__(16) char smem[];
    const int i = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
    const Inst<T> d = insts[i];
    hsteps_body(d, c * wc, wc, step, smem);
}

template <class T>
__global__ void __launch_bounds__(kHT) k_hsolve_one(const Inst<T> d, int wc) {
    extern __shared__ __align__(16) char smem[];
    hsteps_body(d, blockIdx.x * wc, wc, 0, smem);
}

template <class K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        FDE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)bytes));
}

}  // namespace

size_t hsolve_lds_bytes(int Nd, int tslots, int kmax, int nslots, int wc, size_t esz) {
    return ((size_t)Nd + (size_t)tslots * kmax + kHT) * wc * esz + (size_t)nslots * sizeof(int) + 16;
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
