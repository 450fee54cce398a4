// Forward and backward H-substitution (Section 4.1) by pipelined leaf steps, with
// the right-hand sides resident in LDS.
//
// One workgroup (512 threads, eight wavefronts) solves a chunk of wc right-hand-side
// columns of one instance. The chunk (Nd x wc), the short vectors t_B of the
// low-rank blocks in flight, the ranks and one staged diagonal leaf stay in LDS for
// the whole solve; only factor blocks and the step tables are read from HBM. Step p
// (host tables, see HsStep):
//   phase 1, all wavefronts: the chunks of the dense block between leaf p and the
//     leaf solved just before, into per-wavefront partial sums; the increments
//     t_B += V_B(rows of that leaf)^T x of the low-rank blocks whose column cluster
//     holds it (a wavefront per block, reduced by a butterfly over the lanes); the
//     solving wavefronts also read the staged diagonal leaf into registers;
//   phase 2: wavefront j < wc sums the partials of column j and solves with the
//     diagonal leaf (row-scaled unit triangular substitution, readlane broadcasts);
//     the other wavefronts gather every remaining contribution to the next leaf's
//     rows (dense chunks from older leaves, rows of U_B times t_B) and stage the
//     next diagonal leaf in LDS.
// Two barriers per step. Only the dense chunk of the previous leaf and the triangular
// solve are on the dependent chain from one leaf to the next; factor values of the
// next step and step records two steps ahead are loaded while a step runs (vector
// loads, so the waits for them do not serialise with LDS traffic).
#include "hinterp.h"
#include "tri_wave.h"

namespace fde {

namespace {

constexpr int kHT = 512;
constexpr int kHW = kHT / 64;

static_assert(sizeof(HsRec) == 32 && sizeof(HsStep) == 32, "H-solve records are loaded as two 16-byte vectors");

// items per wavefront and step whose factor values are loaded a step ahead (register budget),
// and elements per lane of one batch of the diagonal staging
template <class T>
struct HsDepth {
    static constexpr int kP1 = 2, kP2 = 3, kD = 16;
};
template <>
struct HsDepth<double> {
    static constexpr int kP1 = 1, kP2 = 1, kD = 8;
};

// global-memory view of a pointer: loads through it are vector-memory loads counted by vmcnt
// alone (a flat load also counts on the counter that LDS reads wait for)
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// 32 bytes per lane: a step record (same for every lane) or lane l's record of a step
struct Vec8 {
    int a[8];
};

__device__ inline Vec8 load8(const void* p, bool live) {
    Vec8 v;
    if (live) {
        const auto q = gmem(reinterpret_cast<const int*>(p));
#pragma unroll
        for (int i = 0; i < 8; ++i) v.a[i] = q[i];
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v.a[i] = 0;
    }
    return v;
}

struct StepS {
    int64_t diag;
    int row0, nrow, rec0, nlate, ninc, nearly;
};

__device__ inline StepS step_of(const Vec8& v) {
    StepS s;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane(v.a[0]);
    const int hi = __builtin_amdgcn_readfirstlane(v.a[1]);
    s.diag = ((int64_t)hi << 32) | lo;
    s.row0 = __builtin_amdgcn_readfirstlane(v.a[2]);
    s.nrow = __builtin_amdgcn_readfirstlane(v.a[3]);
    s.rec0 = __builtin_amdgcn_readfirstlane(v.a[4]);
    s.nlate = __builtin_amdgcn_readfirstlane(v.a[5]);
    s.ninc = __builtin_amdgcn_readfirstlane(v.a[6]);
    s.nearly = __builtin_amdgcn_readfirstlane(v.a[7]);
    return s;
}

__device__ inline Vec8 load_step(const HsStep* steps, int s, int nsteps) { return load8(steps + s, s < nsteps); }

// lane l holds record rec0 + l of the step (l < its record count, at most 64)
__device__ inline Vec8 load_recs(const HsRec* recs, const StepS& s, int lane) {
    const int n = s.nlate + s.ninc + s.nearly;
    return load8(recs + s.rec0 + lane, lane < n);
}

struct RecS {
    int64_t off;
    int ld, col0, n, slot, tslot, kind;
};

// record k (wave-uniform) of a step: from the lanes for k < 64, else straight from memory
__device__ inline RecS rec_of(const Vec8& v, int k, const HsRec* recs, const StepS& s) {
    int a[8];
    if (k < 64) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_readlane(v.a[i], k);
    } else {
        const Vec8 w = load8(recs + s.rec0 + k, true);
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_readfirstlane(w.a[i]);
    }
    RecS r;
    r.off = ((int64_t)a[1] << 32) | (unsigned)a[0];
    r.ld = a[2];
    r.col0 = a[3];
    r.n = a[4];
    r.slot = a[5];
    r.tslot = a[6];
    r.kind = a[7];
    return r;
}

// kHsChunk columns of a factor block starting at column c0, row = lane (rows and columns clamped
// into the block, so every load is in bounds and they are all in flight together)
template <class T>
__device__ inline void load_cols(T (&v)[kHsChunk], const T* arena, const RecS& r, int rows, int cols, int c0, int lane) {
    const int li = min(lane, rows - 1), cl = max(cols, 1) - 1;
    const auto a = gmem(arena + r.off + li);
#pragma unroll
    for (int c = 0; c < kHsChunk; ++c) v[c] = a[(int64_t)min(c0 + c, cl) * r.ld];
}

// lane l ends with the sum over the wavefront of v[(l >> 3) & 7]: each exchange halves the
// values a lane holds (10 shuffles for 8 sums instead of 48)
template <class T>
__device__ inline T reduce8(const T (&v)[8], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
    T w[4], u[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T send = b5 ? v[i] : v[i + 4], keep = b5 ? v[i + 4] : v[i];
        w[i] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T send = b4 ? w[i] : w[i + 2], keep = b4 ? w[i + 2] : w[i];
        u[i] = keep + __shfl_xor(send, 16, 64);
    }
    const T send = b3 ? u[0] : u[1], keep = b3 ? u[1] : u[0];
    T s = keep + __shfl_xor(send, 8, 64);
    s += __shfl_xor(s, 4, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 1, 64);
    return s;
}

// WC: columns of a chunk (1, 2, 4 or 8); the last chunk of a solve may use fewer (wce)
template <class T, int WC>
__device__ void hsteps_body(const Inst<T>& d, int c0, int step, char* smem) {
    using D = HsDepth<T>;
    constexpr int wc = WC;
    const int Nd = d.Nd, kmax = d.kmax, nsteps = 2 * d.hs_nleaf;
    const int wce = min(WC, d.nrhs - c0);
    if (wce <= 0) return;
    T* X = reinterpret_cast<T*>(smem);                    // Nd x wc, ld Nd
    T* tb = X + (int64_t)Nd * wc;                          // tslots x kmax x wc
    T* part1 = tb + (int64_t)d.hs_tslots * kmax * wc;      // kHW x 64 x wc (phase 1 partial sums)
    T* part2 = part1 + kHT * wc;                           // 2 x kHW x 64 x wc (early sums, by step parity)
    T* Dg = part2 + 2 * kHT * wc;                          // staged diagonal leaf, ld kHsolveMaxRow
    int* rk = reinterpret_cast<int*>(Dg + kHsolveMaxRow * kHsolveMaxRow);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // phase 2 roles: waves [0, wce) solve; helpers h0 .. h0 + nh - 1 gather for the next leaf
    const int h0 = wc < kHW ? wc : 0, nh = kHW - h0;
    const bool helper = wave >= h0;
    const int hw = wave - h0;
    const T* arena = d.arena;
    const HsStep* steps = d.hs_steps;
    const HsRec* recs = d.hs_recs;
    for (int s = threadIdx.x; s < d.nslots; s += kHT) rk[s] = d.ranks[s];
    const double* Bs = d.B + (int64_t)step * d.bstep + (int64_t)c0 * d.ldb;
    double* Xs = d.X + (int64_t)step * d.xstep + (int64_t)c0 * d.ldx;
    for (int idx = threadIdx.x; idx < Nd * wc; idx += kHT) {
        const int h = idx % Nd, j = idx / Nd;
        X[idx] = j < wce ? (T)Bs[(int64_t)j * d.ldb + d.h2p[h]] : T(0);
    }
    double flops = 0.0;
    StepS S0 = step_of(load_step(steps, 0, nsteps));
    StepS S1 = step_of(load_step(steps, 1, nsteps));
    StepS S2 = step_of(load_step(steps, 2, nsteps));
    Vec8 R0 = load_recs(recs, S0, lane), R1 = load_recs(recs, S1, lane), R2;
    // the diagonal of step 0 (column c of the leaf at Dg + c * kHsolveMaxRow)
    for (int c = wave; c < S0.nrow; c += kHW)
        if (lane < S0.nrow) Dg[lane + c * kHsolveMaxRow] = gmem(arena)[S0.diag + lane + (int64_t)c * S0.nrow];
    __syncthreads();   // ranks in LDS before the prefetches read them
    T av1[D::kP1][kHsChunk], av2[D::kP2][kHsChunk];
    // factor values of this wavefront's first phase-1 items of step S (late chunks: rows of S's
    // leaf; increments: rows of the previous leaf, columns up to the rank)
    auto prefetch1 = [&](const StepS& S, const Vec8& R) {
#pragma unroll
        for (int i = 0; i < D::kP1; ++i) {
            const int k = wave + kHW * i;
            if (k < S.nlate + S.ninc) {
                const RecS r = rec_of(R, k, recs, S);
                if (k < S.nlate) load_cols(av1[i], arena, r, S.nrow, r.n, 0, lane);
                else load_cols(av1[i], arena, r, r.n, rk[r.slot], 0, lane);
            }
        }
    };
    // early items go to kHW partial-sum slots (item e to slot e % kHW), whatever the number of
    // helpers, so the order of every sum is the same for every chunk width; helper hw takes
    // slots hw, hw + nh, ... and their items in that order
    auto prefetch2 = [&](const StepS& S, const Vec8& R, int rows) {
        if (!helper) return;
        int i = 0;
        for (int v = hw; v < min(kHW, S.nearly) && i < D::kP2; v += nh)
            for (int e = v; e < S.nearly && i < D::kP2; e += kHW, ++i) {
                const RecS r = rec_of(R, S.nlate + S.ninc + e, recs, S);
#pragma unroll
                for (int i2 = 0; i2 < D::kP2; ++i2)
                    if (i2 == i) load_cols(av2[i2], arena, r, rows, r.kind == HS_DENSE ? r.n : rk[r.slot], 0, lane);
            }
    };
    prefetch1(S0, R0);
    prefetch2(S0, R0, S1.nrow);
    unsigned long long tph = (d.prof && threadIdx.x == 0) ? wall_clock64() : 0ull;
    auto phase = [&](int k) {   // op profile: step phases (thread 0); TRSM counts the steps
        if (d.prof && threadIdx.x == 0) {
            const unsigned long long t = wall_clock64();
            atomicAdd(&d.prof[2 * kOpCodes + k], t - tph);
            if (k == 7) atomicAdd(&d.prof[2 * OP_TRSM + 1], 1ull);
            tph = t;
        }
    };
    int nearly_prev = 0;   // early items gathered for this step's leaf in the step before
    T tr[kHsolveMaxRow];
    T dinv = T(1);
    for (int s = 0; s < nsteps; ++s) {
        const bool fwd = s < d.hs_nleaf;
        const Vec8 S3v = load_step(steps, s + 3, nsteps);
        // ---------------- phase 1
        const int n = S0.nrow;
        if (wave < wce) {
            // the lane's row, divided by its diagonal entry going backward (unit triangular
            // system); columns c >= n are stale and never used
            const int li = min(lane, n - 1);
            dinv = fwd ? T(1) : T(1) / Dg[li + li * kHsolveMaxRow];
#pragma unroll
            for (int c = 0; c < kHsolveMaxRow; ++c) tr[c] = Dg[li + c * kHsolveMaxRow] * dinv;
        }
        {
            T acc[wc];
#pragma unroll
            for (int j = 0; j < wc; ++j) acc[j] = T(0);
            const int np1 = S0.nlate + S0.ninc;
            for (int k = wave, i = 0; k < np1; k += kHW, ++i) {
                const RecS r = rec_of(R0, k, recs, S0);
                T vv[kHsChunk];
                if (i < D::kP1) {
#pragma unroll
                    for (int i2 = 0; i2 < D::kP1; ++i2)
                        if (i2 == i)
#pragma unroll
                            for (int c = 0; c < kHsChunk; ++c) vv[c] = av1[i2][c];
                } else if (k < S0.nlate) {
                    load_cols(vv, arena, r, n, r.n, 0, lane);
                } else {
                    load_cols(vv, arena, r, r.n, rk[r.slot], 0, lane);
                }
                if (k < S0.nlate) {
                    // late chunk: rows of this leaf times entries of the leaf solved just before
                    if (lane == 0) flops += 2.0 * n * r.n * wc;
#pragma unroll
                    for (int c = 0; c < kHsChunk; ++c)
                        if (c < r.n)
#pragma unroll
                            for (int j = 0; j < wc; ++j) acc[j] += vv[c] * X[r.col0 + c + (int64_t)j * Nd];
                } else {
                    // increment of t_B by the rows of the leaf solved just before
                    const int rank = rk[r.slot], m = r.n;
                    if (lane == 0) flops += 2.0 * m * rank * wc;
                    T* t = tb + (int64_t)r.tslot * kmax * wc;
                    const bool first = r.kind == HS_INC_FIRST;
                    for (int cb = 0; cb < rank; cb += kHsChunk) {
                        if (cb > 0) load_cols(vv, arena, r, m, rank, cb, lane);
#pragma unroll
                        for (int j = 0; j < wc; ++j) {
                            const T xj = lane < m ? X[r.col0 + lane + (int64_t)j * Nd] : T(0);
                            T pr[kHsChunk];
#pragma unroll
                            for (int c = 0; c < kHsChunk; ++c) pr[c] = cb + c < rank ? vv[c] * xj : T(0);
                            const T sum = reduce8(pr, lane);
                            const int c = cb + ((lane >> 3) & 7);
                            if ((lane & 7) == 0 && c < rank) {
                                T* tc = t + (int64_t)c * wc + j;
                                *tc = first ? sum : *tc + sum;
                            }
                        }
                    }
                }
            }
            if (wave < S0.nlate) {
#pragma unroll
                for (int j = 0; j < wc; ++j) part1[(wave * 64 + lane) * wc + j] = acc[j];
            }
        }
        // the next step's phase-1 values; the records two steps ahead
        prefetch1(S1, R1);
        R2 = load_recs(recs, S2, lane);
        __syncthreads();
        phase(6);
        // ---------------- phase 2
        if (wave < wce) {
            // solve: y = b - late partials - early partials; T^{-1} y with the leaf in registers
            const int j = wave;
            const bool act = lane < n;
            T y = act ? X[S0.row0 + lane + (int64_t)j * Nd] : T(0);
            const int nw1 = min(kHW, S0.nlate), nw2 = min(kHW, nearly_prev);
            const T* p2 = part2 + (s & 1) * kHT * wc;
            for (int w = 0; w < nw1; ++w) y -= part1[(w * 64 + lane) * wc + j];
            for (int h = 0; h < nw2; ++h) y -= p2[(h * 64 + lane) * wc + j];
            if (lane == 0) flops += (double)n * n;
            T x = act ? y * dinv : T(0);
            // an opaque copy of the lane index: the 64 per-column lane masks below are then formed
            // where they are used instead of being hoisted out of the step loop (64 mask pairs
            // held in scalar registers across the loop would spill)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            if (fwd) {
#pragma unroll
                for (int c = 0; c < kHsolveMaxRow; ++c) {
                    if (c < n) {
                        const T xs = lane_bcast(x, c);
                        if (ln > c) x -= tr[c] * xs;
                    }
                }
            } else {
#pragma unroll
                for (int c = kHsolveMaxRow - 1; c >= 0; --c) {
                    if (c < n) {
                        const T xs = lane_bcast(x, c);
                        if (ln < c) x -= tr[c] * xs;
                    }
                }
            }
            if (act) X[S0.row0 + lane + (int64_t)j * Nd] = x;
        }
        if (helper) {
            // stage the next diagonal leaf, helper hw taking columns hw, hw + nh, ...; the first
            // batch is in flight during the gather below
            const int nd = S1.nrow;
            const bool rowok = lane < nd;
            T dv[D::kD];
#pragma unroll
            for (int q = 0; q < D::kD; ++q) {
                const int c = hw + q * nh;
                dv[q] = (rowok && c < nd) ? gmem(arena)[S1.diag + lane + (int64_t)c * nd] : T(0);
            }
            // early items: contributions to the next leaf's rows from leaves before this one
            const int m = S1.nrow;
            int i = 0;
            for (int v = hw; v < min(kHW, S0.nearly); v += nh) {
                T acc[wc];
#pragma unroll
                for (int j = 0; j < wc; ++j) acc[j] = T(0);
                for (int e = v; e < S0.nearly; e += kHW, ++i) {
                    const RecS r = rec_of(R0, S0.nlate + S0.ninc + e, recs, S0);
                    const int cols = r.kind == HS_DENSE ? r.n : rk[r.slot];
                    if (lane == 0) flops += 2.0 * m * cols * wc;
                    const T* t = tb + (int64_t)r.tslot * kmax * wc;
                    for (int cb = 0; cb < cols; cb += kHsChunk) {
                        T vv[kHsChunk];
                        if (cb == 0 && i < D::kP2) {
#pragma unroll
                            for (int i2 = 0; i2 < D::kP2; ++i2)
                                if (i2 == i)
#pragma unroll
                                    for (int c = 0; c < kHsChunk; ++c) vv[c] = av2[i2][c];
                        } else {
                            load_cols(vv, arena, r, m, cols, cb, lane);
                        }
                        if (r.kind == HS_DENSE) {
#pragma unroll
                            for (int c = 0; c < kHsChunk; ++c)
                                if (c < cols)
#pragma unroll
                                    for (int j = 0; j < wc; ++j) acc[j] += vv[c] * X[r.col0 + c + (int64_t)j * Nd];
                        } else {
#pragma unroll
                            for (int c = 0; c < kHsChunk; ++c)
                                if (cb + c < cols)
#pragma unroll
                                    for (int j = 0; j < wc; ++j) acc[j] += vv[c] * t[(cb + c) * wc + j];
                        }
                    }
                }
                T* p2 = part2 + ((s + 1) & 1) * kHT * wc;
#pragma unroll
                for (int j = 0; j < wc; ++j) p2[(v * 64 + lane) * wc + j] = acc[j];
            }
            // the next step's early values (rows of the leaf after next)
            prefetch2(S1, R1, S2.nrow);
#pragma unroll
            for (int q = 0; q < D::kD; ++q) {
                const int c = hw + q * nh;
                if (rowok && c < nd) Dg[lane + c * kHsolveMaxRow] = dv[q];
            }
            for (int c = hw + D::kD * nh; c < nd; c += nh)
                if (rowok) Dg[lane + c * kHsolveMaxRow] = gmem(arena)[S1.diag + lane + (int64_t)c * nd];
        }
        __syncthreads();
        phase(7);
        nearly_prev = S0.nearly;
        S0 = S1;
        S1 = S2;
        S2 = step_of(S3v);
        R0 = R1;
        R1 = R2;
    }
    for (int idx = threadIdx.x; idx < Nd * wce; idx += kHT) {
        const int h = idx % Nd, j = idx / Nd;
        Xs[(int64_t)j * d.ldx + d.h2p[h]] = (double)X[idx];
    }
    if (lane == 0) atomicAdd(d.flops, flops);
}

template <class T, int WC>
__global__ void __launch_bounds__(kHT) k_hsolve(const Inst<T>* __restrict__ insts, int nchunk, int step) {
    extern __shared__ __align__(16) char smem[];
    const int i = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
    const Inst<T> d = insts[i];
    hsteps_body<T, WC>(d, c * WC, step, smem);
}

template <class T, int WC>
__global__ void __launch_bounds__(kHT) k_hsolve_one(const Inst<T> d) {
    extern __shared__ __align__(16) char smem[];
    hsteps_body<T, WC>(d, blockIdx.x * WC, 0, smem);
}

template <class K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        FDE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)bytes));
}

}  // namespace

size_t hsolve_lds_bytes(int Nd, int tslots, int kmax, int nslots, int wc, size_t esz) {
    return ((size_t)Nd + (size_t)tslots * kmax + 3 * kHT) * wc * esz + (size_t)kHsolveMaxRow * kHsolveMaxRow * esz +
           (size_t)nslots * sizeof(int) + 16;
}

size_t device_lds_limit(int device) {
    int v = 0;
    FDE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    return (size_t)v;
}

namespace {

template <class T, int WC>
void launch_hsolve_wc(hipStream_t st, int ninst, int nchunk, const Inst<T>* d_insts, int step, size_t lds) {
    allow_lds(k_hsolve<T, WC>, lds);
    hipLaunchKernelGGL((k_hsolve<T, WC>), dim3(ninst * nchunk), dim3(kHT), lds, st, d_insts, nchunk, step);
    FDE_LAUNCH_CHECK();
}

template <class T, int WC>
void launch_hsolve_one_wc(hipStream_t st, const Inst<T>& d, int nchunk, size_t lds) {
    allow_lds(k_hsolve_one<T, WC>, lds);
    hipLaunchKernelGGL((k_hsolve_one<T, WC>), dim3(nchunk), dim3(kHT), lds, st, d);
    FDE_LAUNCH_CHECK();
}

}  // namespace

template <class T>
void launch_hsolve(hipStream_t st, int ninst, int nchunk, int wc, const Inst<T>* d_insts, int step, size_t lds) {
    if (ninst <= 0 || nchunk <= 0) return;
    switch (wc) {
        case 1: launch_hsolve_wc<T, 1>(st, ninst, nchunk, d_insts, step, lds); break;
        case 2: launch_hsolve_wc<T, 2>(st, ninst, nchunk, d_insts, step, lds); break;
        case 4: launch_hsolve_wc<T, 4>(st, ninst, nchunk, d_insts, step, lds); break;
        case 8: launch_hsolve_wc<T, 8>(st, ninst, nchunk, d_insts, step, lds); break;
        default: fail(FDE_EDEVICE, "H-solve chunk width %d is not 1, 2, 4 or 8", wc);
    }
}
template void launch_hsolve<float>(hipStream_t, int, int, int, const Inst<float>*, int, size_t);
template void launch_hsolve<double>(hipStream_t, int, int, int, const Inst<double>*, int, size_t);

template <class T>
void launch_hsolve_one(hipStream_t st, const Inst<T>& d, int nchunk, int wc, size_t lds) {
    if (nchunk <= 0) return;
    switch (wc) {
        case 1: launch_hsolve_one_wc<T, 1>(st, d, nchunk, lds); break;
        case 2: launch_hsolve_one_wc<T, 2>(st, d, nchunk, lds); break;
        case 4: launch_hsolve_one_wc<T, 4>(st, d, nchunk, lds); break;
        case 8: launch_hsolve_one_wc<T, 8>(st, d, nchunk, lds); break;
        default: fail(FDE_EDEVICE, "H-solve chunk width %d is not 1, 2, 4 or 8", wc);
    }
}
template void launch_hsolve_one<float>(hipStream_t, const Inst<float>&, int, int, size_t);
template void launch_hsolve_one<double>(hipStream_t, const Inst<double>&, int, int, size_t);

}  // namespace fde
