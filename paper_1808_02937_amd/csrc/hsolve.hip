// Forward and backward H-substitution (Section 4.1) by pipelined leaf steps, with
// the right-hand sides resident in LDS.
//
// One workgroup (512 threads, eight wavefronts) solves a chunk of wc right-hand-side
// columns of one instance. The chunk (Nd x wc), the short vectors t_B of the
// low-rank blocks in flight, the ranks and the staged diagonal leaves stay in LDS for
// the whole solve; only factor blocks and the step tables are read from HBM. Step p
// (host tables, see HsStep):
//   phase 1, all wavefronts: the chunks of the dense block between leaf p and the
//     leaf solved just before, into per-wavefront partial sums, and the increments
//     t_B += V_B(rows of that leaf)^T x of the low-rank blocks whose column cluster
//     holds it (a wavefront per block, reduced by a butterfly over the lanes);
//   phase 2: wavefront j < wc sums the partials of column j and solves with the
//     staged diagonal leaf (lane = row, readlane broadcasts; the leaf's strict
//     triangle was staged with zeros elsewhere, so the substitution needs no masks);
//     the other wavefronts gather every remaining contribution to the next leaf's
//     rows (dense chunks from older leaves, rows of U_B times t_B) and stage the next
//     diagonal leaf in the other LDS buffer.
// Two barriers per step. Only the dense chunk of the previous leaf and the triangular
// solve are on the dependent chain from one leaf to the next. Factor values of the
// next step, its diagonal leaf and step records two steps ahead are loaded while a
// step runs, as global (vector-memory) loads issued identically by every wavefront,
// so the compiler's waits for them are exact and they stay in flight across barriers.
#include <algorithm>

#include "hinterp.h"
#include "tri_wave.h"

namespace fde {

namespace {

constexpr int kHT = 512;
constexpr int kHW = kHT / 64;

static_assert(sizeof(HsRec) == 32 && sizeof(HsStep) == 32, "H-solve records are loaded as two 16-byte vectors");

// Items per wavefront and step whose factor values are loaded a step ahead, and columns of the
// next diagonal leaf per helper loaded a step ahead (the rest are loaded when needed). The
// loads in flight per wavefront stay within the 63 the vector-memory counter tracks (beyond
// that the compiler can only wait for all of them): 8 kP1 + 8 kP2 + kD + 4 record loads.
template <class T, int WC>
struct HsDepth {
    static constexpr int kP1 = 3, kP2 = 3;
    static constexpr int kD = WC == 1 ? 10 : WC == 2 ? 11 : WC == 4 ? 16 : 10;
};
template <int WC>
struct HsDepth<double, WC> {
    static constexpr int kP1 = 2, kP2 = 2;
    static constexpr int kD = WC == 1 ? 10 : WC == 2 ? 11 : WC == 4 ? 16 : 10;
};

// a * b + c rounded once, whatever the surrounding selects (the masked products below must
// round as the unmasked ones would, in every chunk-width instance of the kernel)
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 32 bytes per lane: a step record (same for every lane) or lane l's record of a step
struct Vec8 {
    int a[8];
};

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

// 32 bytes loaded by every lane whatever `live` (an invalid entry reads `dummy`, a valid
// address, and gives zeros): no load sits on a branch
__device__ inline Vec8 load8_all(const void* p, bool live, const void* dummy) {
    const auto q = gmem(reinterpret_cast<const int*>(live ? p : dummy));
    Vec8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v.a[i] = q[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) v.a[i] = live ? v.a[i] : 0;
    return v;
}

__device__ inline Vec8 load_step(const HsStep* steps, int s, int nsteps) {
    return load8_all(steps + min(s, nsteps - 1), s < nsteps, steps);
}

// lane l holds record rec0 + l of the step (a step has at most 64 records)
__device__ inline Vec8 load_recs(const HsRec* recs, const StepS& s, int lane, const HsStep* steps) {
    const int n = s.nlate + s.ninc + s.nearly;
    return load8_all(recs + s.rec0 + min(lane, max(n - 1, 0)), lane < n, steps);
}

struct RecS {
    int64_t off;
    int ld, col0, n, slot, tslot, kind;
};

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
    // within rows of 16 lanes through DPP: the mirror pairs lane i of a row with lane 15 - i (the
    // other half of the row, same upper lane bits, as xor 8 would); the sums after it run over
    // whole groups of 8 lanes, so any pairing inside a group does (half mirror, then quads)
    const T send = b3 ? u[0] : u[1], keep = b3 ? u[1] : u[0];
    T s = keep + dpp_move<kDppRowMirror>(send);
    s += dpp_move<kDppRowHalfMirror>(s);
    s += dpp_move<kDppXor2>(s);
    s += dpp_move<kDppXor1>(s);
    return s;
}

// fields of record k of a step from the lanes (k < 64, wave-uniform)
__device__ inline RecS rec_lane(const Vec8& v, int k) {
    int a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_readlane(v.a[i], k);
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

// where the factors are: the arena, and (BF) BF16 copies of the low-rank factors from lr_base on
template <class T, bool BF>
struct FacSrc {
    const T* arena;
    const unsigned short* lr16;
    int64_t lr_base;
};

__device__ inline float bf16_bits_to_float(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// kHsChunk columns of a block at `off` (ld), row = lane, rows and columns clamped; a low-rank
// block of BF16 factors is widened to FP32. Both storages are read with one 32-bit load per
// element (for BF16, the word holding the element), so every block issues the same loads: a
// branch between two kinds of load would make the compiler wait for every prefetch in flight
// where the branches join.
template <class T, bool BF>
__device__ inline void load_block(T (&v)[kHsChunk], const FacSrc<T, BF>& f, int64_t off, int ld, int rows, int cols,
                                  int c0, int lane) {
    const int li = min(lane, rows - 1), cl = max(cols, 1) - 1;
    if constexpr (BF) {
        static_assert(sizeof(T) == 4, "BF16 low-rank factors come with FP32 factorisations");
        // one 32-bit load per element from a wave-uniform base, then one byte permute: an FP32 word
        // as it is, or the BF16 half-word of the element moved to the top with zeros below (the
        // element's half follows from the parity of its index, the same for every column when ld is
        // even, alternating when it is odd)
        const bool h16 = f.lr16 && off >= f.lr_base;   // wave-uniform
        const int64_t b = h16 ? off - f.lr_base : off;
        const unsigned* base = h16 ? reinterpret_cast<const unsigned*>(f.lr16) + (b >> 1)   // 4-byte aligned
                                   : reinterpret_cast<const unsigned*>(f.arena) + off;
        const unsigned sh = h16 ? 1u : 0u;
        const unsigned A = (h16 ? (unsigned)(b & 1) : 0u) + (unsigned)li;
        constexpr unsigned kSelLo = 0x01000C0Cu, kSelHi = 0x03020C0Cu, kSelId = 0x03020100u;
        const unsigned sel0 = h16 ? ((A & 1u) ? kSelHi : kSelLo) : kSelId;   // index parity of A
        const unsigned sel1 = h16 ? ((A & 1u) ? kSelLo : kSelHi) : kSelId;   // the other parity
        const auto g = gmem(base);
#pragma unroll
        for (int c = 0; c < kHsChunk; ++c) {
            const unsigned cc = (unsigned)min(c0 + c, cl) * (unsigned)ld;   // wave-uniform
            const unsigned w = g[(A + cc) >> sh];
            v[c] = __uint_as_float(__builtin_amdgcn_perm(0u, w, (cc & 1u) ? sel1 : sel0));
        }
        return;
    }
    const auto a = gmem(f.arena + off + li);
#pragma unroll
    for (int c = 0; c < kHsChunk; ++c) v[c] = a[(int64_t)min(c0 + c, cl) * ld];
}

// One workgroup: chunk c0 / wc of instance d, wc = d.hs_wc <= WC columns (the last chunk may
// use fewer, wce). Every wavefront issues the same global loads in every step, whatever its
// role and the number of items (empty slots load a valid dummy address), so the waits the
// compiler inserts for prefetched values are exact and the prefetches stay in flight across
// the barriers.
template <class T, int WC, bool BF, bool GX>
__device__ __attribute__((always_inline)) void hsteps_body(const Inst<T>& d, int chunk, int step, char* smem) {
    using D = HsDepth<T, WC>;
    const int wc = d.hs_wc;
    const int c0 = chunk * wc;
    const int Nd = d.Nd, kmax = d.kmax, nsteps = 2 * d.hs_nleaf, L = d.hs_nleaf;
    const int wce = min(wc, d.nrhs - c0);
    if (wce <= 0 || wc > WC) return;
    // the chunk's right-hand sides, Nd x wc (ld Nd): in LDS, or (GX, too long for LDS) in the
    // instance's global workspace (columns c0 .. c0 + wc - 1 of d.rhs, L2-resident; the other waves
    // of the workgroup see a wave's stores after each barrier)
    T* X = GX ? d.rhs + (int64_t)c0 * Nd : reinterpret_cast<T*>(smem);
    T* tb = GX ? reinterpret_cast<T*>(smem) : X + (int64_t)Nd * wc;   // tslots x kmax x wc
    T* part1 = tb + (int64_t)d.hs_tslots * kmax * wc;      // kHW x 64 x wc (phase 1 partial sums)
    T* part2 = part1 + kHT * wc;                           // 2 x kHW x 64 x wc (early sums, by step parity)
    // staged diagonal leaf (64 x 64, ld 64) and its diagonal entries, two buffers by step parity:
    // the solve of step s reads buffer s & 1 while the helpers stage step s + 1 in the other; a
    // third row of diagonal slots takes the writes of the lanes off the diagonal
    T* Dg2 = part2 + 2 * kHT * wc;
    T* Dd2 = Dg2 + 2 * kHsolveMaxRow * kHsolveMaxRow;
    int* rk = reinterpret_cast<int*>(Dd2 + 3 * kHsolveMaxRow);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // phase 2 roles: waves [0, wce) solve; helpers h0 .. 7 gather for the next leaf and stage
    const int h0 = wc < kHW ? wc : 0, nh = kHW - h0;
    const bool helper = wave >= h0;
    const int hw = helper ? wave - h0 : 0;
    const FacSrc<T, BF> arena{d.arena, d.lr16, d.lr_base};
    const HsStep* steps = d.hs_steps;
    const HsRec* recs = d.hs_recs;
    for (int s = threadIdx.x; s < d.nslots; s += kHT) rk[s] = d.ranks[s];
    for (int q = threadIdx.x; q < 2 * kHT * wc; q += kHT) part2[q] = T(0);
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
    Vec8 R0 = load_recs(recs, S0, lane, steps), R1 = load_recs(recs, S1, lane, steps), R2;
    // the staged leaf of a step is its solve-ready form (the strict triangle, rows divided by
    // their diagonal entry backward, zero elsewhere and past the leaf, so the substitution needs
    // no masks), copied as it is; its row scales go to Dd
    const T* prep = d.hs_prep;
    auto prep_of = [&](int si) { return prep + (int64_t)min(si, nsteps - 1) * kHsPrepStride; };
    auto stage = [&](T v, int c, int buf) { Dg2[buf * kHsolveMaxRow * kHsolveMaxRow + lane + c * kHsolveMaxRow] = v; };
    // a value loaded off the prefetch path is waited for where it is loaded: no load stays in
    // flight past a branch, which would make the compiler wait for every load at the join
    auto consume = [&](const T(&vv)[kHsChunk]) {
#pragma unroll
        for (int c = 0; c < kHsChunk; ++c) asm volatile("" ::"v"(vv[c]));
    };
    for (int c = wave; c < kHsolveMaxRow; c += kHW) stage(gmem(prep)[lane + c * kHsolveMaxRow], c, 0);
    if (wave == 0) Dd2[lane] = gmem(prep)[kHsolveMaxRow * kHsolveMaxRow + lane];
    __syncthreads();   // ranks and the first leaf in LDS
    T av1[D::kP1][kHsChunk], av2[D::kP2][kHsChunk], dv[D::kD], dvs;
    // phase-1 values of step S: wavefront w takes items w, w + 8, ... (late chunks: rows of S's
    // leaf; increments: rows of the leaf before, columns up to the rank)
    auto prefetch1 = [&](const StepS& S, const Vec8& R) {
        const int np = S.nlate + S.ninc;
#pragma unroll
        for (int i = 0; i < D::kP1; ++i) {
            const int k = wave + kHW * i;
            const bool live = k < np;
            const RecS r = rec_lane(R, min(k, 63));
            const bool late = k < S.nlate;
            const int cols = late ? r.n : kmax;   // low rank: the stored columns (masked by the rank at use)
            load_block(av1[i], arena, live ? r.off : 0, live ? r.ld : 0, live ? (late ? S.nrow : r.n) : 1,
                       live ? cols : 1, 0, lane);
        }
    };
    // early values of step S (rows of the next leaf, `rows`): helper hw takes items hw, hw + nh, ...
    auto prefetch2 = [&](const StepS& S, const Vec8& R, int rows) {
        const int base = S.nlate + S.ninc;
#pragma unroll
        for (int i = 0; i < D::kP2; ++i) {
            const int e = hw + nh * i;
            const bool live = helper && e < S.nearly;
            const RecS r = rec_lane(R, min(base + e, 63));
            const int cols = r.kind == HS_DENSE ? r.n : kmax;
            load_block(av2[i], arena, live ? r.off : 0, live ? r.ld : 0, live ? rows : 1, live ? cols : 1, 0, lane);
        }
    };
    // solve-ready leaf of step si staged by the helpers, helper hw taking columns hw, hw + nh, ...,
    // and its row scales. Every wavefront loads (columns clamped into the leaf, a step past the
    // end reads the last one): straight-line loads, so the compiler counts them exactly and waits
    // for no later prefetch where the values are staged
    auto prefetch_diag = [&](int si) {
        const auto pp = gmem(prep_of(si));
#pragma unroll
        for (int q = 0; q < D::kD; ++q) dv[q] = pp[lane + min(hw + q * nh, kHsolveMaxRow - 1) * kHsolveMaxRow];
        dvs = pp[kHsolveMaxRow * kHsolveMaxRow + lane];
    };
    // the same issue order as at the end of a step (diagonal leaf, then early values): the
    // compiler's wait counts merge the two at the loop head and stay exact
    prefetch1(S0, R0);
    prefetch_diag(1);
    prefetch2(S0, R0, S1.nrow);
    // op profile: step phases timed by thread 0 and the first helper's lane 0, added to the
    // profile once after the loop (no atomics in the loop: a pending flat atomic makes every
    // later wait for a prefetched value a wait for all loads)
    unsigned long long tph = (d.prof && threadIdx.x == 0) ? wall_clock64() : 0ull;
    unsigned long long pt[4] = {0ull, 0ull, 0ull, 0ull};
    auto phase = [&](int k) {
        if (d.prof && threadIdx.x == 0) {
            const unsigned long long t = wall_clock64();
            pt[k - 6] += t - tph;
            tph = t;
        }
    };
    int nearly_prev = 0;   // early items gathered for this step's leaf in the step before
    T dinv = T(1);
    Vec8 S3v;
    for (int s = 0; s < nsteps; ++s) {
        const bool fwd = s < L;
        // ---------------- phase 1
        const int n = S0.nrow;
        if (wave < wce) dinv = Dd2[(s & 1) * kHsolveMaxRow + lane];   // 1 forward, 1 / diagonal backward
        {
            T acc[WC];
#pragma unroll
            for (int j = 0; j < WC; ++j) acc[j] = T(0);
            const int np1 = S0.nlate + S0.ninc;
            // t_B (+)= V_B(rows of the leaf before, columns cb..cb+7)^T x of that leaf
            auto inc_chunk = [&](const RecS& r, const T (&vv)[kHsChunk], int cb) {
                const int rank = rk[r.slot], m = r.n;
                T* t = tb + (int64_t)r.tslot * kmax * wc;
                const bool first = r.kind == HS_INC_FIRST;
#pragma unroll
                for (int j = 0; j < WC; ++j) {
                    if (j >= wc) break;
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
            };
            // one item of phase 1 with its first kHsChunk columns in vv (no load in here)
            auto p1_item = [&](int k, const T (&vv)[kHsChunk]) {
                const RecS r = rec_lane(R0, k);
                if (k < S0.nlate) {
                    // late chunk: rows of this leaf times entries of the leaf solved just before
                    // (columns past the chunk masked, value and factor, without branches)
                    flops += 2.0 * n * r.n * wce;
#pragma unroll
                    for (int c = 0; c < kHsChunk; ++c) {
                        const bool keep = c < r.n;
                        const T a = keep ? vv[c] : T(0);
#pragma unroll
                        for (int j = 0; j < WC; ++j)
                            if (j < wc) {
                                const T xv = X[r.col0 + c + (int64_t)j * Nd];
                                acc[j] = fma_t(a, keep ? xv : T(0), acc[j]);
                            }
                    }
                } else {
                    // increment of t_B by the rows of the leaf solved just before
                    flops += 2.0 * r.n * rk[r.slot] * wce;
                    inc_chunk(r, vv, 0);
                }
            };
            // the prefetched items (static register indices, no load before their use) ...
#pragma unroll
            for (int i = 0; i < D::kP1; ++i) {
                const int k = wave + kHW * i;
                if (k < np1) p1_item(k, av1[i]);
            }
            // ... then, rarely, items beyond the prefetch depth and columns of ranks above kHsChunk
            for (int k = wave + kHW * D::kP1; k < np1; k += kHW) {
                const RecS r = rec_lane(R0, k);
                T vv[kHsChunk];
                if (k < S0.nlate) load_block(vv, arena, r.off, r.ld, n, r.n, 0, lane);
                else load_block(vv, arena, r.off, r.ld, r.n, rk[r.slot], 0, lane);
                consume(vv);
                p1_item(k, vv);
            }
            // (ranks reach past the first chunk only when the rank capacity does)
            for (int k = wave; kmax > kHsChunk && k < np1; k += kHW) {
                if (k < S0.nlate) continue;
                const RecS r = rec_lane(R0, k);
                const int rank = rk[r.slot];
                for (int cb = kHsChunk; cb < rank; cb += kHsChunk) {
                    T vv[kHsChunk];
                    load_block(vv, arena, r.off, r.ld, r.n, rank, cb, lane);
                    consume(vv);
                    inc_chunk(r, vv, cb);
                }
            }
            // every wavefront stores its partial sums (zeros without late chunks)
#pragma unroll
            for (int j = 0; j < WC; ++j)
                if (j < wc) part1[(wave * 64 + lane) * wc + j] = acc[j];
        }
        // the next step's phase-1 values, the records two steps ahead, the step after those
        prefetch1(S1, R1);
        R2 = load_recs(recs, S2, lane, steps);
        S3v = load_step(steps, s + 3, nsteps);
        __syncthreads();
        phase(6);
        // ---------------- phase 2
        if (wave < wce) {
            // solve: y = b - late partials - early partials; T^{-1} y with the leaf in registers
            const int j = wave;
            const int li = min(lane, n - 1);
            T y = X[S0.row0 + li + (int64_t)j * Nd];
            y = lane < n ? y : T(0);
            // every wavefront's partial sums, zero where it had nothing to add (all read at once)
            const T* p2 = part2 + (s & 1) * kHT * wc;
            T ps[2 * kHW];
#pragma unroll
            for (int w = 0; w < kHW; ++w) {
                ps[w] = part1[(w * 64 + lane) * wc + j];
                ps[kHW + w] = p2[(w * 64 + lane) * wc + j];
            }
#pragma unroll
            for (int w = 0; w < 2 * kHW; ++w) y -= ps[w];
            flops += (double)n * n;
            T x = y * dinv;
            // the staged triangle is zero outside the leaf, so blocks of 8 columns up to n need no
            // masks; the lane's row is read from LDS a block ahead of the substitution
            const T* drow = Dg2 + (s & 1) * kHsolveMaxRow * kHsolveMaxRow + lane;
            T cur[8], nxt[8];
            if (fwd) {
#pragma unroll
                for (int i = 0; i < 8; ++i) cur[i] = drow[i * kHsolveMaxRow];
#pragma unroll
                for (int cb = 0; cb < kHsolveMaxRow; cb += 8) {
                    if (cb >= n) break;
                    if (cb + 8 < kHsolveMaxRow)
#pragma unroll
                        for (int i = 0; i < 8; ++i) nxt[i] = drow[(cb + 8 + i) * kHsolveMaxRow];
#pragma unroll
                    for (int i = 0; i < 8; ++i) x -= cur[i] * lane_bcast(x, cb + i);
#pragma unroll
                    for (int i = 0; i < 8; ++i) cur[i] = nxt[i];
                }
            } else {
                const int top = ((n - 1) / 8) * 8;   // first block holding a column < n
#pragma unroll
                for (int i = 0; i < 8; ++i) cur[i] = drow[(top + i) * kHsolveMaxRow];
                for (int cb = top; cb >= 0; cb -= 8) {
                    if (cb >= 8)
#pragma unroll
                        for (int i = 0; i < 8; ++i) nxt[i] = drow[(cb - 8 + i) * kHsolveMaxRow];
#pragma unroll
                    for (int i = 7; i >= 0; --i) x -= cur[i] * lane_bcast(x, cb + i);
#pragma unroll
                    for (int i = 0; i < 8; ++i) cur[i] = nxt[i];
                }
            }
            // rows past the leaf store into the junk diagonal row
            *(lane < n ? X + S0.row0 + lane + (int64_t)j * Nd : Dd2 + 2 * kHsolveMaxRow + lane) = x;
            phase(8);   // thread 0 (a solving wavefront): the triangular solve done
        }
        if (helper) {
            const unsigned long long th0 = (d.prof && lane == 0 && hw == 0) ? wall_clock64() : 0ull;
            // the next leaf into LDS (loaded a step ago)
#pragma unroll
            for (int q = 0; q < D::kD; ++q) {
                const int c = hw + q * nh;
                if (c < kHsolveMaxRow) stage(dv[q], c, (s + 1) & 1);
            }
            if (hw == 0) Dd2[((s + 1) & 1) * kHsolveMaxRow + lane] = dvs;
            // early items: contributions to the next leaf's rows from leaves before this one
            const int m = S1.nrow, base = S0.nlate + S0.ninc;
            {
                T acc[WC];
#pragma unroll
                for (int j = 0; j < WC; ++j) acc[j] = T(0);
                // columns cb..cb+7 of an early item: element (c, j) of the right factor is
                // src[c * sc + j * sj] (dense chunk: x of an older leaf; low rank: t_B); columns from
                // `cols` on are masked, value and factor, without branches
                auto p2_chunk = [&](const RecS& r, const T (&vv)[kHsChunk], int cb, int cols) {
                    const bool dense = r.kind == HS_DENSE;
                    const T* src = dense ? X + r.col0 : tb + (int64_t)r.tslot * kmax * wc;
                    const int sc = dense ? 1 : wc;
                    const int64_t sj = dense ? (int64_t)Nd : 1;
#pragma unroll
                    for (int c = 0; c < kHsChunk; ++c) {
                        const bool keep = cb + c < cols;
                        const T a = keep ? vv[c] : T(0);
#pragma unroll
                        for (int j = 0; j < WC; ++j)
                            if (j < wc) {
                                const T xv = src[(int64_t)(cb + c) * sc + j * sj];
                                acc[j] = fma_t(a, keep ? xv : T(0), acc[j]);
                            }
                    }
                };
                auto cols_of = [&](const RecS& r) { return r.kind == HS_DENSE ? r.n : rk[r.slot]; };
                // the prefetched items first (no load before their use) ...
#pragma unroll
                for (int i = 0; i < D::kP2; ++i) {
                    const int e = hw + nh * i;
                    if (e < S0.nearly) {
                        const RecS r = rec_lane(R0, base + e);
                        const int cols = cols_of(r);
                        flops += 2.0 * m * cols * wce;
                        p2_chunk(r, av2[i], 0, cols);
                    }
                }
                // ... then, rarely, items beyond the prefetch depth and ranks above kHsChunk
                for (int e = hw + nh * D::kP2; e < S0.nearly; e += nh) {
                    const RecS r = rec_lane(R0, base + e);
                    const int cols = cols_of(r);
                    flops += 2.0 * m * cols * wce;
                    T vv[kHsChunk];
                    load_block(vv, arena, r.off, r.ld, m, cols, 0, lane);
                    consume(vv);
                    p2_chunk(r, vv, 0, cols);
                }
                for (int e = hw; kmax > kHsChunk && e < S0.nearly; e += nh) {
                    const RecS r = rec_lane(R0, base + e);
                    const int cols = cols_of(r);
                    for (int cb = kHsChunk; cb < cols; cb += kHsChunk) {
                        T vv[kHsChunk];
                        load_block(vv, arena, r.off, r.ld, m, cols, cb, lane);
                        consume(vv);
                        p2_chunk(r, vv, cb, cols);
                    }
                }
                // every helper stores (zeros without items); slots of non-helpers stay zero
                T* p2 = part2 + ((s + 1) & 1) * kHT * wc;
#pragma unroll
                for (int j = 0; j < WC; ++j)
                    if (j < wc) p2[(hw * 64 + lane) * wc + j] = acc[j];
            }
            // columns of the next leaf beyond the prefetch depth (chunks of several columns)
            for (int c = hw + D::kD * nh; c < kHsolveMaxRow; c += nh) {
                const T v = gmem(prep_of(s + 1))[lane + c * kHsolveMaxRow];
                asm volatile("" ::"v"(v));
                stage(v, c, (s + 1) & 1);
            }
            if (d.prof && lane == 0 && hw == 0) pt[3] += wall_clock64() - th0;   // the first helper
        }
        // every wavefront: the leaf after next, the next step's early values
        prefetch_diag(s + 2);
        prefetch2(S1, R1, S2.nrow);
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
    if (d.prof && (threadIdx.x == 0 || (lane == 0 && helper && hw == 0))) {
        for (int k = 0; k < 4; ++k)
            if (pt[k]) atomicAdd(&d.prof[2 * kOpCodes + 6 + k], pt[k]);
        if (threadIdx.x == 0) atomicAdd(&d.prof[2 * OP_TRSM + 1], (unsigned long long)nsteps);
    }
}

// Solve-ready diagonal leaf of each step (workgroup = step): forward, the strict lower triangle of
// the packed L\U leaf (L has a unit diagonal); backward, the strict upper triangle with row i
// multiplied by 1 / U_ii, and the row scales 1 / U_ii (the substitution then runs without a
// division or a mask). Zero outside the triangle and past the leaf's rows and columns.
template <class T>
__global__ void __launch_bounds__(256) k_hs_prepare(const T* __restrict__ arena, const HsStep* __restrict__ steps,
                                                   int nleaf, T* __restrict__ prep) {
    const int s = blockIdx.x;
    const HsStep st = steps[s];
    const bool fwd = s < nleaf;
    const int n = st.nrow;
    const T* D = arena + st.diag;
    T* P = prep + (int64_t)s * kHsPrepStride;
    for (int q = threadIdx.x; q < kHsolveMaxRow * kHsolveMaxRow; q += blockDim.x) {
        const int i = q % kHsolveMaxRow, c = q / kHsolveMaxRow;
        T v = T(0);
        if (i < n && c < n && (fwd ? c < i : c > i)) {
            v = D[i + (int64_t)c * n];
            if (!fwd) v = v * (T(1) / D[i + (int64_t)i * n]);
        }
        P[q] = v;
    }
    for (int i = threadIdx.x; i < kHsolveMaxRow; i += blockDim.x)
        P[kHsolveMaxRow * kHsolveMaxRow + i] = (fwd || i >= n) ? T(1) : T(1) / D[i + (int64_t)i * n];
}

template <class T, int WC, bool BF, bool GX>
__global__ void __launch_bounds__(kHT) k_hsolve(const Inst<T>* __restrict__ insts, int nchunk, int step) {
    extern __shared__ __align__(16) char smem[];
    const int i = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
    const Inst<T> d = insts[i];
    hsteps_body<T, WC, BF, GX>(d, c, step, smem);
}

template <class T, int WC, bool BF, bool GX>
__global__ void __launch_bounds__(kHT) k_hsolve_one(const Inst<T> d) {
    extern __shared__ __align__(16) char smem[];
    hsteps_body<T, WC, BF, GX>(d, blockIdx.x, 0, smem);
}

__global__ void k_to_bf16(const float* __restrict__ src, int64_t n, unsigned short* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned u = __float_as_uint(src[i]);
        // round to nearest, ties to even, on the upper 16 bits; NaN stays a (quiet) NaN
        const bool nan = (u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu);
        const unsigned r = nan ? (u | 0x00400000u) : u + 0x7fffu + ((u >> 16) & 1u);
        dst[i] = (unsigned short)(r >> 16);
    }
}

__global__ void k_from_bf16(const unsigned short* __restrict__ src, int64_t n, float* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = bf16_bits_to_float(src[i]);
}

template <class K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        FDE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)bytes));
}

}  // namespace

size_t hsolve_lds_bytes(int Nd, int tslots, int kmax, int nslots, int wc, size_t esz, bool global_rhs) {
    return ((global_rhs ? 0 : (size_t)Nd) + (size_t)tslots * kmax + 3 * kHT) * wc * esz +
           (size_t)(2 * kHsolveMaxRow + 3) * kHsolveMaxRow * esz + (size_t)nslots * sizeof(int) + 16;
}

size_t device_lds_limit(int device) {
    int v = 0;
    FDE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    return (size_t)v;
}

int device_cu_count(int device) {
    int v = 0;
    FDE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
    return std::max(v, 1);
}

namespace {

template <class T, int WC, bool BF, bool GX>
void launch_hsolve_wc(hipStream_t st, int ninst, int nchunk, const Inst<T>* d_insts, int step, size_t lds) {
    allow_lds(k_hsolve<T, WC, BF, GX>, lds);
    hipLaunchKernelGGL((k_hsolve<T, WC, BF, GX>), dim3(ninst * nchunk), dim3(kHT), lds, st, d_insts, nchunk, step);
    FDE_LAUNCH_CHECK();
}

template <class T, int WC, bool BF, bool GX>
void launch_hsolve_one_wc(hipStream_t st, const Inst<T>& d, int nchunk, size_t lds) {
    allow_lds(k_hsolve_one<T, WC, BF, GX>, lds);
    hipLaunchKernelGGL((k_hsolve_one<T, WC, BF, GX>), dim3(nchunk), dim3(kHT), lds, st, d);
    FDE_LAUNCH_CHECK();
}

template <class T, int WC>
void launch_hsolve_wc_bf(hipStream_t st, int ninst, int nchunk, const Inst<T>* d_insts, int step, size_t lds,
                         bool bf16, bool gx) {
    if constexpr (sizeof(T) == 4) {
        if (bf16) {
            if (gx) launch_hsolve_wc<T, WC, true, true>(st, ninst, nchunk, d_insts, step, lds);
            else launch_hsolve_wc<T, WC, true, false>(st, ninst, nchunk, d_insts, step, lds);
            return;
        }
    } else {
        if (bf16) fail(FDE_EINVAL, "BF16 low-rank factors come with FP32 factorisations only");
    }
    if (gx) launch_hsolve_wc<T, WC, false, true>(st, ninst, nchunk, d_insts, step, lds);
    else launch_hsolve_wc<T, WC, false, false>(st, ninst, nchunk, d_insts, step, lds);
}

template <class T, int WC>
void launch_hsolve_one_wc_bf(hipStream_t st, const Inst<T>& d, int nchunk, size_t lds, bool bf16, bool gx) {
    if constexpr (sizeof(T) == 4) {
        if (bf16) {
            if (gx) launch_hsolve_one_wc<T, WC, true, true>(st, d, nchunk, lds);
            else launch_hsolve_one_wc<T, WC, true, false>(st, d, nchunk, lds);
            return;
        }
    } else {
        if (bf16) fail(FDE_EINVAL, "BF16 low-rank factors come with FP32 factorisations only");
    }
    if (gx) launch_hsolve_one_wc<T, WC, false, true>(st, d, nchunk, lds);
    else launch_hsolve_one_wc<T, WC, false, false>(st, d, nchunk, lds);
}

}  // namespace

template <class T>
void launch_hs_prepare(hipStream_t st, const T* arena, const HsStep* steps, int nleaf, T* prep) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL((k_hs_prepare<T>), dim3(2 * nleaf), dim3(256), 0, st, arena, steps, nleaf, prep);
    FDE_LAUNCH_CHECK();
}
template void launch_hs_prepare<float>(hipStream_t, const float*, const HsStep*, int, float*);
template void launch_hs_prepare<double>(hipStream_t, const double*, const HsStep*, int, double*);

template <class T>
void launch_hsolve(hipStream_t st, int ninst, int nchunk, int wc, const Inst<T>* d_insts, int step, size_t lds,
                   bool bf16, bool gx) {
    if (ninst <= 0 || nchunk <= 0) return;
    switch (wc) {
        case 1: launch_hsolve_wc_bf<T, 1>(st, ninst, nchunk, d_insts, step, lds, bf16, gx); break;
        case 2: launch_hsolve_wc_bf<T, 2>(st, ninst, nchunk, d_insts, step, lds, bf16, gx); break;
        case 4: launch_hsolve_wc_bf<T, 4>(st, ninst, nchunk, d_insts, step, lds, bf16, gx); break;
        case 8: launch_hsolve_wc_bf<T, 8>(st, ninst, nchunk, d_insts, step, lds, bf16, gx); break;
        default: fail(FDE_EDEVICE, "H-solve chunk width %d is not 1, 2, 4 or 8", wc);
    }
}
template void launch_hsolve<float>(hipStream_t, int, int, int, const Inst<float>*, int, size_t, bool, bool);
template void launch_hsolve<double>(hipStream_t, int, int, int, const Inst<double>*, int, size_t, bool, bool);

template <class T>
void launch_hsolve_one(hipStream_t st, const Inst<T>& d, int nchunk, int wc, size_t lds, bool bf16, bool gx) {
    if (nchunk <= 0) return;
    switch (wc) {
        case 1: launch_hsolve_one_wc_bf<T, 1>(st, d, nchunk, lds, bf16, gx); break;
        case 2: launch_hsolve_one_wc_bf<T, 2>(st, d, nchunk, lds, bf16, gx); break;
        case 4: launch_hsolve_one_wc_bf<T, 4>(st, d, nchunk, lds, bf16, gx); break;
        case 8: launch_hsolve_one_wc_bf<T, 8>(st, d, nchunk, lds, bf16, gx); break;
        default: fail(FDE_EDEVICE, "H-solve chunk width %d is not 1, 2, 4 or 8", wc);
    }
}
template void launch_hsolve_one<float>(hipStream_t, const Inst<float>&, int, int, size_t, bool, bool);
template void launch_hsolve_one<double>(hipStream_t, const Inst<double>&, int, int, size_t, bool, bool);

void launch_to_bf16(hipStream_t st, const float* src, int64_t n, unsigned short* dst) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid), dim3(256), 0, st, src, n, dst);
    FDE_LAUNCH_CHECK();
}

void launch_from_bf16(hipStream_t st, const unsigned short* src, int64_t n, float* dst) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_from_bf16, dim3(grid), dim3(256), 0, st, src, n, dst);
    FDE_LAUNCH_CHECK();
}

}  // namespace fde
