// Triangular solve with a dense leaf of at most 64 rows, one wavefront per right-hand-side
// column (shared by the H-LU and the H-substitutions).
//
// Lane i owns row i. The row is divided by its diagonal entry (lane-local), which turns the
// system into a unit triangular one; the lane's row of the scaled factor stays in registers
// for every column the wavefront solves, and each solved entry is broadcast with readlane,
// so the substitution itself touches neither LDS nor memory and needs no barrier. All factor
// loads are unconditional (addresses clamped into the leaf) so they are in flight together;
// the next column is loaded while the current one is solved.
#pragma once

#include <hip/hip_runtime.h>

namespace fde {

// global-memory view of a pointer: loads through it are vector-memory loads counted by vmcnt
// alone (a flat load also counts on the counter that LDS reads wait for)
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

__device__ inline float lane_bcast(float x, int s) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), s));
}
__device__ inline double lane_bcast(double x, int s) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), s);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane exchange within a row of 16 lanes through the DPP operand modifier (no LDS round trip).
// CTRL is a DPP control word: quad_perm(s0, s1, s2, s3) = s0 | s1 << 2 | s2 << 4 | s3 << 6
// (lane i of each quad reads lane s_i), row_ror(n) = 0x120 + n (lane i of each row reads lane
// (i + n) mod 16 of the row), row_newbcast(n) = 0x150 + n (every lane of each row reads lane n
// of the row).
constexpr int kDppXor1 = 0xB1;   // quad_perm(1, 0, 3, 2)
constexpr int kDppXor2 = 0x4E;   // quad_perm(2, 3, 0, 1)
constexpr int kDppRowMirror = 0x140;       // lane i of each row reads lane 15 - i of the row
constexpr int kDppRowHalfMirror = 0x141;   // lane i of each half row (8 lanes) reads lane 7 - i
constexpr int dpp_row_ror(int n) { return 0x120 + n; }
constexpr int dpp_row_newbcast(int n) { return 0x150 + n; }
template <int CTRL>
__device__ inline int dpp_move(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline float dpp_move(float x) {
    return __int_as_float(dpp_move<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ inline double dpp_move(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_move<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_move<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// X (n x w; element (i, j) at X[i*xrs + j*xcs]) <- T^{-1} X, T n x n (element (i, s) at
// Tm[i*trs + s*tcs]), lower or upper, unit diagonal or not; n <= 64. The calling wavefront
// `wave` of `nwaves` solves columns wave, wave + nwaves, ..., kTriCols of them at a time as
// independent chains (the broadcast of one column's solved entry overlaps the others' updates).
// Rows and steps beyond n carry zeros, so every wavefront runs all 64 steps without branches.
constexpr int kTriCols = 4;
template <class T>
__device__ inline void tri_wave(const T* Tm, int trs, int tcs, int n, bool lower, bool unit, T* X, int xrs, int xcs,
                                int w, int wave, int nwaves) {
    if (wave >= w || n <= 0) return;
    const int lane = threadIdx.x & 63;
    const bool act = lane < n;
    const int li = min(lane, n - 1);
    T tr[64];
#pragma unroll
    for (int s = 0; s < 64; ++s) tr[s] = Tm[(int64_t)li * trs + (int64_t)min(s, n - 1) * tcs];
    const T diag = Tm[(int64_t)li * trs + (int64_t)li * tcs];
    const T dinv = (!unit && act) ? T(1) / diag : T(1);
#pragma unroll
    for (int s = 0; s < 64; ++s) tr[s] = (s < n && act) ? tr[s] * dinv : T(0);
    for (int j0 = wave; j0 < w; j0 += nwaves * kTriCols) {
        T x[kTriCols];
#pragma unroll
        for (int c = 0; c < kTriCols; ++c) {
            const int j = min(j0 + c * nwaves, w - 1);
            x[c] = X[(int64_t)li * xrs + (int64_t)j * xcs];
        }
#pragma unroll
        for (int c = 0; c < kTriCols; ++c) x[c] = act ? x[c] * dinv : T(0);
        if (lower) {
#pragma unroll
            for (int s = 0; s < 64; ++s)
#pragma unroll
                for (int c = 0; c < kTriCols; ++c) {
                    const T xs = lane_bcast(x[c], s);
                    if (lane > s) x[c] -= tr[s] * xs;
                }
        } else {
#pragma unroll
            for (int s = 63; s >= 0; --s)
#pragma unroll
                for (int c = 0; c < kTriCols; ++c) {
                    const T xs = lane_bcast(x[c], s);
                    if (lane < s) x[c] -= tr[s] * xs;
                }
        }
#pragma unroll
        for (int c = 0; c < kTriCols; ++c) {
            const int j = j0 + c * nwaves;
            if (act && j < w) X[(int64_t)lane * xrs + (int64_t)j * xcs] = x[c];
        }
    }
}

}  // namespace fde
