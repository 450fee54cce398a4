// Device interpreter of H-arithmetic programs (H-LU and H-substitutions).
#pragma once

#include "hmatrix.h"

namespace fde {

constexpr int kInterpThreads = 256;
constexpr int kMaxKp = kMaxKprime;

template <class T>
struct Inst {
    const OpRec* ops;
    int nops;
    T* arena;                 // factors
    T* work;                  // temporaries
    T* rhs;                   // right-hand sides (Nd x nrhs, ld Nd) of an H-solve
    int* ranks;               // rank per low-rank block
    T* scr;                   // recompression scratch (T); each OP_LRSUB uses its own part
    double* scrd;             // recompression scratch (FP64 core)
    const int* h2p;
    int Nd;
    const double* B;          // H-solve input (paper order, FP64); B + step * bstep at step `step`
    int ldb;
    double* X;                // H-solve output; X + step * xstep
    int ldx;
    int64_t bstep, xstep;
    int nrhs;
    int nslots;               // low-rank blocks (rank slots)
    int work_rows;            // H-solve temporaries, rows (times the number of right-hand sides)
    const HsStep* hs_steps;   // leaf-step H-solve: 2 * hs_nleaf steps and their records
    const HsRec* hs_recs;
    int hs_nleaf, hs_tslots;
    int hs_wc;                // leaf-step H-solve: columns per workgroup (1, 2, 4 or 8)
    const T* hs_prep;         // leaf-step H-solve: 2 * hs_nleaf solve-ready diagonal leaves (kHsPrepStride each)
    const unsigned short* lr16;   // BF16 low-rank factors (bits), or nullptr: factor offsets >= lr_base
    int64_t lr_base;              // are read from lr16 + (offset - lr_base) (the U, V tail of the arena)
    double tol;
    int kmax;
    double pivot_floor;
    int* status;              // [0] status code, [1] op index of a breakdown
    unsigned long long* prof; // optional: per op code, [2c] wall-clock ticks, [2c+1] count
    double* flops;            // executed floating-point operations (accumulated by thread 0)
    double* op_flops;         // if set: op pc adds its operations to op_flops[pc] (no shared counter)
};

// FDE_PROFILE_OPS=1 in the environment: time every interpreter op by type
bool profile_ops_enabled();
void print_op_profile(const char* what, const unsigned long long* host_prof, int device);

// serial: one workgroup runs the whole op list of each instance (variant as for launch_level;
// a factorisation run serially and by levels uses the same variant, so both give the same bits)
template <class T>
void launch_interp(hipStream_t st, int ninst, const Inst<T>* d_insts, int step = 0, int variant = 0);
template <class T>
void launch_interp_one(hipStream_t st, const Inst<T>& d);
// H-solve with the right-hand sides in LDS: workgroup b solves columns [c*w, c*w + w) of
// instance b / nchunk (c = b % nchunk, w = its hs_wc <= wc, wc in {1, 2, 4, 8}); lds_bytes
// from hsolve_lds_bytes, the largest over the instances
// the solve-ready diagonal leaves of every leaf step (2 * nleaf of them) from the factors
template <class T>
void launch_hs_prepare(hipStream_t st, const T* arena, const HsStep* steps, int nleaf, T* prep);
// bf16: some instance reads BF16 low-rank factors (FP32 only); gx: the right-hand sides stay in
// each instance's global workspace d.rhs (Nd x (nchunk wc) at least) instead of LDS
template <class T>
void launch_hsolve(hipStream_t st, int ninst, int nchunk, int wc, const Inst<T>* d_insts, int step,
                   size_t lds_bytes, bool bf16 = false, bool gx = false);
template <class T>
void launch_hsolve_one(hipStream_t st, const Inst<T>& d, int nchunk, int wc, size_t lds_bytes, bool bf16 = false,
                       bool gx = false);
// dst[i] = src[i] rounded to BF16 (nearest, ties to even), and back to FP32
void launch_to_bf16(hipStream_t st, const float* src, int64_t n, unsigned short* dst);
void launch_from_bf16(hipStream_t st, const unsigned short* src, int64_t n, float* dst);
// LDS bytes of one workgroup of the leaf-step H-solve for wc columns
size_t hsolve_lds_bytes(int Nd, int tslots, int kmax, int nslots, int wc, size_t esz, bool global_rhs = false);
constexpr int kHsolveMaxRow = 64;   // leaf-step H-solve: leaves of at most this many rows
constexpr int kHsolveMaxCols = 8;
// leaf-step H-solve: per step, its diagonal leaf in solve-ready form (64 x 64, column-major, the
// strict lower triangle of L forward, the strict upper triangle of U with each row divided by its
// diagonal entry backward, zero elsewhere), then 64 row scales (1 forward, 1/U_ii backward, 1
// past the leaf)
constexpr int kHsPrepStride = kHsolveMaxRow * kHsolveMaxRow + kHsolveMaxRow;
// largest dynamic LDS of one workgroup on the device (bytes)
size_t device_lds_limit(int device);
int device_cu_count(int device);

// one op of a factorisation in a batch: its record (in the instance's device program), the
// instance and the op's index in its program
struct LevelTask {
    const OpRec* op;
    int inst, pc;
};

// one level of level-scheduled programs: workgroup b runs op tasks[b].pc of instance tasks[b].inst.
// variant: widest recompression the programs can need -- 16 or 32 (small path only), 0 (any)
template <class T>
void launch_level(hipStream_t st, int ntasks, const Inst<T>* d_insts, const LevelTask* d_tasks, int variant);

}  // namespace fde
