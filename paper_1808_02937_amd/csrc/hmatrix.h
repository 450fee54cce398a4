// H-matrix data structures, the op-list ("program") format of the device
// interpreter, and the generator that flattens the recursive H-LU and
// H-substitutions into that list.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "fde_internal.h"

namespace fde {

// --------------------------------------------------------------- trees
struct Cluster {
    int e0, e1;        // elements [e0, e1)
    int d0, d1;        // unknowns [d0, d1) in element-interleaved order
    double lo, hi;     // union of the supports of its basis functions
    int level;
    int child[2] = {-1, -1};
    bool leaf() const { return child[0] < 0; }
    int size() const { return d1 - d0; }
};

enum BlockKind { kDense = 0, kLowRank = 1, kHier = 2 };

struct Block {
    int kind;
    int tau, sigma;        // cluster ids (rows, cols)
    int child[4] = {-1, -1, -1, -1};   // 2 x 2, row-major
    // storage (element offsets in the factor arena)
    int64_t off = 0;       // dense: m x n column-major (ld = m)
    int64_t uoff = 0, voff = 0;   // low rank: U m x kmax (ld m), V n x kmax (ld n)
    int slot = -1;         // rank slot (low rank)
    int lr_id = -1;        // index among low-rank blocks
    bool lower = false;    // low rank: row cluster right of the column cluster
};

// per low-rank block: how its Taylor factors are formed (Section 3.1-3.2)
struct FactorSide {
    int singular;      // 1: c_nu-type (x-c)^{1-alpha-nu} side, 0: ((x-c)/r)^nu side
    double center, radius, sgn, mult;
    int cluster;
};

struct LowRankDesc {
    int block;
    FactorSide u, v;   // U rows (block rows), V rows (block cols)
};

// --------------------------------------------------------------- program
constexpr int kMaxKprime = 256;   // widest [U, X] recompressed in one OP_LRSUB

// OP_LRMV (H-substitutions): Y += alpha U (V^T X) for low-rank block blk, through temporary v[2]
enum OpCode { OP_GETRF = 1, OP_TRSM = 2, OP_GEMM = 3, OP_LRSUB = 4, OP_ZERO = 5, OP_LOAD = 6, OP_STORE = 7, OP_LRMV = 8 };
constexpr int kOpCodes = 9;
constexpr int kProfPhases = 10;            // small recompression phases, then H-solve step phases
constexpr int kProfSlots = 2 * kOpCodes + kProfPhases;   // per op code: wall-clock ticks, count; phases
enum Base { B_ARENA = 0, B_WORK = 1, B_RHS = 2, B_WORK_NRHS = 3 };

struct View {
    int base;          // B_ARENA (factors) or B_WORK (right-hand sides and temporaries)
    int rs, cs;        // element (i, j) at off + i*rs + j*cs
    int64_t off;
};

// a low-rank block as an op on it sees it: factor offsets in the arena, rows, columns, rank slot;
// rank >= 0 is its rank when the op runs (resolved on the device), -1 to read it from the slot
struct LRBlockDev {
    int64_t uoff, voff;
    int m, n, slot, rank;
};

struct OpRec {
    int code;
    int flags;         // TRSM: bit0 lower, bit1 unit diagonal
    int dim[3];        // m, n, k; >= 0 static, -1 = number of right-hand sides, <= -2: rank slot -2-d
    int blk;           // LRSUB: low-rank block id
    float alpha, beta; // GEMM
    View v[3];         // GEMM: C, A, B; TRSM: X, T; GETRF: A; LRSUB: X, Y; ZERO: X; LRMV: Y, X, t
    int64_t sofs_t;    // LRSUB: private scratch (elements of the factor type, then doubles)
    int64_t sofs_d;
    LRBlockDev lb;     // LRSUB, LRMV: block blk (filled in the device copy of a program)
};

struct TempRegion {
    int64_t off;       // element offset in the work space
    int rows, cols;    // column-major, ld = rows
};

struct Program {
    std::vector<OpRec> ops;
    int64_t work_elems = 0;   // temporaries (H-solve: in rows, times the number of right-hand sides)
    int kx_max = 0;           // widest update X Y^T recompressed into a low-rank block
    std::vector<TempRegion> temps;   // factorisation: every temporary, never reused before scheduling
    // level schedule (schedule_levels): ops[level_off[l] .. level_off[l+1]) are independent
    std::vector<int> level_off;
    std::vector<int> origin;         // program-order index of every scheduled op
    int64_t scr_t = 0, scr_d = 0;    // recompression scratch of one level (factor type, doubles)
    // dependencies (schedule_levels with_deps): scheduled op i may start once the scheduled ops
    // deps[dep_off[i] .. dep_off[i+1]) have finished (all earlier in the level order). They cover
    // every conflicting access to the same memory, temporaries sharing memory included; recompression
    // scratch is private to a level and not covered.
    std::vector<int> dep_off, deps;
};

// --------------------------------------------------------------- leaf-step H-solve
// The forward (L, unit lower) and backward (U) H-substitutions as 2 x (number of leaves)
// steps, pipelined by one leaf. Step p of a direction solves the leaf at position p:
//   phase 1: the contributions of leaf p-1 (solved in the step before) to the rows of leaf p
//            (chunks of <= kHsChunk columns of dense blocks), and the increments
//            t_B += V_B(rows of leaf p-1)^T x_{p-1} of the low-rank blocks whose column
//            cluster sigma holds leaf p-1;
//   phase 2: the triangular solve of leaf p and, meanwhile, every other contribution to the
//            rows of leaf p+1: dense chunks from leaves <= p-1 and rows U_B t_B of low-rank
//            blocks whose sigma ends at or before leaf p-1.
// The pipelining needs every low-rank block to couple leaves at least two apart, which holds
// when admissible clusters are separated by a cluster; the generator checks it.
constexpr int kHsChunk = 8;

enum HsKind { HS_DENSE = 0, HS_LOWRANK = 1, HS_INC_FIRST = 2, HS_INC = 3 };

struct HsRec {         // one unit of work of a step (32 bytes)
    int64_t off;       // dense: the chunk's first column; low rank: U_B (or V_B) at the leaf's first row
    int ld;            // leading dimension (dense: rows of the row leaf; U_B: |tau|; V_B: |sigma|)
    int col0;          // dense: x index of the chunk's first column; increment: x index of the leaf's first row
    int n;             // dense: columns (1..kHsChunk); increment: rows of the leaf; low rank: 0
    int slot;          // low rank and increments: rank slot of B
    int tslot;         // low rank and increments: t buffer slot of B
    int kind;          // HsKind
};

struct HsStep {        // 32 bytes
    int64_t diag;      // dense diagonal leaf (packed L\U), ld = nrow
    int row0, nrow;    // the leaf solved in this step
    int rec0;          // records [rec0, rec0 + nlate + ninc + nearly): late chunks, increments, early items
    int nlate, ninc, nearly;
};

struct HsTables {
    std::vector<HsStep> steps;   // forward (leaf order), then backward (reverse leaf order)
    std::vector<HsRec> recs;
    int nleaf = 0, tslots = 0, maxrow = 0, maxrec = 0;
    bool ok = false;             // false: the structure does not allow the pipelined steps
};

// --------------------------------------------------------------- H-matrix
// host-side trees and storage layout (copyable: each factorisation lays out its own copy)
struct HTree {
    Op* op = nullptr;
    int R = 8, leaf = 8;
    double lambda = 1.0;
    std::vector<int> h2p;          // internal index -> paper index
    std::vector<Cluster> cl;
    std::vector<Block> bl;
    int root = 0;
    std::vector<int> lr_blocks;    // block ids of low-rank leaves
    std::vector<int> dense_blocks;
    int kmax = 8;                  // rank capacity of U, V storage
    int64_t arena_elems = 0;
    int nslots = 0;
    int max_lr_rows = 0;           // largest m or n of a low-rank block
};

struct HMat {
    HTree t;
    std::vector<int> init_rank;    // rank of each low-rank block after the build (R or 0)
    // FP64 copy of A~ on the device in the layout of t (kmax = R)
    DevBuf<double> d_arena;
    DevBuf<int> d_h2p;
};

void gen_hsolve_steps(const HTree& hm, HsTables& tab);   // sets tab.ok
// every table entry inside the factor storage and the vector, before the tables reach the device
void validate_hsolve_steps(const HTree& hm, const HsTables& tab);

void build_trees(HTree* hm);
void assign_storage(HTree* hm, int kmax);
void build_hmatrix_device(HMat* hm);   // hbuild.hip

// program generation (progs.cpp)
void gen_hlu(const HTree& hm, Program& prog);
void gen_hsolve(const HTree& hm, Program& prog);
int lrsub_kprime_max(const HTree& hm, const Program& lu);
// scratch one OP_LRSUB needs at most (elements of the factor type, doubles)
void lrsub_need(const HTree& hm, const OpRec& o, int64_t* t_elems, int64_t* d_elems);
// schedule.cpp: reorder a factorisation program into levels of mutually independent ops
// (every op after all ops it conflicts with), give the temporaries memory by their level
// lifetimes and every OP_LRSUB private scratch within its level
// with_deps: also the per-op dependency lists (dep_off, deps; otherwise left empty)
void schedule_levels(const HTree& hm, Program& prog, bool with_deps);
// element-by-element check of a schedule against the program order it came from
// (host, slow: tests and diagnostics); fails with FDE_EDEVICE on a violated dependency
void check_schedule(const HTree& hm, const Program& original, const Program& scheduled);
void validate_program(const HTree& hm, const Program& prog, int64_t arena_elems, int64_t work_elems,
                      int nrhs_max, bool solve);

}  // namespace fde
