// Launchers and device tables of the H-matrix construction.
#pragma once

#include "hmatrix.h"

namespace fde {

struct DenseBlkDev {   // dense leaf: rows [r0, r0+m), cols [c0, c0+n) of the internal order
    int64_t off;
    int r0, c0, m, n;
};

struct FacSideDev {    // one factor (U or V) of a low-rank leaf
    int64_t off;       // destination, column-major, ld = rows
    int d0, rows;      // internal indices [d0, d0+rows)
    int sing, alt;     // sing: mult*coef_nu*r^nu*(sgn(x-c))^{1-alpha-nu}; else mult*((x-c)/r)^nu
    double c, r, sgn, mult;
    int nq, pad;       // Gauss-Legendre nodes per element
};

struct SegDev {        // contiguous copy with conversion
    int64_t src, dst, len;
};

struct LeafDev {       // leaf block for reconstruction
    int64_t off, uoff, voff;
    int r0, c0, m, n, lowrank, slot;
};

// blocks of at most max_elems entries
void launch_hbuild_dense(Op* op, int nblk, int max_elems, const DenseBlkDev* d_blks, const int* d_h2p, double* arena);
// sides: host copy of the table at d_sides (the launch splits every side into chunks of rows)
void launch_hbuild_factors(Op* op, int R, const std::vector<FacSideDev>& sides, const FacSideDev* d_sides,
                           double* arena);
template <class S, class D>
void launch_segcopy(hipStream_t st, int nseg, const SegDev* d_segs, const S* src, D* dst);
template <class T>
void launch_to_dense(hipStream_t st, int nleaf, const LeafDev* d_leaves, const T* arena, const int* ranks,
                     const int* perm, double* out, int ld);
// degree per element (hp.hip): leaves of an H-matrix built at the largest degree with the rows
// and columns of the outside unknowns zeroed and their diagonal entries 1 (h2p: internal ->
// extended paper index)
void hp_mask_leaves(Op* op, int nleaf, const LeafDev* d_leaves, const int* d_ranks, const int* d_h2p, double* arena,
                    hipStream_t st);

}  // namespace fde
