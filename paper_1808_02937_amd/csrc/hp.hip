// A polynomial degree per element (the space S_N^P with degrees P_i, Section 2.2).
//
// The bubbles psi_p = L_{p-1} - L_{p+1} do not depend on P_i, so the space with degrees P_i is
// spanned by a subset of the basis of the one-degree space with P = max P_i on the same mesh,
// and its system A_hp is the principal submatrix of that space's A on the unknowns it keeps.
// The operator is therefore built at the largest degree, on extended unknowns, and the other
// unknowns are decoupled: their rows and columns of every product are replaced by those of the
// identity. A vector that vanishes on them stays so under the products, under the H-matrix
// built the same way (rows and columns of the outside unknowns zeroed, unit diagonal), under its
// H-LU factors (the outside unknowns eliminate with pivot 1 and no coupling, so the factors
// restricted to the kept unknowns are those of A~_hp) and under every Krylov step. The public
// calls exchange vectors of the space's own Nd = sum P_i - 1 unknowns (its order: the bubbles
// element by element, then the hats) and scatter and gather them here.
#include "fde_internal.h"
#include "hbuild.h"

namespace fde {

namespace {

constexpr int kT = 256;

// Y = keep * Y + (1 - keep) * X on the extended unknowns (X null: 0)
__global__ void k_hp_decouple(int Nd, int nrhs, const double* __restrict__ keep, const double* __restrict__ X,
                              int ldx, double* __restrict__ Y, int ldy) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= (int64_t)Nd * nrhs) return;
    const int i = (int)(q % Nd), r = (int)(q / Nd);
    if (keep[i] == 0.0) Y[(int64_t)r * ldy + i] = X ? X[(int64_t)r * ldx + i] : 0.0;
}

__global__ void k_hp_zero(int Nd, int nrhs, double* __restrict__ Y, int ldy) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= (int64_t)Nd * nrhs) return;
    Y[(q / Nd) * ldy + q % Nd] = 0.0;
}

// Xe[map[i], r] = Xp[i, r]
__global__ void k_hp_scatter(int n, int nrhs, const int* __restrict__ map, const double* __restrict__ Xp, int ldp,
                             double* __restrict__ Xe, int lde) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= (int64_t)n * nrhs) return;
    const int i = (int)(q % n), r = (int)(q / n);
    Xe[(int64_t)r * lde + map[i]] = Xp[(int64_t)r * ldp + i];
}

// Xp[i, r] = Xe[map[i], r]
__global__ void k_hp_gather(int n, int nrhs, const int* __restrict__ map, const double* __restrict__ Xe, int lde,
                            double* __restrict__ Xp, int ldp) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= (int64_t)n * nrhs) return;
    const int i = (int)(q % n), r = (int)(q / n);
    Xp[(int64_t)r * ldp + i] = Xe[(int64_t)r * lde + map[i]];
}

// Ap[i, j] = Ae[map[i], map[j]] (column-major)
__global__ void k_hp_gather_matrix(int n, const int* __restrict__ map, const double* __restrict__ Ae, int lde,
                                   double* __restrict__ Ap, int ldp) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= (int64_t)n * n) return;
    const int i = (int)(q % n), j = (int)(q / n);
    Ap[(int64_t)j * ldp + i] = Ae[(int64_t)map[j] * lde + map[i]];
}

// one leaf per workgroup: the rows and columns of outside unknowns vanish (low rank: their rows
// of U and V), the diagonal entry of an outside unknown is 1
__global__ void k_hp_mask_leaves(const LeafDev* __restrict__ leaves, const int* __restrict__ ranks,
                                 const int* __restrict__ h2p, const double* __restrict__ keep,
                                 double* __restrict__ arena) {
    const LeafDev b = leaves[blockIdx.x];
    if (b.lowrank) {
        const int k = b.slot >= 0 ? ranks[b.slot] : 0;
        for (int q = threadIdx.x; q < b.m * k; q += blockDim.x) {
            const int i = q % b.m, l = q / b.m;
            if (keep[h2p[b.r0 + i]] == 0.0) arena[b.uoff + i + (int64_t)l * b.m] = 0.0;
        }
        for (int q = threadIdx.x; q < b.n * k; q += blockDim.x) {
            const int j = q % b.n, l = q / b.n;
            if (keep[h2p[b.c0 + j]] == 0.0) arena[b.voff + j + (int64_t)l * b.n] = 0.0;
        }
    } else {
        for (int q = threadIdx.x; q < b.m * b.n; q += blockDim.x) {
            const int i = q % b.m, j = q / b.m;
            const int r = b.r0 + i, c = b.c0 + j;
            if (keep[h2p[r]] == 0.0 || keep[h2p[c]] == 0.0) arena[b.off + q] = r == c ? 1.0 : 0.0;
        }
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void hp_decouple(Op* op, int nrhs, const double* X, int ldx, double* Y, int ldy, hipStream_t st) {
    const int64_t n = (int64_t)op->Nd * nrhs;
    if (!op->hp || n == 0) return;
    hipLaunchKernelGGL(k_hp_decouple, dim3(blocks_for(n)), dim3(kT), 0, st, op->Nd, nrhs, op->d_hp_keep.p, X, ldx, Y,
                       ldy);
    FDE_LAUNCH_CHECK();
}

void hp_scatter(Op* op, int nrhs, const double* Xp, int ldp, double* Xe, int lde, hipStream_t st) {
    const int64_t ne = (int64_t)op->Nd * nrhs, np = (int64_t)op->hp_nd * nrhs;
    if (ne == 0) return;
    hipLaunchKernelGGL(k_hp_zero, dim3(blocks_for(ne)), dim3(kT), 0, st, op->Nd, nrhs, Xe, lde);
    FDE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_hp_scatter, dim3(blocks_for(np)), dim3(kT), 0, st, op->hp_nd, nrhs, op->d_hp_map.p, Xp, ldp,
                       Xe, lde);
    FDE_LAUNCH_CHECK();
}

void hp_gather(Op* op, int nrhs, const double* Xe, int lde, double* Xp, int ldp, hipStream_t st) {
    const int64_t np = (int64_t)op->hp_nd * nrhs;
    if (np == 0) return;
    hipLaunchKernelGGL(k_hp_gather, dim3(blocks_for(np)), dim3(kT), 0, st, op->hp_nd, nrhs, op->d_hp_map.p, Xe, lde,
                       Xp, ldp);
    FDE_LAUNCH_CHECK();
}

void hp_gather_matrix(Op* op, const double* Ae, int lde, double* Ap, int ldp, hipStream_t st) {
    const int64_t n2 = (int64_t)op->hp_nd * op->hp_nd;
    if (n2 == 0) return;
    hipLaunchKernelGGL(k_hp_gather_matrix, dim3(blocks_for(n2)), dim3(kT), 0, st, op->hp_nd, op->d_hp_map.p, Ae, lde,
                       Ap, ldp);
    FDE_LAUNCH_CHECK();
}

void hp_mask_leaves(Op* op, int nleaf, const LeafDev* d_leaves, const int* d_ranks, const int* d_h2p, double* arena,
                    hipStream_t st) {
    if (!op->hp || nleaf == 0) return;
    hipLaunchKernelGGL(k_hp_mask_leaves, dim3(nleaf), dim3(kT), 0, st, d_leaves, d_ranks, d_h2p, op->d_hp_keep.p,
                       arena);
    FDE_LAUNCH_CHECK();
}

}  // namespace fde
