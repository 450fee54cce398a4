// H-matrix construction on the device (Section 3), FP64.
//
// Dense blocks hold the exact entries of A = rho M + S (text after eq.
// (approxmat)); low-rank blocks hold the factors of the truncated Taylor
// expansion of (t-s)^{1-alpha} (eq. (eqn:Lexpan)):
//   Q_{i,nu} = gamma0 int h_nu(t) phi_i'(t) dt,   W_{j,nu} = int g_nu(s) phi_j'(s) ds
// (Section 3.2), each integral a Gauss-Legendre sum over the one or two
// elements supporting phi_i. Powers are normalised by the expansion
// cluster's radius r, (s - s0)^nu -> ((s - s0)/r)^nu with r^nu moved to the
// other factor, so both factors stay O(1) in FP32.
#include "hbuild.h"
#include "sem_device.h"

namespace fde {

namespace {

// workgroup (x, y): entries [y kDenseChunk, (y + 1) kDenseChunk) of block x (a few entries per
// thread: each entry is a chain of dependent loads, so many workgroups hide their latency)
constexpr int kDenseChunk = 1024;
__global__ void k_hbuild_dense(SemDev s, const DenseBlkDev* __restrict__ blks, const int* __restrict__ h2p,
                               double* __restrict__ arena) {
    const DenseBlkDev b = blks[blockIdx.x];
    const int q1 = min(b.m * b.n, (int)(blockIdx.y + 1) * kDenseChunk);
    for (int q = blockIdx.y * kDenseChunk + threadIdx.x; q < q1; q += blockDim.x) {
        const int i = q % b.m, j = q / b.m;
        arena[b.off + q] = sem_entry(s, h2p[b.r0 + i], h2p[b.c0 + j]);
    }
}

// One thread per row of a factor side, a workgroup per chunk of kRowsPerChunk rows of one side
// (sides range from a leaf to half the matrix, so chunks keep the workgroups even); all R
// expansion terms of the row at once: at each quadrature node the first power is one pow()
// (none for the regular side's nu = 0) and the following ones come by repeated multiplication
// with the same ratio ((x-c)/r, or 1/(sgn(x-c)) for the singular side). The workgroup first
// stages its Gauss-Legendre rule and the Legendre values L_m(x_k), m <= P, in LDS, so the node
// loop reads neither memory nor a recurrence.
constexpr int kNuChunk = 16;
constexpr int kRowsPerChunk = 128;
constexpr int kFacMaxP = 32;
__global__ void __launch_bounds__(kRowsPerChunk) k_hbuild_factors(int P, int R, double alpha,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ h,
                                                                  const double* __restrict__ gl,
                                                                  const FacSideDev* __restrict__ sides,
                                                                  const int2* __restrict__ chunks,
                                                                  double* __restrict__ arena) {
    __shared__ double s_x[kMaxGL], s_w[kMaxGL], s_leg[(kFacMaxP + 1) * kMaxGL];
    const int2 ch = chunks[blockIdx.x];
    const FacSideDev f = sides[ch.x];
    const int nq = min(kMaxGL, f.nq);   // chosen per side on the host
    const int off_n = nq * (nq - 1) / 2;
    const int wbase = kMaxGL * (kMaxGL + 1) / 2;
    for (int k = threadIdx.x; k < nq; k += blockDim.x) {
        const double xk = gl[off_n + k];
        s_x[k] = xk;
        s_w[k] = gl[wbase + off_n + k];
        double pm = 1.0, pc = xk;   // L_0, L_1
        s_leg[k] = 1.0;
        if (P >= 1) s_leg[kMaxGL + k] = xk;
        for (int m = 1; m < P; ++m) {
            const double pn = ((2 * m + 1) * xk * pc - m * pm) / (m + 1);
            pm = pc;
            pc = pn;
            s_leg[(m + 1) * kMaxGL + k] = pc;
        }
    }
    __syncthreads();
    const int i = ch.y + threadIdx.x;
    if (i >= f.rows) return;
    if (f.mult == 0.0) {
        for (int nu = 0; nu < R; ++nu) arena[f.off + i + (int64_t)nu * f.rows] = 0.0;
        return;
    }
    const int d = f.d0 + i;
    const int e = d / P, l = d % P;
    int ne, el[2], mm[2];
    double cf[2];
    if (l < P - 1) {
        ne = 1;
        el[0] = e;
        mm[0] = l + 1;
        cf[0] = -(2.0 * (l + 1) + 1.0) * 2.0 / h[e];
    } else {
        ne = 2;
        el[0] = e;
        mm[0] = 0;
        cf[0] = 1.0 / h[e];
        el[1] = e + 1;
        mm[1] = 0;
        cf[1] = -1.0 / h[e + 1];
    }
    for (int nu0 = 0; nu0 < R; nu0 += kNuChunk) {
        double acc[kNuChunk];
#pragma unroll
        for (int u = 0; u < kNuChunk; ++u) acc[u] = 0.0;
        for (int a = 0; a < ne; ++a) {
            const int ee = el[a];
            const double xl = x[ee], he = h[ee];
            const double scale = cf[a] * 0.5 * he;
            const double* leg = s_leg + mm[a] * kMaxGL;
            for (int k = 0; k < nq; ++k) {
                const double xr = s_x[k], w = s_w[k];
                const double xx = xl + 0.5 * he * (1.0 + xr);
                double F, step;
                if (f.sing) {
                    const double b = f.sgn * (xx - f.c);
                    F = pow(b, 1.0 - alpha - nu0);
                    step = 1.0 / b;
                } else {
                    const double b = (xx - f.c) / f.r;
                    F = nu0 == 0 ? 1.0 : pow(b, (double)nu0);
                    step = b;
                }
                const double wl = scale * w * leg[k];
#pragma unroll
                for (int u = 0; u < kNuChunk; ++u) {
                    acc[u] += wl * F;
                    F *= step;
                }
            }
        }
        for (int u = 0; u < kNuChunk && nu0 + u < R; ++u) {
            const int nu = nu0 + u;
            double coef = 1.0;
            if (f.sing) {
                for (int k = 1; k <= nu; ++k) coef *= (alpha + k - 2.0) / k;
                if (f.alt && (nu & 1)) coef = -coef;
                coef *= pow(f.r, (double)nu);
            }
            arena[f.off + i + (int64_t)nu * f.rows] = acc[u] * f.mult * coef;
        }
    }
}

template <class S, class D>
__global__ void k_segcopy(const S* __restrict__ src, D* __restrict__ dst, const SegDev* __restrict__ segs) {
    const SegDev sg = segs[blockIdx.x];
    for (int64_t q = threadIdx.x; q < sg.len; q += blockDim.x) dst[sg.dst + q] = (D)src[sg.src + q];
}

template <class T>
__global__ void k_to_dense(const T* __restrict__ arena, const int* __restrict__ ranks,
                           const LeafDev* __restrict__ leaves, const int* __restrict__ perm, int unit_lower,
                           double* __restrict__ out, int ld) {
    const LeafDev b = leaves[blockIdx.x];
    const int k = b.slot >= 0 ? ranks[b.slot] : 0;
    for (int q = threadIdx.x; q < b.m * b.n; q += blockDim.x) {
        const int i = q % b.m, j = q / b.m;
        double v;
        if (b.lowrank) {
            v = 0.0;
            for (int l = 0; l < k; ++l)
                v += (double)arena[b.uoff + i + (int64_t)l * b.m] * (double)arena[b.voff + j + (int64_t)l * b.n];
        } else {
            v = (double)arena[b.off + q];
        }
        int r = b.r0 + i, c = b.c0 + j;
        (void)unit_lower;
        if (perm) {
            r = perm[r];
            c = perm[c];
        }
        out[(int64_t)c * ld + r] = v;
    }
}

}  // namespace

void launch_hbuild_dense(Op* op, int nblk, int max_elems, const DenseBlkDev* d_blks, const int* d_h2p,
                         double* arena) {
    if (nblk == 0 || max_elems <= 0) return;
    const unsigned chunks = (unsigned)((max_elems + kDenseChunk - 1) / kDenseChunk);
    hipLaunchKernelGGL(k_hbuild_dense, dim3(nblk, chunks), dim3(256), 0, op->ctx->stream, sem_dev(op), d_blks,
                       d_h2p, arena);
    FDE_LAUNCH_CHECK();
}

void launch_hbuild_factors(Op* op, int R, const std::vector<FacSideDev>& sides, const FacSideDev* d_sides,
                           double* arena) {
    if (sides.empty()) return;
    if (op->P > kFacMaxP) fail(FDE_EUNSUPPORTED, "H-matrix factors: P <= %d (got %d)", kFacMaxP, op->P);
    std::vector<int2> chunks;
    for (size_t k = 0; k < sides.size(); ++k)
        for (int r0 = 0; r0 < sides[k].rows; r0 += kRowsPerChunk) chunks.push_back(make_int2((int)k, r0));
    if (chunks.empty()) return;
    DevBuf<int2> d_chunks;
    d_chunks.alloc(op->ctx, chunks.size());
    upload(op->ctx, d_chunks.p, chunks.data(), chunks.size() * sizeof(int2));
    hipLaunchKernelGGL(k_hbuild_factors, dim3((unsigned)chunks.size()), dim3(kRowsPerChunk), 0, op->ctx->stream,
                       op->P, R, op->alpha, op->d_x.p, op->d_h.p, op->ctx->gl.p, d_sides, d_chunks.p, arena);
    FDE_LAUNCH_CHECK();
}

template <class S, class D>
void launch_segcopy(hipStream_t st, int nseg, const SegDev* d_segs, const S* src, D* dst) {
    if (nseg == 0) return;
    hipLaunchKernelGGL((k_segcopy<S, D>), dim3(nseg), dim3(256), 0, st, src, dst, d_segs);
    FDE_LAUNCH_CHECK();
}
template void launch_segcopy<double, double>(hipStream_t, int, const SegDev*, const double*, double*);
template void launch_segcopy<double, float>(hipStream_t, int, const SegDev*, const double*, float*);

template <class T>
void launch_to_dense(hipStream_t st, int nleaf, const LeafDev* d_leaves, const T* arena, const int* ranks,
                     const int* perm, double* out, int ld) {
    if (nleaf == 0) return;
    hipLaunchKernelGGL((k_to_dense<T>), dim3(nleaf), dim3(256), 0, st, arena, ranks, d_leaves, perm, 0, out, ld);
    FDE_LAUNCH_CHECK();
}
template void launch_to_dense<double>(hipStream_t, int, const LeafDev*, const double*, const int*, const int*,
                                      double*, int);
template void launch_to_dense<float>(hipStream_t, int, const LeafDev*, const float*, const int*, const int*,
                                     double*, int);

}  // namespace fde
