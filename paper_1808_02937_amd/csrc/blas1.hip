// Small FP64 vector kernels used around the solver (lifting, Krylov updates).
#include "fde_internal.h"

namespace fde {

namespace {
__global__ void k_axpy_cols(int n, int ncol, double a, const double* __restrict__ x, int ldx,
                            double* __restrict__ y, int ldy) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * ncol) return;
    const int c = (int)(idx / n), i = (int)(idx % n);
    y[(int64_t)c * ldy + i] += a * x[(int64_t)c * ldx + i];
}
}  // namespace

void axpy_cols(hipStream_t st, int n, int ncol, double a, const double* x, int ldx, double* y, int ldy) {
    const int64_t tot = (int64_t)n * ncol;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, ncol, a, x,
                       ldx, y, ldy);
    FDE_LAUNCH_CHECK();
}

}  // namespace fde
