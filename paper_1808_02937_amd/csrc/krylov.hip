// Kernels of the batched FGMRES: one 1024-thread workgroup per system (one
// right-hand side of one operator) for every reduction, so each system's
// arithmetic is independent of what else is in the batch (a result is the
// same alone and in a mix).
//
// Arnoldi step (fused): classical Gram-Schmidt against the basis, repeated
// once (CGS2), normalisation, Givens update of the Hessenberg column and of
// the residual estimate |g_{j+1}|.
#include <cmath>

#include "krylov.h"

namespace fde {

namespace {

constexpr int kT = 1024;   // a system's vectors (Nd up to tens of thousands) over 16 wavefronts
constexpr int kW = kT / 64;
constexpr int kChunk = 16;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Red {
    double w[kW][kChunk];
    double dots[kMaxRestart + 1];
    double s;
};

__device__ inline double block_sum(double v, Red& r) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) r.w[wave][0] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kW; ++w) s += r.w[w][0];
    __syncthreads();
    return s;
}

// dots[i] = v_i . w for i < nv (vectors v_i = base + i*stride), deterministic order
__device__ void block_dots(const double* base, int64_t stride, int nv, const double* w, int n, Red& r) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = 0; c0 < nv; c0 += kChunk) {
        const int cn = min(kChunk, nv - c0);
        double part[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) part[c] = 0.0;
        for (int i = threadIdx.x; i < n; i += kT) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < kChunk; ++c)
                if (c < cn) part[c] += base[(int64_t)(c0 + c) * stride + i] * wi;
        }
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            if (c < cn) {   // uniform: only the vectors of this chunk are reduced
                const double v = wave_sum(part[c]);
                if (lane == 0) r.w[wave][c] = v;
            }
        __syncthreads();
        if (threadIdx.x < cn) {
            double s = 0.0;
            for (int q = 0; q < kW; ++q) s += r.w[q][threadIdx.x];
            r.dots[c0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

__global__ void k_gnorm(const SysDev* __restrict__ sys, SysState* __restrict__ ss, const int* __restrict__ sel) {
    __shared__ Red r;
    const int slot = sel ? sel[blockIdx.x] : blockIdx.x;
    const SysDev d = sys[slot];
    double v = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) v += d.G[i] * d.G[i];
    v = block_sum(v, r);
    if (threadIdx.x == 0) {
        SysState& s = ss[slot];
        s.gnorm = sqrt(v);
        s.iters = 0;
        s.conv = 0;
        s.status = 0;
        s.active = 0;
        s.jend = 0;
        s.relres = 1.0;
        if (!(s.gnorm > 0.0)) {
            s.conv = 1;
            s.relres = 0.0;
            if (!(s.gnorm == 0.0)) s.status = -5;   // not finite
        }
    }
}

__global__ void k_zero_x(const SysDev* __restrict__ sys, const int* __restrict__ sel) {
    const SysDev d = sys[sel ? sel[blockIdx.y] : blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.Nd; i += gridDim.x * blockDim.x) d.X[i] = 0.0;
}

__global__ void k_cycle_start(const SysDev* __restrict__ sys, SysState* __restrict__ ss, int first, int maxit,
                              const int* __restrict__ sel) {
    __shared__ Red r;
    const int slot = sel ? sel[blockIdx.x] : blockIdx.x;
    const SysDev d = sys[slot];
    SysState& s = ss[slot];
    if (s.conv || s.iters >= maxit) {
        if (threadIdx.x == 0) s.active = 0;
        return;
    }
    double* v0 = d.V + (int64_t)d.c * d.Nd;
    const double* Rc = d.R + (int64_t)d.c * d.Nd;
    double nn = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double ri = d.G[i] - (first ? 0.0 : Rc[i]);
        v0[i] = ri;
        nn += ri * ri;
    }
    const double beta = sqrt(block_sum(nn, r));
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) v0[i] *= inv;
    if (threadIdx.x == 0) {
        for (int k = 0; k <= kMaxRestart; ++k) s.g[k] = 0.0;
        s.g[0] = beta;
        s.jend = 0;
        s.active = beta > 0.0 ? 1 : 0;
        s.est = beta;
    }
}

__global__ void k_copy_step(const SysDev* __restrict__ sys, const int* __restrict__ mask, int j,
                            const int* __restrict__ sel, const int* __restrict__ jv) {
    const int slot = sel ? sel[blockIdx.y] : blockIdx.y;
    const SysDev d = sys[slot];
    if (!mask[slot]) return;
    if (jv) j = jv[blockIdx.y];
    const double* v = d.V + (int64_t)j * d.bs + (int64_t)d.c * d.Nd;
    double* z = d.Z + (int64_t)j * d.bs + (int64_t)d.c * d.Nd;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.Nd; i += gridDim.x * blockDim.x) z[i] = v[i];
}

__global__ void __launch_bounds__(kT) k_arnoldi(const SysDev* __restrict__ sys, SysState* __restrict__ ss, int j,
                                                int m, double rtol, int maxit, const int* __restrict__ sel,
                                                const int* __restrict__ jv) {
    __shared__ Red r;
    __shared__ double hcol[kMaxRestart + 1];
    const int slot = sel ? sel[blockIdx.x] : blockIdx.x;
    if (jv) j = jv[blockIdx.x];
    const SysDev d = sys[slot];
    SysState& s = ss[slot];
    if (!s.active) return;
    const int n = d.Nd;
    double* w = d.W + (int64_t)d.c * n;
    const double* V0 = d.V + (int64_t)d.c * n;
    for (int pass = 0; pass < 2; ++pass) {
        block_dots(V0, d.bs, j + 1, w, n, r);
        for (int i = threadIdx.x; i < n; i += kT) {
            double acc = 0.0;
            for (int k = 0; k <= j; ++k) acc += r.dots[k] * V0[(int64_t)k * d.bs + i];
            w[i] -= acc;
        }
        if (threadIdx.x <= j) hcol[threadIdx.x] = (pass == 0 ? 0.0 : hcol[threadIdx.x]) + r.dots[threadIdx.x];
        __syncthreads();
    }
    double nn = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) nn += w[i] * w[i];
    const double hn = sqrt(block_sum(nn, r));
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    double* v1 = d.V + (int64_t)(j + 1) * d.bs + (int64_t)d.c * n;
    if (j + 1 < m + 1)
        for (int i = threadIdx.x; i < n; i += kT) v1[i] = w[i] * inv;
    if (threadIdx.x == 0) {
        hcol[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            const double t = s.cs[i] * hcol[i] + s.sn[i] * hcol[i + 1];
            hcol[i + 1] = -s.sn[i] * hcol[i] + s.cs[i] * hcol[i + 1];
            hcol[i] = t;
        }
        const double den = hypot(hcol[j], hcol[j + 1]);
        const double c = den > 0.0 ? hcol[j] / den : 1.0, sn = den > 0.0 ? hcol[j + 1] / den : 0.0;
        s.cs[j] = c;
        s.sn[j] = sn;
        hcol[j] = den;
        hcol[j + 1] = 0.0;
        for (int i = 0; i <= j + 1; ++i) s.H[i + j * (kMaxRestart + 1)] = hcol[i];
        s.g[j + 1] = -sn * s.g[j];
        s.g[j] = c * s.g[j];
        s.est = fabs(s.g[j + 1]);
        s.iters += 1;
        const bool done = !(s.est > rtol * s.gnorm) || j + 1 >= m || s.iters >= maxit || !(hn > 0.0) ||
                          !isfinite(s.est);
        if (done) {
            s.active = 0;
            s.jend = j + 1;
        }
    }
}

__global__ void k_count_active(const SysState* __restrict__ ss, int ns, int* out) {
    __shared__ Red r;
    double v = 0.0;
    for (int i = threadIdx.x; i < ns; i += kT) v += ss[i].active;
    v = block_sum(v, r);
    if (threadIdx.x == 0) *out = (int)v;
}

__global__ void k_update(const SysDev* __restrict__ sys, SysState* __restrict__ ss, const int* __restrict__ sel) {
    const int slot = sel ? sel[blockIdx.x] : blockIdx.x;
    const SysDev d = sys[slot];
    SysState& s = ss[slot];
    const int k = s.jend;
    if (k <= 0) return;
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double t = s.g[i];
            for (int l = i + 1; l < k; ++l) t -= s.H[i + l * (kMaxRestart + 1)] * s.y[l];
            s.y[i] = t / s.H[i + i * (kMaxRestart + 1)];
        }
    }
    __syncthreads();
    const double* Z0 = d.Z + (int64_t)d.c * d.Nd;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += s.y[l] * Z0[(int64_t)l * d.bs + i];
        d.X[i] += acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) s.jend = 0;
}

__global__ void k_check(const SysDev* __restrict__ sys, SysState* __restrict__ ss, double rtol,
                        const int* __restrict__ sel) {
    __shared__ Red r;
    const int slot = sel ? sel[blockIdx.x] : blockIdx.x;
    const SysDev d = sys[slot];
    SysState& s = ss[slot];
    if (s.conv) return;
    const double* Rc = d.R + (int64_t)d.c * d.Nd;
    double nn = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double ri = d.G[i] - Rc[i];
        nn += ri * ri;
    }
    const double rn = sqrt(block_sum(nn, r));
    if (threadIdx.x == 0) {
        s.relres = rn / s.gnorm;
        s.conv = s.relres <= rtol ? 1 : 0;
        if (!isfinite(s.relres)) s.status = -5;
    }
}

// compact status of the selected systems (one 32-byte record each) for the host
__global__ void k_gather_status(const SysState* __restrict__ ss, const int* __restrict__ sel, int n,
                                SysStatus* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const SysState& s = ss[sel ? sel[i] : i];
    out[i] = SysStatus{s.relres, s.active, s.conv, s.status, s.iters, s.jend, 0};
}

// Singular values of the m x m upper triangular R that the Arnoldi process of system 0 left in
// its Hessenberg storage (Givens-rotated, so R has the singular values of the (m+1) x m
// Hessenberg matrix): one-sided Jacobi on the columns of R in LDS, one 1024-thread workgroup,
// pairs of columns in 32 groups of 32 threads. out[0] = largest, out[1] = smallest.
__global__ void __launch_bounds__(kT) k_sigma_jacobi(const SysState* __restrict__ ss, int m, double* __restrict__ out) {
    __shared__ double Rm[kMaxRestart][kMaxRestart + 1];   // column c in Rm[c][.]
    __shared__ int flag;
    const SysState& s = ss[0];
    if (s.jend > 0 && s.jend < m) m = s.jend;   // the Krylov space was exhausted early
    for (int q = threadIdx.x; q < kMaxRestart * kMaxRestart; q += kT) {
        const int c = q / kMaxRestart, r = q % kMaxRestart;
        Rm[c][r] = (c < m && r <= c) ? s.H[r + c * (kMaxRestart + 1)] : 0.0;
    }
    __syncthreads();
    const int n2 = m + (m & 1), npairs = n2 / 2;
    const int grp = threadIdx.x / 32, gl = threadIdx.x % 32;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) flag = 0;
        __syncthreads();
        for (int round = 0; round < n2 - 1; ++round) {
            if (grp < npairs) {
                int p, q;
                if (grp == 0) {
                    p = round;
                    q = n2 - 1;
                } else {
                    p = (round + grp) % (n2 - 1);
                    q = (round - grp + n2 - 1) % (n2 - 1);
                }
                if (p < m && q < m) {
                    double a = 0.0, b = 0.0, g = 0.0;
                    for (int r = gl; r < m; r += 32) {
                        const double x = Rm[p][r], y = Rm[q][r];
                        a += x * x;
                        b += y * y;
                        g += x * y;
                    }
                    for (int o = 16; o > 0; o >>= 1) {
                        a += __shfl_xor(a, o, 32);
                        b += __shfl_xor(b, o, 32);
                        g += __shfl_xor(g, o, 32);
                    }
                    if (g != 0.0 && fabs(g) > 1e-15 * sqrt(a * b)) {
                        const double zeta = (b - a) / (2.0 * g);
                        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                        for (int r = gl; r < m; r += 32) {
                            const double x = Rm[p][r], y = Rm[q][r];
                            Rm[p][r] = cs * x - sn * y;
                            Rm[q][r] = sn * x + cs * y;
                        }
                        if (gl == 0) flag = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int rot = flag;
        __syncthreads();
        if (!rot) break;
    }
    if (threadIdx.x < 32) {
        double mx = 0.0, mn = 1e300;
        for (int c = threadIdx.x; c < m; c += 32) {
            double nn = 0.0;
            for (int r = 0; r < m; ++r) nn += Rm[c][r] * Rm[c][r];
            const double sv = sqrt(nn);
            mx = fmax(mx, sv);
            mn = fmin(mn, sv);
        }
        for (int o = 16; o > 0; o >>= 1) {
            mx = fmax(mx, __shfl_xor(mx, o, 32));
            mn = fmin(mn, __shfl_xor(mn, o, 32));
        }
        if (threadIdx.x == 0) {
            out[0] = mx;
            out[1] = mn;
        }
    }
}

}  // namespace

void fg_sigma(hipStream_t st, const SysState* ss, int m, double* out) {
    hipLaunchKernelGGL(k_sigma_jacobi, dim3(1), dim3(kT), 0, st, ss, m, out);
    FDE_LAUNCH_CHECK();
}

void fg_gnorm(hipStream_t st, int ns, const SysDev* sys, SysState* ss, const int* sel) {
    hipLaunchKernelGGL(k_gnorm, dim3(ns), dim3(kT), 0, st, sys, ss, sel);
    FDE_LAUNCH_CHECK();
}
void fg_zero_x(hipStream_t st, int ns, const SysDev* sys, const int* sel) {
    hipLaunchKernelGGL(k_zero_x, dim3(16, ns), dim3(256), 0, st, sys, sel);
    FDE_LAUNCH_CHECK();
}
void fg_cycle_start(hipStream_t st, int ns, const SysDev* sys, SysState* ss, int first, int maxit, const int* sel) {
    hipLaunchKernelGGL(k_cycle_start, dim3(ns), dim3(kT), 0, st, sys, ss, first, maxit, sel);
    FDE_LAUNCH_CHECK();
}
void fg_copy_step(hipStream_t st, int ns, const SysDev* sys, const int* mask, int j, const int* sel, const int* jv) {
    hipLaunchKernelGGL(k_copy_step, dim3(16, ns), dim3(256), 0, st, sys, mask, j, sel, jv);
    FDE_LAUNCH_CHECK();
}
void fg_arnoldi(hipStream_t st, int ns, const SysDev* sys, SysState* ss, int j, int m, double rtol, int maxit,
                const int* sel, const int* jv) {
    hipLaunchKernelGGL(k_arnoldi, dim3(ns), dim3(kT), 0, st, sys, ss, j, m, rtol, maxit, sel, jv);
    FDE_LAUNCH_CHECK();
}
void fg_count_active(hipStream_t st, int ns, const SysState* ss, int* out) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(kT), 0, st, ss, ns, out);
    FDE_LAUNCH_CHECK();
}
void fg_update(hipStream_t st, int ns, const SysDev* sys, SysState* ss, const int* sel) {
    hipLaunchKernelGGL(k_update, dim3(ns), dim3(kT), 0, st, sys, ss, sel);
    FDE_LAUNCH_CHECK();
}
void fg_check(hipStream_t st, int ns, const SysDev* sys, SysState* ss, double rtol, const int* sel) {
    hipLaunchKernelGGL(k_check, dim3(ns), dim3(kT), 0, st, sys, ss, rtol, sel);
    FDE_LAUNCH_CHECK();
}
void fg_gather_status(hipStream_t st, int n, const SysState* ss, const int* sel, SysStatus* out) {
    hipLaunchKernelGGL(k_gather_status, dim3((n + 255) / 256), dim3(256), 0, st, ss, sel, n, out);
    FDE_LAUNCH_CHECK();
}

}  // namespace fde
