// Kernels of the batched, left-preconditioned BiCGSTAB (Section 4.2, eq. (precondsys)): the
// paper's iteration on A~^{-1} A X = A~^{-1} G, with the H-LU of A~ as the preconditioner. One
// 1024-thread workgroup per system (one right-hand side of one operator) for every reduction, so
// each system's arithmetic is independent of the rest of the batch.
//
// A step of van der Vorst's method, with M = A~^{-1}:
//   v = M A p;  alpha = rho / (rh . v);  s = r - alpha v;  x += alpha p;  stop if |s| <= tol |b|
//   t = M A s;  omega = (t . s) / (t . t);  x += omega s;  r = s - omega t;  stop if |r| <= tol |b|
//   rho' = rh . r;  beta = (rho' / rho)(alpha / omega);  p = r + beta (p - omega v)
// with b = M G, r_0 = rh = p_0 = b, x_0 = 0. The stopping test is on the preconditioned residual,
// as in the paper; the true residual |G - A x| / |G| is reported at the end.
#include <cmath>

#include "bicgstab.h"

namespace fde {

namespace {

constexpr int kT = 1024;
constexpr int kW = kT / 64;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// two sums over the workgroup in one round of barriers (deterministic order)
__device__ inline void block_sum2(double& a, double& b, double (*w)[2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) {
        w[wave][0] = a;
        w[wave][1] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < kW; ++q) {
        sa += w[q][0];
        sb += w[q][1];
    }
    __syncthreads();
    a = sa;
    b = sb;
}

__device__ inline double* col(double* base, const BicgDev& d) { return base + (int64_t)d.c * d.Nd; }

// r = b (already M G, or G itself without a preconditioner), rh = p = r, x = 0, |G|, |b|, rho
__global__ void __launch_bounds__(kT) k_bc_init(const BicgDev* __restrict__ sys, BicgState* __restrict__ ss,
                                                int maxit) {
    __shared__ double w[kW][2];
    const BicgDev d = sys[blockIdx.x];
    BicgState& s = ss[blockIdx.x];
    double* r = col(d.r, d);
    double* rh = col(d.rh, d);
    double* p = col(d.p, d);
    double gg = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double ri = r[i], gi = d.G[i];
        rh[i] = ri;
        p[i] = ri;
        d.X[i] = 0.0;
        gg += gi * gi;
        bb += ri * ri;
    }
    block_sum2(gg, bb, w);
    if (threadIdx.x == 0) {
        s.gnorm = sqrt(gg);
        s.bnorm = sqrt(bb);
        s.rho = bb;
        s.alpha = s.omega = 1.0;
        s.iters = 0;
        s.conv = 0;
        s.status = 0;
        s.relres = 1.0;
        s.active = 1;
        if (!(s.bnorm > 0.0) || !(s.gnorm > 0.0)) {   // zero right-hand side: x = 0 is the solution
            s.active = 0;
            s.conv = 1;
            s.relres = 0.0;
            if (!isfinite(bb) || !isfinite(gg)) s.status = -5;
        }
        if (maxit <= 0) s.active = 0;
    }
}

// first half: v = M A p is in place; alpha, s = r - alpha v, x += alpha p, test |s|
__global__ void __launch_bounds__(kT) k_bc_half1(const BicgDev* __restrict__ sys, BicgState* __restrict__ ss,
                                                 double tol) {
    __shared__ double w[kW][2];
    const BicgDev d = sys[blockIdx.x];
    BicgState& s = ss[blockIdx.x];
    if (!s.active) return;
    const double* v = col(d.v, d);
    const double* rh = col(d.rh, d);
    double rv = 0.0, dummy = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) rv += rh[i] * v[i];
    block_sum2(rv, dummy, w);
    const double alpha = s.rho / rv;
    if (!(rv != 0.0) || !isfinite(alpha)) {   // breakdown: (rh . v) vanished
        if (threadIdx.x == 0) {
            s.active = 0;
            s.status = -3;
        }
        return;
    }
    const double* r = col(d.r, d);
    const double* p = col(d.p, d);
    double* sv = col(d.s, d);
    double ss2 = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double si = r[i] - alpha * v[i];
        sv[i] = si;
        d.X[i] += alpha * p[i];
        ss2 += si * si;
    }
    block_sum2(ss2, dummy, w);
    if (threadIdx.x == 0) {
        s.alpha = alpha;
        const double rel = sqrt(ss2) / s.bnorm;
        if (rel <= tol) {   // converged at the half step: r = s
            s.relres = rel;
            s.iters += 1;
            s.conv = 1;
            s.active = 0;
        }
    }
}

// second half: t = M A s is in place; omega, x += omega s, r = s - omega t, test |r|, then p
__global__ void __launch_bounds__(kT) k_bc_half2(const BicgDev* __restrict__ sys, BicgState* __restrict__ ss,
                                                 double tol, int maxit) {
    __shared__ double w[kW][2];
    const BicgDev d = sys[blockIdx.x];
    BicgState& s = ss[blockIdx.x];
    if (!s.active) return;
    const double* t = col(d.t, d);
    const double* sv = col(d.s, d);
    double ts = 0.0, tt = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        ts += t[i] * sv[i];
        tt += t[i] * t[i];
    }
    block_sum2(ts, tt, w);
    const double omega = ts / tt;
    if (!(tt > 0.0) || !(omega != 0.0) || !isfinite(omega)) {   // breakdown: omega vanished
        if (threadIdx.x == 0) {
            s.active = 0;
            s.status = -3;
        }
        return;
    }
    double* r = col(d.r, d);
    const double* rh = col(d.rh, d);
    double rr = 0.0, rhr = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double si = sv[i];
        d.X[i] += omega * si;
        const double ri = si - omega * t[i];
        r[i] = ri;
        rr += ri * ri;
        rhr += rh[i] * ri;
    }
    block_sum2(rr, rhr, w);
    const double rel = sqrt(rr) / s.bnorm;
    const bool done = rel <= tol;
    const double beta = (rhr / s.rho) * (s.alpha / omega);
    if (!done) {
        double* p = col(d.p, d);
        const double* v = col(d.v, d);
        for (int i = threadIdx.x; i < d.Nd; i += kT) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    }
    if (threadIdx.x == 0) {
        s.omega = omega;
        s.rho = rhr;
        s.relres = rel;
        s.iters += 1;
        if (done) {
            s.conv = 1;
            s.active = 0;
        } else if (s.iters >= maxit || !(rhr != 0.0)) {
            s.active = 0;
            if (!(rhr != 0.0)) s.status = -3;
        }
    }
}

// copy src -> dst (column c of each system), for systems without a preconditioner (M = I)
__global__ void k_bc_copy(const BicgDev* __restrict__ sys, const int* __restrict__ mask, int which) {
    const BicgDev d = sys[blockIdx.y];
    if (!mask[blockIdx.y]) return;
    const double* src = which == 0 ? d.G : col(d.W, d);
    double* dst = which == 0 ? col(d.r, d) : (which == 1 ? col(d.v, d) : col(d.t, d));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.Nd; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void k_bc_count(const BicgState* __restrict__ ss, int ns, int* out) {
    __shared__ int w[kW];
    int a = 0;
    for (int i = threadIdx.x; i < ns; i += kT) a += ss[i].active;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < kW; ++q) t += w[q];
        *out = t;
    }
}

// true residual |G - A x| / |G| with A x in W
__global__ void __launch_bounds__(kT) k_bc_true(const BicgDev* __restrict__ sys, BicgState* __restrict__ ss) {
    __shared__ double w[kW][2];
    const BicgDev d = sys[blockIdx.x];
    BicgState& s = ss[blockIdx.x];
    const double* ax = col(d.W, d);
    double nn = 0.0, dummy = 0.0;
    for (int i = threadIdx.x; i < d.Nd; i += kT) {
        const double ri = d.G[i] - ax[i];
        nn += ri * ri;
    }
    block_sum2(nn, dummy, w);
    if (threadIdx.x == 0) {
        s.truerel = s.gnorm > 0.0 ? sqrt(nn) / s.gnorm : 0.0;
        if (!isfinite(s.truerel)) s.status = -5;
    }
}

}  // namespace

void bc_init(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, int maxit) {
    hipLaunchKernelGGL(k_bc_init, dim3(ns), dim3(kT), 0, st, sys, ss, maxit);
    FDE_LAUNCH_CHECK();
}
void bc_half1(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, double tol) {
    hipLaunchKernelGGL(k_bc_half1, dim3(ns), dim3(kT), 0, st, sys, ss, tol);
    FDE_LAUNCH_CHECK();
}
void bc_half2(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss, double tol, int maxit) {
    hipLaunchKernelGGL(k_bc_half2, dim3(ns), dim3(kT), 0, st, sys, ss, tol, maxit);
    FDE_LAUNCH_CHECK();
}
void bc_copy(hipStream_t st, int ns, const BicgDev* sys, const int* mask, int which) {
    hipLaunchKernelGGL(k_bc_copy, dim3(16, ns), dim3(256), 0, st, sys, mask, which);
    FDE_LAUNCH_CHECK();
}
void bc_count_active(hipStream_t st, int ns, const BicgState* ss, int* out) {
    hipLaunchKernelGGL(k_bc_count, dim3(1), dim3(kT), 0, st, ss, ns, out);
    FDE_LAUNCH_CHECK();
}
void bc_true_residual(hipStream_t st, int ns, const BicgDev* sys, BicgState* ss) {
    hipLaunchKernelGGL(k_bc_true, dim3(ns), dim3(kT), 0, st, sys, ss);
    FDE_LAUNCH_CHECK();
}

}  // namespace fde
