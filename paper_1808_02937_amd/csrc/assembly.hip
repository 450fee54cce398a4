// Element-pair moment blocks of the SEM stiffness matrix (FP64, gfx950).
//
// Section 2.2 with the kernel form of the weak form (Section 2.1) and the
// entry formula of Section 3.2: every basis derivative is a Legendre series
// on each element (psi_p' = -(2p+1) L_p), so S_l = D^T K D with
//   K^{ef}_{mn} = gamma0 int_{I_e} int_{I_f} (t-s)_+^{1-alpha} L_m(xi_e(t)) L_n(xi_f(s)) ds dt.
// One 64-lane wavefront computes one P x P block:
//   same element  : Duffy map s = t - (1+xi) w, tensor Gauss-Jacobi (exact);
//   adjacent      : square split on its diagonal, Duffy map per triangle,
//                   Gauss-Jacobi in the radial variable, Gauss-Legendre panels
//                   graded toward the nearest singular point in the angle;
//   separated     : tensor Gauss-Legendre on panels graded geometrically
//                   toward the gap, the node count per panel from the
//                   Bernstein-ellipse bound of the kernel.
// The far-field blocks are pow-bound FP64 ALU work; each is staged through LDS
// as (weights * kernel) -> (Legendre_t * .) -> (. * Legendre_s) contractions.
#include <algorithm>
#include <cmath>

#include "fde_internal.h"
#include "sem_device.h"

namespace fde {

namespace {

constexpr int kWave = 64;
constexpr int kMaxPanelNodes = 48;   // a graded panel never needs more (rho >= 3.7)
constexpr int kMaxP = 32;
constexpr int kAccPerLane = (kMaxP * kMaxP + kWave - 1) / kWave;

struct Geo {
    double he, hf, gap;  // element sizes and the gap between them (gap < 0: not separated)
    int kind;            // 0 same element, 1 adjacent, 2 separated
};

__device__ inline double legendre(int n, double x) {
    if (n == 0) return 1.0;
    double pm = 1.0, p = x;
    for (int k = 1; k < n; ++k) {
        const double pn = ((2 * k + 1) * x * p - k * pm) / (k + 1);
        pm = p;
        p = pn;
    }
    return p;
}

// nodes for a panel of length len whose nearest singular point lies dist beyond
// its start; error target ~1e-16 for a kernel times a degree-(P-1) polynomial
__device__ inline int panel_nodes(double len, double dist, int P) {
    const double a = 1.0 + 2.0 * dist / len;
    const double rho = a + sqrt(a * a - 1.0);
    int n = (int)ceil(0.5 * (P - 1 + 36.8 / log(rho))) + 1;
    if (n < 1) n = 1;
    if (n > kMaxPanelNodes) n = kMaxPanelNodes;
    return n;
}

// panel j of [0, len] graded toward 0 with gap g: [g(2^j-1), g(2^{j+1}-1)] clipped
__device__ inline int panel_count(double len, double g) {
    if (g >= len) return 1;
    int j = 0;
    while (g * (exp2((double)(j + 1)) - 1.0) < len) ++j;
    return j + 1;
}
__device__ inline void panel_bounds(double len, double g, int j, double* lo, double* hi) {
    if (g >= len) {
        *lo = 0.0;
        *hi = len;
        return;
    }
    *lo = g * (exp2((double)j) - 1.0);
    const double h = g * (exp2((double)(j + 1)) - 1.0);
    *hi = h < len ? h : len;
}

__device__ inline void gl_rule(const double* gl, int n, int i, double lo, double hi, double* x,
                               double* w) {
    const int off = n * (n - 1) / 2;
    const double xr = gl[off + i];
    const double wr = gl[kMaxGL * (kMaxGL + 1) / 2 + off + i];
    *x = 0.5 * (hi - lo) * xr + 0.5 * (hi + lo);
    *w = 0.5 * (hi - lo) * wr;
}

// shared memory layout for one wavefront
struct Smem {
    double* Lt;   // P x kMaxPanelNodes
    double* Ls;   // P x kMaxPanelNodes
    double* T;    // P x kMaxPanelNodes
    double* Kw;   // kMaxPanelNodes^2
    double* nodes; // 4 x kMaxPanelNodes
};

__device__ void block_separated(const Geo& g, int P, double alpha, double gamma0,
                                const double* gl, Smem sm, double* acc) {
    const int lane = threadIdx.x;
    const int pt = panel_count(g.he, g.gap);
    const int ps = panel_count(g.hf, g.gap);
    double* tu = sm.nodes;                         // t-panel nodes u = t - x_e and weights
    double* tw = sm.nodes + kMaxPanelNodes;
    double* sv = sm.nodes + 2 * kMaxPanelNodes;    // s-panel nodes v = x_{f+1} - s and weights
    double* sw = sm.nodes + 3 * kMaxPanelNodes;
    for (int jt = 0; jt < pt; ++jt) {
        double tlo, thi;
        panel_bounds(g.he, g.gap, jt, &tlo, &thi);
        for (int js = 0; js < ps; ++js) {
            double slo, shi;
            panel_bounds(g.hf, g.gap, js, &slo, &shi);
            const double d = g.gap + tlo + slo;  // smallest t - s over the panel pair
            const int nt = panel_nodes(thi - tlo, d, P);
            const int ns = panel_nodes(shi - slo, d, P);
            for (int i = lane; i < nt + ns; i += kWave) {
                const bool is_t = i < nt;
                const int j = is_t ? i : i - nt;
                double v, wv;
                if (is_t)
                    gl_rule(gl, nt, j, tlo, thi, &v, &wv);
                else
                    gl_rule(gl, ns, j, slo, shi, &v, &wv);
                const double xi = is_t ? 2.0 * v / g.he - 1.0 : 1.0 - 2.0 * v / g.hf;
                double* Lrow = is_t ? sm.Lt : sm.Ls;
                double pm = 1.0, p = xi;
                Lrow[j] = 1.0;
                if (P > 1) Lrow[kMaxPanelNodes + j] = xi;
                for (int k = 1; k + 1 < P; ++k) {
                    const double pn = ((2 * k + 1) * xi * p - k * pm) / (k + 1);
                    pm = p;
                    p = pn;
                    Lrow[(k + 1) * kMaxPanelNodes + j] = pn;
                }
                if (is_t) {
                    tu[j] = v;
                    tw[j] = wv;
                } else {
                    sv[j] = v;
                    sw[j] = wv;
                }
            }
            __syncthreads();
            for (int q = lane; q < nt * ns; q += kWave) {
                const int i = q / ns, j = q % ns;
                sm.Kw[i * kMaxPanelNodes + j] = tw[i] * sw[j] * pow(g.gap + tu[i] + sv[j], 1.0 - alpha);
            }
            __syncthreads();
            // T[m][j] = sum_i Lt[m][i] Kw[i][j]
            for (int q = lane; q < P * ns; q += kWave) {
                const int m = q / ns, j = q % ns;
                double s = 0.0;
                for (int i = 0; i < nt; ++i) s += sm.Lt[m * kMaxPanelNodes + i] * sm.Kw[i * kMaxPanelNodes + j];
                sm.T[m * kMaxPanelNodes + j] = s;
            }
            __syncthreads();
            // acc[m][n] += sum_j T[m][j] Ls[n][j]
            int a = 0;
            for (int q = lane; q < P * P; q += kWave, ++a) {
                const int m = q / P, n = q % P;
                double s = 0.0;
                for (int j = 0; j < ns; ++j) s += sm.T[m * kMaxPanelNodes + j] * sm.Ls[n * kMaxPanelNodes + j];
                acc[a] += gamma0 * s;
            }
            __syncthreads();
        }
    }
}

__device__ void block_same(const Geo& g, int P, double alpha, double gamma0, const double* rules,
                           Smem sm, double* acc) {
    const int lane = threadIdx.x;
    const int no = P + 1, ni = P;
    const double* xo = rules;
    const double* wo = rules + no;
    const double* xi_in = rules + 2 * no;
    const double* wi_in = rules + 2 * no + ni;
    const double scale_in = exp2(alpha - 2.0);   // w = (1+y)/2, w^{1-alpha} dw = 2^{alpha-2} (1+y)^{1-alpha} dy
    // T[n][o] = sum_i wi L_n(xi_o - (1+xi_o) w_i)
    for (int q = lane; q < P * no; q += kWave) {
        const int n = q / no, o = q % no;
        double s = 0.0;
        for (int i = 0; i < ni; ++i) {
            const double w = 0.5 * (1.0 + xi_in[i]);
            s += wi_in[i] * scale_in * legendre(n, xo[o] - (1.0 + xo[o]) * w);
        }
        sm.T[n * kMaxPanelNodes + o] = s;
    }
    __syncthreads();
    const double c = gamma0 * pow(0.5 * g.he, 3.0 - alpha);
    int a = 0;
    for (int q = lane; q < P * P; q += kWave, ++a) {
        const int m = q / P, n = q % P;
        double s = 0.0;
        for (int o = 0; o < no; ++o) s += wo[o] * legendre(m, xo[o]) * sm.T[n * kMaxPanelNodes + o];
        acc[a] += c * s;
    }
    __syncthreads();
}

__device__ void block_adjacent(const Geo& g, int P, double alpha, double gamma0, const double* rules,
                               const double* gl, Smem sm, double* acc) {
    const int lane = threadIdx.x;
    const int nr = P + 1;
    const double* xr = rules;      // GJ(0, 2-alpha), n = P+1
    const double* wr = rules + nr;
    const double rscale = exp2(alpha - 3.0);   // r = (1+y)/2: r^{2-alpha} dr = 2^{alpha-3}(1+y)^{2-alpha} dy
    const double e1 = 1.0 - alpha;
    // triangle 1 (b <= a): I1[n][r] = sum_w (he + hf w)^{1-alpha} L_n(1 - 2 a_r w)
    // triangle 2 (a <= b): I2[m][r] = sum_w (he w + hf)^{1-alpha} L_m(2 b_r w - 1)
    for (int tri_ = 0; tri_ < 2; ++tri_) {
        const double gw = tri_ == 0 ? g.he / g.hf : g.hf / g.he;   // singular point at w = -gw
        const int np = panel_count(1.0, gw);
        for (int q = lane; q < P * nr; q += kWave) {
            const int n = q / nr, r = q % nr;
            const double ar = 0.5 * (1.0 + xr[r]);
            double s = 0.0;
            for (int j = 0; j < np; ++j) {
                double lo, hi;
                panel_bounds(1.0, gw, j, &lo, &hi);
                const int nw = panel_nodes(hi - lo, lo + gw, P);
                for (int i = 0; i < nw; ++i) {
                    double w, ww;
                    gl_rule(gl, nw, i, lo, hi, &w, &ww);
                    if (tri_ == 0)
                        s += ww * pow(g.he + g.hf * w, e1) * legendre(n, 1.0 - 2.0 * ar * w);
                    else
                        s += ww * pow(g.he * w + g.hf, e1) * legendre(n, 2.0 * ar * w - 1.0);
                }
            }
            sm.T[n * kMaxPanelNodes + r] = s;
        }
        __syncthreads();
        const double c = gamma0 * g.he * g.hf * rscale;
        int a = 0;
        for (int q = lane; q < P * P; q += kWave, ++a) {
            const int m = q / P, n = q % P;
            double s = 0.0;
            for (int r = 0; r < nr; ++r) {
                const double ar = 0.5 * (1.0 + xr[r]);
                if (tri_ == 0)
                    s += wr[r] * legendre(m, 2.0 * ar - 1.0) * sm.T[n * kMaxPanelNodes + r];
                else
                    s += wr[r] * legendre(n, 1.0 - 2.0 * ar) * sm.T[m * kMaxPanelNodes + r];
            }
            acc[a] += c * s;
        }
        __syncthreads();
    }
}

__device__ void compute_block(const Geo& g, int P, double alpha, double gamma0, const double* rules,
                              const double* gl, double scale, double* out) {
    extern __shared__ double smem[];
    Smem sm;
    sm.Lt = smem;
    sm.Ls = sm.Lt + P * kMaxPanelNodes;
    sm.T = sm.Ls + P * kMaxPanelNodes;
    sm.Kw = sm.T + (P < 2 ? 2 : P) * kMaxPanelNodes;
    sm.nodes = sm.Kw + kMaxPanelNodes * kMaxPanelNodes;
    double acc[kAccPerLane];
    for (int a = 0; a < kAccPerLane; ++a) acc[a] = 0.0;
    if (g.kind == 0)
        block_same(g, P, alpha, gamma0, rules, sm, acc);
    else if (g.kind == 1)
        block_adjacent(g, P, alpha, gamma0, rules, gl, sm, acc);
    else
        block_separated(g, P, alpha, gamma0, gl, sm, acc);
    int a = 0;
    for (int q = threadIdx.x; q < P * P; q += kWave, ++a) out[q] = scale * acc[a];
}

__global__ void __launch_bounds__(kWave) k_moments_dense(int N, int P, double alpha, double gamma0,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ h,
                                                        const double* __restrict__ rules,
                                                        const double* __restrict__ gl,
                                                        double* __restrict__ mom, int64_t npairs) {
    for (int64_t pid = blockIdx.x; pid < npairs; pid += gridDim.x) {
        // pair index -> (e, f), f <= e, row-major over the lower triangle
        int64_t e = (int64_t)((sqrt(8.0 * (double)pid + 1.0) - 1.0) * 0.5);
        while (tri(e + 1) <= pid) ++e;
        while (tri(e) > pid) --e;
        const int64_t f = pid - tri(e);
        Geo g;
        g.he = h[e];
        g.hf = h[f];
        g.kind = (e == f) ? 0 : (f == e - 1 ? 1 : 2);
        g.gap = (g.kind == 2) ? x[e] - x[f + 1] : 0.0;
        compute_block(g, P, alpha, gamma0, rules, gl, 1.0, mom + pid * P * P);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kWave) k_moments_list(int P, double alpha, double gamma0,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ h,
                                                       const double* __restrict__ rules,
                                                       const double* __restrict__ gl,
                                                       const int* __restrict__ ev,
                                                       const int* __restrict__ fv,
                                                       double* __restrict__ out, int npairs) {
    const int pid = blockIdx.x;
    if (pid >= npairs) return;
    const int e = ev[pid], f = fv[pid];
    Geo g;
    g.he = h[e];
    g.hf = h[f];
    g.kind = (e == f) ? 0 : (f == e - 1 ? 1 : 2);
    g.gap = (g.kind == 2) ? x[e] - x[f + 1] : 0.0;
    compute_block(g, P, alpha, gamma0, rules, gl, 1.0, out + (int64_t)pid * P * P);
}

// Toeplitz generators Khat_k at h_e = 2 with ratio r = h_{e+1}/h_e:
// K^{ef} = (h_e/2)^{2-alpha} (h_f/2) Khat_{e-f} (Section 4.3, eq. (eq420)).
__global__ void __launch_bounds__(kWave) k_generators(int N, int P, double alpha, double gamma0,
                                                     double r, const double* __restrict__ rules,
                                                     const double* __restrict__ gl,
                                                     double* __restrict__ gen) {
    const int k = blockIdx.x;
    if (k >= N) return;
    Geo g;
    g.he = 2.0;
    g.hf = 2.0 * pow(r, -(double)k);
    g.kind = k == 0 ? 0 : (k == 1 ? 1 : 2);
    // the k-1 elements between: 2 sum_{j=1}^{k-1} q^j, q = 1/r, in closed form
    // (q expm1((k-1) ln q) / expm1(ln q), accurate also for q near 1)
    double gap = 0.0;
    if (k > 1) {
        if (r == 1.0) {
            gap = 2.0 * (k - 1);
        } else {
            const double lq = -log(r);
            gap = 2.0 * exp(lq) * expm1((k - 1) * lq) / expm1(lq);
        }
    }
    g.gap = gap;
    compute_block(g, P, alpha, gamma0, rules, gl, 1.0 / (0.5 * g.hf), gen + (int64_t)k * P * P);
}

size_t moments_smem(int P) {
    return sizeof(double) * (size_t)(3 * (P < 2 ? 2 : P) * kMaxPanelNodes + kMaxPanelNodes * kMaxPanelNodes +
                                     4 * kMaxPanelNodes);
}

// ---------------------------------------------------------------- dense A
__global__ void k_dense_matrix(SemDev s, double* __restrict__ A, int lda) {
    const int Nd = s.N * s.P - 1;
    const int i = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nd || j >= Nd) return;
    A[(int64_t)j * lda + i] = sem_entry(s, i, j);
}

// ---------------------------------------------------------------- load vector
// G_i = sum_q w_q f(x_q) phi_i(x_q) over the quadrature nodes of the elements in supp(phi_i).
// One wavefront per element, the lanes striding over the element's nodes (24 on most elements,
// hundreds on the graded end elements): at a node the Legendre values L_0..L_P by the
// three-term recurrence give the bubbles psi_p = L_{p-1} - L_{p+1}; the per-lane sums are
// reduced over the wavefront. The two hat halves (1 -+ xi)/2 of the element go to `hat`, and a
// second kernel adds the halves of the two elements around each interior node.
constexpr int kLvMaxP = 32;

// lane l ends with the wavefront sum of v[(l >> 1) & 31] (31 shuffles for 32 sums)
__device__ __attribute__((always_inline)) inline double reduce32(double (&a)[32], int lane) {
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int o = 32 >> st, half = 16 >> st;
        const bool hi = lane & o;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            // the two values as opaque registers: a select between array elements would otherwise
            // become a load at a lane-dependent index (the array then lives in scratch memory)
            double lo = a[i], up = a[i + half];
            asm volatile("" : "+v"(lo), "+v"(up));
            const double send = hi ? lo : up, keep = hi ? up : lo;
            a[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    return a[0] + __shfl_xor(a[0], 1, 64);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_load_elements(int N, int P, const int* __restrict__ off,
                                                       const double* __restrict__ xi, const double* __restrict__ w,
                                                       const double* __restrict__ f, double* __restrict__ G,
                                                       double* __restrict__ hat) {
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= N) return;
    double acc[32], hl = 0.0, hr = 0.0;
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0.0;
    for (int q = off[e] + lane; q < off[e + 1]; q += 64) {
        const double x = xi[q], wf = w[q] * f[q];
        // psi_p = L_{p-1} - L_{p+1}, with L_{p+1} from the three-term recurrence as p advances
        double Lm = 1.0, Lc = x;   // L_{p-1}, L_p
#pragma unroll
        for (int p = 1; p < kLvMaxP; ++p)
            if (p < P) {
                const double Ln = ((2.0 * p + 1.0) * x * Lc - p * Lm) * (1.0 / (p + 1.0));
                acc[p - 1] += wf * (Lm - Ln);
                Lm = Lc;
                Lc = Ln;
            }
        hl += wf * 0.5 * (1.0 - x);
        hr += wf * 0.5 * (1.0 + x);
    }
    const double sb = reduce32(acc, lane);
    const int p = ((lane >> 1) & 31) + 1;
    if ((lane & 1) == 0 && p < P) G[(int64_t)e * (P - 1) + p - 1] = sb;
    hl = wave_sum(hl);
    hr = wave_sum(hr);
    if (lane == 0) {
        hat[2 * e] = hl;
        hat[2 * e + 1] = hr;
    }
}

// hat j (interior node j = 1..N-1): right half of element j-1 plus left half of element j
__global__ void k_load_hats(int N, int P, const double* __restrict__ hat, double* __restrict__ G) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j >= N) return;
    G[(int64_t)N * (P - 1) + j - 1] = hat[2 * (j - 1) + 1] + hat[2 * j];
}

}  // namespace

void launch_pair_moments_dense(Op* op) {
    const int64_t npairs = tri(op->N);
    const int grid = (int)(npairs < (1 << 22) ? npairs : (1 << 22));
    hipLaunchKernelGGL(k_moments_dense, dim3(grid), dim3(kWave), moments_smem(op->P), op->ctx->stream,
                       op->N, op->P, op->alpha, op->gamma0, op->d_x.p, op->d_h.p, op->d_rules.p,
                       op->ctx->gl.p, op->d_mom.p, npairs);
    FDE_LAUNCH_CHECK();
}

void launch_generators(Op* op) {
    hipLaunchKernelGGL(k_generators, dim3(op->N), dim3(kWave), moments_smem(op->P), op->ctx->stream,
                       op->N, op->P, op->alpha, op->gamma0, op->ratio, op->d_rules.p, op->ctx->gl.p,
                       op->d_gen.p);
    FDE_LAUNCH_CHECK();
}

void launch_pair_moments_list(Op* op, int npairs, const int* d_e, const int* d_f, double* d_out) {
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_moments_list, dim3(npairs), dim3(kWave), moments_smem(op->P), op->ctx->stream,
                       op->P, op->alpha, op->gamma0, op->d_x.p, op->d_h.p, op->d_rules.p,
                       op->ctx->gl.p, d_e, d_f, d_out, npairs);
    FDE_LAUNCH_CHECK();
}

void launch_dense_matrix(Op* op, double* A, int lda) {
    const int Nd = op->Nd;
    dim3 grid(ceil_div(Nd, 128), Nd);
    hipLaunchKernelGGL(k_dense_matrix, grid, dim3(128), 0, op->ctx->stream, sem_dev(op), A, lda);
    FDE_LAUNCH_CHECK();
}

namespace {
// f(x_q) = sum_k coef_k d_k^{expo_k} at every load-vector node, d_k the exact distance to a
// (side 0) or to b (side 1)
// load-vector nodes, one wavefront per panel, lane i = node i: a Gauss-Legendre node mapped to the
// panel [lo, hi] measured from the element end `side`, with its reference coordinate, weight and
// distances to a and b formed from the element's own end distances (no cancellation near the
// ends); explicit panels are copied
__global__ void k_load_rule(int np, const LoadPanel* __restrict__ pan, const double* __restrict__ ex,
                            const double* __restrict__ gl, const double* __restrict__ xm, int N, double* __restrict__ x,
                            double* __restrict__ xi, double* __restrict__ w, double* __restrict__ da,
                            double* __restrict__ db) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6), i = threadIdx.x & 63;
    if (p >= np) return;
    const LoadPanel pn = pan[p];
    if (i >= pn.n) return;
    const int q = pn.node0 + i;
    if (pn.ex >= 0) {
        const double* e = ex + 5 * (size_t)(pn.ex + i);
        x[q] = e[0];
        xi[q] = e[1];
        w[q] = e[2];
        da[q] = e[3];
        db[q] = e[4];
        return;
    }
    const double a = xm[0], b = xm[N];
    const double xl = xm[pn.elem], xr = xm[pn.elem + 1], he = xr - xl;
    const double da_l = xl - a, db_r = b - xr;
    const int off = pn.n * (pn.n - 1) / 2;
    const double gx = gl[off + i], gw = gl[kMaxGL * (kMaxGL + 1) / 2 + off + i];
    const double u = 0.5 * (pn.hi - pn.lo) * gx + 0.5 * (pn.hi + pn.lo);
    w[q] = 0.5 * (pn.hi - pn.lo) * gw;
    if (pn.side == 0) {
        double xv = xl + u;
        if (xv <= xl) xv = nextafter(xl, xr);
        x[q] = xv;
        xi[q] = 2.0 * u / he - 1.0;
        da[q] = da_l + u;
        db[q] = db_r + (he - u);
    } else {
        double xv = xr - u;
        if (xv >= xr) xv = nextafter(xr, xl);
        x[q] = xv;
        xi[q] = 1.0 - 2.0 * u / he;
        da[q] = da_l + (he - u);
        db[q] = db_r + u;
    }
}

__global__ void k_eval_powers(int nq, const double* __restrict__ da, const double* __restrict__ db, int nt,
                              const double* __restrict__ coef, const double* __restrict__ expo,
                              const int* __restrict__ side, double* __restrict__ f) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const double a = da[q], b = db[q];
        double s = 0.0;
        for (int k = 0; k < nt; ++k) s += coef[k] * pow(side[k] ? b : a, expo[k]);
        f[q] = s;
    }
}
}  // namespace

void launch_load_rule(Op* op, int npanels, const LoadPanel* d_panels, const double* d_ex) {
    if (npanels <= 0) return;
    hipLaunchKernelGGL(k_load_rule, dim3(ceil_div(npanels, 4)), dim3(256), 0, op->ctx->stream, npanels, d_panels, d_ex,
                       op->ctx->gl.p, op->d_x.p, op->N, op->d_lq_x.p, op->d_lq_xi.p, op->d_lq_w.p, op->d_lq_da.p,
                       op->d_lq_db.p);
    FDE_LAUNCH_CHECK();
}

void launch_eval_powers(Op* op, int nt, const double* d_coef, const double* d_expo, const int* d_side) {
    const int nq = op->lq_n;
    hipLaunchKernelGGL(k_eval_powers, dim3(std::min(ceil_div(nq, 256), 1024)), dim3(256), 0, op->ctx->stream, nq,
                       op->d_lq_da.p, op->d_lq_db.p, nt, d_coef, d_expo, d_side, op->d_lq_f.p);
    FDE_LAUNCH_CHECK();
}

void launch_load_vector(Op* op, double* G) {
    if (op->P > kLvMaxP) fail(FDE_EUNSUPPORTED, "load vector: P <= %d", kLvMaxP);
    DevBuf<double> hat;
    hat.alloc(op->ctx, 2 * (size_t)op->N);
    hipLaunchKernelGGL(k_load_elements, dim3(ceil_div(op->N, 4)), dim3(256), 0, op->ctx->stream, op->N, op->P,
                       op->d_lq_off.p, op->d_lq_xi.p, op->d_lq_w.p, op->d_lq_f.p, G, hat.p);
    FDE_LAUNCH_CHECK();
    if (op->N > 1) {
        hipLaunchKernelGGL(k_load_hats, dim3(ceil_div(op->N - 1, 256)), dim3(256), 0, op->ctx->stream, op->N, op->P,
                           hat.p, G);
        FDE_LAUNCH_CHECK();
    }
}

}  // namespace fde
