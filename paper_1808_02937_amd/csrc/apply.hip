// Stiffness apply Y = A X = rho M X + D^T (theta K + (1-theta) K^T) D X (FP64, gfx950).
//
// D maps the unknowns to per-element Legendre coefficients of the derivative
// (Section 2.2: hats have slope +-1/h, (phi_e^p)' = -(2p+1)(2/h_e) L_p), K is the
// block-lower element operator of the moments K^{ef}.
//
// Dense apply (any mesh; the O(Nd^2) product of Section 4.2): the packed lower
// triangle of K is streamed once in tiles of T x T element pairs (T = 64 / P)
// through LDS, with wide non-temporal loads and the next tile in flight; each
// tile yields a row partial (K c) and a column partial (K^T c), so every moment
// byte is read from HBM once and used for both S_l and S_l^T (Section 4.3 forms
// S_l^T X the same way from S_l). Partials are reduced in a fixed order
// (deterministic, no atomics).
//
// Block-Toeplitz apply (uniform or constant-ratio meshes, Section 4.3 and
// Appendix A): K^{ef} = (h_e/2)^{2-alpha} (h_f/2) Khat_{e-f}; the causal block
// convolution and its transpose are diagonalised by a zero-padded FFT of length
// L >= 2N (circulant embedding). Each real sequence of length L is transformed
// as a complex sequence of length L/2 (even/odd packing) by an in-place radix-2
// FFT in LDS, one workgroup per channel. Per frequency the P x P complex
// symbol is applied; on a uniform mesh theta Khat + (1-theta) Khat^H is one
// symbol, on a geometric mesh the two parts carry different diagonal scalings
// and are transformed separately.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "fde_internal.h"

namespace fde {

// Workspace of the allocation-free apply (fde_stiffness_apply_noalloc): one array on every GPU the
// library runs on, held until the process ends. Host code never uses this name as an address; it
// uses the per-device address that init_apply_scratch takes from the runtime.
static __device__ __align__(256) double scratch[kApplyScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device ordinal
}  // namespace

void init_apply_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return;
    int cur = -1;
    FDE_HIP(hipGetDevice(&cur));
    if (cur != device) fail(FDE_EDEVICE, "apply scratch: device %d is not current (%d is)", device, cur);
    void* p = nullptr;
    FDE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(FDE_EDEVICE, "apply scratch: no device address on device %d", device);
    g_scratch_ptr[device] = static_cast<double*>(p);
}

double* apply_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_ptr.size() || !g_scratch_ptr[device])
        fail(FDE_EDEVICE, "apply scratch of device %d was not set up (fde_ctx_create does that)", device);
    return g_scratch_ptr[device];
}

namespace {

constexpr int kThreads = 256;

__device__ inline double hat_value(const double* x, int j, int N, int P, double bc0, double bcN) {
    if (j == 0) return bc0;
    if (j == N) return bcN;
    return x ? x[N * (P - 1) + j - 1] : 0.0;
}

// Legendre coefficient m of the derivative on element e
__device__ inline double deriv_coef(const double* x, int e, int m, int N, int P, const double* h,
                                   double bc0, double bcN) {
    if (m == 0)
        return (hat_value(x, e + 1, N, P, bc0, bcN) - hat_value(x, e, N, P, bc0, bcN)) / h[e];
    if (!x) return 0.0;
    return -(2.0 * m + 1.0) * 2.0 / h[e] * x[e * (P - 1) + m - 1];
}

// ----------------------------------------------------------------- gather
__global__ void k_gather(int N, int P, const double* __restrict__ h, const double* __restrict__ X,
                         int ldx, int nrhs, double bc0, double bcN, double* __restrict__ c) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)nrhs * N * P;
    if (idx >= tot) return;
    const int r = (int)(idx / ((int64_t)N * P));
    const int rem = (int)(idx % ((int64_t)N * P));
    const int e = rem / P, m = rem % P;
    c[idx] = deriv_coef(X ? X + (int64_t)r * ldx : nullptr, e, m, N, P, h, bc0, bcN);
}

// the same coefficients for chunks of up to kc right-hand sides, each chunk stored unknown-major:
// chunk k (columns [k kc, k kc + nr)) at c + k kc N P, entry (e P + m) nr + r
__global__ void k_gather_t(int N, int P, const double* __restrict__ h, const double* __restrict__ X, int ldx,
                           int nrhs, int kc, double bc0, double bcN, double* __restrict__ c) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t NP = (int64_t)N * P;
    if (idx >= (int64_t)nrhs * NP) return;
    const int64_t k = idx / (kc * NP), rem = idx % (kc * NP);
    const int nr = (int)std::min<int64_t>(kc, nrhs - k * kc);
    const int64_t row = rem / nr;
    const int r = (int)(rem % nr), e = (int)(row / P), m = (int)(row % P);
    const int col = (int)(k * kc) + r;
    c[idx] = deriv_coef(X ? X + (int64_t)col * ldx : nullptr, e, m, N, P, h, bc0, bcN);
}

// ----------------------------------------------------------------- scatter
__global__ void k_scatter(int N, int P, double rho, const double* __restrict__ h,
                          const double* __restrict__ lmass, const double* __restrict__ z,
                          const double* __restrict__ X, int ldx, int nrhs, double bc0, double bcN,
                          double* __restrict__ Y, int ldy) {
    const int Nd = N * P - 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nrhs * Nd) return;
    const int r = (int)(idx / Nd);
    const int i = (int)(idx % Nd);
    const double* x = X ? X + (int64_t)r * ldx : nullptr;
    const double* zr = z + (int64_t)r * N * P;
    const int nb = N * (P - 1);
    const int P1 = P + 1;
    double y;
    auto local = [&](int e, int b) -> double {  // local coefficient b of element e
        if (b == 0) return hat_value(x, e, N, P, bc0, bcN);
        if (b == 1) return hat_value(x, e + 1, N, P, bc0, bcN);
        return x ? x[e * (P - 1) + b - 2] : 0.0;
    };
    if (i < nb) {
        const int e = i / (P - 1), p = i % (P - 1) + 1;
        y = -(2.0 * p + 1.0) * 2.0 / h[e] * zr[e * P + p];
        if (rho != 0.0) {
            double s = 0.0;
            for (int b = 0; b < P1; ++b) s += lmass[(1 + p) * P1 + b] * local(e, b);
            y += rho * 0.5 * h[e] * s;
        }
    } else {
        const int j = i - nb + 1;
        y = zr[(j - 1) * P] / h[j - 1] - zr[j * P] / h[j];
        if (rho != 0.0) {
            double s1 = 0.0, s0 = 0.0;
            for (int b = 0; b < P1; ++b) {
                s1 += lmass[1 * P1 + b] * local(j - 1, b);
                s0 += lmass[0 * P1 + b] * local(j, b);
            }
            y += rho * (0.5 * h[j - 1] * s1 + 0.5 * h[j] * s0);
        }
    }
    Y[(int64_t)r * ldy + i] = y;
}

// ----------------------------------------------------------------- dense tiles
__device__ inline void tile_ij(int64_t t, int* I, int* J) {
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (tri(i + 1) <= t) ++i;
    while (tri(i) > t) --i;
    *I = (int)i;
    *J = (int)(t - tri(i));
}

// Streaming dense apply for up to kStreamRhs right-hand sides. The packed lower triangle of the
// moments is cut into tiles of T x T element pairs (T P <= 64, about 32 KB of moments per tile);
// workgroups loop over the tiles. A tile's rows are contiguous runs of T P^2 doubles in HBM; each
// thread fetches its share with 16-byte loads (8-byte loads for odd P, whose pair blocks start at
// odd offsets), all issued at once, and the next tile's loads are in flight while the current tile
// is used from LDS. In LDS a pair block's rows have stride P + 1, so the row-partial threads
// (consecutive m) read distinct banks. Row partials (K c)_e and column partials (K^T c)_f of the
// tile go to `part` in the layout k_dense_reduce sums (fixed order: deterministic).
constexpr int kStreamRhs = 4;
constexpr int kStreamThreads = 256;

template <int P>
struct StreamTile {
    static constexpr int T = P >= 64 ? 1 : 64 / P;   // elements per tile side
    static constexpr int PP = P * P;
    static constexpr int LDP = P + 1;                // padded row of a pair block in LDS
    static constexpr int BLK = P * LDP;              // padded pair block
    static constexpr bool W16 = (P % 2) == 0;        // pair blocks start at even offsets
    static constexpr int GW = W16 ? 2 : 1;           // doubles per granule
    static constexpr int GR = T * PP / GW;           // granules per tile row
    static constexpr int KL = (T * GR + kStreamThreads - 1) / kStreamThreads;   // granules per thread
    static constexpr int TP = T * P;
};

template <int P>
__device__ __attribute__((always_inline)) inline void stream_load(const double* __restrict__ mom, int N, int64_t t,
                                                                  double (&v)[StreamTile<P>::KL][2]) {
    using S = StreamTile<P>;
    int I, J;
    tile_ij(t, &I, &J);
    const int e0 = I * S::T, f0 = J * S::T;
    const int ne = min(S::T, N - e0), nf = min(S::T, N - f0);
#pragma unroll
    for (int j = 0; j < S::KL; ++j) {
        const int g = j * kStreamThreads + threadIdx.x;
        const int el = g / S::GR, off = (g % S::GR) * S::GW;
        const int e = e0 + el;
        const int nvalid = el < ne ? min(nf, e - f0 + 1) : 0;   // pairs (e, f) with f <= e
        const bool ok = g < S::T * S::GR && off < nvalid * S::PP;
        const double* src = ok ? mom + (tri(e) + f0) * S::PP + off : mom;
        // read once: non-temporal loads keep the stream out of the caches
        if constexpr (S::W16) {
            typedef double d2v __attribute__((ext_vector_type(2)));
            const d2v w = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(src));
            v[j][0] = ok ? w[0] : 0.0;
            v[j][1] = ok ? w[1] : 0.0;
        } else {
            const double w = __builtin_nontemporal_load(src);
            v[j][0] = ok ? w : 0.0;
        }
    }
}

template <int P>
__global__ void __launch_bounds__(kStreamThreads) k_dense_stream(int N, const double* __restrict__ mom,
                                                                 const double* __restrict__ c, int nrhs,
                                                                 double* __restrict__ part, int64_t ntiles) {
    using S = StreamTile<P>;
    __shared__ double Kt[S::T * S::T * S::BLK];
    __shared__ double ce[kStreamRhs][S::TP], cf[kStreamRhs][S::TP];
    const int tid = threadIdx.x;
    const int nout = 2 * S::TP;
    double v[S::KL][2];
    int64_t t = blockIdx.x;
    if (t < ntiles) stream_load<P>(mom, N, t, v);
    for (; t < ntiles; t += gridDim.x) {
        int I, J;
        tile_ij(t, &I, &J);
        const int e0 = I * S::T, f0 = J * S::T;
        // this tile's moments into LDS (padded pair rows), its coefficient vectors beside them
#pragma unroll
        for (int j = 0; j < S::KL; ++j) {
            const int g = j * kStreamThreads + tid;
            if (g < S::T * S::GR) {
                const int el = g / S::GR, k = (g % S::GR) * S::GW;
                const int fl = k / S::PP, w = k % S::PP, m = w / P, n = w % P;
                double* dst = Kt + (el * S::T + fl) * S::BLK + m * S::LDP + n;
                dst[0] = v[j][0];
                if constexpr (S::W16) dst[1] = v[j][1];
            }
        }
        for (int q = tid; q < nrhs * S::TP; q += kStreamThreads) {
            const int r = q / S::TP, i = q % S::TP;
            const int ei = e0 * P + i, fi = f0 * P + i;
            ce[r][i] = ei < N * P ? c[(int64_t)r * N * P + ei] : 0.0;
            cf[r][i] = fi < N * P ? c[(int64_t)r * N * P + fi] : 0.0;
        }
        __syncthreads();
        // the next tile's loads fly while this one is used
        if (t + gridDim.x < ntiles) stream_load<P>(mom, N, t + gridDim.x, v);
        // threads [0, 2 TP): row partials, two half sums over fl per output; [128, 128 + 2 TP):
        // column partials, two half sums over el
        const bool row = tid < 128;
        const int u = row ? tid : tid - 128;
        const int o = u >> 1, h = u & 1;
        if (o < S::TP) {
            double acc[kStreamRhs];
#pragma unroll
            for (int r = 0; r < kStreamRhs; ++r) acc[r] = 0.0;
            const int a = o / P, b = o % P;   // row: (el, m); column: (fl, n)
            const int lo = h ? S::T / 2 : 0, hi = h ? S::T : S::T / 2;
            for (int x = lo; x < hi; ++x) {
#pragma unroll
                for (int y = 0; y < P; ++y) {
                    // row: K[el=a][fl=x][m=b][n=y] c_f[x][y]; column: K[el=x][fl=a][m=y][n=b] c_e[x][y]
                    const double kv = row ? Kt[(a * S::T + x) * S::BLK + b * S::LDP + y]
                                          : Kt[(x * S::T + a) * S::BLK + y * S::LDP + b];
#pragma unroll
                    for (int r = 0; r < kStreamRhs; ++r)
                        if (r < nrhs) acc[r] += kv * (row ? cf[r][x * P + y] : ce[r][x * P + y]);
                }
            }
#pragma unroll
            for (int r = 0; r < kStreamRhs; ++r) {
                const double tot = acc[r] + __shfl_xor(acc[r], 1, 64);
                if (r < nrhs && h == 0) part[((int64_t)r * ntiles + t) * nout + (row ? 0 : S::TP) + o] = tot;
            }
        }
        __syncthreads();
    }
}

// Dense apply for many right-hand sides on the FP64 matrix cores. Same tiles, same streamed loads
// and LDS layout as k_dense_stream; a tile is the TP x TP matrix M[(el, m)][(fl, n)] (TP = T P <=
// 64), and its partials are two small products per chunk of up to kMfmaRhs right-hand sides:
//   rows:    R = M C_f   (TP x nr),     columns: Q = M^T C_e   (TP x nr),
// with C_f, C_e the tile's coefficient rows staged in LDS. Each product runs in 16 x 16 output
// tiles of v_mfma_f64_16x16x4 (A: 16 x 4, B: 4 x 16, accumulated over TP / 4 steps); wave w
// takes output rows [16 w, 16 w + 16) of both products for every 16-column block of the chunk.
// Operands past TP read as zero.
constexpr int kMfmaRhs = 64;
constexpr int kMfmaMin = 8;   // fewer right-hand sides take the vector stream
typedef double v4d_apply __attribute__((ext_vector_type(4)));

template <int P>
__global__ void __launch_bounds__(kStreamThreads) k_dense_mfma(int N, const double* __restrict__ mom,
                                                               const double* __restrict__ c, int nrhs,
                                                               double* __restrict__ part, int64_t ntiles) {
    using S = StreamTile<P>;
    constexpr int NB = kMfmaRhs / 16;   // 16-column blocks of a full chunk
    __shared__ double Kt[S::T * S::T * S::BLK];
    constexpr int LDR = kMfmaRhs + 1;   // odd row stride: the staging stores hit distinct banks
    __shared__ double cf[64 * LDR], ce[64 * LDR];   // [row (fl, n) or (el, m)][rhs]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nout = 2 * S::TP;
    const int nb = (nrhs + 15) / 16;
    double v[S::KL][2];
    int64_t t = blockIdx.x;
    if (t < ntiles) stream_load<P>(mom, N, t, v);
    for (; t < ntiles; t += gridDim.x) {
        int I, J;
        tile_ij(t, &I, &J);
        const int e0 = I * S::T, f0 = J * S::T;
#pragma unroll
        for (int j = 0; j < S::KL; ++j) {
            const int g = j * kStreamThreads + tid;
            if (g < S::T * S::GR) {
                const int el = g / S::GR, k = (g % S::GR) * S::GW;
                const int fl = k / S::PP, w = k % S::PP, m = w / P, n = w % P;
                double* dst = Kt + (el * S::T + fl) * S::BLK + m * S::LDP + n;
                dst[0] = v[j][0];
                if constexpr (S::W16) dst[1] = v[j][1];
            }
        }
        // coefficient rows of the tile: c is unknown-major for this chunk, so the rows of the
        // tile are one contiguous run each (TP nrhs doubles); all loads of a round in flight at once
        {
            const int len = S::TP * nrhs;
            const double* srce = c + (int64_t)e0 * P * nrhs;
            const double* srcf = c + (int64_t)f0 * P * nrhs;
            const int lim_e = (int)std::min<int64_t>(len, ((int64_t)N * P - (int64_t)e0 * P) * nrhs);
            const int lim_f = (int)std::min<int64_t>(len, ((int64_t)N * P - (int64_t)f0 * P) * nrhs);
            for (int base = 0; base < 64 * kMfmaRhs; base += 8 * kStreamThreads) {
                double a[8], b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = base + u * kStreamThreads + tid;
                    a[u] = q < lim_e ? srce[q] : 0.0;
                    b[u] = q < lim_f ? srcf[q] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = base + u * kStreamThreads + tid;
                    if (q < len) {
                        const int i = q / nrhs, r = q % nrhs;
                        ce[i * LDR + r] = a[u];
                        cf[i * LDR + r] = b[u];
                    }
                }
            }
            // columns past nrhs and rows past TP read as zero in the products
            for (int q = tid; q < 64 * LDR; q += kStreamThreads) {
                const int i = q / LDR, r = q % LDR;
                if (r >= nrhs || i >= S::TP) {
                    ce[q] = 0.0;
                    cf[q] = 0.0;
                }
            }
        }
        __syncthreads();
        if (t + gridDim.x < ntiles) stream_load<P>(mom, N, t + gridDim.x, v);
        // lane roles: i = lane % 16 (row of A, column of B), kq = lane / 16 (k within a step)
        const int i = lane & 15, kq = lane >> 4;
        const int row = 16 * wave + i;   // output row of this wave's tiles
        v4d_apply accR[NB], accC[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            accR[b] = v4d_apply{0.0, 0.0, 0.0, 0.0};
            accC[b] = v4d_apply{0.0, 0.0, 0.0, 0.0};
        }
        if (16 * wave < S::TP) {
            const int ra = row / P, rm = row % P;   // (el, m) for R = M C_f; (fl, n) for Q = M^T C_e
#pragma unroll 2
            for (int ks = 0; ks < (S::TP + 3) / 4; ++ks) {
                const int k = 4 * ks + kq;
                const int ka = k / P, km = k % P;
                const bool ok = row < S::TP && k < S::TP;
                // R: A[row][k] = M[(ra, rm)][(ka, km)];  Q: A[row][k] = M[(ka, km)][(ra, rm)]
                const double aR = ok ? Kt[(ra * S::T + ka) * S::BLK + rm * S::LDP + km] : 0.0;
                const double aC = ok ? Kt[(ka * S::T + ra) * S::BLK + km * S::LDP + rm] : 0.0;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b < nb) {
                        const double bR = cf[k * LDR + 16 * b + i];
                        const double bC = ce[k * LDR + 16 * b + i];
                        accR[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR, bR, accR[b], 0, 0, 0);
                        accC[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aC, bC, accC[b], 0, 0, 0);
                    }
                }
            }
            // register u of lane l holds output (16 wave + 4 u + l / 16, 16 b + l % 16); the tile's
            // partials are stored [output][rhs] (rhs fastest: 16 lanes write 128 contiguous bytes)
            double* pr = part + t * (int64_t)nout * nrhs;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int r = 16 * b + i;
                if (b < nb && r < nrhs) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int o = 16 * wave + 4 * u + kq;
                        if (o < S::TP) {
                            pr[(int64_t)o * nrhs + r] = accR[b][u];
                            pr[(int64_t)(S::TP + o) * nrhs + r] = accC[b][u];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int P>
void launch_mfma_p(hipStream_t st, int N, const double* mom, const double* c, int nrhs, double* part,
                   int64_t ntiles) {
    const int64_t grid = std::min<int64_t>(ntiles, 1024);
    hipLaunchKernelGGL(k_dense_mfma<P>, dim3((unsigned)grid), dim3(kStreamThreads), 0, st, N, mom, c, nrhs, part,
                       ntiles);
    FDE_LAUNCH_CHECK();
}

bool launch_mfma(hipStream_t st, int N, int P, const double* mom, const double* c, int nrhs, double* part,
                 int64_t ntiles) {
    switch (P) {
#define FDE_MFMA_P(p) \
    case p: launch_mfma_p<p>(st, N, mom, c, nrhs, part, ntiles); return true;
        FDE_MFMA_P(2) FDE_MFMA_P(3) FDE_MFMA_P(4) FDE_MFMA_P(5) FDE_MFMA_P(6) FDE_MFMA_P(7) FDE_MFMA_P(8)
        FDE_MFMA_P(9) FDE_MFMA_P(10) FDE_MFMA_P(11) FDE_MFMA_P(12) FDE_MFMA_P(13) FDE_MFMA_P(14) FDE_MFMA_P(15)
        FDE_MFMA_P(16)
#undef FDE_MFMA_P
        default: return false;
    }
}

// z = theta (K c) + (1 - theta) (K^T c) from the tile partials: workgroup (I, r) sums, for the TE
// elements of tile row I, the row partials of tiles (I, J <= I) and the column partials of tiles
// (I' >= I, I); 16 groups of 64 threads take every 16th tile, then the groups are added in order
// (deterministic).
constexpr int kReduceThreads = 1024;
__global__ void __launch_bounds__(kReduceThreads) k_dense_reduce(int N, int P, int TE, int nT, double theta,
                                                               const double* __restrict__ part, int64_t ntiles,
                                                               double* __restrict__ z) {
    constexpr int kG = kReduceThreads / 64;
    __shared__ double sr[kG][64], sc[kG][64];
    const int I = blockIdx.x, r = blockIdx.y;
    const int TP = TE * P, nout = 2 * TP;
    const int o = threadIdx.x & 63, k = threadIdx.x >> 6;
    const double* pr = part + (int64_t)r * ntiles * nout;
    double a = 0.0, b = 0.0;
    if (o < TP) {
        for (int J = k; J <= I; J += kG) a += pr[(tri(I) + J) * nout + o];
        for (int Ip = I + k; Ip < nT; Ip += kG) b += pr[(tri(Ip) + I) * nout + TP + o];
    }
    sr[k][o] = a;
    sc[k][o] = b;
    __syncthreads();
    if (threadIdx.x < TP) {
        double ra = 0.0, cb = 0.0;
        for (int q = 0; q < kG; ++q) {
            ra += sr[q][threadIdx.x];
            cb += sc[q][threadIdx.x];
        }
        const int e = I * TE + threadIdx.x / P;
        if (e < N) z[((int64_t)r * N + e) * P + threadIdx.x % P] = theta * ra + (1.0 - theta) * cb;
    }
}

// The same sums for the matrix-core partials ([tile][output][rhs], nr right-hand sides of a chunk):
// workgroup (I, chunk) of 1024 threads, thread (o, r) pairs in 16 groups over the tiles.
__global__ void __launch_bounds__(256) k_dense_reduce_rhs(int N, int P, int TE, int nT, double theta,
                                                         const double* __restrict__ part, int64_t ntiles, int nr,
                                                         int r0, int nrhs, double* __restrict__ z) {
    const int I = blockIdx.x;
    const int TP = TE * P, nout = 2 * TP;
    const int q = blockIdx.y * 256 + threadIdx.x;   // output (o, r) of this tile row and chunk
    if (q < TP * nr) {
        const int o = q / nr, r = q % nr;
        double a = 0.0, b = 0.0;
        for (int J = 0; J <= I; ++J) a += part[((tri(I) + J) * nout + o) * (int64_t)nr + r];
        for (int Ip = I; Ip < nT; ++Ip) b += part[((tri(Ip) + I) * nout + TP + o) * (int64_t)nr + r];
        const int e = I * TE + o / P;
        if (e < N) z[((int64_t)(r0 + r) * N + e) * P + o % P] = theta * a + (1.0 - theta) * b;
    }
}

// ----------------------------------------------------------------- FFT
__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ inline unsigned bitrev(unsigned k, int logM) { return __brev(k) >> (32 - logM); }

// in-place radix-2 DIT on buf[0..M) holding bit-reversed input; tw[j] = exp(-2 pi i j / L), L = 2M
__device__ void fft_dit(double2* buf, int M, int logM, const double2* __restrict__ tw, bool inverse) {
    for (int s = 1; s <= logM; ++s) {
        const int half = 1 << (s - 1);
        const int stride = M >> (s - 1);       // W_M^{pos M/(2 half)} = W_L^{2 pos M/(2 half)}
        for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
            const int grp = b / half, pos = b % half;
            const int i = grp * 2 * half + pos;
            const int j = i + half;
            double2 w = tw[pos * stride];
            if (inverse) w = cconj(w);
            const double2 u = buf[i];
            const double2 v = cmul(buf[j], w);
            buf[i] = cadd(u, v);
            buf[j] = csub(u, v);
        }
        __syncthreads();
    }
}

struct FwdIn {
    // mode 0: element coefficients from X (channel m, part: 0 omega-scaled, 1 sigma-scaled, 2 unscaled)
    // mode 1: generator entries gen[e][c]
    int mode;
    const double* X;
    int ldx;
    double bc0, bcN;
    const double* h;
    double alpha;
    const double* gen;
};

__device__ inline double fwd_value(const FwdIn& in, int N, int P, int r, int ch, int part, int e) {
    if (e >= N) return 0.0;
    if (in.mode == 1) return in.gen[(int64_t)e * P * P + ch];
    const double* x = in.X ? in.X + (int64_t)r * in.ldx : nullptr;
    const double v = deriv_coef(x, e, ch, N, P, in.h, in.bc0, in.bcN);
    if (part == 0) return v * 0.5 * in.h[e];
    if (part == 1) return v * pow(0.5 * in.h[e], 2.0 - in.alpha);
    return v;
}

// grid (channels, nrhs, parts): spectrum of the real sequence, k = 0..M, into out[((r*parts+part)*nch+ch)*(M+1)+k]
__global__ void __launch_bounds__(kThreads) k_rfft_forward(int N, int P, int M, int logM, int nch, FwdIn in,
                                                         int part_base, const double2* __restrict__ tw,
                                                         double2* __restrict__ out) {
    extern __shared__ double2 buf[];
    const int ch = blockIdx.x, r = blockIdx.y, part = blockIdx.z;
    const int mode_part = in.mode == 1 ? 0 : part_base + part;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        const int src = (int)bitrev((unsigned)k, logM);
        buf[k] = make_double2(fwd_value(in, N, P, r, ch, mode_part, 2 * src),
                              fwd_value(in, N, P, r, ch, mode_part, 2 * src + 1));
    }
    __syncthreads();
    fft_dit(buf, M, logM, tw, false);
    double2* o = out + (((int64_t)r * gridDim.z + part) * nch + ch) * (M + 1);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) {
        const double2 zk = buf[k % M];
        const double2 zc = cconj(buf[(M - k) % M]);
        const double2 E = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
        const double2 d = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y - zc.y));
        const double2 O = make_double2(d.y, -d.x);   // d / i
        o[k] = cadd(E, cmul(tw[k], O));
    }
}

// grid (P, nrhs): z[r][e][m] = sum over parts of scale_part(e) * irfft(spec)[e]
struct InvOut {
    int parts;            // 1 uniform, 2 geometric
    double s_uniform;     // uniform: (h/2)^{3-alpha}
    double theta, alpha;
    const double* h;
};

__global__ void __launch_bounds__(kThreads) k_rfft_inverse(int N, int P, int M, int logM, InvOut io,
                                                         const double2* __restrict__ tw,
                                                         const double2* __restrict__ spec,
                                                         double* __restrict__ z) {
    extern __shared__ double2 buf[];
    const int m = blockIdx.x, r = blockIdx.y;
    for (int part = 0; part < io.parts; ++part) {
        const double2* X = spec + (((int64_t)r * io.parts + part) * P + m) * (M + 1);
        for (int k = threadIdx.x; k < M; k += blockDim.x) {
            const double2 xk = X[k];
            const double2 xc = cconj(X[M - k]);
            const double2 E = make_double2(0.5 * (xk.x + xc.x), 0.5 * (xk.y + xc.y));
            const double2 d = make_double2(0.5 * (xk.x - xc.x), 0.5 * (xk.y - xc.y));
            const double2 O = cmul(d, cconj(tw[k]));
            buf[bitrev((unsigned)k, logM)] = make_double2(E.x - O.y, E.y + O.x);   // E + i O
        }
        __syncthreads();
        fft_dit(buf, M, logM, tw, true);
        const double inv = 1.0 / M;
        for (int k = threadIdx.x; k < M; k += blockDim.x) {
            for (int s = 0; s < 2; ++s) {
                const int e = 2 * k + s;
                if (e >= N) continue;
                const double v = (s == 0 ? buf[k].x : buf[k].y) * inv;
                double* zp = z + ((int64_t)r * N + e) * P + m;
                if (io.parts == 1) {
                    *zp = io.s_uniform * v;
                } else if (part == 0) {
                    *zp = io.theta * pow(0.5 * io.h[e], 2.0 - io.alpha) * v;
                } else {
                    *zp += (1.0 - io.theta) * 0.5 * io.h[e] * v;
                }
            }
        }
        __syncthreads();
    }
}

// per frequency: uniform  Y[m] = sum_n S[m][n] X[n];
//                geometric Yc[m] = sum_n K[m][n] Xc[n],  Yr[m] = sum_n conj(K[n][m]) Xr[n]
// (one thread per right-hand side, output row m and frequency k)
__global__ void k_symbol_apply(int P, int M, int parts, const double2* __restrict__ sym,
                               const double2* __restrict__ spec, int nrhs, double2* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K1 = M + 1;
    if (idx >= (int64_t)nrhs * P * K1) return;
    const int r = (int)(idx / ((int64_t)P * K1)), rem = (int)(idx % ((int64_t)P * K1));
    const int m = rem / K1, k = rem % K1;
    for (int part = 0; part < parts; ++part) {
        const double2* X = spec + ((int64_t)r * parts + part) * P * K1;
        double2* Y = out + ((int64_t)r * parts + part) * P * K1;
        {
            double2 s = make_double2(0.0, 0.0);
            for (int n = 0; n < P; ++n) {
                double2 a;
                if (part == 0)
                    a = sym[((int64_t)m * P + n) * K1 + k];
                else
                    a = cconj(sym[((int64_t)n * P + m) * K1 + k]);
                s = cadd(s, cmul(a, X[(int64_t)n * K1 + k]));
            }
            Y[(int64_t)m * K1 + k] = s;
        }
    }
}

// symbol from the generator spectra Kw[c][k] (c = m*P + n): uniform S = theta Kw + (1-theta) Kw^H
__global__ void k_symbol_build(int P, int M, int uniform, double theta, const double2* __restrict__ Kw,
                               double2* __restrict__ sym) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K1 = M + 1;
    if (idx >= (int64_t)P * P * K1) return;
    const int c = (int)(idx / K1), k = (int)(idx % K1);
    const int m = c / P, n = c % P;
    if (!uniform) {
        sym[idx] = Kw[idx];
        return;
    }
    const double2 a = Kw[(int64_t)c * K1 + k];
    const double2 b = cconj(Kw[((int64_t)n * P + m) * K1 + k]);
    sym[idx] = make_double2(theta * a.x + (1.0 - theta) * b.x, theta * a.y + (1.0 - theta) * b.y);
}

int dense_tile_elems(int P) {
    int te = 64 / P;
    if (te < 1) te = 1;
    if (te > 32) te = 32;
    return te;
}

// launch the streaming dense apply for degree P (tile side 64 / P: the same tiles as
// dense_tile_elems for every P in [2, 32])
template <int P>
void launch_stream_p(hipStream_t st, int N, const double* mom, const double* c, int nrhs, double* part,
                     int64_t ntiles) {
    static_assert(StreamTile<P>::T * P <= 64, "row partial threads");
    // a few workgroups per CU loop over the tiles (grids of 2048 to 8192 measured the same)
    const int64_t grid = std::min<int64_t>(ntiles, 2048);
    hipLaunchKernelGGL(k_dense_stream<P>, dim3((unsigned)grid), dim3(kStreamThreads), 0, st, N, mom, c, nrhs, part,
                       ntiles);
    FDE_LAUNCH_CHECK();
}

bool launch_stream(hipStream_t st, int N, int P, const double* mom, const double* c, int nrhs, double* part,
                   int64_t ntiles) {
    switch (P) {
#define FDE_STREAM_P(p) \
    case p: launch_stream_p<p>(st, N, mom, c, nrhs, part, ntiles); return true;
        FDE_STREAM_P(2) FDE_STREAM_P(3) FDE_STREAM_P(4) FDE_STREAM_P(5) FDE_STREAM_P(6) FDE_STREAM_P(7)
        FDE_STREAM_P(8) FDE_STREAM_P(9) FDE_STREAM_P(10) FDE_STREAM_P(11) FDE_STREAM_P(12) FDE_STREAM_P(13)
        FDE_STREAM_P(14) FDE_STREAM_P(15) FDE_STREAM_P(16) FDE_STREAM_P(17) FDE_STREAM_P(18) FDE_STREAM_P(19)
        FDE_STREAM_P(20) FDE_STREAM_P(21) FDE_STREAM_P(22) FDE_STREAM_P(23) FDE_STREAM_P(24) FDE_STREAM_P(25)
        FDE_STREAM_P(26) FDE_STREAM_P(27) FDE_STREAM_P(28) FDE_STREAM_P(29) FDE_STREAM_P(30) FDE_STREAM_P(31)
        FDE_STREAM_P(32)
#undef FDE_STREAM_P
        default: return false;
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

size_t Op::apply_ws_doubles(int nrhs) const {
    const size_t cz = 2 * (size_t)nrhs * N * P;   // c and z
    if (!toeplitz) {
        const int TE = dense_tile_elems(P);
        const int64_t nT = ceil_div(N, TE);
        const size_t parts = (size_t)nrhs * tri(nT) * 2 * TE * P;
        return cz + parts;
    }
    const int M = L / 2;
    const int parts = uniform ? 1 : 2;
    return cz + 2 * 2 * (size_t)nrhs * parts * P * (M + 1);   // two complex spectra buffers
}

void build_symbol(Op* op) {
    // spectra of the P^2 generator sequences, then the symbol
    const int P = op->P, M = op->L / 2, logM = ilog2(M);
    DevBuf<double2> kw;
    kw.alloc(op->ctx, (size_t)P * P * (M + 1));
    FwdIn in{};
    in.mode = 1;
    in.gen = op->d_gen.p;
    hipLaunchKernelGGL(k_rfft_forward, dim3(P * P, 1, 1), dim3(kThreads), sizeof(double2) * M,
                       op->ctx->stream, op->N, P, M, logM, P * P, in, 0, op->d_tw.p, kw.p);
    FDE_LAUNCH_CHECK();
    const int64_t tot = (int64_t)P * P * (M + 1);
    hipLaunchKernelGGL(k_symbol_build, dim3((unsigned)ceil_div((int)tot, 256)), dim3(256), 0,
                       op->ctx->stream, P, M, op->uniform ? 1 : 0, op->theta, kw.p, op->d_sym.p);
    FDE_LAUNCH_CHECK();
    // kw goes back to the context's stream-ordered cache: work queued later on the stream reuses it
}

void stiffness_apply(Op* op, int nrhs, const double* X, int ldx, double* Y, int ldy, double bc0,
                     double bcN, bool zero_x, hipStream_t on, double* ws, hipEvent_t* core_events) {
    const int N = op->N, P = op->P, Nd = op->Nd;
    hipStream_t st = on ? on : op->ctx->stream;
    if (!ws) {
        const size_t need = op->apply_ws_doubles(nrhs);
        if (op->ws.n < need) {
            // blocks come from the context's cache, ordered on its stream: another stream must not get one
            if (on && on != op->ctx->stream) fail(FDE_EDEVICE, "apply workspace not reserved before a side-stream apply");
            op->ws.alloc(op->ctx, need);
        }
        ws = op->ws.p;
    }
    double* c = ws;
    double* z = c + (size_t)nrhs * N * P;
    double* rest = z + (size_t)nrhs * N * P;
    const double* Xin = zero_x ? nullptr : X;
    const int64_t nzp = (int64_t)nrhs * N * P;
    if (!op->toeplitz) {
        const int TE = dense_tile_elems(P);
        const int nT = ceil_div(N, TE);
        const int64_t ntiles = tri(nT);
        // many columns: chunks of up to kMfmaRhs on the matrix cores (P <= 16), their coefficients
        // unknown-major per chunk; otherwise up to kStreamRhs columns per streaming pass (each pass
        // reads the moments once)
        const bool mfma = nrhs >= kMfmaMin && P <= 16;
        const int chunk = mfma ? kMfmaRhs : kStreamRhs;
        if (mfma)
            hipLaunchKernelGGL(k_gather_t, dim3((unsigned)((nzp + 255) / 256)), dim3(256), 0, st, N, P, op->d_h.p,
                               Xin, ldx, nrhs, chunk, bc0, bcN, c);
        else
            hipLaunchKernelGGL(k_gather, dim3((unsigned)((nzp + 255) / 256)), dim3(256), 0, st, N, P,
                               op->d_h.p, Xin, ldx, nrhs, bc0, bcN, c);
        FDE_LAUNCH_CHECK();
        if (core_events) FDE_HIP(hipEventRecord(core_events[0], st));
        for (int r0 = 0; r0 < nrhs; r0 += chunk) {
            const int nr = std::min(chunk, nrhs - r0);
            const double* cr = c + (int64_t)r0 * N * P;
            double* pr = rest + (int64_t)r0 * ntiles * 2 * TE * P;
            const bool ok = mfma ? launch_mfma(st, N, P, op->d_mom.p, cr, nr, pr, ntiles)
                                 : launch_stream(st, N, P, op->d_mom.p, cr, nr, pr, ntiles);
            if (!ok) fail(FDE_EUNSUPPORTED, "dense apply: no kernel for P = %d", P);
        }
        if (core_events) FDE_HIP(hipEventRecord(core_events[1], st));
        if (mfma) {
            for (int r0 = 0; r0 < nrhs; r0 += chunk) {
                const int nr = std::min(chunk, nrhs - r0);
                hipLaunchKernelGGL(k_dense_reduce_rhs, dim3((unsigned)nT, (unsigned)ceil_div(TE * P * nr, 256)),
                                   dim3(256), 0, st, N, P, TE, nT, op->theta,
                                   rest + (int64_t)r0 * ntiles * 2 * TE * P, ntiles, nr, r0, nrhs, z);
                FDE_LAUNCH_CHECK();
            }
        } else {
            hipLaunchKernelGGL(k_dense_reduce, dim3((unsigned)nT, (unsigned)nrhs), dim3(kReduceThreads), 0, st, N,
                               P, TE, nT, op->theta, rest, ntiles, z);
        }
        FDE_LAUNCH_CHECK();
    } else {
        const int M = op->L / 2, logM = ilog2(M);
        const int parts = op->uniform ? 1 : 2;
        double2* specA = reinterpret_cast<double2*>(rest);
        double2* specB = specA + (size_t)nrhs * parts * P * (M + 1);
        FwdIn in{};
        in.mode = 0;
        in.X = Xin;
        in.ldx = ldx;
        in.bc0 = bc0;
        in.bcN = bcN;
        in.h = op->d_h.p;
        in.alpha = op->alpha;
        hipLaunchKernelGGL(k_rfft_forward, dim3(P, nrhs, parts), dim3(kThreads), sizeof(double2) * M, st,
                           N, P, M, logM, P, in, op->uniform ? 2 : 0, op->d_tw.p, specA);
        FDE_LAUNCH_CHECK();
        if (core_events) FDE_HIP(hipEventRecord(core_events[0], st));
        const int64_t nk = (int64_t)nrhs * P * (M + 1);
        hipLaunchKernelGGL(k_symbol_apply, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st, P, M,
                           parts, op->d_sym.p, specA, nrhs, specB);
        FDE_LAUNCH_CHECK();
        if (core_events) FDE_HIP(hipEventRecord(core_events[1], st));
        InvOut io;
        io.parts = parts;
        io.s_uniform = std::pow(0.5 * op->h[0], 3.0 - op->alpha);
        io.theta = op->theta;
        io.alpha = op->alpha;
        io.h = op->d_h.p;
        hipLaunchKernelGGL(k_rfft_inverse, dim3(P, nrhs), dim3(kThreads), sizeof(double2) * M, st, N, P,
                           M, logM, io, op->d_tw.p, specB, z);
        FDE_LAUNCH_CHECK();
    }
    const int64_t ny = (int64_t)nrhs * Nd;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, st, N, P, op->rho,
                       op->d_h.p, op->d_lmass.p, z, Xin, ldx, nrhs, bc0, bcN, Y, ldy);
    FDE_LAUNCH_CHECK();
    hp_decouple(op, nrhs, Xin, ldx, Y, ldy, st);   // degree per element: the outside unknowns
}

}  // namespace fde
