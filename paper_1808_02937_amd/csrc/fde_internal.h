// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include <cstdarg>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fde.h"

namespace fde {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
struct Error {
    int code;
    std::string msg;
};
// Throw inside the library; the C entry points catch and translate.
[[noreturn]] void fail(int code, const char* fmt, ...);

#define FDE_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::fde::fail(FDE_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                               \
    } while (0)

#define FDE_LAUNCH_CHECK() FDE_HIP(hipGetLastError())

// C entry points: library errors become status codes and a message (no exception crosses the ABI)
#define FDE_API_BEGIN try {
#define FDE_API_END                                 \
    }                                               \
    catch (const fde::Error& e) {                   \
        fde::set_error("%s", e.msg.c_str());        \
        return e.code;                              \
    }                                               \
    catch (const std::bad_alloc&) {                 \
        fde::set_error("host allocation failed");   \
        return FDE_ENOMEM;                          \
    }                                               \
    catch (...) {                                   \
        fde::set_error("unexpected internal error"); \
        return FDE_EDEVICE;                         \
    }                                               \
    return FDE_OK;

// a status from another entry point, as an error of this one (its message is kept)
inline void check_rc(int rc) {
    if (rc != FDE_OK) {
        const char* m = fde_last_error();
        throw Error{rc, m ? std::string(m) : std::string()};
    }
}

// ---------------------------------------------------------------- quadrature
// n-point Gauss rule for (1-x)^a (1+x)^b on [-1,1]; nodes ascending.
void gauss_jacobi(int n, double a, double b, double* x, double* w);

constexpr int kMaxGL = 64;  // Gauss-Legendre rules n = 1..kMaxGL live on the device
// Gauss-Legendre rules n = 1..kMaxGL: nodes of rule n at offset n(n-1)/2, the weights
// kMaxGL(kMaxGL+1)/2 entries further; computed on first use, read-only afterwards
const double* gauss_legendre_table();

// ---------------------------------------------------------------- memory
struct Ctx;
void* dev_alloc(Ctx* c, size_t bytes);
void dev_free(Ctx* c, void* p, size_t bytes);
// host -> device copy on the context stream; returns at once (the source may be reused)
void upload(Ctx* c, void* dst, const void* src, size_t bytes);

template <class T>
struct DevBuf {
    Ctx* ctx = nullptr;
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void alloc(Ctx* c, size_t count) {
        reset();
        ctx = c;
        n = count;
        p = count ? static_cast<T*>(dev_alloc(c, count * sizeof(T))) : nullptr;
    }
    void reset() {
        if (p) dev_free(ctx, p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

struct Plan;   // H-LU and H-solve programs of one H-matrix structure (hlu.h)

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;   // 0: unlimited
    size_t in_use = 0;   // bytes of live blocks
    // Stream-ordered cache of device blocks: a block freed by the library is kept and handed to
    // a later request on the same stream (work queued on one stream runs in order, so no wait is
    // needed). Cached bytes count against the budget and are released first when it is tight.
    std::multimap<size_t, void*> pool;    // free blocks by size
    std::unordered_map<void*, size_t> live;
    size_t pooled = 0;
    // Pinned staging ring for host-to-device uploads: the data is copied into the ring and the
    // copy to the device is asynchronous (an upload from pageable memory would wait for all work
    // queued on the stream); a region is reused once the event recorded after its copy has fired.
    struct Staged {
        size_t start, end;
        hipEvent_t ev;
    };
    char* stage = nullptr;
    size_t stage_head = 0;
    std::deque<Staged> staged;
    std::vector<hipEvent_t> spare_events;
    ~Ctx();
    DevBuf<double> gl;   // Gauss-Legendre n=1..kMaxGL: nodes then weights, offset n(n-1)/2
    size_t lds_limit = 0;   // largest dynamic LDS of one workgroup (bytes)
    int num_cu = 0;         // compute units of the device
    // most recently used plans first, keyed by the structure they were made for
    std::vector<std::pair<std::string, std::shared_ptr<Plan>>> plans;
    // plans whose host part was built ahead (in parallel) and that wait for their upload
    std::map<std::string, std::shared_ptr<Plan>> host_plans;
    // task list of the last batched factorisation (it depends only on the batch's plans)
    std::shared_ptr<void> lu_tasks;
    // side streams (default priority) for independent small work forked from and joined back into
    // `stream`: the per-operator applies of a batched Krylov step
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork_ev = nullptr;
    int nside = 3;   // side streams the applies may use (0: everything on `stream`)
};

// ---------------------------------------------------------------- operator
struct Op {
    Ctx* ctx = nullptr;
    int N = 0, P = 0, Nd = 0;
    double alpha = 0, theta = 0, rho = 0, gamma0 = 0;
    std::vector<double> x, h;
    bool toeplitz = false;
    bool uniform = false;
    double ratio = 1.0;  // h_{e+1}/h_e on constant-ratio meshes
    int L = 0;           // FFT length (power of two >= 2N)
    // device data
    DevBuf<double> d_x, d_h;
    DevBuf<double> d_hpow;       // (h_e / 2)^(2 - alpha) per element (the Toeplitz moments' scale)
    DevBuf<double> d_rules;      // GJ(0,2-alpha) n=P+1 then GJ(0,1-alpha) n=P: x then w
    DevBuf<double> d_lmass;      // (P+1)^2 local mass in [phi_L, phi_R, psi_1..]
    DevBuf<double> d_mom;        // dense: N(N+1)/2 pairs x P x P
    DevBuf<double> d_gen;        // Toeplitz: N generators x P x P
    DevBuf<double2> d_sym;       // Toeplitz: (L/2+1) x P x P spectrum of the generators
    DevBuf<double2> d_tw;        // twiddles for the half-length complex FFT
    // load-vector quadrature: lq_n nodes on the device (element e owns [lq_off[e], lq_off[e+1]));
    // host copies of x and the end distances only once asked for
    int lq_n = 0;
    std::vector<int> lq_off;     // N+1 offsets
    std::vector<double> lq_x, lq_da, lq_db;
    DevBuf<double> d_lq_x, d_lq_xi, d_lq_w, d_lq_f, d_lq_da, d_lq_db;
    DevBuf<int> d_lq_off;
    // apply workspace
    DevBuf<double> ws;
    size_t apply_ws_doubles(int nrhs) const;
    // a degree per element (the space S_N^P with degrees P_i, Section 2.2): the operator is built
    // at P = max P_i on its Nd extended unknowns (the one-degree order); the space's own hp_nd
    // unknowns (its order: bubbles element by element, then the hats) sit at d_hp_map among
    // them, d_hp_keep marks them (1) and the outside ones (0), which every product decouples
    bool hp = false;
    int hp_nd = 0;
    std::vector<int> hp_P;
    DevBuf<int> d_hp_map;
    DevBuf<double> d_hp_keep;
    int pub_nd() const { return hp ? hp_nd : Nd; }   // unknowns of the public calls' vectors
};

// degree per element (hp.hip): Y = keep Y + (1 - keep) X over the extended unknowns (X null: 0;
// nothing on a one-degree operator); public hp_nd-row columns <-> extended Nd-row columns
// (scatter zero-fills the outside rows); Ap[i, j] = Ae[map i, map j]
void hp_decouple(Op* op, int nrhs, const double* X, int ldx, double* Y, int ldy, hipStream_t st);
void hp_scatter(Op* op, int nrhs, const double* Xp, int ldp, double* Xe, int lde, hipStream_t st);
void hp_gather(Op* op, int nrhs, const double* Xe, int lde, double* Xp, int ldp, hipStream_t st);
void hp_gather_matrix(Op* op, const double* Ae, int lde, double* Ap, int ldp, hipStream_t st);

// a Gauss-Legendre panel [lo, hi] (distances from the end `side` of element elem: 0 left, 1 right)
// of n nodes, the first at node0; ex >= 0: n nodes given explicitly from entry ex of the explicit
// list (x, xi, w, d_a, d_b per node)
struct LoadPanel {
    double lo, hi;
    int elem, side, n, node0, ex, pad;
};
// expand npanels panels into the operator's load-vector nodes (d_lq_x, d_lq_xi, d_lq_w, d_lq_da, d_lq_db)
void launch_load_rule(Op* op, int npanels, const LoadPanel* d_panels, const double* d_ex);

// device bytes an operator on nodes x (N elements, degree P) holds after an apply of nrhs columns
size_t op_device_bytes(const double* x, int N, int P, int nrhs);

// kernels (assembly.hip)
void launch_pair_moments_dense(Op* op);
void launch_generators(Op* op);
void launch_pair_moments_list(Op* op, int npairs, const int* d_e, const int* d_f, double* d_out);
void launch_load_vector(Op* op, double* G);
// d_lq_f <- sum_k coef_k d_k^{expo_k} at the load-vector nodes (device coefficient arrays)
void launch_eval_powers(Op* op, int nt, const double* d_coef, const double* d_expo, const int* d_side);
void launch_dense_matrix(Op* op, double* A, int lda);

// apply (apply.hip): Y = A X (+ boundary values bc0/bcN of the lifting)
// on: the stream to run on (nullptr: the context's); on another stream the workspace for nrhs
// columns must already exist (reserve_apply on the context's stream)
// ws: the workspace (op->apply_ws_doubles(nrhs) doubles) or nullptr for the operator's own
// core_events: if set, [0] and [1] are recorded around the kernels that read the operator (the
// moment stream of the dense apply, the symbol product of the Toeplitz apply)
void stiffness_apply(Op* op, int nrhs, const double* X, int ldx, double* Y, int ldy, double bc0,
                     double bcN, bool zero_x, hipStream_t on = nullptr, double* ws = nullptr,
                     hipEvent_t* core_events = nullptr);
// allocation-free apply: a fixed device array per GPU (8 MiB), its address taken once per device
constexpr size_t kApplyScratchDoubles = size_t(1) << 20;
void init_apply_scratch(int device);   // with `device` current; once per device (later calls return)
double* apply_scratch(int device);
void build_symbol(Op* op);

// blas1.hip
void axpy_cols(hipStream_t st, int n, int ncol, double a, const double* x, int ldx, double* y, int ldy);

// tiny helpers
__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t tri(int64_t e) { return e * (e + 1) / 2; }

}  // namespace fde

struct fde_ctx : fde::Ctx {};
struct fde_op : fde::Op {};
