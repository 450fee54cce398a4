/*
 * fde.h -- C ABI of the MI355X (gfx950) solver for the spectral element
 * discretisation of the one-dimensional two-sided Riemann-Liouville
 * fractional diffusion equation, with an H-matrix preconditioner.
 *
 * Problem (Section 1, eq. (Model)):
 *   -D^2 ( theta aI_x^{2-alpha} u + (1-theta) xI_b^{2-alpha} u ) + rho u = f  on (a,b),
 *   u(a) = c1, u(b) = c2,   1 < alpha < 2,  0 <= theta <= 1,  rho >= 0.
 * Discretisation (Section 2.2, eq. (lsys)): A X = G with A = rho M + S,
 *   S = theta S_l + (1-theta) S_l^T, on the space S_N^P of N elements of degree P.
 *
 * Conventions shared by every call:
 *  - Every function returns an int status: FDE_OK (0) or a negative FDE_E* code;
 *    fde_last_error() gives a message for the calling thread's last failure.
 *    No C++ exception crosses this boundary.
 *  - Vectors are in the paper's unknown order (the vector X below eq. (lsys)):
 *    [u^1_1..u^{P-1}_1; ...; u^1_N..u^{P-1}_N; hat_1..hat_{N-1}], Nd = N*P - 1
 *    entries, bubbles element-major, then the hat (nodal) coefficients.
 *    Multi-column arrays are column-major with a leading dimension >= Nd.
 *  - Pointers named *_dev are device (HBM) pointers on the context's device;
 *    *_host are host pointers. The caller owns every array it passes in; the
 *    library owns the opaque handles and releases them in *_destroy.
 *  - Work is issued on the context's HIP stream. Calls return after their
 *    device work is enqueued unless stated otherwise (calls that fill host
 *    outputs synchronise the stream first).
 *  - Handles are thread-compatible, not thread-safe: use one context per
 *    thread, or serialise calls on a context.
 *  - Device memory the library allocates counts against the context's HBM
 *    budget; a call that would exceed it fails with FDE_ENOMEM and frees
 *    what it allocated.
 */
#ifndef FDE_H
#define FDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FDE_OK            0
#define FDE_EINVAL       -1   /* bad argument: alpha not in (1,2), theta not in [0,1], P < 2, non-increasing mesh, ... */
#define FDE_ENOMEM       -2   /* the context's HBM budget (or the device) cannot hold the request */
#define FDE_EBREAKDOWN   -3   /* H-LU met a pivot below its floor (A~ not factorisable without pivoting) */
#define FDE_ENOCONV      -4   /* the Krylov iteration hit maxit; X holds the last iterate, info.relres is set */
#define FDE_EDEVICE      -5   /* a HIP runtime call failed */
#define FDE_EUNSUPPORTED -6   /* a structure the library does not handle (message says which) */

/* precision of the H-LU factors and H-solves */
#define FDE_FP64          0   /* everything in FP64 (the plain FP64 path) */
#define FDE_FP32          1   /* H-LU factors and H-solves in FP32 */
#define FDE_FP32_BF16UV   2   /* FP32 H-LU; afterwards the low-rank factors U, V are kept in BF16 only
                                 (dense blocks FP32) and the H-solves widen them to FP32 */

/* Krylov method */
#define FDE_FGMRES        0   /* right-preconditioned flexible GMRES(restart) */
#define FDE_BICGSTAB      1   /* left-preconditioned BiCGSTAB on A~^{-1} A X = A~^{-1} G (Section 4.2,
                                 eq. (precondsys)): stops when the preconditioned residual
                                 |A~^{-1}(G - A X)| <= rtol |A~^{-1} G|, as the paper does; info.relres
                                 is the true |G - A X| / |G| at exit, info.iters counts full steps
                                 (two preconditioned products each); restart is ignored */

/* stiffness-apply strategy */
#define FDE_APPLY_AUTO     0  /* FFT block-Toeplitz on uniform / constant-ratio meshes, dense otherwise */
#define FDE_APPLY_DENSE    1  /* stream the element-pair moments of S_l (any mesh) */
#define FDE_APPLY_TOEPLITZ 2  /* FFT block-Toeplitz (fails with FDE_EINVAL on other meshes) */

typedef struct fde_ctx  fde_ctx;   /* device, stream, HBM budget */
typedef struct fde_op   fde_op;    /* the FP64 SEM operator A = rho M + S on one mesh */
typedef struct fde_hmat fde_hmat;  /* H-matrix approximation A~ = rho M + H (Section 3) */
typedef struct fde_hlu  fde_hlu;   /* H-LU factors L_H U_H of A~ (Section 4.1) */

/* H-matrix parameters (Section 3): R = number of Taylor terms (eq. (eqn:Lexpan)),
 * lambda = admissibility parameter of eq. (admis), leaf_elems = largest leaf
 * cluster in elements (>= 2). Defaults: R = 8, lambda = 1, leaf_elems = 8. */
typedef struct { int R; double lambda; int leaf_elems; } fde_hparams;

/* H-LU parameters (Section 4.1): after every low-rank sum the block is
 * recompressed to the singular values above tol * sigma_1, at most rank_cap
 * (<= 0: R) of them. precision: FDE_FP64, FDE_FP32 or FDE_FP32_BF16UV. pivot_floor: a leaf
 * pivot of magnitude <= pivot_floor * max|leaf| is a breakdown. */
typedef struct { double tol; int rank_cap; int precision; double pivot_floor; } fde_hlu_params;

/* Krylov parameters (Section 4.2): stop when ||G - A X||_2 / ||G||_2 <= rtol
 * for the true FP64 residual; restart = Krylov subspace size; maxit bounds the
 * total number of preconditioned matrix-vector products per right-hand side. */
typedef struct { int method; int restart; int maxit; double rtol; } fde_solve_params;

/* per right-hand side result */
typedef struct { int iters; double relres; int status; } fde_solve_info;

/* f(x) evaluated by the caller, for fde_load_vector_fn */
typedef double (*fde_fn)(double x, void* user);

/* ---- context ------------------------------------------------------------ */

/* device: HIP ordinal. hip_stream: a hipStream_t (e.g. torch's current stream)
 * or NULL for the null stream. hbm_budget_bytes: 0 = no limit beyond the device.
 * The context keeps device blocks its objects free and hands them to later
 * requests (stream-ordered: all library work is queued on the context stream);
 * those cached bytes count against the budget and are returned to the device
 * first when a request would exceed it, and when the context is destroyed.
 * Destroy every object of a context before the context. */
int  fde_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, fde_ctx** out);
void fde_ctx_destroy(fde_ctx* ctx);
/* switch the context to another stream (waits for the work queued on the old one) */
int  fde_ctx_set_stream(fde_ctx* ctx, void* hip_stream);
/* Side streams (0 to 3, default 3; default priority) the context may fork the
 * per-operator applies of a batched Krylov step onto. 0 keeps all of a
 * context's work on its stream: for several contexts driven side by side,
 * where every stream takes one of the process's few hardware queues. */
int  fde_ctx_set_apply_streams(fde_ctx* ctx, int n);
/* bytes of device memory the context's live objects currently hold (rounded up
 * to the allocator's block sizes; cached free blocks are not counted) */
size_t fde_ctx_bytes_in_use(const fde_ctx* ctx);

/* ---- operator (Section 2.2) ------------------------------------------- */

/* Build A = rho M + theta S_l + (1-theta) S_l^T on the partition
 * nodes_host[0] = a < ... < nodes_host[N] = b (eq. (Partition)) with degree P
 * on every element. Assembles the FP64 element-pair moments
 *   K^{ef}_{mn} = gamma0 int_{I_e} int_{I_f} (t-s)_+^{1-alpha} L_m(xi_e(t)) L_n(xi_f(s)) ds dt
 * on the device: all N(N+1)/2 pairs for the dense apply, or the N
 * block-Toeplitz generators on uniform / constant-ratio meshes (Section 4.3).
 * Errors: FDE_EINVAL, FDE_ENOMEM, FDE_EDEVICE. */
int  fde_op_create(fde_ctx* ctx, const double* nodes_host, int N, int P, double alpha,
                   double theta, double rho, int apply_mode, fde_op** out);
/* The same with degree P_host[i] on element i (the space S_N^P with degrees
 * P_i of Section 2.2; each in [1, 32], the largest >= 2). Its Nd = sum P_i - 1
 * unknowns are ordered as in eq. (lsys): the P_i - 1 bubbles of each element,
 * element by element, then the N - 1 hats; every call below that takes or
 * returns vectors or matrices of the operator (apply, load vectors, dense
 * forms, H-matrix, H-solves, Krylov solves) uses that order and size. The
 * bubbles do not depend on P_i, so this system is the principal submatrix of
 * the one-degree system with P = max P_i on the same mesh: the operator is
 * built at that degree (pair moments, Toeplitz symbol, H-matrix structure) and
 * the other unknowns are decoupled (their rows and columns become those of the
 * identity), which keeps the H-LU of the space's own A~. Not available on such
 * an operator (FDE_EUNSUPPORTED): fde_stiffness_apply_timed,
 * fde_stiffness_apply_noalloc, fde_hlu_to_dense, fde_sigma_estimate.
 * fde_op_pair_moments returns the max P_i x max P_i moments. */
int  fde_op_create_hp(fde_ctx* ctx, const double* nodes_host, int N, const int* P_host, double alpha,
                      double theta, double rho, int apply_mode, fde_op** out);
void fde_op_destroy(fde_op* op);
/* Nd = N*P - 1 (sum P_i - 1 with a degree per element) */
int  fde_op_ndof(const fde_op* op);
/* 1 if the operator uses the FFT block-Toeplitz apply, 0 for the dense apply */
int  fde_op_is_toeplitz(const fde_op* op);

/* Element-pair moments K^{ef} (P x P, row m = Legendre index on element e) for
 * `npairs` pairs with 0 <= f <= e < N (0-based elements); out_host holds
 * npairs*P*P doubles, pair-major, row-major inside a pair. Synchronises. */
int  fde_op_pair_moments(fde_op* op, int npairs, const int* e_host, const int* f_host,
                         double* out_host);

/* Materialise A (Nd x Nd, column-major, paper order) into A_dev (lda >= Nd).
 * Meant for checks at small N; O(Nd^2) memory belongs to the caller. */
int  fde_op_dense(fde_op* op, double* A_dev, int lda);

/* ---- load vector (below eq. (lsys)) ------------------------------------ */

/* Quadrature nodes at which f is needed: *nq receives the count; x_host,
 * da_host, db_host (each may be NULL) receive the nodes and their distances
 * x - a and b - x, computed without cancellation (nq doubles each). Elements
 * that touch a or b carry panels graded geometrically toward the endpoint and
 * a Gauss-Jacobi end panel for the weight d^{1-alpha}, so f with an endpoint
 * singularity d^{-alpha} x (smooth) is integrated to ~1e-15 relative when f
 * is evaluated through the distances (x itself cannot resolve b - x below
 * ulp(b)). */
int  fde_load_nodes(fde_op* op, int* nq, double* x_host, double* da_host, double* db_host);
/* G_dev (Nd) = (f, phi_i) - c1 a(phi_0, phi_i) - c2 a(phi_N, phi_i) with f given
 * by its values f_host[q] at the nodes of fde_load_nodes (lifting of the
 * boundary values with the boundary hats). */
int  fde_load_vector(fde_op* op, const double* f_host, double c1, double c2, double* G_dev);
/* Same, with f evaluated through a host callback. */
int  fde_load_vector_fn(fde_op* op, fde_fn f, void* user, double c1, double c2, double* G_dev);
/* Same, for f(x) = sum_k coef[k] d_k(x)^expo[k] with d_k = x - a (side[k] = 0)
 * or b - x (side[k] = 1), evaluated on the device at the nodes of
 * fde_load_nodes through their exact distances. This is the form of the
 * right-hand side that Section 5 derives from a solution given as a sum of
 * powers (a Riemann-Liouville derivative of d^mu is a multiple of
 * d^{mu-alpha}). nterms <= 64; host arrays, read before return. */
int  fde_load_vector_powers(fde_op* op, int nterms, const double* coef_host, const double* expo_host,
                            const int* side_host, double c1, double c2, double* G_dev);

/* ---- stiffness apply (Section 4.3) ------------------------------------- */

/* Y = A X for nrhs columns (FP64). Dense apply streams the lower-triangular
 * moments once and uses each block for both S_l and S_l^T; the Toeplitz apply
 * is a zero-padded real FFT of length >= 2N along the elements. */
int  fde_stiffness_apply(fde_op* op, int nrhs, const double* X_dev, int ldx,
                         double* Y_dev, int ldy);

/* fde_stiffness_apply, then wait for it; *core_ms_host is the HIP-event time on
 * the context's stream of the kernels that read the operator (the moment stream
 * of the dense apply, the per-frequency symbol product of the Toeplitz apply).
 * For measurement; nrhs >= 1. */
int  fde_stiffness_apply_timed(fde_op* op, int nrhs, const double* X_dev, int ldx,
                               double* Y_dev, int ldy, double* core_ms_host);

/* Same result as fde_stiffness_apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the workspace
 * (gathered coefficients, tile partials or FFT spectra) is a fixed 8 MiB device
 * array per GPU, set up by fde_ctx_create and held until the process ends; no
 * hipMalloc, hipFree or allocating library call is made. Every call on one GPU
 * shares that array, so calls that overlap on one GPU (other streams, other
 * threads, other contexts) race. Returns FDE_EINVAL when nrhs columns of this
 * operator need more workspace than the array holds (Toeplitz apply:
 * 2 nrhs N P + 4 nrhs parts P (L/2 + 1) doubles; dense apply:
 * 2 nrhs N P + nrhs T(T+1) TE P doubles, TE = max(1, 64 / P), T = ceil(N / TE)). */
int  fde_stiffness_apply_noalloc(fde_op* op, int nrhs, const double* X_dev, int ldx,
                                 double* Y_dev, int ldy);

/* ---- H-matrix (Section 3) --------------------------------------------- */

int  fde_build_hmatrix(fde_op* op, const fde_hparams* prm, fde_hmat** out);
void fde_hmat_destroy(fde_hmat* hm);
/* number of dense and low-rank leaf blocks */
int  fde_hmat_counts(const fde_hmat* hm, int* n_dense, int* n_lowrank);
/* A~ (Nd x Nd, column-major, paper order) into out_dev. */
int  fde_hmat_to_dense(fde_hmat* hm, double* out_dev, int ld);

/* ---- H-LU and H-solves (Section 4.1) ---------------------------------- */

/* The recursion of Section 4.1 is flattened into an op list and scheduled in
 * levels: the ops of a level are independent (they touch no element another
 * op of the level writes) and run concurrently, one workgroup each, one
 * kernel launch per level. The op lists depend only on the structure (mesh,
 * H-matrix parameters, rank capacity); a context keeps the 8 most recently
 * used ones and frees them when it is destroyed. */
int  fde_hlu_factor(fde_hmat* hm, const fde_hlu_params* prm, fde_hlu** out);
/* Factor n H-matrices (any sizes) with the same parameters together: launch l
 * runs level l of every factorisation; out[i] receives each factor. On any
 * failure no factor is returned (out[] all NULL) and the status of the first
 * failing H-matrix is returned. */
int  fde_hlu_factor_batched(int n, fde_hmat* const* hms, const fde_hlu_params* prm, fde_hlu** out);

/* Host-only plan of the H-LU of an operator on `nodes` (N+1 increasing
 * abscissae, polynomial degree P) with H-matrix parameters hp (NULL: defaults)
 * and rank capacity rank_cap (<= 0: R): sizes of its op lists and schedule and
 * the device memory one factorisation allocates. Needs no device. check != 0
 * also replays the program element by element and verifies that the schedule
 * orders every pair of conflicting accesses and that temporaries sharing
 * memory are never live in the same level (slow: for tests); a violation
 * returns FDE_EDEVICE. */
typedef struct {
    long long ops;             /* ops of the H-LU program */
    int levels;                /* levels of its schedule (critical path, in ops) */
    int max_width;             /* most ops in one level */
    long long solve_ops;       /* ops of the H-solve program */
    long long arena_elems;     /* factor storage, elements of the factor precision */
    long long work_elems;      /* H-LU temporaries, elements of the factor precision */
    long long scratch_elems;   /* recompression scratch, elements of the factor precision */
    long long scratch_f64;     /* recompression scratch, doubles */
    long long bytes_fp32;      /* device bytes one FP32 factorisation allocates */
    long long bytes_fp64;      /* device bytes one FP64 factorisation allocates */
    int lr_blocks;             /* low-rank blocks of the H-matrix */
    int hsolve_steps;          /* leaf steps of the leaf-step H-solve (0: the op-list H-solve runs) */
    int hsolve_tslots;         /* its temporaries (slots of R values per column) */
    long long hsolve_lds_fp32; /* its LDS bytes per workgroup, FP32, one column, right-hand side in LDS */
    long long hsolve_lds_fp32_global_rhs;   /* the same with the right-hand side in global memory */
} fde_hlu_plan_info;
int  fde_hlu_plan(const double* nodes_host, int N, int P, const fde_hparams* hp, int rank_cap, int check,
                  fde_hlu_plan_info* out);
void fde_hlu_destroy(fde_hlu* f);
/* L_H (strict lower part, unit diagonal implied) and U_H packed in one
 * Nd x Nd column-major matrix in the H-matrix's internal order; h2p_host (if
 * not NULL) receives that order as paper indices (Nd ints). */
int  fde_hlu_to_dense(fde_hlu* f, double* out_dev, int ld, int* h2p_host);
/* Work of the last factorisation and of the H-solves since the factorisation:
 * floating-point operations the device executed (counted per op with its
 * actual dimensions and ranks) and the factorisation launch time measured with
 * HIP events on the context stream (ms; for a batched factorisation the whole
 * launch). Any output may be NULL. Synchronises. */
int  fde_hlu_stats(fde_hlu* f, double* factor_flops, double* factor_kernel_ms, double* solve_flops);
/* largest rank over the low-rank blocks of the factors (synchronises) */
int  fde_hlu_max_rank(fde_hlu* f, int* max_rank);
/* X = U_H^{-1} L_H^{-1} B (forward then backward H-substitution), nrhs columns,
 * FP64 in and out; the substitution runs in the factor precision. */
int  fde_hlu_solve(fde_hlu* f, int nrhs, const double* B_dev, int ldb, double* X_dev, int ldx);
/* Which H-solve a solve of nrhs columns on f runs (host query, no device work):
 * FDE_HSOLVE_LDS, the leaf-step solve (one workgroup per chunk of *cols columns,
 * *lds_bytes of LDS each) with the right-hand sides in LDS; FDE_HSOLVE_GLOBAL_RHS,
 * the same with them in a global workspace (Nd too large for LDS);
 * FDE_HSOLVE_OPS, the op-list interpreter (*cols = 0). One column per workgroup
 * unless a launch would pass the device's compute units. The environment
 * variables FDE_HSOLVE_VARIANT=global or =ops force the latter two and
 * FDE_HSOLVE_COLS=1|2|4|8 a chunk width (for checks of one variant against
 * another). Any output may be NULL. */
#define FDE_HSOLVE_OPS 0
#define FDE_HSOLVE_LDS 1
#define FDE_HSOLVE_GLOBAL_RHS 2
int  fde_hlu_solve_variant(fde_hlu* f, int nrhs, int* variant, int* cols, long long* lds_bytes);

/* ---- preconditioned Krylov (Section 4.2) ------------------------------- */

/* Solve A X = G for nrhs columns with the H-LU as preconditioner (prec may be
 * NULL: no preconditioner). X is overwritten (zero initial guess). info_host:
 * nrhs entries. Returns FDE_ENOCONV if any column missed rtol. */
int  fde_solve(fde_op* op, fde_hlu* prec, int nrhs, const double* G_dev, int ldg,
               double* X_dev, int ldx, const fde_solve_params* prm, fde_solve_info* info_host);

/* Solve n independent systems (different operators, meshes and sizes) in
 * lock-step: every kernel of an iteration serves all of them in one launch.
 * ops[i], precs[i] (may be NULL), nrhs[i] columns, G[i]/X[i] device arrays
 * with leading dimensions ldg[i]/ldx[i]; info_host has sum(nrhs) entries. */
int  fde_solve_batched(fde_ctx* ctx, int n, fde_op* const* ops, fde_hlu* const* precs,
                       const int* nrhs, const double* const* G_dev, const int* ldg,
                       double* const* X_dev, const int* ldx, const fde_solve_params* prm,
                       fde_solve_info* info_host);

/* ---- utilities --------------------------------------------------------- */

/* n-point Gauss rule for the weight (1-x)^a (1+x)^b on [-1,1] (host; the
 * library's own generator, used for every rule above). */
int  fde_gauss_jacobi(int n, double a, double b, double* x_host, double* w_host);
/* ---- condition-number diagnostics (Section 5's condition-number figures) -- */

#define FDE_SIGMA_A            0   /* B = A                                                    */
#define FDE_SIGMA_AINV         1   /* B = A^{-1}: each product a FGMRES solve (rtol 1e-13, f)  */
#define FDE_SIGMA_ATILDE_INV   2   /* B = (L_H U_H)^{-1}: the H-LU solve with f                */
#define FDE_SIGMA_PRECOND      3   /* B = (L_H U_H)^{-1} A, the preconditioned operator        */
/* Largest and smallest singular values of the (steps + 1) x steps Hessenberg
 * matrix of `steps` Arnoldi steps on B from a start vector seeded by `seed`
 * (device Arnoldi with two Gram-Schmidt passes, device one-sided Jacobi). They
 * lie in [sigma_min(B), sigma_max(B)] and reach them as the Krylov space fills
 * (exactly when steps = Nd). Condition numbers follow as
 * kappa(A) ~ smax(A) smax(A^{-1}), kappa(A~) ~ smax(A) smax(A~^{-1}) when f
 * factors A~ exactly (tol 1e-13; sigma_max(A~) = sigma_max(A) up to the
 * H-matrix error), kappa(A~^{-1} A) ~ smax / smin of FDE_SIGMA_PRECOND.
 * 1 <= steps <= min(64, Nd); f may be NULL for FDE_SIGMA_A. Synchronous. */
int  fde_sigma_estimate(fde_op* op, fde_hlu* f, int kind, int steps, unsigned long long seed,
                        double* smax_host, double* smin_host);

/* ---- serving (many problems, many right-hand sides) -------------------- */

/* A problem: the operator of eq. (Model) on nodes[0..N] with degree P. */
typedef struct { const double* nodes; int N; int P; double alpha; double theta; double rho; } fde_problem;
typedef struct fde_server fde_server;   /* solver cache over one context */

/* A server keeps, per problem, the operator and the H-LU factors (H-matrix
 * parameters hp, H-LU parameters lp; NULL: defaults) and serves batches of
 * right-hand sides with the Krylov parameters sp. budget_bytes (0: none)
 * bounds the device bytes its cached problems hold: before factors are built
 * the least recently used problems that the batch does not use are evicted. */
int  fde_server_create(fde_ctx* ctx, const fde_hparams* hp, const fde_hlu_params* lp,
                       const fde_solve_params* sp, size_t budget_bytes, fde_server** out);
void fde_server_destroy(fde_server* s);
/* Solve n requests: request i asks for nrhs[i] solutions X[i] (device, ld
 * ldx[i]) of problem probs[i] with right-hand sides G[i] (device, ld ldg[i]).
 * Problems without cached factors are built in one batched H-LU, then all
 * right-hand sides are solved by one batched FGMRES. info: sum(nrhs) entries
 * in request order (host); cached[i] (host, optional): 1 if the factors were
 * cached. A problem that cannot fit the budget gets status FDE_ENOMEM in
 * its info entries and the call returns FDE_ENOMEM after serving the rest. */
int  fde_server_solve(fde_server* s, int n, const fde_problem* probs, const int* nrhs,
                      const double* const* G_dev, const int* ldg, double* const* X_dev, const int* ldx,
                      fde_solve_info* info, int* cached);
/* Continuous serving. fde_server_submit queues a request (problem, nrhs
 * right-hand sides G, solutions X: device arrays the caller keeps alive until
 * the request is done) and returns its ticket at once. Each fde_server_step
 * admits queued requests in arrival order as engine slots (256 right-hand
 * sides in flight) and the HBM budget allow -- building, in one batched H-LU,
 * the factors of problems not cached yet, and evicting unused cached problems
 * -- then advances every request in flight by one FGMRES step in shared
 * launches and retires the requests that have converged; requests join and
 * leave between steps, while others are on the device. A request's arithmetic
 * does not depend on what else is in flight, so its X is the same alone and in
 * a mix. *in_flight (optional): requests queued or running after the step.
 * fde_server_poll reports whether a ticket is done; once done it fills info
 * (nrhs entries, host) and cached (1 if its factors were cached at admission),
 * forgets the ticket, and returns the request's status (FDE_ENOMEM if its
 * problem can never fit the budget, FDE_ENOCONV, a build failure). */
int  fde_server_submit(fde_server* s, const fde_problem* prob, int nrhs, const double* G_dev, int ldg,
                       double* X_dev, int ldx, long long* ticket);
int  fde_server_step(fde_server* s, int* in_flight);
int  fde_server_poll(fde_server* s, long long ticket, int* done, fde_solve_info* info_host, int* cached);
/* cached problems, their device bytes, and the cache's hits, misses and evictions */
int  fde_server_stats(const fde_server* s, int* entries, size_t* bytes, long long* hits, long long* misses,
                      long long* evictions);

const char* fde_last_error(void);
const char* fde_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDE_H */
