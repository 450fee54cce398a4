// Flattening of the recursive H-LU (Section 4.1) and of the forward/backward
// H-substitutions into an op list executed by the device interpreter.
//
// The recursion is the block-recursive H-LU of Borm, Grasedyck and Hackbusch
// cited in Section 4.1:
//   LU(A) : LU(A00); A01 <- L00^{-1} A01; A10 <- A10 U00^{-1};
//           A11 <- A11 - A10 A01 (truncated); LU(A11)
// with triangular solves and products recursing over the block tree, low-rank
// products formed through their factors and every low-rank sum recompressed
// (OP_LRSUB). Ranks are data dependent, so dimensions that equal a block's
// current rank are encoded as rank slots and read on the device.
#include <algorithm>
#include <cstdio>

#include "hmatrix.h"

namespace fde {

namespace {

struct Slab {
    View v;
    int rows;
    int width;   // dimension code
};

inline int rank_code(const Block& b) { return -2 - b.slot; }

class Gen {
   public:
    Gen(const HTree& hm, Program& p, bool solve) : hm_(hm), p_(p), solve_(solve) {}

    // ---- views
    int rows(int b) const { return hm_.cl[hm_.bl[b].tau].size(); }
    int cols(int b) const { return hm_.cl[hm_.bl[b].sigma].size(); }
    const Block& B(int b) const { return hm_.bl[b]; }
    int ch(int b, int i, int j) const { return hm_.bl[b].child[2 * i + j]; }
    View dense(int b) const { return View{B_ARENA, 1, rows(b), B(b).off}; }
    View denseT(int b) const { return View{B_ARENA, rows(b), 1, B(b).off}; }
    Slab U(int b) const { return Slab{View{B_ARENA, 1, rows(b), B(b).uoff}, rows(b), rank_code(B(b))}; }
    Slab V(int b) const { return Slab{View{B_ARENA, 1, cols(b), B(b).voff}, cols(b), rank_code(B(b))}; }
    static View T(const View& v) { return View{v.base, v.cs, v.rs, v.off}; }
    static Slab rows_of(const Slab& s, int r0, int nr) {
        Slab o = s;
        o.v.off += (int64_t)r0 * s.v.rs;
        o.rows = nr;
        return o;
    }
    // split a slab along the two children of the row cluster
    Slab half(const Slab& s, int cluster, int which) const {
        const Cluster& c = hm_.cl[cluster];
        const Cluster& c0 = hm_.cl[c.child[0]];
        if (which == 0) return rows_of(s, 0, c0.size());
        return rows_of(s, c0.size(), c.size() - c0.size());
    }

    // ---- temporaries: a stack in the H-substitutions; in the factorisation every
    // temporary is distinct (the level schedule gives them memory afterwards)
    Slab alloc(int rows_, int width, int cap) {
        Slab s;
        s.rows = rows_;
        s.width = width;
        if (solve_) {
            s.v = View{3, 1, rows_, top_};   // base 3: offset and columns scale with nrhs
            top_ += rows_;
        } else {
            s.v = View{B_WORK, 1, rows_, top_};
            p_.temps.push_back(TempRegion{top_, rows_, cap});
            top_ += (int64_t)rows_ * cap;
        }
        high_ = std::max(high_, top_);
        return s;
    }
    void release(const Slab& s) {
        if (solve_) top_ = s.v.off;
    }
    int cap(int width) const { return width >= 0 ? width : hm_.kmax; }

    // ---- emitters
    void gemm(const View& C, const View& A, const View& Bv, int m, int n, int k, float alpha, float beta) {
        OpRec o{};
        o.code = OP_GEMM;
        o.v[0] = C;
        o.v[1] = A;
        o.v[2] = Bv;
        o.dim[0] = m;
        o.dim[1] = n;
        o.dim[2] = k;
        o.alpha = alpha;
        o.beta = beta;
        p_.ops.push_back(o);
    }
    void trsm(const View& Tv, int n, const Slab& X, bool lower, bool unit) {
        OpRec o{};
        o.code = OP_TRSM;
        o.flags = (lower ? 1 : 0) | (unit ? 2 : 0);
        o.v[0] = X.v;
        o.v[1] = Tv;
        o.dim[0] = n;
        o.dim[1] = X.width;
        p_.ops.push_back(o);
    }
    void lrsub(int b, const Slab& X, const Slab& Y) {
        OpRec o{};
        o.code = OP_LRSUB;
        o.blk = B(b).lr_id;
        o.v[0] = X.v;
        o.v[1] = Y.v;
        o.dim[2] = X.width;
        kx_max_ = std::max(kx_max_, X.width >= 0 ? X.width : hm_.kmax);
        p_.ops.push_back(o);
    }

    // ---- H-arithmetic (same recursion and order as the FP64 reference)
    // Y += alpha A X; with `first`, Y = alpha A X: the first product into each row range of Y
    // overwrites it (beta = 0, the same bits as adding to zeros), so no op clears Y beforehand
    void matmul_add(int A, const Slab& X, const Slab& Y, float alpha, bool first = false) {
        const Block& a = B(A);
        const float beta = first ? 0.f : 1.f;
        if (first && solve_) fail(FDE_EDEVICE, "H-solve program: overwriting product");
        if (a.kind == kDense) {
            gemm(Y.v, dense(A), X.v, rows(A), X.width, cols(A), alpha, beta);
        } else if (a.kind == kLowRank) {
            Slab t = alloc(hm_.kmax, X.width, solve_ ? 1 : cap(X.width));
            if (solve_) {
                OpRec o{};
                o.code = OP_LRMV;
                o.blk = a.lr_id;
                o.v[0] = Y.v;
                o.v[1] = X.v;
                o.v[2] = t.v;
                o.dim[0] = rows(A);
                o.dim[1] = X.width;
                o.dim[2] = rank_code(a);
                o.alpha = alpha;
                p_.ops.push_back(o);
            } else {
                gemm(t.v, T(V(A).v), X.v, rank_code(a), X.width, cols(A), 1.f, 0.f);
                gemm(Y.v, U(A).v, t.v, rows(A), X.width, rank_code(a), alpha, beta);
            }
            release(t);
        } else {
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    matmul_add(ch(A, i, j), half(X, a.sigma, j), half(Y, a.tau, i), alpha, first && j == 0);
        }
    }
    // Y += alpha A^T X (Y = alpha A^T X with `first`, as above)
    void matmulT_add(int A, const Slab& X, const Slab& Y, float alpha, bool first = false) {
        const Block& a = B(A);
        const float beta = first ? 0.f : 1.f;
        if (first && solve_) fail(FDE_EDEVICE, "H-solve program: overwriting product");
        if (a.kind == kDense) {
            gemm(Y.v, denseT(A), X.v, cols(A), X.width, rows(A), alpha, beta);
        } else if (a.kind == kLowRank) {
            Slab t = alloc(hm_.kmax, X.width, solve_ ? 1 : cap(X.width));
            gemm(t.v, T(U(A).v), X.v, rank_code(a), X.width, rows(A), 1.f, 0.f);
            gemm(Y.v, V(A).v, t.v, cols(A), X.width, rank_code(a), alpha, beta);
            release(t);
        } else {
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i)
                    matmulT_add(ch(A, i, j), half(X, a.tau, i), half(Y, a.sigma, j), alpha, first && i == 0);
        }
    }
    void lr_sub(int C, const Slab& X, const Slab& Y) {   // C <- C - X Y^T
        const Block& c = B(C);
        if (c.kind == kDense) {
            gemm(dense(C), X.v, T(Y.v), rows(C), cols(C), X.width, -1.f, 1.f);
        } else if (c.kind == kLowRank) {
            lrsub(C, X, Y);
        } else {
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) lr_sub(ch(C, i, j), half(X, c.tau, i), half(Y, c.sigma, j));
        }
    }
    void gemm_sub(int C, int A, int Bb) {   // C <- C - A B
        const Block &a = B(A), &b = B(Bb), &c = B(C);
        if (a.kind == kLowRank) {
            Slab W = alloc(cols(Bb), rank_code(a), hm_.kmax);
            matmulT_add(Bb, V(A), W, 1.f, true);
            lr_sub(C, U(A), W);
            release(W);
        } else if (b.kind == kLowRank) {
            Slab Z = alloc(rows(A), rank_code(b), hm_.kmax);
            matmul_add(A, U(Bb), Z, 1.f, true);
            lr_sub(C, Z, V(Bb));
            release(Z);
        } else if (a.kind == kDense && b.kind == kDense) {
            if (c.kind == kDense) {
                gemm(dense(C), dense(A), dense(Bb), rows(C), cols(C), cols(A), -1.f, 1.f);
            } else if (c.kind == kLowRank) {
                lr_sub(C, Slab{dense(A), rows(A), cols(A)}, Slab{denseT(Bb), cols(Bb), rows(Bb)});
                hm_max_inner_ = std::max(hm_max_inner_, cols(A));
            } else {
                fail(FDE_EUNSUPPORTED, "H-LU: dense product into a hierarchical block");
            }
        } else if (a.kind == kHier && b.kind == kHier && c.kind == kHier) {
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int l = 0; l < 2; ++l) gemm_sub(ch(C, i, j), ch(A, i, l), ch(Bb, l, j));
        } else {
            fail(FDE_EUNSUPPORTED, "H-LU: product of kinds %d x %d into kind %d is not handled", a.kind,
                 b.kind, c.kind);
        }
    }
    void solve_L(int L, const Slab& X) {   // X <- L^{-1} X, unit lower
        const Block& l = B(L);
        if (l.kind == kDense) {
            trsm(dense(L), rows(L), X, true, true);
            return;
        }
        const Slab X0 = half(X, l.tau, 0), X1 = half(X, l.tau, 1);
        solve_L(ch(L, 0, 0), X0);
        matmul_add(ch(L, 1, 0), X0, X1, -1.f);
        solve_L(ch(L, 1, 1), X1);
    }
    void solve_U(int Uu, const Slab& X) {   // X <- U^{-1} X
        const Block& u = B(Uu);
        if (u.kind == kDense) {
            trsm(dense(Uu), rows(Uu), X, false, false);
            return;
        }
        const Slab X0 = half(X, u.tau, 0), X1 = half(X, u.tau, 1);
        solve_U(ch(Uu, 1, 1), X1);
        matmul_add(ch(Uu, 0, 1), X1, X0, -1.f);
        solve_U(ch(Uu, 0, 0), X0);
    }
    void solve_UT(int Uu, const Slab& X) {   // X <- U^{-T} X
        const Block& u = B(Uu);
        if (u.kind == kDense) {
            trsm(denseT(Uu), rows(Uu), X, true, false);
            return;
        }
        const Slab X0 = half(X, u.tau, 0), X1 = half(X, u.tau, 1);
        solve_UT(ch(Uu, 0, 0), X0);
        matmulT_add(ch(Uu, 0, 1), X0, X1, -1.f);
        solve_UT(ch(Uu, 1, 1), X1);
    }
    void trsm_L(int L, int Bb) {   // B <- L^{-1} B
        const Block& b = B(Bb);
        if (b.kind == kLowRank) {
            solve_L(L, U(Bb));
        } else if (b.kind == kDense) {
            solve_L(L, Slab{dense(Bb), rows(Bb), cols(Bb)});
        } else {
            trsm_L(ch(L, 0, 0), ch(Bb, 0, 0));
            trsm_L(ch(L, 0, 0), ch(Bb, 0, 1));
            gemm_sub(ch(Bb, 1, 0), ch(L, 1, 0), ch(Bb, 0, 0));
            gemm_sub(ch(Bb, 1, 1), ch(L, 1, 0), ch(Bb, 0, 1));
            trsm_L(ch(L, 1, 1), ch(Bb, 1, 0));
            trsm_L(ch(L, 1, 1), ch(Bb, 1, 1));
        }
    }
    void trsm_U(int Uu, int Bb) {   // B <- B U^{-1}
        const Block& b = B(Bb);
        if (b.kind == kLowRank) {
            solve_UT(Uu, V(Bb));
        } else if (b.kind == kDense) {
            solve_UT(Uu, Slab{denseT(Bb), cols(Bb), rows(Bb)});
        } else {
            trsm_U(ch(Uu, 0, 0), ch(Bb, 0, 0));
            trsm_U(ch(Uu, 0, 0), ch(Bb, 1, 0));
            gemm_sub(ch(Bb, 0, 1), ch(Bb, 0, 0), ch(Uu, 0, 1));
            gemm_sub(ch(Bb, 1, 1), ch(Bb, 1, 0), ch(Uu, 0, 1));
            trsm_U(ch(Uu, 1, 1), ch(Bb, 0, 1));
            trsm_U(ch(Uu, 1, 1), ch(Bb, 1, 1));
        }
    }
    void hlu(int A) {
        const Block& a = B(A);
        if (a.kind == kDense) {
            OpRec o{};
            o.code = OP_GETRF;
            o.v[0] = dense(A);
            o.dim[0] = rows(A);
            p_.ops.push_back(o);
            return;
        }
        hlu(ch(A, 0, 0));
        trsm_L(ch(A, 0, 0), ch(A, 0, 1));
        trsm_U(ch(A, 0, 0), ch(A, 1, 0));
        gemm_sub(ch(A, 1, 1), ch(A, 1, 0), ch(A, 0, 1));
        hlu(ch(A, 1, 1));
    }

    int64_t high() const { return high_; }
    int kx_max() const { return kx_max_; }
    int max_inner() const { return hm_max_inner_; }

   private:
    const HTree& hm_;
    Program& p_;
    bool solve_;
    int64_t top_ = 0, high_ = 0;
    int kx_max_ = 0;
    int hm_max_inner_ = 0;
};

}  // namespace

void gen_hlu(const HTree& hm, Program& prog) {
    prog = Program{};
    Gen g(hm, prog, false);
    g.hlu(hm.root);
    prog.work_elems = g.high();
    prog.kx_max = g.kx_max();
}

void gen_hsolve(const HTree& hm, Program& prog) {
    prog = Program{};
    Gen g(hm, prog, true);
    OpRec ld{};
    ld.code = OP_LOAD;
    prog.ops.push_back(ld);
    const int Nd = hm.op->Nd;
    Slab X{View{B_RHS, 1, Nd, 0}, Nd, -1};
    g.solve_L(hm.root, X);
    g.solve_U(hm.root, X);
    OpRec st{};
    st.code = OP_STORE;
    prog.ops.push_back(st);
    prog.work_elems = g.high();   // in row units (times nrhs on the device)
    prog.kx_max = 0;
}

int lrsub_kprime_max(const HTree& hm, const Program& lu) { return hm.kmax + std::max(lu.kx_max, 1); }

void lrsub_need(const HTree& hm, const OpRec& o, int64_t* t_elems, int64_t* d_elems) {
    const Block& b = hm.bl[hm.lr_blocks[o.blk]];
    const int64_t m = hm.cl[b.tau].size(), n = hm.cl[b.sigma].size();
    const int64_t kp = hm.kmax + (o.dim[2] >= 0 ? o.dim[2] : hm.kmax);
    const int64_t kf = std::min<int64_t>(kp, 32);
    // QR path: [U, -X] and [V, Y] copies and both triangles; FP64 core, rotations, singular values
    *t_elems = (m + n) * kp + 2 * kp * kp;
    // Gram path (k' <= 32): twelve k' x k' FP64 matrices, three 32-vectors, one side's rows x k'
    *d_elems = std::max(2 * kp * kp + 2 * kp, 12 * kf * kf + 3 * 32 + std::max(m, n) * kf);
}

// Every view an op touches must stay inside its region; checked on the host with
// dynamic dimensions at their upper bounds before any program reaches the device.
void validate_program(const HTree& hm, const Program& prog, int64_t arena_elems, int64_t work_elems,
                      int nrhs_max, bool solve) {
    const int Nd = hm.op->Nd;
    auto dimv = [&](int d) -> int64_t {
        if (d >= 0) return d;
        if (d == -1) return nrhs_max;
        return hm.kmax;
    };
    auto check = [&](const View& v, int64_t r, int64_t c, int pc, const char* what) {
        if (r <= 0 || c <= 0) return;
        if (v.rs < 0 || v.cs < 0 || v.off < 0) fail(FDE_EDEVICE, "program op %d (%s): negative view", pc, what);
        int64_t off = v.off, cs = v.cs, lim;
        switch (v.base) {
            case B_ARENA: lim = arena_elems; break;
            case B_WORK: lim = work_elems; break;
            case B_RHS: lim = (int64_t)Nd * nrhs_max; break;
            case 3: off *= nrhs_max; lim = work_elems * nrhs_max; break;
            default: fail(FDE_EDEVICE, "program op %d: bad base %d", pc, v.base);
        }
        const int64_t last = off + (r - 1) * v.rs + (c - 1) * cs;
        if (last >= lim) fail(FDE_EDEVICE, "program op %d (%s): view reaches %lld >= %lld (base %d)", pc, what,
                              (long long)last, (long long)lim, v.base);
    };
    for (size_t pc = 0; pc < prog.ops.size(); ++pc) {
        const OpRec& o = prog.ops[pc];
        switch (o.code) {
            case OP_GEMM: {
                const int64_t m = dimv(o.dim[0]), n = dimv(o.dim[1]), k = dimv(o.dim[2]);
                check(o.v[0], m, n, (int)pc, "gemm C");
                check(o.v[1], m, k, (int)pc, "gemm A");
                check(o.v[2], k, n, (int)pc, "gemm B");
                break;
            }
            case OP_TRSM: {
                const int64_t n = dimv(o.dim[0]), w = dimv(o.dim[1]);
                check(o.v[0], n, w, (int)pc, "trsm X");
                check(o.v[1], n, n, (int)pc, "trsm T");
                break;
            }
            case OP_GETRF: check(o.v[0], o.dim[0], o.dim[0], (int)pc, "getrf"); break;
            case OP_ZERO: check(o.v[0], dimv(o.dim[0]), dimv(o.dim[1]), (int)pc, "zero"); break;
            case OP_LRSUB: {
                if (o.blk < 0 || o.blk >= (int)hm.lr_blocks.size()) fail(FDE_EDEVICE, "program op %zu: bad block", pc);
                const Block& b = hm.bl[hm.lr_blocks[o.blk]];
                const int64_t k = dimv(o.dim[2]);
                check(o.v[0], hm.cl[b.tau].size(), k, (int)pc, "lrsub X");
                check(o.v[1], hm.cl[b.sigma].size(), k, (int)pc, "lrsub Y");
                if (hm.kmax + k > kMaxKprime) fail(FDE_EUNSUPPORTED, "program op %zu: recompression width %lld > %d", pc,
                                                   (long long)(hm.kmax + k), kMaxKprime);
                int64_t nt, nd;
                lrsub_need(hm, o, &nt, &nd);
                if (o.sofs_t < 0 || o.sofs_d < 0 || o.sofs_t + nt > prog.scr_t || o.sofs_d + nd > prog.scr_d)
                    fail(FDE_EDEVICE, "program op %zu: recompression scratch out of range", pc);
                break;
            }
            case OP_LRMV: {
                if (!solve) fail(FDE_EDEVICE, "program op %zu: low-rank product op in a factorisation", pc);
                if (o.blk < 0 || o.blk >= (int)hm.lr_blocks.size()) fail(FDE_EDEVICE, "program op %zu: bad block", pc);
                const Block& b = hm.bl[hm.lr_blocks[o.blk]];
                const int64_t w = dimv(o.dim[1]);
                if (o.dim[0] != hm.cl[b.tau].size() || o.dim[2] != -2 - b.slot)
                    fail(FDE_EDEVICE, "program op %zu: low-rank product dimensions", pc);
                check(o.v[0], hm.cl[b.tau].size(), w, (int)pc, "lrmv Y");
                check(o.v[1], hm.cl[b.sigma].size(), w, (int)pc, "lrmv X");
                check(o.v[2], hm.kmax, w, (int)pc, "lrmv t");
                break;
            }
            case OP_LOAD:
            case OP_STORE:
                if (!solve) fail(FDE_EDEVICE, "load/store in a factorisation program");
                break;
            default: fail(FDE_EDEVICE, "program op %zu: unknown code %d", pc, o.code);
        }
    }
}

}  // namespace fde
