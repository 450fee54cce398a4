// Level schedule of an H-LU program.
//
// The recursion of Section 4.1 is written down as one op list in program
// order, but most of its ops are independent: the two triangular solves of a
// step, the four quadrant updates of a product, the recompressions of
// different blocks. On a GPU with 256 compute units the factorisation of one
// operator runs as a sequence of levels; every op of a level depends only on
// ops of earlier levels, and the ops of a level run concurrently, one
// workgroup each.
//
// Dependencies are found from the memory each op reads and writes. Every view
// of a program lies in one storage region -- a dense block, the U or V factor
// of a low-rank block, one temporary -- and covers a rectangle of it (a row
// range of a column-major slab, or of its transpose). An op's level is one
// more than the highest level of an earlier access to an overlapping
// rectangle that conflicts with it (read after write, write after read or
// write). After the levels are known, temporaries whose level lifetimes do not
// overlap share memory, and every recompression gets private scratch inside
// its level.
#include <algorithm>
#include <map>
#include <numeric>
#include <queue>

#include "hmatrix.h"

namespace fde {

namespace {

struct Region {
    int64_t start;
    int ld, rows, cols;
    int base;
};

struct Rect {
    int region;
    int r0, r1, c0, c1;   // half-open
};

struct Acc {
    int r0, r1, c0, c1;
    int level;
    bool write;
};

class Regions {
   public:
    Regions(const HTree& hm, const Program& prog) {
        for (int b : hm.dense_blocks) {
            const Block& B = hm.bl[b];
            const int m = hm.cl[B.tau].size(), n = hm.cl[B.sigma].size();
            add(Region{B.off, m, m, n, B_ARENA});
        }
        for (int b : hm.lr_blocks) {
            const Block& B = hm.bl[b];
            const int m = hm.cl[B.tau].size(), n = hm.cl[B.sigma].size();
            add(Region{B.uoff, m, m, hm.kmax, B_ARENA});
            add(Region{B.voff, n, n, hm.kmax, B_ARENA});
        }
        for (const TempRegion& t : prog.temps) add(Region{t.off, t.rows, t.rows, t.cols, B_WORK});
        slot0_ = (int)reg_.size();
        for (int s = 0; s < hm.nslots; ++s) reg_.push_back(Region{0, 1, 1, 1, -1});
        for (int base : {B_ARENA, B_WORK}) {
            auto& v = order_[base == B_ARENA ? 0 : 1];
            for (int i = 0; i < slot0_; ++i)
                if (reg_[i].base == base) v.push_back(i);
            std::sort(v.begin(), v.end(), [&](int a, int b) { return reg_[a].start < reg_[b].start; });
        }
    }
    int size() const { return (int)reg_.size(); }
    const Region& operator[](int i) const { return reg_[i]; }
    int slot(int s) const { return slot0_ + s; }

    // rectangle of region coordinates covered by a view of m x n elements (element (i, j) at
    // off + i rs + j cs); the whole region where the view does not match its layout
    Rect rect(const View& v, int64_t m, int64_t n) const {
        if (v.base != B_ARENA && v.base != B_WORK) fail(FDE_EDEVICE, "schedule: view base %d in a factorisation", v.base);
        const auto& ord = order_[v.base == B_ARENA ? 0 : 1];
        auto it = std::upper_bound(ord.begin(), ord.end(), v.off,
                                   [&](int64_t off, int r) { return off < reg_[r].start; });
        if (it == ord.begin()) fail(FDE_EDEVICE, "schedule: view at %lld lies in no region", (long long)v.off);
        const int r = *(it - 1);
        const Region& R = reg_[r];
        const int64_t o = v.off - R.start;
        const int64_t r0 = o % R.ld, c0 = o / R.ld;
        Rect x{r, 0, R.rows, 0, R.cols};
        if (v.rs == 1 && v.cs == R.ld) {
            x = Rect{r, (int)r0, (int)(r0 + m), (int)c0, (int)(c0 + n)};
        } else if (v.rs == R.ld && v.cs == 1) {
            x = Rect{r, (int)r0, (int)(r0 + n), (int)c0, (int)(c0 + m)};
        }
        if (x.r0 < 0 || x.c0 < 0 || x.r1 > R.rows || x.c1 > R.cols || x.r0 >= x.r1 || x.c0 >= x.c1)
            fail(FDE_EDEVICE, "schedule: view of %lld x %lld at %lld leaves its region", (long long)m, (long long)n,
                 (long long)v.off);
        return x;
    }

   private:
    void add(const Region& r) { reg_.push_back(r); }
    std::vector<Region> reg_;
    std::vector<int> order_[2];
    int slot0_ = 0;
};

// an earlier access as the dependency list sees it: every op on its own (no merged reads)
struct OpAcc {
    int r0, r1, c0, c1;
    int pc;
    bool write;
};

template <class A>
inline bool overlap(const Rect& a, const A& b) {
    return a.r0 < b.r1 && b.r0 < a.r1 && a.c0 < b.c1 && b.c0 < a.c1;
}
template <class A>
inline bool contains(const Rect& a, const A& b) {
    return a.r0 <= b.r0 && b.r1 <= a.r1 && a.c0 <= b.c0 && b.c1 <= a.c1;
}

// reads and writes of one op, dynamic dimensions at their bounds
void accesses(const HTree& hm, const Regions& R, const OpRec& o, std::vector<Rect>& rd, std::vector<Rect>& wr) {
    rd.clear();
    wr.clear();
    auto dimv = [&](int d) -> int64_t { return d >= 0 ? d : hm.kmax; };
    auto slot = [&](int d) {
        if (d <= -2) rd.push_back(Rect{R.slot(-2 - d), 0, 1, 0, 1});
    };
    for (int k = 0; k < 3; ++k) slot(o.dim[k]);
    switch (o.code) {
        case OP_GEMM: {
            const int64_t m = dimv(o.dim[0]), n = dimv(o.dim[1]), k = dimv(o.dim[2]);
            if (m <= 0 || n <= 0) break;
            if (k > 0) {
                rd.push_back(R.rect(o.v[1], m, k));
                rd.push_back(R.rect(o.v[2], k, n));
            }
            wr.push_back(R.rect(o.v[0], m, n));   // also read when beta != 0: the write covers it
            break;
        }
        case OP_TRSM: {
            const int64_t n = dimv(o.dim[0]), w = dimv(o.dim[1]);
            if (n <= 0 || w <= 0) break;
            rd.push_back(R.rect(o.v[1], n, n));
            wr.push_back(R.rect(o.v[0], n, w));
            break;
        }
        case OP_GETRF:
            if (o.dim[0] > 0) wr.push_back(R.rect(o.v[0], o.dim[0], o.dim[0]));
            break;
        case OP_ZERO: {
            const int64_t m = dimv(o.dim[0]), n = dimv(o.dim[1]);
            if (m > 0 && n > 0) wr.push_back(R.rect(o.v[0], m, n));
            break;
        }
        case OP_LRSUB: {
            const Block& b = hm.bl[hm.lr_blocks[o.blk]];
            const int64_t m = hm.cl[b.tau].size(), n = hm.cl[b.sigma].size(), k = dimv(o.dim[2]);
            if (k > 0) {
                rd.push_back(R.rect(o.v[0], m, k));
                rd.push_back(R.rect(o.v[1], n, k));
            }
            wr.push_back(R.rect(View{B_ARENA, 1, (int)m, b.uoff}, m, hm.kmax));
            wr.push_back(R.rect(View{B_ARENA, 1, (int)n, b.voff}, n, hm.kmax));
            wr.push_back(Rect{R.slot(b.slot), 0, 1, 0, 1});
            break;
        }
        default: fail(FDE_EDEVICE, "schedule: op code %d in a factorisation", o.code);
    }
}

}  // namespace

void schedule_levels(const HTree& hm, Program& prog, bool with_deps) {
    const size_t nops = prog.ops.size();
    Regions R(hm, prog);
    std::vector<std::vector<Acc>> hist(R.size());
    std::vector<std::vector<OpAcc>> ohist(R.size());
    std::vector<std::vector<int>> preds(nops);   // program order
    std::vector<int> level(nops, 0);
    std::vector<Rect> rd, wr;
    int nlev = 0;
    for (size_t pc = 0; pc < nops; ++pc) {
        accesses(hm, R, prog.ops[pc], rd, wr);
        // dependencies: the last writes of what the op reads, every access since of what it writes
        // (kept per op, unmerged, so they cost more than the levels: only when asked for)
        if (with_deps) {
            std::vector<int>& pp = preds[pc];
            for (const Rect& x : rd)
                for (const OpAcc& a : ohist[x.region])
                    if (a.write && overlap(x, a)) pp.push_back(a.pc);
            for (const Rect& x : wr)
                for (const OpAcc& a : ohist[x.region])
                    if (overlap(x, a)) pp.push_back(a.pc);
            for (const Rect& x : wr) {
                auto& h = ohist[x.region];
                h.erase(std::remove_if(h.begin(), h.end(), [&](const OpAcc& a) { return contains(x, a); }), h.end());
            }
            for (const Rect& x : rd) ohist[x.region].push_back(OpAcc{x.r0, x.r1, x.c0, x.c1, (int)pc, false});
            for (const Rect& x : wr) ohist[x.region].push_back(OpAcc{x.r0, x.r1, x.c0, x.c1, (int)pc, true});
        }
        int L = 0;
        for (const Rect& x : rd)
            for (const Acc& a : hist[x.region])
                if (a.write && overlap(x, a)) L = std::max(L, a.level);
        for (const Rect& x : wr)
            for (const Acc& a : hist[x.region])
                if (overlap(x, a)) L = std::max(L, a.level);
        L += 1;
        level[pc] = L;
        nlev = std::max(nlev, L);
        for (const Rect& x : wr) {
            auto& h = hist[x.region];
            h.erase(std::remove_if(h.begin(), h.end(), [&](const Acc& a) { return contains(x, a); }), h.end());
            h.push_back(Acc{x.r0, x.r1, x.c0, x.c1, L, true});
        }
        for (const Rect& x : rd) {
            // repeated reads of one rectangle keep one entry at the highest level
            auto& h = hist[x.region];
            bool merged = false;
            for (Acc& a : h)
                if (!a.write && a.r0 == x.r0 && a.r1 == x.r1 && a.c0 == x.c0 && a.c1 == x.c1) {
                    a.level = std::max(a.level, L);
                    merged = true;
                    break;
                }
            if (!merged) h.push_back(Acc{x.r0, x.r1, x.c0, x.c1, L, false});
        }
    }

    // temporaries: level lifetimes, then memory shared between lifetimes that do not overlap
    const size_t nt = prog.temps.size();
    std::vector<int> first(nt, nlev + 1), last(nt, 0);
    std::vector<int64_t> tstart(nt);
    for (size_t t = 0; t < nt; ++t) tstart[t] = prog.temps[t].off;
    auto temp_of = [&](int64_t off) -> size_t {
        auto it = std::upper_bound(tstart.begin(), tstart.end(), off);
        return (size_t)(it - tstart.begin()) - 1;
    };
    std::vector<std::vector<int>> temp_ops(nt);   // ops (program order) that use each temporary
    auto touch = [&](size_t pc, const View& v) {
        if (v.base != B_WORK || nt == 0) return;
        const size_t t = temp_of(v.off);
        first[t] = std::min(first[t], level[pc]);
        last[t] = std::max(last[t], level[pc]);
        if (temp_ops[t].empty() || temp_ops[t].back() != (int)pc) temp_ops[t].push_back((int)pc);
    };
    auto views_used = [](const OpRec& o) {
        switch (o.code) {
            case OP_GEMM: return 3;
            case OP_TRSM: case OP_LRSUB: return 2;
            case OP_GETRF: case OP_ZERO: return 1;
            default: return 0;
        }
    };
    for (size_t pc = 0; pc < nops; ++pc)
        for (int k = 0; k < views_used(prog.ops[pc]); ++k) touch(pc, prog.ops[pc].v[k]);
    std::vector<size_t> torder(nt);
    std::iota(torder.begin(), torder.end(), 0);
    std::stable_sort(torder.begin(), torder.end(), [&](size_t a, size_t b) { return first[a] < first[b]; });
    std::vector<int64_t> newoff(nt, 0);
    std::map<int64_t, std::vector<int64_t>> free_by_size;
    using Live = std::pair<int, size_t>;   // (last level, temp)
    std::priority_queue<Live, std::vector<Live>, std::greater<Live>> live;
    int64_t top = 0;
    std::map<int64_t, size_t> owner;   // offset -> temporary that used the memory last
    for (size_t t : torder) {
        if (first[t] > last[t]) continue;   // never used
        while (!live.empty() && live.top().first < first[t]) {
            const size_t u = live.top().second;
            live.pop();
            free_by_size[(int64_t)prog.temps[u].rows * prog.temps[u].cols].push_back(newoff[u]);
        }
        const int64_t sz = (int64_t)prog.temps[t].rows * prog.temps[t].cols;
        auto& fl = free_by_size[sz];
        if (!fl.empty()) {
            newoff[t] = fl.back();
            fl.pop_back();
            // memory handed on: every op on t waits for every op on its previous owner
            if (with_deps)
                for (int pc : temp_ops[t])
                    for (int q : temp_ops[owner.at(newoff[t])]) preds[pc].push_back(q);
        } else {
            newoff[t] = top;
            top += sz;
        }
        live.push(Live{last[t], t});
        owner[newoff[t]] = t;
    }
    for (size_t pc = 0; pc < nops; ++pc) {
        OpRec& o = prog.ops[pc];
        for (int k = 0; k < views_used(o); ++k) {
            View& v = o.v[k];
            if (v.base != B_WORK) continue;
            const size_t t = temp_of(v.off);
            v.off = newoff[t] + (v.off - tstart[t]);
        }
    }
    for (size_t t = 0; t < nt; ++t) prog.temps[t].off = newoff[t];
    prog.work_elems = top;

    // level order (stable: program order inside a level)
    std::vector<size_t> idx(nops);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return level[a] < level[b]; });
    std::vector<OpRec> ops(nops);
    prog.origin.resize(nops);
    for (size_t i = 0; i < nops; ++i) {
        ops[i] = prog.ops[idx[i]];
        prog.origin[i] = (int)idx[i];
    }
    prog.ops.swap(ops);
    // dependency lists in the level order (sorted, no repeats); empty when not asked for
    prog.dep_off.clear();
    prog.deps.clear();
    if (with_deps) {
        std::vector<int> where(nops);
        for (size_t i = 0; i < nops; ++i) where[idx[i]] = (int)i;
        prog.dep_off.assign(nops + 1, 0);
        prog.deps.clear();
        for (size_t i = 0; i < nops; ++i) {
            std::vector<int> d;
            for (int q : preds[idx[i]]) d.push_back(where[q]);
            std::sort(d.begin(), d.end());
            d.erase(std::unique(d.begin(), d.end()), d.end());
            for (int q : d)
                if (q >= (int)i) fail(FDE_EDEVICE, "schedule: op %zu depends on a later op", i);
            prog.deps.insert(prog.deps.end(), d.begin(), d.end());
            prog.dep_off[i + 1] = (int)prog.deps.size();
        }
    }
    prog.level_off.assign(nlev + 1, 0);
    for (size_t i = 0; i < nops; ++i) prog.level_off[level[idx[i]]]++;   // counts at index level
    // counts sit at 1..nlev; turn into offsets of levels 0..nlev-1
    {
        std::vector<int> off(nlev + 1, 0);
        for (int l = 1; l <= nlev; ++l) off[l] = off[l - 1] + prog.level_off[l];
        prog.level_off.swap(off);
    }

    // private scratch of every recompression inside its level (64-element aligned)
    prog.scr_t = prog.scr_d = 0;
    for (int l = 0; l < nlev; ++l) {
        int64_t ut = 0, ud = 0;
        for (int i = prog.level_off[l]; i < prog.level_off[l + 1]; ++i) {
            OpRec& o = prog.ops[i];
            if (o.code != OP_LRSUB) continue;
            int64_t nt_, nd_;
            lrsub_need(hm, o, &nt_, &nd_);
            o.sofs_t = ut;
            o.sofs_d = ud;
            ut += (nt_ + 63) / 64 * 64;
            ud += (nd_ + 63) / 64 * 64;
        }
        prog.scr_t = std::max(prog.scr_t, ut);
        prog.scr_d = std::max(prog.scr_d, ud);
    }
    prog.scr_t = std::max<int64_t>(prog.scr_t, 1);
    prog.scr_d = std::max<int64_t>(prog.scr_d, 1);
}

namespace {

// memory an op touches, element by element: views (m x n, read or written) and rank slots, with
// dynamic dimensions at their bounds (the views of recompression scratch are not included)
struct Use {
    View v;
    int64_t m, n;
    bool write;
};
void op_uses(const HTree& hm, const OpRec& o, size_t pc, std::vector<Use>& uses, std::vector<std::pair<int, bool>>& slots) {
    auto dimv = [&](int d) -> int64_t { return d >= 0 ? d : hm.kmax; };
    uses.clear();
    slots.clear();
    for (int k = 0; k < 3; ++k)
        if (o.dim[k] <= -2) slots.push_back({-2 - o.dim[k], false});
    switch (o.code) {
        case OP_GEMM: {
            const int64_t m = dimv(o.dim[0]), n = dimv(o.dim[1]), k = dimv(o.dim[2]);
            uses.push_back({o.v[1], m, k, false});
            uses.push_back({o.v[2], k, n, false});
            if (o.beta != 0.f) uses.push_back({o.v[0], m, n, false});   // C is read unless beta = 0
            uses.push_back({o.v[0], m, n, true});
            break;
        }
        case OP_TRSM:
            uses.push_back({o.v[1], dimv(o.dim[0]), dimv(o.dim[0]), false});
            uses.push_back({o.v[0], dimv(o.dim[0]), dimv(o.dim[1]), true});
            break;
        case OP_GETRF: uses.push_back({o.v[0], o.dim[0], o.dim[0], true}); break;
        case OP_ZERO: uses.push_back({o.v[0], dimv(o.dim[0]), dimv(o.dim[1]), true}); break;
        case OP_LRSUB: {
            const Block& b = hm.bl[hm.lr_blocks[o.blk]];
            const int64_t m = hm.cl[b.tau].size(), n = hm.cl[b.sigma].size(), k = dimv(o.dim[2]);
            uses.push_back({o.v[0], m, k, false});
            uses.push_back({o.v[1], n, k, false});
            uses.push_back({View{B_ARENA, 1, (int)m, b.uoff}, m, hm.kmax, true});
            uses.push_back({View{B_ARENA, 1, (int)n, b.voff}, n, hm.kmax, true});
            slots.push_back({b.slot, true});
            break;
        }
        default: fail(FDE_EDEVICE, "schedule check: op %zu has code %d", pc, o.code);
    }
}

// every element of a use, as an index into [arena | work space]
template <class F>
void each_element(const Use& u, int64_t AE, F&& fn) {
    for (int64_t j = 0; j < u.n; ++j)
        for (int64_t i = 0; i < u.m; ++i) {
            const int64_t o = u.v.off + i * u.v.rs + j * u.v.cs;
            fn(u.v.base == B_ARENA ? o : AE + o);
        }
}

// Dependency lists: replay the scheduled program in its level order over the memory it really
// uses (temporaries sharing memory included) and verify that every pair of conflicting accesses is
// ordered by the dependency graph (the earlier op is an ancestor of the later one). Ancestor sets
// are quadratic in the op count: programs above 20000 ops get only the cheap checks.
void check_deps(const HTree& hm, const Program& sp) {
    const size_t nops = sp.ops.size();
    if (sp.dep_off.size() != nops + 1 || (size_t)sp.dep_off.back() != sp.deps.size())
        fail(FDE_EDEVICE, "dependency check: table does not cover the program");
    for (size_t i = 0; i < nops; ++i)
        for (int k = sp.dep_off[i]; k < sp.dep_off[i + 1]; ++k)
            if (sp.deps[k] < 0 || (size_t)sp.deps[k] >= i) fail(FDE_EDEVICE, "dependency check: op %zu waits for a later op", i);
    if (nops > 20000) return;
    const size_t W = (nops + 63) / 64;
    std::vector<uint64_t> anc(nops * W, 0);
    for (size_t i = 0; i < nops; ++i)
        for (int k = sp.dep_off[i]; k < sp.dep_off[i + 1]; ++k) {
            const size_t q = sp.deps[k];
            for (size_t w = 0; w < W; ++w) anc[i * W + w] |= anc[q * W + w];
            anc[i * W + q / 64] |= 1ull << (q % 64);
        }
    auto ancestor = [&](size_t q, size_t i) { return (anc[i * W + q / 64] >> (q % 64)) & 1ull; };
    const int64_t AE = hm.arena_elems, WE = sp.work_elems, NS = hm.nslots;
    std::vector<int> lastw(AE + WE + NS, -1);
    std::vector<std::vector<int>> readers(AE + WE + NS);
    std::vector<Use> uses;
    std::vector<std::pair<int, bool>> slots;
    for (size_t i = 0; i < nops; ++i) {
        op_uses(hm, sp.ops[i], i, uses, slots);
        auto verify = [&](int64_t e, bool write) {
            if (e < 0 || e >= AE + WE + NS) fail(FDE_EDEVICE, "dependency check: op %zu outside its memory", i);
            if (lastw[e] >= 0 && (size_t)lastw[e] != i && !ancestor(lastw[e], i))
                fail(FDE_EDEVICE, "dependency check: op %zu does not wait for op %d", i, lastw[e]);
            if (write)
                for (int r : readers[e])
                    if ((size_t)r != i && !ancestor(r, i)) fail(FDE_EDEVICE, "dependency check: op %zu does not wait for op %d", i, r);
        };
        for (const Use& u : uses) each_element(u, AE, [&](int64_t e) { verify(e, u.write); });
        for (auto& sl : slots) verify(AE + WE + sl.first, sl.second);
        auto record = [&](int64_t e, bool write) {
            if (write) {
                lastw[e] = (int)i;
                readers[e].clear();
            } else if (readers[e].empty() || readers[e].back() != (int)i) {
                readers[e].push_back((int)i);
            }
        };
        for (const Use& u : uses)
            if (!u.write) each_element(u, AE, [&](int64_t e) { record(e, false); });
        for (const Use& u : uses)
            if (u.write) each_element(u, AE, [&](int64_t e) { record(e, true); });
        for (auto& sl : slots) record(AE + WE + sl.first, sl.second);
    }
}

}  // namespace

// Independent check: replay the original program element by element and verify that every
// pair of conflicting accesses is ordered by the levels of the scheduled ops, and that no two
// temporaries sharing memory in the schedule are live in the same level.
void check_schedule(const HTree& hm, const Program& original, const Program& scheduled) {
    const size_t nops = original.ops.size();
    if (scheduled.ops.size() != nops) fail(FDE_EDEVICE, "schedule check: op count changed");
    const int nlev = (int)scheduled.level_off.size() - 1;
    if ((size_t)scheduled.level_off.back() != nops || scheduled.origin.size() != nops)
        fail(FDE_EDEVICE, "schedule check: level table does not cover the program");
    std::vector<size_t> where(nops, nops);
    std::vector<int> level(nops, 0);
    for (int l = 0; l < nlev; ++l)
        for (int i = scheduled.level_off[l]; i < scheduled.level_off[l + 1]; ++i) {
            const int pc = scheduled.origin[i];
            if (pc < 0 || (size_t)pc >= nops || where[pc] != nops) fail(FDE_EDEVICE, "schedule check: bad permutation");
            where[pc] = i;
            level[pc] = l + 1;
        }
    for (size_t pc = 0; pc < nops; ++pc) {
        OpRec a = original.ops[pc], b = scheduled.ops[where[pc]];
        for (int k = 0; k < 3; ++k)
            if (a.v[k].base == B_WORK) a.v[k].off = b.v[k].off = 0;   // temporaries move (checked below)
        a.sofs_t = b.sofs_t = a.sofs_d = b.sofs_d = 0;
        bool same = a.code == b.code && a.flags == b.flags && a.blk == b.blk && a.alpha == b.alpha && a.beta == b.beta;
        for (int k = 0; k < 3; ++k)
            same = same && a.dim[k] == b.dim[k] && a.v[k].base == b.v[k].base && a.v[k].rs == b.v[k].rs &&
                   a.v[k].cs == b.v[k].cs && a.v[k].off == b.v[k].off;
        if (!same) fail(FDE_EDEVICE, "schedule check: op %zu changed", pc);
    }
    // element-wise replay in program order over the arena, the slots and the ORIGINAL temporaries
    const int64_t AE = hm.arena_elems, WE = original.work_elems, NS = hm.nslots;
    std::vector<int> lw(AE + WE + NS, 0), lr(AE + WE + NS, 0);
    std::vector<char> wrote(WE, 0);   // temporaries start undefined: none is read before a write
    std::vector<Use> uses;
    std::vector<std::pair<int, bool>> slots;
    // every access of an op is checked against the earlier ops before any of them is recorded
    // (an op may read and write the same elements)
    auto each = [&](const Use& u, auto&& fn) { each_element(u, AE, fn); };
    for (size_t pc = 0; pc < nops; ++pc) {
        const OpRec& o = original.ops[pc];
        const int L = level[pc];
        op_uses(hm, o, pc, uses, slots);
        auto verify = [&](int64_t e, bool write) {
            if (e < 0 || e >= AE + WE + NS) fail(FDE_EDEVICE, "schedule check: op %zu outside its memory", pc);
            if (L <= lw[e] || (write && L <= lr[e]))
                fail(FDE_EDEVICE, "schedule check: op %zu (level %d) conflicts with level %d", pc, L,
                     std::max(lw[e], write ? lr[e] : 0));
            if (!write && e >= AE && e < AE + WE && !wrote[e - AE])
                fail(FDE_EDEVICE, "schedule check: op %zu reads a temporary no earlier op wrote", pc);
        };
        auto record = [&](int64_t e, bool write) {
            if (write) {
                if (e >= AE && e < AE + WE) wrote[e - AE] = 1;
                lw[e] = L;
                lr[e] = 0;
            } else {
                lr[e] = std::max(lr[e], L);
            }
        };
        for (const Use& u : uses) {
            if (u.v.base == B_WORK && u.m > 0 && u.n > 0) {
                const int64_t last = u.v.off + (u.m - 1) * u.v.rs + (u.n - 1) * u.v.cs;
                if (u.v.off < 0 || last >= WE) fail(FDE_EDEVICE, "schedule check: op %zu outside the work space", pc);
            }
            each(u, [&](int64_t e) { verify(e, u.write); });
        }
        for (auto& s : slots) verify(AE + WE + s.first, s.second);
        for (const Use& u : uses)
            if (!u.write) each(u, [&](int64_t e) { record(e, false); });
        for (const Use& u : uses)
            if (u.write) each(u, [&](int64_t e) { record(e, true); });
        for (auto& s : slots) record(AE + WE + s.first, s.second);
    }
    // shared temporaries: for each level, no element of the scheduled work space is used by two
    // different original temporaries whose level lifetimes overlap
    const size_t nt = original.temps.size();
    if (nt != scheduled.temps.size()) fail(FDE_EDEVICE, "schedule check: temporaries changed");
    std::vector<int> first(nt, nlev + 1), last(nt, 0);
    std::vector<int64_t> ostart(nt);
    for (size_t t = 0; t < nt; ++t) ostart[t] = original.temps[t].off;
    for (size_t pc = 0; pc < nops; ++pc) {
        const OpRec& o = original.ops[pc];
        const int nv = o.code == OP_GEMM ? 3 : (o.code == OP_TRSM || o.code == OP_LRSUB) ? 2 : 1;
        for (int k = 0; k < nv; ++k) {
            if (o.v[k].base != B_WORK) continue;
            const size_t t = (size_t)(std::upper_bound(ostart.begin(), ostart.end(), o.v[k].off) - ostart.begin()) - 1;
            first[t] = std::min(first[t], level[pc]);
            last[t] = std::max(last[t], level[pc]);
            // the scheduled op addresses the same offset inside the moved temporary
            const View& sv = scheduled.ops[where[pc]].v[k];
            if (sv.base != B_WORK || sv.off - scheduled.temps[t].off != o.v[k].off - ostart[t])
                fail(FDE_EDEVICE, "schedule check: op %zu view %d not relocated with its temporary", pc, k);
        }
    }
    std::vector<std::pair<int64_t, size_t>> byoff;
    for (size_t t = 0; t < nt; ++t)
        if (first[t] <= last[t]) byoff.push_back({scheduled.temps[t].off, t});
    std::sort(byoff.begin(), byoff.end());
    for (size_t a = 0; a < byoff.size(); ++a) {
        const size_t t = byoff[a].second;
        const int64_t end = scheduled.temps[t].off + (int64_t)scheduled.temps[t].rows * scheduled.temps[t].cols;
        if (end > scheduled.work_elems) fail(FDE_EDEVICE, "schedule check: temporary beyond the work space");
        for (size_t b = a + 1; b < byoff.size() && byoff[b].first < end; ++b) {
            const size_t u = byoff[b].second;
            if (!(last[t] < first[u] || last[u] < first[t]))
                fail(FDE_EDEVICE, "schedule check: temporaries %zu and %zu share memory while both live", t, u);
        }
    }
    check_deps(hm, scheduled);
}

}  // namespace fde
