// Leaf-step form of the forward and backward H-substitutions (Section 4.1).
//
// The op-list form of the substitutions follows the block recursion and issues
// one small dependent op per leaf block. Here the same triangular solves are
// reorganised by leaf rows and pipelined by one leaf (the two phases of a step
// are described with HsStep). A low-rank block B = U_B V_B^T contributes
// U_B t_B with t_B = V_B^T x_sigma; t_B is accumulated leaf by leaf as the
// leaves of sigma are solved, and kept in a slot until the last leaf of tau has
// used it. Slots are shared between blocks whose lifetimes (in steps) do not
// overlap.
#include <algorithm>
#include <map>
#include <queue>

#include "hmatrix.h"

namespace fde {

namespace {

struct Leaf {
    int cl;      // cluster id
    int d0, d1;  // internal rows
};

}  // namespace

void gen_hsolve_steps(const HTree& hm, HsTables& tab) {
    tab = HsTables{};
    std::vector<Leaf> leaves;
    for (size_t c = 0; c < hm.cl.size(); ++c)
        if (hm.cl[c].leaf()) leaves.push_back(Leaf{(int)c, hm.cl[c].d0, hm.cl[c].d1});
    std::sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) { return a.d0 < b.d0; });
    const int L = (int)leaves.size();
    tab.nleaf = L;
    std::map<int, int> leaf_of_cluster;
    for (int i = 0; i < L; ++i) leaf_of_cluster[leaves[i].cl] = i;
    auto first_leaf = [&](int cl) {   // leaf index holding the first row of cluster cl
        const int d0 = hm.cl[cl].d0;
        int i = 0;
        while (i + 1 < L && leaves[i + 1].d0 <= d0) ++i;
        return i;
    };
    auto last_leaf = [&](int cl) {
        const int d1 = hm.cl[cl].d1;
        int i = L - 1;
        while (i > 0 && leaves[i].d0 >= d1) --i;
        return i;
    };
    std::vector<HsStep> steps;
    std::vector<HsRec> recs;
    int tslots = 0;
    for (int dir = 0; dir < 2; ++dir) {   // 0: forward with the lower blocks, 1: backward with the upper blocks
        auto pos = [&](int leaf) { return dir == 0 ? leaf : L - 1 - leaf; };
        // per step position: late chunks, t increments, early items (for the next position)
        std::vector<std::vector<HsRec>> late(L), inc(L), early(L);
        std::vector<int64_t> diag(L, -1);
        struct Ref {
            int list, p;
            size_t k;
        };
        struct Life {
            int start, end;   // first step (phase 1) that writes t, last step (phase 2) that reads it
            std::vector<Ref> refs;
        };
        std::vector<Life> lives;
        for (int b : hm.dense_blocks) {
            const Block& B = hm.bl[b];
            const Cluster &tc = hm.cl[B.tau], &sc = hm.cl[B.sigma];
            if (B.tau == B.sigma) {
                diag[leaf_of_cluster.at(B.tau)] = B.off;
                continue;
            }
            const bool lower = tc.d0 > sc.d0;
            if (lower != (dir == 0)) continue;
            const int p = pos(leaf_of_cluster.at(B.tau)), q = pos(leaf_of_cluster.at(B.sigma));
            if (q >= p) fail(FDE_EDEVICE, "H-solve: dense block outside its triangle");
            const int m = tc.size(), n = sc.size();
            for (int c0 = 0; c0 < n; c0 += kHsChunk) {
                const HsRec r{B.off + (int64_t)c0 * m, m, sc.d0 + c0, std::min(kHsChunk, n - c0), -1, -1, HS_DENSE};
                if (q == p - 1) late[p].push_back(r);
                else early[p - 1].push_back(r);
            }
        }
        for (int b : hm.lr_blocks) {
            const Block& B = hm.bl[b];
            const Cluster &tc = hm.cl[B.tau], &sc = hm.cl[B.sigma];
            const bool lower = tc.d0 > sc.d0;
            if (lower != (dir == 0)) continue;
            const int fs = first_leaf(B.sigma), ls = last_leaf(B.sigma);
            const int ft = first_leaf(B.tau), lt = last_leaf(B.tau);
            const int qmin = std::min(pos(fs), pos(ls)), qmax = std::max(pos(fs), pos(ls));
            const int pmin = std::min(pos(ft), pos(lt)), pmax = std::max(pos(ft), pos(lt));
            if (qmax > pmin - 2) return;   // tab.ok stays false
            Life lf;
            lf.start = qmin + 1;
            lf.end = pmax - 1;
            for (int l = fs; l <= ls; ++l) {
                const int q = pos(l);
                const Leaf& lv = leaves[l];
                inc[q + 1].push_back(HsRec{B.voff + (lv.d0 - sc.d0), sc.size(), lv.d0, lv.d1 - lv.d0, B.slot, -1,
                                           q == qmin ? HS_INC_FIRST : HS_INC});
                lf.refs.push_back(Ref{1, q + 1, inc[q + 1].size() - 1});
            }
            for (int i = ft; i <= lt; ++i) {
                const int p = pos(i);
                const Leaf& lv = leaves[i];
                early[p - 1].push_back(HsRec{B.uoff + (lv.d0 - tc.d0), tc.size(), 0, 0, B.slot, -1, HS_LOWRANK});
                lf.refs.push_back(Ref{2, p - 1, early[p - 1].size() - 1});
            }
            lives.push_back(std::move(lf));
        }
        // t slots: a slot is free for a new block from the step after its last reader
        std::vector<size_t> ord(lives.size());
        for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
        std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return lives[a].start < lives[b].start; });
        std::priority_queue<std::pair<int, int>, std::vector<std::pair<int, int>>, std::greater<std::pair<int, int>>> busy;
        std::vector<int> free_slots;
        int nslot = 0;
        for (size_t k : ord) {
            Life& lf = lives[k];
            while (!busy.empty() && busy.top().first < lf.start) {
                free_slots.push_back(busy.top().second);
                busy.pop();
            }
            int sl;
            if (!free_slots.empty()) {
                sl = free_slots.back();
                free_slots.pop_back();
            } else {
                sl = nslot++;
            }
            busy.push({lf.end, sl});
            for (const Ref& r : lf.refs) (r.list == 1 ? inc : early)[r.p][r.k].tslot = sl;
        }
        tslots = std::max(tslots, nslot);
        for (int p = 0; p < L; ++p) {
            const int i = dir == 0 ? p : L - 1 - p;
            if (diag[i] < 0) fail(FDE_EDEVICE, "leaf %d has no dense diagonal block", i);
            HsStep st;
            st.diag = diag[i];
            st.row0 = leaves[i].d0;
            st.nrow = leaves[i].d1 - leaves[i].d0;
            st.rec0 = (int)recs.size();
            st.nlate = (int)late[p].size();
            st.ninc = (int)inc[p].size();
            st.nearly = (int)early[p].size();
            for (auto* v : {&late[p], &inc[p], &early[p]}) recs.insert(recs.end(), v->begin(), v->end());
            steps.push_back(st);
            tab.maxrow = std::max(tab.maxrow, st.nrow);
            tab.maxrec = std::max(tab.maxrec, st.nlate + st.ninc + st.nearly);
        }
    }
    tab.steps = std::move(steps);
    tab.recs = std::move(recs);
    tab.tslots = tslots;
    tab.ok = true;
}

void validate_hsolve_steps(const HTree& hm, const HsTables& tab) {
    if (!tab.ok) return;
    const int64_t arena = hm.arena_elems;
    const int Nd = hm.op ? hm.op->Nd : 0;
    const int L = tab.nleaf, kmax = hm.kmax;
    if ((int)tab.steps.size() != 2 * L) fail(FDE_EDEVICE, "H-solve steps: %zu for %d leaves", tab.steps.size(), L);
    struct LR {
        int64_t uoff, voff;
        int t0, t1, s0, s1;   // tau and sigma rows
    };
    std::map<int, LR> by_slot;
    for (int b : hm.lr_blocks) {
        const Block& B = hm.bl[b];
        const Cluster &tc = hm.cl[B.tau], &sc = hm.cl[B.sigma];
        by_slot[B.slot] = LR{B.uoff, B.voff, tc.d0, tc.d1, sc.d0, sc.d1};
    }
    auto in_arena = [&](int64_t off, int rows, int cols, int ld) {
        return off >= 0 && rows >= 1 && cols >= 1 && ld >= rows && off + (rows - 1) + (int64_t)(cols - 1) * ld < arena;
    };
    for (int dir = 0; dir < 2; ++dir) {
        // step position at which each x row is solved
        std::vector<int> solved_at(Nd, -1);
        std::vector<int> owner(tab.tslots, -1), lo(tab.tslots, 0), hi(tab.tslots, 0);
        int64_t area = 0;
        for (int p = 0; p < L; ++p) {
            const HsStep& st = tab.steps[dir * L + p];
            const int n = st.nrow;
            if (n < 1 || st.row0 < 0 || st.row0 + n > Nd) fail(FDE_EDEVICE, "H-solve step rows out of range");
            if (!in_arena(st.diag, n, n, n)) fail(FDE_EDEVICE, "H-solve diagonal out of range");
            if (st.nlate < 0 || st.ninc < 0 || st.nearly < 0 || st.rec0 < 0 ||
                (size_t)st.rec0 + st.nlate + st.ninc + st.nearly > tab.recs.size())
                fail(FDE_EDEVICE, "H-solve records out of range");
            const HsStep* prev = p > 0 ? &tab.steps[dir * L + p - 1] : nullptr;
            const HsStep* next = p + 1 < L ? &tab.steps[dir * L + p + 1] : nullptr;
            if ((st.nlate > 0 || st.ninc > 0) && !prev) fail(FDE_EDEVICE, "H-solve: phase 1 work without a solved leaf");
            if (st.nearly > 0 && !next) fail(FDE_EDEVICE, "H-solve: early items without a next leaf");
            area += (int64_t)n * (n - 1) / 2;
            // phase 1: late chunks read the previous leaf; increments add the previous leaf's rows
            for (int k = 0; k < st.nlate + st.ninc; ++k) {
                const HsRec& r = tab.recs[st.rec0 + k];
                if (k < st.nlate) {
                    if (r.kind != HS_DENSE || r.n < 1 || r.n > kHsChunk || !in_arena(r.off, n, r.n, r.ld) ||
                        r.col0 < prev->row0 || r.col0 + r.n > prev->row0 + prev->nrow)
                        fail(FDE_EDEVICE, "H-solve late chunk");
                    area += (int64_t)n * r.n;
                } else {
                    if ((r.kind != HS_INC_FIRST && r.kind != HS_INC) || r.slot < 0 || r.tslot < 0 ||
                        r.tslot >= tab.tslots || !by_slot.count(r.slot))
                        fail(FDE_EDEVICE, "H-solve increment record");
                    const LR& b = by_slot.at(r.slot);
                    if (r.col0 != prev->row0 || r.n != prev->nrow || r.col0 < b.s0 || r.col0 + r.n > b.s1 ||
                        r.ld != b.s1 - b.s0 || r.off != b.voff + (r.col0 - b.s0) || !in_arena(r.off, r.n, kmax, r.ld))
                        fail(FDE_EDEVICE, "H-solve increment out of its block");
                    if (r.kind == HS_INC_FIRST) {
                        owner[r.tslot] = r.slot;
                        lo[r.tslot] = r.col0;
                        hi[r.tslot] = r.col0 + r.n;
                    } else {
                        if (owner[r.tslot] != r.slot) fail(FDE_EDEVICE, "H-solve t slot taken over while in use");
                        if (r.col0 + r.n == lo[r.tslot]) lo[r.tslot] = r.col0;
                        else if (r.col0 == hi[r.tslot]) hi[r.tslot] += r.n;
                        else fail(FDE_EDEVICE, "H-solve increments not contiguous");
                    }
                }
            }
            // phase 2: the leaf is solved; early items for the next leaf read only leaves <= p-1
            for (int k = 0; k < st.nearly; ++k) {
                const HsRec& r = tab.recs[st.rec0 + st.nlate + st.ninc + k];
                const int m = next->nrow;
                if (r.kind == HS_DENSE) {
                    if (r.n < 1 || r.n > kHsChunk || !in_arena(r.off, m, r.n, r.ld) || r.col0 < 0 || r.col0 + r.n > Nd)
                        fail(FDE_EDEVICE, "H-solve early chunk");
                    for (int c = r.col0; c < r.col0 + r.n; ++c)
                        if (solved_at[c] < 0 || solved_at[c] > p - 1) fail(FDE_EDEVICE, "H-solve early chunk reads unsolved x");
                    area += (int64_t)m * r.n;
                } else if (r.kind == HS_LOWRANK) {
                    if (r.tslot < 0 || r.tslot >= tab.tslots || !by_slot.count(r.slot))
                        fail(FDE_EDEVICE, "H-solve low-rank item record");
                    const LR& b = by_slot.at(r.slot);
                    if (next->row0 < b.t0 || next->row0 + m > b.t1 || r.ld != b.t1 - b.t0 ||
                        r.off != b.uoff + (next->row0 - b.t0) || !in_arena(r.off, m, kmax, r.ld))
                        fail(FDE_EDEVICE, "H-solve low-rank item out of its block");
                    if (owner[r.tslot] != r.slot || lo[r.tslot] != b.s0 || hi[r.tslot] != b.s1)
                        fail(FDE_EDEVICE, "H-solve low-rank item uses an incomplete t");
                    area += (int64_t)m * (b.s1 - b.s0);
                } else {
                    fail(FDE_EDEVICE, "H-solve early record kind");
                }
            }
            for (int r = st.row0; r < st.row0 + n; ++r) {
                if (solved_at[r] >= 0) fail(FDE_EDEVICE, "H-solve row solved twice");
                solved_at[r] = p;
            }
        }
        if (area != (int64_t)Nd * (Nd - 1) / 2)
            fail(FDE_EDEVICE, "H-solve steps cover %lld entries of a triangle of %lld", (long long)area,
                 (long long)Nd * (Nd - 1) / 2);
    }
}

}  // namespace fde
