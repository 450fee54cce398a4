// Leaf-step form of the forward and backward H-substitutions (Section 4.1).
//
// The op-list form of the substitutions follows the block recursion and issues
// one small dependent op per leaf block. Here the same triangular solves are
// reorganised by leaf rows: the step of leaf i gathers every contribution of
// already solved leaves to its rows at once and then solves with the diagonal
// leaf. A low-rank block B = U_B V_B^T contributes U_B (V_B^T x_sigma): the
// short vector t_B = V_B^T x_sigma is formed once, right after the last leaf of
// sigma is solved, and kept in a slot until the last leaf of tau has used it.
// Slots are shared between blocks whose lifetimes (in steps) do not overlap.
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
    for (int dir = 0; dir < 2; ++dir) {   // 0: forward with the lower blocks, 1: backward with the upper blocks
        // contributions per leaf, t computations per leaf, and t lifetimes
        std::vector<std::vector<HsItem>> items(L);
        std::vector<std::vector<HsTcomp>> tcs(L);
        std::vector<int64_t> diag(L, -1);
        struct Life {
            int start, end;   // step positions (in this direction's order)
            int leaf_tc;      // leaf whose step computes t
            size_t tc_index;
            std::vector<std::pair<int, size_t>> users;   // (leaf, item index)
        };
        std::vector<Life> lives;
        auto pos = [&](int leaf) { return dir == 0 ? leaf : L - 1 - leaf; };
        for (int b : hm.dense_blocks) {
            const Block& B = hm.bl[b];
            const Cluster &tc = hm.cl[B.tau], &sc = hm.cl[B.sigma];
            if (B.tau == B.sigma) {
                diag[leaf_of_cluster.at(B.tau)] = B.off;
                continue;
            }
            const bool lower = tc.d0 > sc.d0;
            if (lower != (dir == 0)) continue;
            const int i = leaf_of_cluster.at(B.tau);
            const int m = tc.size(), n = sc.size();
            for (int c0 = 0; c0 < n; c0 += kHsChunk)
                items[i].push_back(HsItem{B.off + (int64_t)c0 * m, m, sc.d0 + c0, std::min(kHsChunk, n - c0), -1, -1});
        }
        for (int b : hm.lr_blocks) {
            const Block& B = hm.bl[b];
            const Cluster &tc = hm.cl[B.tau], &sc = hm.cl[B.sigma];
            const bool lower = tc.d0 > sc.d0;
            if (lower != (dir == 0)) continue;
            Life lf;
            // sigma solved: at its last leaf going forward, at its first leaf going backward
            lf.leaf_tc = dir == 0 ? last_leaf(B.sigma) : first_leaf(B.sigma);
            lf.start = pos(lf.leaf_tc);
            tcs[lf.leaf_tc].push_back(HsTcomp{B.voff, sc.size(), sc.d0, B.slot, -1});
            lf.tc_index = tcs[lf.leaf_tc].size() - 1;
            lf.end = lf.start;
            for (int i = first_leaf(B.tau); i <= last_leaf(B.tau); ++i) {
                const Leaf& lv = leaves[i];
                items[i].push_back(HsItem{B.uoff + (lv.d0 - tc.d0), tc.size(), 0, 0, B.slot, -1});
                lf.users.push_back({i, items[i].size() - 1});
                lf.end = std::max(lf.end, pos(i));
            }
            lives.push_back(lf);
        }
        // t slots: a block's t is written in the step at `start` and read up to the step at `end`
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
            tcs[lf.leaf_tc][lf.tc_index].tslot = sl;
            for (auto& u : lf.users) items[u.first][u.second].tslot = sl;
        }
        tab.tslots = std::max(tab.tslots, nslot);
        for (int s = 0; s < L; ++s) {
            const int i = dir == 0 ? s : L - 1 - s;
            if (diag[i] < 0) fail(FDE_EDEVICE, "leaf %d has no dense diagonal block", i);
            HsStep st;
            st.diag = diag[i];
            st.row0 = leaves[i].d0;
            st.nrow = leaves[i].d1 - leaves[i].d0;
            st.it0 = (int)tab.items.size();
            tab.items.insert(tab.items.end(), items[i].begin(), items[i].end());
            st.it1 = (int)tab.items.size();
            st.tc0 = (int)tab.tcomp.size();
            tab.tcomp.insert(tab.tcomp.end(), tcs[i].begin(), tcs[i].end());
            st.tc1 = (int)tab.tcomp.size();
            tab.steps.push_back(st);
            tab.maxrow = std::max(tab.maxrow, st.nrow);
        }
    }
}

void validate_hsolve_steps(const HTree& hm, const HsTables& tab) {
    const int64_t arena = hm.arena_elems;
    const int Nd = hm.op ? hm.op->Nd : 0;
    const int L = tab.nleaf;
    if ((int)tab.steps.size() != 2 * L) fail(FDE_EDEVICE, "H-solve steps: %zu for %d leaves", tab.steps.size(), L);
    // coverage: per direction, the contributions and the diagonal leaves tile one triangle of
    // the Nd x Nd matrix exactly (low-rank items cover their leaf rows times all of sigma)
    for (int dir = 0; dir < 2; ++dir) {
        int64_t area = 0;
        for (int s = dir * L; s < (dir + 1) * L; ++s) {
            const HsStep& st = tab.steps[s];
            area += (int64_t)st.nrow * (st.nrow - 1) / 2;
            for (int it = st.it0; it < st.it1; ++it) {
                const HsItem& m = tab.items[it];
                if (m.ncol > 0) {
                    area += (int64_t)st.nrow * m.ncol;
                } else {
                    // find the t computation of this item's slot in the same direction with the matching U block
                    int64_t cols = -1;
                    for (int b : hm.lr_blocks) {
                        const Block& B = hm.bl[b];
                        const Cluster& tc = hm.cl[B.tau];
                        if (m.off >= B.uoff && m.off < B.uoff + tc.size() && m.ld == tc.size() && m.slot == B.slot) {
                            cols = hm.cl[B.sigma].size();
                            break;
                        }
                    }
                    if (cols < 0) fail(FDE_EDEVICE, "H-solve item refers to no low-rank block");
                    area += (int64_t)st.nrow * cols;
                }
            }
        }
        if (area != (int64_t)Nd * (Nd - 1) / 2)
            fail(FDE_EDEVICE, "H-solve steps cover %lld entries of a triangle of %lld", (long long)area,
                 (long long)Nd * (Nd - 1) / 2);
    }
    for (const HsStep& st : tab.steps) {
        if (st.nrow < 1 || st.row0 < 0 || st.row0 + st.nrow > Nd) fail(FDE_EDEVICE, "H-solve step rows out of range");
        if (st.diag < 0 || st.diag + (int64_t)st.nrow * st.nrow > arena) fail(FDE_EDEVICE, "H-solve diagonal out of range");
        if (st.it0 < 0 || st.it1 < st.it0 || st.it1 > (int)tab.items.size()) fail(FDE_EDEVICE, "H-solve items out of range");
        if (st.tc0 < 0 || st.tc1 < st.tc0 || st.tc1 > (int)tab.tcomp.size()) fail(FDE_EDEVICE, "H-solve t range");
        for (int it = st.it0; it < st.it1; ++it) {
            const HsItem& m = tab.items[it];
            const int cols = m.ncol > 0 ? m.ncol : hm.kmax;
            if (m.ncol > kHsChunk || m.ld < st.nrow) fail(FDE_EDEVICE, "H-solve item shape");
            if (m.off < 0 || m.off + (st.nrow - 1) + (int64_t)(cols - 1) * m.ld >= arena)
                fail(FDE_EDEVICE, "H-solve item out of the factor storage");
            if (m.ncol > 0) {
                if (m.col0 < 0 || m.col0 + m.ncol > Nd) fail(FDE_EDEVICE, "H-solve item columns out of range");
            } else if (m.slot < 0 || m.slot >= hm.nslots || m.tslot < 0 || m.tslot >= tab.tslots) {
                fail(FDE_EDEVICE, "H-solve item slot out of range");
            }
        }
        for (int e = st.tc0; e < st.tc1; ++e) {
            const HsTcomp& t = tab.tcomp[e];
            if (t.voff < 0 || t.voff + (int64_t)hm.kmax * t.ld > arena) fail(FDE_EDEVICE, "H-solve V out of range");
            if (t.col0 < 0 || t.col0 + t.ld > Nd) fail(FDE_EDEVICE, "H-solve t columns out of range");
            if (t.slot < 0 || t.slot >= hm.nslots || t.tslot < 0 || t.tslot >= tab.tslots)
                fail(FDE_EDEVICE, "H-solve t slot out of range");
        }
    }
}

}  // namespace fde
