// Cluster tree, block tree and storage layout of the H-matrix (Section 3).
//
// Readings of what Section 3 leaves open (the same choices as the FP64 CPU
// reference used by the tests):
//  * unknowns are reordered element by element -- the bubbles of element e,
//    then the hat at its right node -- so a cluster of elements owns a
//    contiguous index range; the paper's order is restored at the boundary;
//  * a cluster's geometric extent is the union of its basis supports
//    (Section 3.2), i.e. [x_{e0}, x_{min(e1+1, N)}] because of the hat overhang;
//  * the cluster tree bisects element ranges to the common depth
//    ceil(log2(N / leaf)); blocks pair same-level clusters; admissible blocks
//    (eq. (admis), dist > 0) are low rank, leaf pairs dense, others 2 x 2;
//  * the expansion of (t-s)^{1-alpha} is taken about the centre of the cluster
//    with the smaller radius (Remark after the Lemma), in s on a tie;
//  * for an admissible pair with the row cluster right of the column cluster,
//    S = theta S_l ~ theta Q W^T; the mirrored block is (1-theta) W Q^T.
#include <algorithm>
#include <cmath>

#include "hmatrix.h"

namespace fde {

namespace {

int make_cluster(HTree* hm, int e0, int e1, int level, int depth) {
    const Op* op = hm->op;
    const int N = op->N, P = op->P;
    Cluster c;
    c.e0 = e0;
    c.e1 = e1;
    c.d0 = e0 * P;
    c.d1 = std::min(e1 * P, N * P - 1);
    c.lo = op->x[e0];
    c.hi = op->x[std::min(e1 + 1, N)];
    c.level = level;
    const int id = (int)hm->cl.size();
    hm->cl.push_back(c);
    if (level < depth) {
        const int mid = e0 + (e1 - e0) / 2;
        const int a = make_cluster(hm, e0, mid, level + 1, depth);
        const int b = make_cluster(hm, mid, e1, level + 1, depth);
        hm->cl[id].child[0] = a;
        hm->cl[id].child[1] = b;
    }
    return id;
}

bool admissible(const Cluster& t, const Cluster& s, double lam) {
    const double dist = std::max({0.0, s.lo - t.hi, t.lo - s.hi});
    const double diam = std::max(t.hi - t.lo, s.hi - s.lo);
    return dist > 0.0 && diam <= lam * dist;
}

int make_block(HTree* hm, int t, int s) {
    Block b;
    b.tau = t;
    b.sigma = s;
    const Cluster& ct = hm->cl[t];
    const Cluster& cs = hm->cl[s];
    const int id = (int)hm->bl.size();
    if (admissible(ct, cs, hm->lambda)) {
        b.kind = kLowRank;
        b.lower = ct.lo >= cs.hi;
        hm->bl.push_back(b);
        return id;
    }
    if (ct.leaf() || cs.leaf()) {
        b.kind = kDense;
        hm->bl.push_back(b);
        return id;
    }
    b.kind = kHier;
    hm->bl.push_back(b);
    int ch[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) ch[2 * i + j] = make_block(hm, ct.child[i], cs.child[j]);
    for (int k = 0; k < 4; ++k) hm->bl[id].child[k] = ch[k];
    return id;
}

void collect(HTree* hm, int b) {
    Block& B = hm->bl[b];
    if (B.kind == kHier) {
        for (int k = 0; k < 4; ++k) collect(hm, B.child[k]);
        return;
    }
    if (B.kind == kDense)
        hm->dense_blocks.push_back(b);
    else
        hm->lr_blocks.push_back(b);
}

}  // namespace

void build_trees(HTree* hm) {
    const Op* op = hm->op;
    const int N = op->N, P = op->P;
    // internal order
    hm->h2p.clear();
    for (int e = 0; e < N; ++e) {
        for (int p = 1; p < P; ++p) hm->h2p.push_back(e * (P - 1) + p - 1);
        if (e < N - 1) hm->h2p.push_back(N * (P - 1) + e);
    }
    const int depth = N <= hm->leaf ? 0 : (int)std::ceil(std::log2((double)N / hm->leaf) - 1e-12);
    hm->cl.clear();
    hm->bl.clear();
    make_cluster(hm, 0, N, 0, depth);
    hm->root = make_block(hm, 0, 0);
    hm->dense_blocks.clear();
    hm->lr_blocks.clear();
    collect(hm, hm->root);
    assign_storage(hm, hm->kmax);
}

// storage: dense blocks, then U and V of the low-rank blocks with kmax columns each
void assign_storage(HTree* hm, int kmax) {
    hm->kmax = kmax;
    int64_t off = 0;
    hm->max_lr_rows = 0;
    for (int b : hm->dense_blocks) {
        Block& B = hm->bl[b];
        B.off = off;
        off += (int64_t)hm->cl[B.tau].size() * hm->cl[B.sigma].size();
    }
    int slot = 0;
    for (size_t k = 0; k < hm->lr_blocks.size(); ++k) {
        Block& B = hm->bl[hm->lr_blocks[k]];
        const int m = hm->cl[B.tau].size(), n = hm->cl[B.sigma].size();
        B.uoff = off;
        off += (int64_t)m * hm->kmax;
        B.voff = off;
        off += (int64_t)n * hm->kmax;
        B.slot = slot++;
        B.lr_id = (int)k;
        hm->max_lr_rows = std::max({hm->max_lr_rows, m, n});
    }
    hm->arena_elems = off;
    hm->nslots = slot;
}

}  // namespace fde
