// The per-target code of dimension PCMS_EMU_DIM, for the CPU emulation
// (compiled once per dimension).
#include <cmath>
#include <cstdlib>
#include <utility>

#include "emu_common.h"

namespace emu {

template <>
void dispatch_dim<PCMS_EMU_DIM>(int op, const KArgs &a, const GridParams &gp, int group,
                                int degree, int precision, bool unit)
{
    if (unit) dispatch<PCMS_EMU_DIM, true>(op, a, gp, group, degree, precision);
    else dispatch<PCMS_EMU_DIM, false>(op, a, gp, group, degree, precision);
}

template <>
void morton_keys<PCMS_EMU_DIM>(const GridParams &gp, const double *pts, int n,
                               std::vector<unsigned> &keys)
{
    keys.resize(n);
    for (int i = 0; i < n; ++i) keys[i] = bvh_morton<PCMS_EMU_DIM>(gp, pts + (size_t)i * PCMS_EMU_DIM);
}

template <>
int lbvh_tree<PCMS_EMU_DIM>(const unsigned *codes, int n, const double *spts, float *nodes)
{
    constexpr int D = PCMS_EMU_DIM, S = bvh_stride(D);
    auto fail = [](const char *what, int x) {
        std::fprintf(stderr, "lbvh: %s (%d)\n", what, x);
        std::abort();
    };
    // leaves: cuts from the tree over the sources, then a serial scan
    std::vector<int> cut(std::max(n - 1, 1), -1);
    const char *env = std::getenv("PCMS_LBVH_LEAF");
    const int max_leaf = env && std::atoi(env) >= 1 ? std::atoi(env) : kBvhLeaf;
    for (int i = 0; i < n - 1; ++i) bvh_point_cut(codes, n, i, max_leaf, cut.data());
    for (int i = 0; i < n - 1; ++i)
        if (cut[i] != 0 && cut[i] != 1) fail("split not written", i);
    std::vector<int> leaf_start;
    for (int i = 0; i < n; ++i)
        if (i == 0 || cut[i - 1]) leaf_start.push_back(i);
    const int nl = (int)leaf_start.size();
    leaf_start.push_back(n);
    // the leaves are the largest subtrees of at most max_leaf sources: split
    // [a, b) at the highest bit in which the keys (code, position) of its
    // ends differ until the ranges are small enough, and compare
    {
        auto key = [&](int i) { return ((uint64_t)codes[i] << 32) | (uint32_t)i; };
        std::vector<int> ref;
        std::vector<std::pair<int, int>> todo{{0, n}};
        while (!todo.empty()) {
            auto [a, b] = todo.back();
            todo.pop_back();
            if (b - a <= max_leaf) {
                ref.push_back(a);
                continue;
            }
            const int bit = 63 - __builtin_clzll(key(a) ^ key(b - 1));
            int m = a;
            while (!((key(m) >> bit) & 1)) ++m;
            todo.push_back({m, b});
            todo.push_back({a, m});
        }
        if ((int)ref.size() != nl) fail("leaf count differs from the recursive split", (int)ref.size());
        for (int l = 0; l < nl; ++l)
            if (ref[l] != leaf_start[l]) fail("leaf start differs from the recursive split", l);
    }
    const int nr = 2 * nl - 1;
    std::vector<int> parent(nr, -1), child1(std::max(nl - 1, 1), -1),
        split_right(std::max(nl - 1, 1), -1);
    for (int i = 0; i < nl - 1; ++i)
        bvh_radix_node<D>(codes, leaf_start.data(), nl, i, nodes, parent.data(),
                          child1.data(), split_right.data());
    for (int r = 1; r < nr; ++r)
        if (parent[r] < 0 || parent[r] >= nl - 1) fail("record has no parent", r);
    for (int b = 0; b < nl - 1; ++b)
        if (split_right[b] < 0) fail("no node splits after leaf", b);
    for (int r = 0; r < nr; ++r)
        bvh_rope<D>(nl, r, nodes, leaf_start.data(), split_right.data());
    int max_depth = 0;
    for (int l = 0; l < nl; ++l) {
        int depth = 0;
        for (int r = nl - 1 + l; r != 0; r = parent[r]) ++depth;
        max_depth = std::max(max_depth, depth);
    }
    if (max_depth > 64) fail("tree deeper than 64", max_depth);
    // boxes as the device computes them: the leaves', then the internal
    // nodes level by level from the deepest (depth = parent hops to the root)
    for (int l = 0; l < nl; ++l) {
        float lo[D], hi[D];
        bvh_leaf_box<D>(spts, leaf_start[l], leaf_start[l + 1], lo, hi);
        float *nd = nodes + (size_t)(nl - 1 + l) * S;
        for (int k = 0; k < D; ++k) {
            nd[k] = lo[k];
            nd[D + k] = hi[k];
        }
    }
    std::vector<std::vector<int>> level(64);
    for (int i = 0; i < nl - 1; ++i) {
        int d = 0;
        for (int r = i; r != 0; r = parent[r]) ++d;
        if (d > 63) fail("internal node deeper than 63", d);
        level[d].push_back(i);
    }
    for (int d = 63; d >= 0; --d)
        for (int i : level[d]) {
            float *nd = nodes + (size_t)i * S;
            const float *a = nodes + (size_t)bvh_int(nd, 2 * D) * S;
            const float *b = nodes + (size_t)child1[i] * S;
            for (int k = 0; k < D; ++k) {
                if (std::isnan(a[k]) || std::isnan(b[k])) fail("child box not ready", i);
                nd[k] = std::fmin(a[k], b[k]);
                nd[D + k] = std::fmax(a[D + k], b[D + k]);
            }
        }
    // every box contains its children's, every record covers the sources of
    // its children, and the ropes chain through the leaves in order (a full
    // walk with an infinite ball)
    int r = 0, expect = 0;
    while (r >= 0) {
        const float *nd = nodes + (size_t)r * S;
        const int c0 = bvh_int(nd, 2 * D);
        if (c0 < 0) {
            if (r - (nl - 1) != expect) fail("walk reached the wrong leaf", r - (nl - 1));
            if (bvh_int(nd, 2 * D + 2) != leaf_start[expect] ||
                bvh_int(nd, 2 * D + 3) != leaf_start[expect + 1])
                fail("leaf record range", expect);
            ++expect;
            r = bvh_int(nd, 2 * D + 1);
        } else {
            const float *a = nodes + (size_t)c0 * S;
            const float *b = nodes + (size_t)child1[r] * S;
            if (bvh_int(a, 2 * D + 1) != child1[r]) fail("first child's rope is not the second child", r);
            if (bvh_int(nd, 2 * D + 2) != bvh_int(a, 2 * D + 2) ||
                bvh_int(nd, 2 * D + 3) != bvh_int(b, 2 * D + 3) ||
                bvh_int(a, 2 * D + 3) != bvh_int(b, 2 * D + 2))
                fail("node range is not its children's", r);
            for (int k = 0; k < D; ++k)
                if (!(nd[k] <= a[k] && nd[k] <= b[k] && nd[D + k] >= a[D + k] && nd[D + k] >= b[D + k]))
                    fail("box does not contain its children", r);
            r = c0;
        }
    }
    if (expect != nl) fail("walk visited fewer leaves", expect);
    return nl;
}

}  // namespace emu
