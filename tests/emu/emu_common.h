// Shared pieces of the CPU emulation of the kernels (pcms_emu.cpp holds the
// driver; emu_dim.cpp instantiates the per-target code of one dimension, so
// the dimensions compile in parallel).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "fit.h"

// Spinning barrier for the few threads of one lane group.
struct SpinBarrier {
    int n;
    std::atomic<int> count{0};
    std::atomic<unsigned> gen{0};
    explicit SpinBarrier(int n_) : n(n_) {}
    void arrive_and_wait()
    {
        const unsigned g0 = gen.load(std::memory_order_acquire);
        if (count.fetch_add(1, std::memory_order_acq_rel) + 1 == n) {
            count.store(0, std::memory_order_relaxed);
            gen.fetch_add(1, std::memory_order_acq_rel);
        } else {
            int spins = 0;
            while (gen.load(std::memory_order_acquire) == g0)
                if (++spins > 4096) std::this_thread::yield();
        }
    }
};

// The G lanes of a group run as G threads; every collective operation is a
// barrier round in which each lane publishes its value, then all read.
struct EmuGroup {
    int G;
    SpinBarrier bar;
    double d[16];
    float f[16];
    int i[16];
    bool b[16];
    explicit EmuGroup(int g) : G(g), bar(g) {}
};

extern long long g_rows, g_cands, g_walks, g_exact, g_nodes;

namespace emu {

using namespace pcms;

// Runs body(i, L, grp) for every target on G threads (lane q = thread q),
// each target with its own poisoned LDS words; reports work per wave.  The
// kernels run one lane per target; G > 1 exercises the cooperative paths.
template <int kGroup, class Body>
void run_groups(const KArgs &a, Body body)
{
    std::vector<int> lds((size_t)std::max(a.n_tgt, 1) * a.words, 0x7f7f7f7f);
    EmuGroup ctx(kGroup);
    std::vector<long long> walks(a.n_tgt), cands(a.n_tgt);
    std::vector<std::thread> th;
    for (int q = 0; q < kGroup; ++q) {
        th.emplace_back([&, q]() {
            for (int i = 0; i < a.n_tgt; ++i) {
                const long long w0 = pcms_emu_walks, c0 = pcms_emu_cands;
                body(i, lds.data() + (size_t)i * a.words, Grp<kGroup>{q, &ctx});
                if (q == 0) {
                    walks[i] = pcms_emu_walks - w0;
                    cands[i] = pcms_emu_cands - c0;
                }
                ctx.bar.arrive_and_wait();
            }
            if (q == 0) {
                g_rows = pcms_emu_rows;
                g_cands = pcms_emu_cands;
                g_walks = pcms_emu_walks;
                g_exact = pcms_emu_exact;
                g_nodes = pcms_emu_nodes;
            }
        });
    }
    for (auto &t : th) t.join();
    // divergence: a wave holds 64 / kGroup consecutive targets
    const int tw = 64 / kGroup;
    double mw = 0, mc = 0;
    long long nw = 0;
    for (int i0 = 0; i0 < a.n_tgt; i0 += tw) {
        long long w = 0, c = 0;
        for (int i = i0; i < std::min(a.n_tgt, i0 + tw); ++i) {
            w = std::max(w, walks[i]);
            c = std::max(c, cands[i]);
        }
        mw += w;
        mc += c;
        ++nw;
    }
    if (nw)
        std::fprintf(stderr, "divergence: per wave max walks %.2f cands %.1f vs target mean %.2f %.1f\n",
                     mw / nw, mc / nw, (double)g_walks / a.n_tgt, (double)g_cands / a.n_tgt);
}

template <int D, bool UNIT, int G>
void run_nbr(const KArgs &a, const GridParams &gp)
{
    if (a.bvh_nodes)
        run_groups<G>(a, [&](int i, int *L, Grp<G> g) { nbr_target<D, UNIT, G, true>(a, gp, i, L, g); });
    else
        run_groups<G>(a, [&](int i, int *L, Grp<G> g) { nbr_target<D, UNIT, G>(a, gp, i, L, g); });
}

template <int D, int P, int PREC, bool UNIT, int G>
void run_xfer(const KArgs &a, const GridParams &gp)
{
    if (a.bvh_nodes)
        run_groups<G>(a, [&](int i, int *L, Grp<G> g) {
            xfer_target<D, P, PREC, UNIT, G, false, true>(a, gp, i, L, g);
        });
    else
        run_groups<G>(a, [&](int i, int *L, Grp<G> g) { xfer_target<D, P, PREC, UNIT, G>(a, gp, i, L, g); });
}

template <int D, int P, int PREC, bool UNIT, int G>
void run_op(const KArgs &a, const GridParams &gp)
{
    run_groups<G>(a, [&](int i, int *L, Grp<G> g) {
        xfer_target<D, P, PREC, UNIT, G, true>(a, gp, i, L, g);
    });
}

template <int D, bool UNIT, int G>
void dispatch_g(int op, const KArgs &a, const GridParams &gp, int degree, int precision)
{
    if (op == 0) return run_nbr<D, UNIT, G>(a, gp);
#define X(PP)                                                                  \
    if (degree == PP && op == 2) {                                             \
        if (precision == PCMS_MIXED) return run_op<D, PP, PCMS_MIXED, UNIT, G>(a, gp); \
        if (precision == PCMS_MIXED_REFINE)                                    \
            return run_op<D, PP, PCMS_MIXED_REFINE, UNIT, G>(a, gp);            \
        return run_op<D, PP, PCMS_FP64, UNIT, G>(a, gp);                       \
    }                                                                          \
    if (degree == PP) {                                                        \
        if (precision == PCMS_MIXED) return run_xfer<D, PP, PCMS_MIXED, UNIT, G>(a, gp); \
        if (precision == PCMS_MIXED_REFINE)                                    \
            return run_xfer<D, PP, PCMS_MIXED_REFINE, UNIT, G>(a, gp);          \
        return run_xfer<D, PP, PCMS_FP64, UNIT, G>(a, gp);                     \
    }
    X(0) X(1) X(2)
#undef X
}

template <int D, bool UNIT>
inline void dispatch(int op, const KArgs &a, const GridParams &gp, int group, int degree, int precision)
{
    if (group == 4) return dispatch_g<D, UNIT, 4>(op, a, gp, degree, precision);
    return dispatch_g<D, UNIT, 1>(op, a, gp, degree, precision);
}

// Defined per dimension in emu_dim.cpp.
template <int D>
void dispatch_dim(int op, const KArgs &a, const GridParams &gp, int group, int degree,
                  int precision, bool unit);

// LBVH steps (emu_dim.cpp), serial versions of the device build with its
// per-item functions: Morton codes of n points in the single-bucket box of
// gp; the tree over the sorted codes and sorted records spts (nodes sized
// by the caller for 2n - 1 records, returns the leaf count; aborts on a
// malformed tree).
template <int D>
void morton_keys(const GridParams &gp, const double *pts, int n, std::vector<unsigned> &keys);
template <int D>
int lbvh_tree(const unsigned *codes, int n, const double *spts, float *nodes);

}  // namespace emu
