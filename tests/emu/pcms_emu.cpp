// CPU emulation of the HIP library's kernels, for indexing checks under the
// address and undefined-behaviour sanitisers.  It runs the per-target search
// and fit code of fit.h / search.h unchanged (compiled for the host), and the
// grid build with the same bucket sizing, keys and radix-sort scatter pieces
// (device_common.h), following the kernels' block/round/wave structure.
// Every LDS word access is bounds-checked per lane.
//
// Usage: pcms_emu <input.bin> <output.bin>   (format written by emu_driver.py)
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "emu_common.h"

thread_local long long pcms_emu_rows = 0, pcms_emu_cands = 0, pcms_emu_walks = 0,
                       pcms_emu_exact = 0, pcms_emu_nodes = 0;

unsigned pcms_emu_ballot(EmuGroup *g, int q, bool p)
{
    g->b[q] = p;
    g->bar.arrive_and_wait();
    unsigned m = 0;
    for (int x = 0; x < g->G; ++x) m |= (unsigned)g->b[x] << x;
    g->bar.arrive_and_wait();
    return m;
}

// the same butterfly as the kernels' xor shuffles, lower lane's value first
template <class T>
static T butterfly(EmuGroup *g, int q, T x, T *slot, bool is_min)
{
    slot[q] = x;
    g->bar.arrive_and_wait();
    T v[16];
    for (int k = 0; k < g->G; ++k) v[k] = slot[k];
    for (int off = g->G / 2; off > 0; off >>= 1) {
        T nv[16];
        for (int k = 0; k < g->G; ++k) {
            T mine = v[k], other = v[k ^ off];
            if (is_min) nv[k] = other < mine ? other : mine;
            else nv[k] = (k & off) ? other + mine : mine + other;
        }
        for (int k = 0; k < g->G; ++k) v[k] = nv[k];
    }
    g->bar.arrive_and_wait();
    return v[q];
}

double pcms_emu_sum(EmuGroup *g, int q, double x) { return butterfly(g, q, x, g->d, false); }
float pcms_emu_sum(EmuGroup *g, int q, float x) { return butterfly(g, q, x, g->f, false); }
int pcms_emu_sum(EmuGroup *g, int q, int x) { return butterfly(g, q, x, g->i, false); }
double pcms_emu_min(EmuGroup *g, int q, double x) { return butterfly(g, q, x, g->d, true); }
int pcms_emu_min(EmuGroup *g, int q, int x) { return butterfly(g, q, x, g->i, true); }
void pcms_emu_sync(EmuGroup *g, int q)
{
    (void)q;
    g->bar.arrive_and_wait();
}

long long g_rows = 0, g_cands = 0, g_walks = 0, g_exact = 0, g_nodes = 0;

[[noreturn]] void pcms_emu_lds_fault(int e, int words)
{
    std::fprintf(stderr, "LDS word %d outside the lane's %d words\n", e, words);
    std::abort();
}

namespace {

using namespace pcms;

[[noreturn]] void die(const char *m)
{
    std::fprintf(stderr, "pcms_emu: %s\n", m);
    std::abort();
}

struct Reader {
    FILE *f;
    int64_t i64()
    {
        int64_t v;
        if (std::fread(&v, 8, 1, f) != 1) die("short read");
        return v;
    }
    double f64()
    {
        double v;
        if (std::fread(&v, 8, 1, f) != 1) die("short read");
        return v;
    }
    template <class T>
    std::vector<T> arr(size_t n)
    {
        std::vector<T> v(n);
        if (n && std::fread(v.data(), sizeof(T), n, f) != n) die("short read");
        return v;
    }
};

constexpr int kSortThreads = 256, kSortRounds = 16, kSortItems = kSortThreads * kSortRounds;

// Stable LSD radix sort with the kernels' structure: per-block digit
// histograms (digit-major), exclusive scan, then per-block rounds of 256
// items in 4 waves, ranked with the ballot pieces the kernel uses.
void radix_sort_emu(std::vector<unsigned> &keys, std::vector<int> &vals, int bits)
{
    const int n = (int)keys.size();
    const int nb = (n + kSortItems - 1) / kSortItems;
    std::vector<unsigned> kout(n);
    std::vector<int> vout(n);
    const int passes = std::max(1, (bits + 7) / 8);
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        std::vector<int> hist((size_t)256 * nb, 0);
        for (int b = 0; b < nb; ++b)
            for (int r = 0; r < kSortRounds; ++r)
                for (int t = 0; t < kSortThreads; ++t) {
                    int i = b * kSortItems + r * kSortThreads + t;
                    if (i < n) hist[(size_t)((keys[i] >> shift) & 255) * nb + b]++;
                }
        int run = 0;
        for (auto &h : hist) {
            int c = h;
            h = run;
            run += c;
        }
        for (int b = 0; b < nb; ++b) {
            int running[256];
            for (int d = 0; d < 256; ++d) running[d] = hist[(size_t)d * nb + b];
            for (int r = 0; r < kSortRounds; ++r) {
                const int base = b * kSortItems + r * kSortThreads;
                if (base >= n) break;
                unsigned key[256];
                int val[256], digit[256];
                bool valid[256];
                for (int t = 0; t < 256; ++t) {
                    int i = base + t;
                    valid[t] = i < n;
                    key[t] = valid[t] ? keys[i] : 0u;
                    val[t] = valid[t] ? vals[i] : 0;
                    digit[t] = (key[t] >> shift) & 255;
                }
                unsigned long long vb[4] = {0, 0, 0, 0}, bb[4][8] = {};
                for (int t = 0; t < 256; ++t) {
                    int w = t >> 6, lane = t & 63;
                    if (valid[t]) vb[w] |= 1ull << lane;
                    for (int q = 0; q < 8; ++q)
                        if ((digit[t] >> q) & 1) bb[w][q] |= 1ull << lane;
                }
                unsigned long long mask[256];
                int wave_cnt[4][256];
                std::memset(wave_cnt, 0, sizeof(wave_cnt));
                for (int t = 0; t < 256; ++t) mask[t] = digit_match(vb[t >> 6], bb[t >> 6], digit[t]);
                for (int t = 0; t < 256; ++t)
                    if (valid[t] && (mask[t] & lanes_below(t & 63)) == 0)
                        wave_cnt[t >> 6][digit[t]] = __builtin_popcountll(mask[t]);
                for (int t = 0; t < 256; ++t) {
                    if (!valid[t]) continue;
                    int pos = scatter_slot(running[digit[t]], wave_cnt, t >> 6, digit[t], mask[t], t & 63);
                    if (pos < 0 || pos >= n) die("radix scatter slot out of range");
                    kout[pos] = key[t];
                    vout[pos] = val[t];
                }
                for (int d = 0; d < 256; ++d)
                    running[d] += wave_cnt[0][d] + wave_cnt[1][d] + wave_cnt[2][d] + wave_cnt[3][d];
            }
        }
        keys.swap(kout);
        vals.swap(vout);
    }
}

int key_bits(int cap)
{
    int b = 0;
    while (b < 31 && (1u << b) < (unsigned)cap) ++b;
    return b;
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc != 3) die("usage: pcms_emu in.bin out.bin");
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) die("cannot open input");
    Reader rd{f};
    if (rd.i64() != 0x50434d53454d55LL) die("bad magic");
    const int op_word = (int)rd.i64();
    const int op = op_word & 0xf;
    const bool lbvh = (op_word & 0x10) != 0;   // the LBVH in place of the uniform grid
    const int64_t n_src = rd.i64(), dim = rd.i64(), n_tgt = rd.i64(), nf = rd.i64();
    const int degree = (int)rd.i64(), mode = (int)rd.i64(), k = (int)rd.i64();
    const int n_min = (int)rd.i64(), max_iter = (int)rd.i64(), k_cap = (int)rd.i64();
    const int weight = (int)rd.i64(), precision = (int)rd.i64(), group = (int)rd.i64();
    const double r = rd.f64(), lambda = rd.f64(), cell_width = rd.f64(), ppc = rd.f64();
    // slices of dimension 0 per bucket width, as the library's grids take
    // them (the same accepted overrides)
    const char *env_sub = std::getenv("PCMS_ROW_SLICES");
    const int sub_env = env_sub ? std::atoi(env_sub) : 0;
    const int row_slices =
        sub_env == 1 || sub_env == 2 || sub_env == 4 || sub_env == 8 || sub_env == 16 ? sub_env
                                                                                      : kRowSlices;
    double g[kMaxDim];
    for (int q = 0; q < kMaxDim; ++q) g[q] = rd.f64();
    auto src = rd.arr<double>((size_t)(n_src * dim));
    auto vals = rd.arr<double>((size_t)(nf * n_src));
    auto tgt = rd.arr<double>((size_t)(n_tgt * dim));
    std::fclose(f);

    // grid build
    double lo[kMaxDim], hi[kMaxDim];
    for (int q = 0; q < dim; ++q) {
        lo[q] = INFINITY;
        hi[q] = -INFINITY;
        for (int64_t j = 0; j < n_src; ++j) {
            lo[q] = std::fmin(lo[q], src[j * dim + q]);
            hi[q] = std::fmax(hi[q], src[j * dim + q]);
        }
    }
    // an LBVH: one bucket over the box, sources in Morton order
    const int cap = lbvh ? 1 : (int)std::min<int64_t>(2 * n_src + 64, (int64_t)1 << 30);
    GridParams gp;
    if (lbvh)
        grid_params_compute(lo, hi, (int)dim, n_src, g, 0.0, (double)n_src, 1, 1, &gp);
    else
        grid_params_compute(lo, hi, (int)dim, n_src, g, cell_width, ppc, cap, row_slices, &gp);
    if (gp.n_cells > cap) die("bucket count above the allocation");
    std::vector<unsigned> keys(n_src);
    std::vector<int> perm(n_src);
#define MORTON(DD)                                                              \
    case DD:                                                                    \
        emu::morton_keys<DD>(gp, src.data(), (int)n_src, keys);                 \
        break;
    if (lbvh) {
        switch (dim) { MORTON(1) MORTON(2) MORTON(3) MORTON(4) MORTON(5) }
        for (int64_t j = 0; j < n_src; ++j) perm[j] = (int)j;
        radix_sort_emu(keys, perm, 32);
    } else {
        for (int64_t j = 0; j < n_src; ++j) {
            keys[j] = bucket_key(gp, &src[j * dim]);
            perm[j] = (int)j;
            if (keys[j] >= (unsigned)gp.n_cells) die("bucket key out of range");
        }
        radix_sort_emu(keys, perm, key_bits(cap));
    }
    for (int64_t j = 1; j < n_src; ++j)
        if (keys[j - 1] > keys[j] || (keys[j - 1] == keys[j] && perm[j - 1] > perm[j]))
            die("radix sort is not stable-sorted");
    std::vector<int> cs((size_t)cap + 1, -1);
    for (int c = 0; c <= gp.n_cells; ++c) {
        if (lbvh) {
            cs[c] = c == 0 ? 0 : (int)n_src;
            continue;
        }
        int l = 0, h = (int)n_src;
        while (l < h) {
            int mid = (l + h) >> 1;
            if (keys[mid] < (unsigned)c) l = mid + 1;
            else h = mid;
        }
        cs[c] = l;
    }
    // the device's one-pass bucket offsets (cell_run) must give the same
    if (!lbvh) {
        std::vector<int> cs_runs((size_t)gp.n_cells + 1, -1);
        for (int i = 0; i <= (int)n_src; ++i) {
            int lo, hi;
            cell_run(keys.data(), (int)n_src, gp.n_cells, i, lo, hi);
            for (int c = lo; c <= hi; ++c) {
                if (c < 0 || c > gp.n_cells || cs_runs[c] != -1) die("bucket runs overlap");
                cs_runs[c] = i;
            }
        }
        for (int c = 0; c <= gp.n_cells; ++c)
            if (cs_runs[c] != cs[c]) die("one-pass bucket offsets differ from the binary search");
    }
    // the kernels may read only [0, n_cells]: keep exactly that for the sanitiser
    cs = std::vector<int>(cs.begin(), cs.begin() + gp.n_cells + 1);
    const int dp = padded_dim(dim);
    std::vector<double> spts((size_t)(n_src * dp), 0.0);
    for (int64_t p = 0; p < n_src; ++p)
        for (int q = 0; q < dim; ++q) spts[p * dp + q] = src[(size_t)perm[p] * dim + q];
    // FP32 records as the gather kernel writes them
    const int dp32 = padded_dim32(dim);
    std::vector<float> spts32((size_t)(n_src * dp32), 0.0f);
    for (int64_t p = 0; p < n_src; ++p)
        for (int q = 0; q < dim; ++q)
            spts32[p * dp32 + q] = (float)(src[(size_t)perm[p] * dim + q] - gp.lo[q]);
    // fixed-point records as the gather kernel writes them
    std::vector<uint32_t> sq((size_t)(n_src * dim), 0u);
    for (int64_t p = 0; p < n_src; ++p)
        for (int q = 0; q < dim; ++q)
            sq[p * dim + q] = quantize(src[(size_t)perm[p] * dim + q], gp.lo[q], gp.iqs[q]);
    // the tree (records poisoned with NaN; lbvh_tree checks that every node
    // is completed by both children and that the ropes chain the leaves)
    // (16-byte aligned: the walks read records as float4)
    std::vector<float4> node_store((size_t)bvh_stride((int)dim) * (2 * n_src - 1) / 4,
                                   float4{NAN, NAN, NAN, NAN});
    float *nodes = &node_store[0].x;
    int n_leaves = 0;
#define TREE(DD)                                                                 \
    case DD:                                                                     \
        n_leaves = emu::lbvh_tree<DD>(keys.data(), (int)n_src, spts.data(), nodes);   \
        break;
    if (lbvh) {
        switch (dim) { TREE(1) TREE(2) TREE(3) TREE(4) TREE(5) }
    }
    // targets, in the kernels' processing order
    std::vector<unsigned> tkeys(n_tgt);
    std::vector<int> tperm(n_tgt);
    const double bound = tile_key_bound((double)cap, dim);
    const bool tiled = bound < 4294967295.0;
    int tbits = key_bits(cap);
    if (lbvh) {
        switch (dim) {
#define TMORTON(DD)                                                              \
    case DD:                                                                     \
        emu::morton_keys<DD>(gp, tgt.data(), (int)n_tgt, tkeys);                 \
        break;
            TMORTON(1) TMORTON(2) TMORTON(3) TMORTON(4) TMORTON(5)
        }
        for (int64_t i = 0; i < n_tgt; ++i) tperm[i] = (int)i;
        tbits = 32;
    } else {
        for (int64_t i = 0; i < n_tgt; ++i) {
            tkeys[i] = tiled ? target_key(gp, &tgt[i * dim]) : bucket_key(gp, &tgt[i * dim]);
            tperm[i] = (int)i;
        }
        if (tiled) {
            tbits = 0;
            while (tbits < 32 && (double)(1ull << tbits) < bound) ++tbits;
        }
    }
    // the library sorts on the key's top 24 bits only
    if (tbits > 24) {
        for (auto &k : tkeys) k >>= (tbits - 24);
        tbits = 24;
    }
    radix_sort_emu(tkeys, tperm, tbits);
    const int nfs = padded_dim((int)nf);
    std::vector<double> svals((size_t)(n_src * nfs), 0.0);
    for (int64_t p = 0; p < n_src; ++p)
        for (int l = 0; l < nf; ++l) svals[p * nfs + l] = vals[(size_t)l * n_src + perm[p]];

    KArgs a{};
    a.gp = &gp;
    a.cs = cs.data();
    a.spts = spts.data();
    a.spts32 = spts32.data();
    a.sq = sq.data();
    a.bvh_nodes = lbvh ? nodes : nullptr;
    if (lbvh) std::fprintf(stderr, "lbvh: %d leaves over %lld sources\n", n_leaves, (long long)n_src);
    a.perm = perm.data();
    a.tgt = tgt.data();
    a.tperm = tperm.data();
    a.n_tgt = (int)n_tgt;
    a.mode = mode;
    a.k = k;
    a.n_min = n_min;
    a.max_iter = max_iter;
    a.r = r;
    a.k_cap = k_cap;
    a.words = target_words(mode, k, k_cap);
    a.stride = a.words | 1;
    a.svals = svals.data();
    a.nf = (int)nf;
    a.nfs = nfs;
    a.weight = weight;
    a.lambda = lambda;
    std::vector<double> out((size_t)(nf * n_tgt), 0.0);
    std::vector<int32_t> nbr((size_t)(n_tgt * k_cap), -1), n_kept(n_tgt), n_found(n_tgt);
    std::vector<double> r2(n_tgt);
    std::vector<uint8_t> status(n_tgt);
    // operator slots [words][n_tgt] (poisoned: unwritten slots are never read)
    std::vector<double> op_w((size_t)a.words * n_tgt, NAN);
    std::vector<int32_t> op_c((size_t)a.words * n_tgt, -7), op_n(n_tgt, -9);
    a.op_w = op_w.data();
    a.op_c = op_c.data();
    a.op_n = op_n.data();
    a.out = out.data();
    // transfers stage each target's fields as one record, as the one-problem
    // launches do (poisoned: every record must be written in full)
    std::vector<double> stage((size_t)n_tgt * a.nfs, -777.0);
    if (op == 1) a.stage = stage.data();
    a.nbr = nbr.data();
    a.n_kept = n_kept.data();
    a.n_found = n_found.data();
    a.r2 = r2.data();
    a.status = status.data();
    bool unit = true;
    for (int q = 0; q < dim; ++q) unit = unit && g[q] == 1.0;
#define DIMCASE(DD)                                                                 \
    case DD:                                                                        \
        emu::dispatch_dim<DD>(op, a, gp, group, degree, precision, unit);           \
        break;
    switch (dim) {
        DIMCASE(1) DIMCASE(2) DIMCASE(3) DIMCASE(4) DIMCASE(5)
        default: die("bad dim");
    }
#undef DIMCASE
    if (op == 1) {
        // the output transpose of the staged records
        for (int64_t t = 0; t < n_tgt; ++t)
            for (int l = 0; l < a.nfs; ++l) {
                const double v = stage[(size_t)t * a.nfs + l];
                if (v == -777.0) die("staged record not written in full");
                if (l < nf) out[(size_t)l * n_tgt + t] = v;
            }
    }
    std::fprintf(stderr, "work: walks %lld rows %lld candidates %lld per target: %.2f %.2f %.2f"
                 " exact rechecks %.3f\n",
                 g_walks, g_rows, g_cands, (double)g_walks / n_tgt, (double)g_rows / n_tgt,
                 (double)g_cands / n_tgt, (double)g_exact / n_tgt);
    if (lbvh) std::fprintf(stderr, "lbvh records visited per target: %.2f\n", (double)g_nodes / n_tgt);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) die("cannot open output");
    if (op == 0) {
        std::fwrite(nbr.data(), 4, nbr.size(), o);
        std::fwrite(n_kept.data(), 4, n_kept.size(), o);
        std::fwrite(n_found.data(), 4, n_found.size(), o);
        std::fwrite(r2.data(), 8, r2.size(), o);
    } else if (op == 2) {
        // original target order, k_cap slots per target, as the export entry point
        std::vector<int32_t> nk(n_tgt), cols((size_t)(n_tgt * k_cap), -1);
        std::vector<double> w((size_t)(n_tgt * k_cap), 0.0);
        for (int64_t i = 0; i < n_tgt; ++i) {
            const int64_t ti = tperm[i];
            const int n = op_n[i];
            nk[ti] = n;
            for (int e = 0; e < n; ++e) {
                cols[ti * k_cap + e] = perm[op_c[(size_t)e * n_tgt + i]];
                w[ti * k_cap + e] = op_w[(size_t)e * n_tgt + i];
            }
        }
        std::fwrite(nk.data(), 4, nk.size(), o);
        std::fwrite(cols.data(), 4, cols.size(), o);
        std::fwrite(w.data(), 8, w.size(), o);
    } else {
        std::fwrite(out.data(), 8, out.size(), o);
    }
    std::fwrite(status.data(), 1, status.size(), o);
    std::fclose(o);
    return 0;
}
