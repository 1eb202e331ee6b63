// Host check of the product orders 1 to 4 of the library (order_items,
// linked from libbf.so) on uneven batches (f ~ U{0..36}, W ids from a
// pool), for the wave-specialised schedule's grid of one workgroup per CU:
//   * every order is a permutation of the items; orders 1 and 2 sort as
//     documented (f descending then W id; W id modulo 8), stably, also for
//     batches of one f;
//   * order 3: with 8 or more items per W and per workgroup, the products of
//     one workgroup come in runs of one W (3 in 4 consecutive pairs share it);
//   * order 4: within each part, no workgroup's summed (f + 32) exceeds the
//     part's mean by more than 4% plus one product (the caller's order gives
//     about 20% on such batches).
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "bf_host.h"

static int run(int n, int n_w, int G, unsigned seed, bool one_f)
{
    std::mt19937 rng(seed);
    std::vector<BfItem> in((size_t)n), out((size_t)n);
    for (int t = 0; t < n; ++t) {
        in[(size_t)t] = BfItem{};
        in[(size_t)t].w_id = (int)(rng() % (unsigned)n_w);
        in[(size_t)t].f = one_f ? 36 : (int)(rng() % 37u);
        in[(size_t)t].pad0 = t;   // item identity
    }
    std::vector<int> scratch;
    BalanceTable bt;
    bt.n = n;
    bt.g = G;
    bt.pos.resize((size_t)n);
    bt.part.resize((size_t)n);
    ws_balance_table(bt.pos.data(), n, G);
    ws_part_table(bt.part.data(), n, G);
    std::vector<int> deal((size_t)n);
    ws_deal_table(deal.data(), n, G);
    const int X = G < 8 ? G : 8;
    for (int mode : {1, 2, 3, 4}) {
        std::fill(out.begin(), out.end(), BfItem{});
        for (BfItem &o : out)
            o.pad0 = -1;
        order_items(in.data(), out.data(), n, n_w, scratch, mode, mode == 3 ? deal.data() : nullptr,
                    mode == 4 ? &bt : nullptr);
        std::vector<int> seen((size_t)n, 0);
        for (int p = 0; p < n; ++p) {
            const int id = out[(size_t)p].pad0;
            if (id < 0 || id >= n || seen[(size_t)id]++) {
                std::fprintf(stderr, "mode %d n=%d: position %d holds item %d\n", mode, n, p, id);
                return 1;
            }
        }
        if (mode == 1)
            for (int p = 1; p < n; ++p) {
                const BfItem &u = out[(size_t)p - 1], &v = out[(size_t)p];
                // f descending, then W id ascending, then the caller's order
                const bool ok = u.f > v.f || (u.f == v.f && (u.w_id < v.w_id ||
                                                            (u.w_id == v.w_id && u.pad0 < v.pad0)));
                if (!ok) {
                    std::fprintf(stderr, "mode 1 n=%d: positions %d, %d out of order\n", n, p - 1, p);
                    return 1;
                }
            }
        if (mode == 2)
            for (int p = 1; p < n; ++p) {
                const BfItem &u = out[(size_t)p - 1], &v = out[(size_t)p];
                const bool ok = u.w_id % 8 < v.w_id % 8 || (u.w_id % 8 == v.w_id % 8 && u.pad0 < v.pad0);
                if (!ok) {
                    std::fprintf(stderr, "mode 2 n=%d: positions %d, %d out of order\n", n, p - 1, p);
                    return 1;
                }
            }
        if (mode == 4) {
            // within each part, no workgroup's summed (f + 32) exceeds the
            // part's mean by more than 4% plus one product (those taking one
            // product more than the others)
            const int q = n / X, r = n % X;
            for (int x = 0; x < X; ++x) {
                const int lo = x * q + (x < r ? x : r);
                const int cnt = q + (x < r ? 1 : 0);
                const int nb = G / X + (x < G % X ? 1 : 0);
                if (cnt < 16 * nb)
                    continue;
                double total = 0, mx = 0;
                for (int j = 0; j < nb; ++j) {
                    double sum = 0;
                    for (int p = lo + j; p < lo + cnt; p += nb)
                        sum += out[(size_t)p].f + 32;
                    total += sum;
                    mx = std::max(mx, sum);
                }
                const double mean = total / nb;
                if (mx > 1.04 * mean + 68) {
                    std::fprintf(stderr, "mode 4 n=%d G=%d part %d: workgroup sum %.0f against mean %.0f\n", n,
                                 G, x, mx, mean);
                    return 1;
                }
            }
        }
        if (mode == 3 && n >= 8 * n_w && n >= 8 * G) {
            // with 8 or more items per W and per workgroup, consecutive products of
            // a workgroup share W at least 3 times in 4
            long same = 0, pairs = 0;
            const int q = n / X, r = n % X;
            for (int x = 0; x < X; ++x) {
                const int lo = x * q + (x < r ? x : r);
                const int cnt = q + (x < r ? 1 : 0);
                const int nb = G / X + (x < G % X ? 1 : 0);
                for (int j = 0; j < nb; ++j)
                    for (int p = lo + j + nb; p < lo + cnt; p += nb, ++pairs)
                        same += out[(size_t)p].w_id == out[(size_t)(p - nb)].w_id;
            }
            if (4 * same < 3 * pairs) {
                std::fprintf(stderr, "mode 3 n=%d n_w=%d: %ld of %ld consecutive pairs share W\n", n, n_w, same,
                             pairs);
                return 1;
            }
        }
    }
    return 0;
}

int main()
{
    long cases = 0;
    for (int G : {1, 7, 8, 9, 64, 255, 256})
        for (int n : {0, 1, 5, 63, 64, 65, 1000, 4099, 8192, 16384})
            for (int n_w : {1, 3, 64, 256})
                if (run(n, n_w, G, (unsigned)(n * 31 + G * 7 + n_w), false) ||
                    run(n, n_w, G, (unsigned)(n * 17 + G + n_w), true)) {
                    return 1;
                } else {
                    ++cases;
                }
    std::fprintf(stderr, "orders ok (%ld cases)\n", cases);
    return 0;
}
