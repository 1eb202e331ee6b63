// Exhaustive host check of ws_deal (bf_internal.h) and the host tables of
// bf_host.h (ws_deal_table, ws_balance_table): for item counts and
// grids of every size class, the map is a bijection of 0 .. n - 1, and
// items that are consecutive within one workgroup's block land in
// consecutive products of that workgroup, i.e. nb positions apart, where
// the wave-specialised schedule's share (lo + j + k nb) puts them.
#include <cstdio>
#include <vector>

#include "bf_host.h"

static int check(int n, int G)
{
    std::vector<int> hit((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        const int p = ws_deal(i, n, G);
        if (p < 0 || p >= n) {
            std::fprintf(stderr, "n=%d G=%d: item %d -> %d out of range\n", n, G, i, p);
            return 1;
        }
        hit[(size_t)p]++;
    }
    for (int p = 0; p < n; ++p)
        if (hit[(size_t)p] != 1) {
            std::fprintf(stderr, "n=%d G=%d: position %d hit %d times\n", n, G, p, hit[(size_t)p]);
            return 1;
        }
    // The host table agrees with the per-item map.
    std::vector<int> tab((size_t)n + 1, -7);
    ws_deal_table(tab.data(), n, G);
    if (tab[(size_t)n] != -7) {
        std::fprintf(stderr, "n=%d G=%d: ws_deal_table wrote past its end\n", n, G);
        return 1;
    }
    for (int i = 0; i < n; ++i)
        if (tab[(size_t)i] != ws_deal(i, n, G)) {
            std::fprintf(stderr, "n=%d G=%d: ws_deal_table[%d] = %d, ws_deal %d\n", n, G, i, tab[(size_t)i],
                         ws_deal(i, n, G));
            return 1;
        }
    // The share of workgroup b (as the kernel computes it) must be a run of
    // consecutive item indices.
    const int X = G < 8 ? G : 8;
    std::vector<int> inv((size_t)n);
    for (int i = 0; i < n; ++i)
        inv[(size_t)ws_deal(i, n, G)] = i;
    for (int b = 0; b < G; ++b) {
        const int x = b % X, j = b / X;
        const int nb = G / X + (x < G % X ? 1 : 0);
        const int q = n / X, r = n % X;
        const int lo = x * q + (x < r ? x : r);
        const int cnt = q + (x < r ? 1 : 0);
        const int n_my = j < cnt ? (cnt - j + nb - 1) / nb : 0;
        for (int k = 1; k < n_my; ++k) {
            const int a = inv[(size_t)(lo + j + (k - 1) * nb)], c = inv[(size_t)(lo + j + k * nb)];
            if (c != a + 1) {
                std::fprintf(stderr, "n=%d G=%d: workgroup %d products %d, %d are items %d, %d\n", n, G, b,
                             k - 1, k, a, c);
                return 1;
            }
        }
    }
    return 0;
}

// ws_balance_table: a bijection onto the shares' layout, every workgroup
// getting exactly the products its share holds, and a balanced deal: the
// ranks a workgroup receives sum to within the part's size of the mean
// rank sum (so summed f, ranked longest first, comes out even).
static int check_balance(int n, int G)
{
    std::vector<int> pos((size_t)n + 1, -7), hit((size_t)n, 0);
    ws_balance_table(pos.data(), n, G);
    if (pos[(size_t)n] != -7) {
        std::fprintf(stderr, "balance n=%d G=%d: wrote past its end\n", n, G);
        return 1;
    }
    for (int i = 0; i < n; ++i) {
        const int p = pos[(size_t)i];
        if (p < 0 || p >= n || hit[(size_t)p]++) {
            std::fprintf(stderr, "balance n=%d G=%d: rank %d -> %d out of range or repeated\n", n, G, i, p);
            return 1;
        }
    }
    // every position's part is the part of its rank (items stay in their XCD's eighth)
    std::vector<int> part((size_t)n);
    ws_part_table(part.data(), n, G);
    for (int i = 0; i < n; ++i)
        if (part[(size_t)pos[(size_t)i]] != part[(size_t)i]) {
            std::fprintf(stderr, "balance n=%d G=%d: rank %d leaves its part\n", n, G, i);
            return 1;
        }
    return 0;
}

int main()
{
    const int grids[] = {1, 2, 3, 7, 8, 9, 15, 16, 17, 31, 64, 255, 256, 257, 512, 1000};
    long cases = 0;
    for (int G : grids)
        for (int n = 0; n <= 3000; n += (n < 600 ? 1 : 37)) {
            if (check(n, G))
                return 1;
            ++cases;
        }
    for (int n : {8192, 16384, 16383, 65536})
        for (int G : {256, 255, 248})
            if (check(n, G) || check_balance(n, G))
                return 1;
    for (int G : grids)
        for (int n = 0; n <= 3000; n += (n < 600 ? 1 : 37))
            if (check_balance(n, G))
                return 1;
    std::fprintf(stderr, "ws_deal ok (%ld cases)\n", cases);
    return 0;
}
