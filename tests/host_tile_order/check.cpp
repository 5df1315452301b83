// Host check of the charged step's tile order: the multiply-high division is exact, and the
// mapping from a work-group's linear id to its tile is a bijection onto the launch's tiles.
#include "lbmix_step.h"

#include <cstdio>
#include <random>
#include <vector>

using namespace lbmix;

static int fail(const char *what, unsigned long long a, unsigned long long b, unsigned long long c) {
    std::printf("FAIL %s %llu %llu %llu\n", what, a, b, c);
    return 1;
}

int main() {
    std::mt19937_64 rng(7);
    // division: every divisor up to 2^16 against dense and random dividends, then random divisors
    for (uint32_t d = 1; d <= 65536; ++d) {
        const FastDiv f = fast_div(d);
        for (uint32_t n = 0; n < 4096; ++n)
            if (fdiv(n, f) != n / d) return fail("fdiv", n, d, fdiv(n, f));
        for (int i = 0; i < 64; ++i) {
            const uint32_t n = (uint32_t)(rng() & 0x7fffffffu);
            if (fdiv(n, f) != n / d) return fail("fdiv", n, d, fdiv(n, f));
            const uint32_t m = (n / d) * d;   // at and just below multiples of d
            if (fdiv(m, f) != m / d || (m > 0 && fdiv(m - 1, f) != (m - 1) / d)) return fail("fdiv edge", m, d, 0);
        }
    }
    for (int i = 0; i < 200000; ++i) {
        const uint32_t d = 1 + (uint32_t)(rng() % 0x7fffffffu), n = (uint32_t)(rng() & 0x7fffffffu);
        if (fdiv(n, fast_div(d)) != n / d) return fail("fdiv", n, d, 0);
    }
    // tile order: every in-plane grid of up to 6 x 64 work-groups, and the launch grids of the
    // tests and the bench workloads
    std::vector<unsigned char> seen;
    auto grid = [&](uint32_t gx, uint32_t gy) -> int {
        const TileOrder t = tile_order(gx, gy);
        const uint32_t p = gx * gy;
        if (t.band != (p % 8 == 0 ? 1u : 0u)) return fail("band flag", gx, gy, t.band);
        if (!t.band) return 0;
        seen.assign(p, 0);
        for (uint32_t by = 0; by < gy; ++by)
            for (uint32_t bx = 0; bx < gx; ++bx) {
                uint32_t tx, ty;
                xcd_tile(bx, by, t, gx, tx, ty);
                if (tx >= gx || ty >= gy) return fail("tile out of range", gx, gy, bx + gx * by);
                if (seen[tx + gx * ty]++) return fail("tile twice", gx, gy, bx + gx * by);
                // XCD (j mod 8) receives the band [xcd P/8, (xcd + 1) P/8)
                const uint32_t j = bx + gx * by, tile = tx + gx * ty;
                if (tile / (p / 8) != j % 8) return fail("band", gx, gy, j);
            }
        return 0;
    };
    for (uint32_t gx = 1; gx <= 6; ++gx)
        for (uint32_t gy = 1; gy <= 64; ++gy)
            if (grid(gx, gy)) return 1;
    const uint32_t big[][2] = {{1, 128}, {1, 32}, {1, 8}, {1, 256}, {2, 256}, {2, 512}, {3, 160}, {1, 4096}};
    for (auto &g : big)
        if (grid(g[0], g[1])) return 1;
    std::printf("tile order checks passed\n");
    return 0;
}
