// Host checks of the fused step's data handling:
// - the population layout: the element that the step stores for every (node, slot, species)
//   is a bijection onto the allocation, and the element that direction p pulls at a node is
//   the one stored for the upstream node (or, next to a wall, the node's own value of the
//   opposite slot);
// - the stochastic rounding of FP64 values to FP32 stores: over all 2^16 random inputs the
//   result is one of the two FP32 values that bracket the exact one, and their mean is the
//   exact value to 2^-17 of the gap.
#include "lbmix_step_kernel.h"

#include <cmath>
#include <cstdio>
#include <type_traits>
#include <vector>

using namespace lbmix;

template <int P, class F>
static void for_p(F &&f) {
    if constexpr (P > 0) {
        for_p<P - 1>(f);
        f(std::integral_constant<int, P - 1>{});
    }
}

template <class S>
static int check(uint32_t nx, uint32_t ny, uint32_t nzf, int ns, bool slit, uint32_t blog) {
    const uint32_t N = nx << blog;
    const size_t total = (size_t)Q * nx * ny * nzf * ns;
    std::vector<unsigned char> seen(total, 0);
    auto walls = [&](uint32_t z) -> uint32_t {
        if (!slit) return 0u;
        return (z == 0 ? 1u : 0u) | (z + 1 == nzf ? 2u : 0u);
    };
    auto stored = [&](uint32_t x, uint32_t y, uint32_t z, int arr, int s) -> size_t {
        const Pull pl(x, y, z, nx, ny, nzf, walls(z), blog);
        return elem_at<S>(s, arr, pl.q0, pl.own_inplane(), pl.own_blk(), N, ns);
    };
    int bad = 0;
    for (uint32_t z = 0; z < nzf; ++z)
        for (uint32_t y = 0; y < ny; ++y)
            for (uint32_t x = 0; x < nx; ++x)
                for (int p = 0; p < Q; ++p)
                    for (int s = 0; s < ns; ++s) {
                        const size_t e = stored(x, y, z, p, s);
                        if (e >= total || seen[e]++) ++bad;
                    }
    for (size_t e = 0; e < total; ++e)
        if (seen[e] != 1) ++bad;
    for (uint32_t z = 0; z < nzf; ++z)
        for (uint32_t y = 0; y < ny; ++y)
            for (uint32_t x = 0; x < nx; ++x) {
                const Pull pl(x, y, z, nx, ny, nzf, walls(z), blog);
                for_p<Q>([&](auto pc) {
                    constexpr int p = decltype(pc)::value;
                    int arr;
                    uint32_t plane, inplane, blk;
                    pl.template src<p>(arr, plane, inplane, blk);
                    const bool bb = (cz(p) == 1 && z == 0 && slit) || (cz(p) == -1 && z + 1 == nzf && slit);
                    const uint32_t sx = (x + nx - cx(p)) % nx, sy = (y + ny - cy(p)) % ny, sz = (z + nzf - cz(p)) % nzf;
                    for (int s = 0; s < ns; ++s) {
                        const size_t got = elem_at<S>(s, arr, plane, inplane, blk, N, ns);
                        const size_t want = bb ? stored(x, y, z, opp(p), s) : stored(sx, sy, sz, p, s);
                        if (got != want) ++bad;
                    }
                });
            }
    if (bad)
        std::printf("FAIL %u x %u x %u, %d species of %zu bytes, slit %d, blocks of %u rows: %d\n", nx, ny, nzf, ns,
                    sizeof(S), slit, 1u << blog, bad);
    return bad;
}

static int check_rounding() {
    int bad = 0;
    std::vector<double> vals = {0.0, -0.0, 1.0, -1.0, 0.1, -0.1, 1.5 + 1e-12, 3.0e-5, -7.25e-3, 123456.789,
                                1.0 - 1e-17, 2.0 - 1e-12, 1e30, -4.2e-30, double(0.1f), std::nextafter(1.0, 2.0)};
    unsigned long long x = 88172645463325252ull;   // xorshift64 for more values over 60 decades
    for (int i = 0; i < 200; ++i) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        const double m = 1.0 + double(x >> 11) * 0x1.0p-53, e = double(int(x % 121) - 60);
        vals.push_back(((x >> 3) & 1 ? -m : m) * std::pow(10.0, e / 2.0));
    }
    for (double v : vals) {
        const float n = float(v);   // nearest; the other bracketing value is its neighbour toward v
        float lo = n, hi = n;
        if (double(n) < v) hi = std::nextafter(n, INFINITY);
        if (double(n) > v) lo = std::nextafter(n, -INFINITY);
        double sum = 0.0;
        for (uint32_t k = 0; k < 65536; ++k) {
            const float f = f64_to_f32_sr(v, k << 16);
            if (f != lo && f != hi) {
                ++bad;
                break;
            }
            sum += double(f);
        }
        const double gap = double(hi) - double(lo);
        if (gap > 0.0 && std::fabs(sum / 65536.0 - v) > 0x1.0p-17 * gap * 1.0000001) ++bad;
        if (gap == 0.0 && sum != 65536.0 * v) ++bad;
    }
    if (bad) std::printf("FAIL stochastic rounding: %d values\n", bad);
    return bad;
}

int main() {
    const uint32_t shapes[][3] = {{256, 8, 3}, {5, 7, 4}, {16, 12, 5}, {64, 2, 3}, {3, 24, 2}, {8, 6, 6},
                                  {1, 1, 3}, {40, 36, 3}, {7, 16, 4}, {4, 64, 3}, {2, 128, 2}};
    int bad = 0;
    // every block height that divides ny (1 to 64 rows)
    for (auto &sh : shapes)
        for (uint32_t blog = 0; blog <= 6 && sh[1] % (1u << blog) == 0; ++blog)
            for (int ns = 1; ns <= 4; ++ns)
                for (bool slit : {false, true}) {
                    if (slit && sh[2] < 2) continue;
                    bad += check<double>(sh[0], sh[1], sh[2], ns, slit, blog);
                    bad += check<float>(sh[0], sh[1], sh[2], ns, slit, blog);
                    bad += check<uint16_t>(sh[0], sh[1], sh[2], ns, slit, blog);
                }
    // the block height chosen for a plane: a slot's block of about 32 KB that divides ny
    const uint32_t cases[][5] = {{256, 256, 2, 4, 4}, {512, 512, 2, 4, 3}, {256, 256, 2, 2, 5}, {128, 128, 3, 2, 5},
                                 {32, 32, 3, 2, 5}, {256, 256, 2, 8, 3}, {64, 6, 3, 4, 1}, {1000, 7, 2, 8, 0},
                                 {8, 64, 1, 2, 6}};
    for (auto &c : cases)
        if (pop_block_log2(c[0], c[1], c[2], c[3]) != c[4]) {
            std::printf("FAIL block rows of %u x %u, %u species of %u bytes: 2^%u\n", c[0], c[1], c[2], c[3],
                        pop_block_log2(c[0], c[1], c[2], c[3]));
            ++bad;
        }
    bad += check_rounding();
    if (bad) return 1;
    std::printf("layout checks passed\n");
    return 0;
}
