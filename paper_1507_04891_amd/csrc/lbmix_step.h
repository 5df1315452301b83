// Internal interface between the C-ABI runtime and the gfx950 kernels of the fused step.
// Not installed; the public interface is include/lbmix.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbmix {

constexpr int Q = 19;
constexpr int MAXS = 4;
constexpr int BLOCK = 256;        // threads per work-group row of the node kernels
constexpr int STEP_BLOCK = 512;   // threads per work-group of stream_collide (two rows)

enum class Store : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

// One fluid plane of a geometry with walls (a slit, or a stack of slit channels along z that
// share the lateral extent): its wall neighbours, its channel and the channel's parameters.
struct PlaneInfo {
    double omega_d;       // drag frequency of the channel
    double ghost_lo;      // 4 pi l_B sigma of the wall below (used when walls & 1)
    double ghost_hi;      // 4 pi l_B sigma of the wall above (used when walls & 2)
    double lump;          // wall charge per node lumped into this plane (Poisson)
    uint32_t walls;       // bit 0: the plane below is a wall; bit 1: the plane above is a wall
    uint32_t chan;        // channel index
    uint32_t zfull;       // index of the plane in the full-lattice arrays
    uint32_t zloc;        // index of the plane in its own channel's lattice (walls counted)
};

// Rows of a block of the population layout: the power of two (at most 64) that makes a slot's
// block about 32 KB (a row holds nx ns esize bytes), or the largest below it that divides ny.
// Measured on the 256^3 binary step in FP32 (2 KB rows): 0.871, 0.849, 0.826, 0.838 and 0.856
// ms per step with blocks of 4, 8, 16, 32 and 64 rows; at 512^3 (4 KB rows): 6.92, 7.13 and
// 7.60 ms with 8, 16 and 32 rows.
inline uint32_t pop_block_log2(uint32_t nx, uint32_t ny, uint32_t ns, uint32_t esize) {
    const unsigned long long row = (unsigned long long)nx * ns * esize;
    uint32_t l = 0;
    while (l < 6 && (row << (l + 1)) <= 32768ull) ++l;
    while (l > 0 && ny % (1u << l) != 0) --l;
    return l;
}

// Division by a fixed divisor d >= 1 as a multiply-high, an add and a shift (the round-up
// method of Granlund and Montgomery): m = floor(2^32 (2^s - d) / d) + 1 with s = ceil(log2 d).
// Exact for every n < 2^31.
struct FastDiv {
    uint32_t d, m, s;
};
inline FastDiv fast_div(uint32_t d) {
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    return FastDiv{d, (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1), s};
}
__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
    const uint32_t t = (uint32_t)(((unsigned long long)n * f.m) >> 32);
    return (t + n) >> f.s;
}

// Tile order of the charged step.  The hardware deals the work-groups of a launch to the eight
// XCDs in turn (linear id b to XCD b mod 8), each XCD with its own L2, so in dispatch order the
// rows y - 1, y and y + 1 of a plane sit in three L2s and each row of the potential, which the
// gradient reads at the six neighbours of a node, is fetched three times.  When a plane has a
// multiple of 8 work-groups, the XCD of a work-group is set by its index j within the plane, and
// the j-th work-group takes tile (j mod 8) P/8 + j/8 of the P in the plane instead: each XCD
// works on a band of consecutive rows of every plane, and the chip still works through the
// planes in order.  Any order is correct; this one only changes which L2 serves which tile.
struct TileOrder {
    uint32_t band;        // 1: bands of rows per XCD; 0: dispatch order
    uint32_t per_xcd;     // work-groups of a plane per XCD (P / 8)
    FastDiv per_row;      // work-groups along x
};
__host__ __device__ inline void xcd_tile(uint32_t bx, uint32_t by, const TileOrder &t, uint32_t gx, uint32_t &tx,
                                         uint32_t &ty) {
    const uint32_t j = bx + gx * by;
    const uint32_t tile = (j & 7u) * t.per_xcd + (j >> 3);
    ty = fdiv(tile, t.per_row);
    tx = tile - ty * gx;
}
inline TileOrder tile_order(uint32_t gx, uint32_t gy) {
    const uint32_t p = gx * gy;
    return TileOrder{p % 8 == 0 ? 1u : 0u, p / 8, fast_div(gx)};
}

// Arguments of the fused stream-collide launch.  Populations are stored over the fluid
// planes only, [zf][y / B][p][y mod B][x][species] with B = 2^blog rows per block (the
// 16-bit three-species form splits each block of a slot into pairs and singles), in the
// storage type; a stored value is (f_p - w_p rho_bar) * scale_p.  The potential and the
// charge density are indexed by node = x + nx * (y + ny * zf).
struct StepArgs {
    const void *fin;
    void *fout;
    uint32_t nx, ny, nzf;
    uint32_t N;                      // slot stride of the populations: B nx nodes
    uint32_t blog;                   // log2 B, B the rows of a block (B divides ny; pop_block_log2)
    int ns;                          // species count (element stride of the layout)
    double rho_bar[MAXS];            // storage shift per species (0: plain f)
    float scale[MAXS][Q];            // 16-bit forms: power-of-two scale (1 otherwise)
    float inv_scale[MAXS][Q];
    // per species and weight class k (rest, axis, diagonal): w_k scale_k and
    // w_k omega_visc scale_k, in FP64 and FP32
    double cw[MAXS][3], cwo[MAXS][3];
    float cwf[MAXS][3], cwof[MAXS][3];
    double inv_scale_k[MAXS][3];     // inv_scale of weight class k, in FP64
    double omega_v, omega_d;
    // the same parameters in FP32 for the FP32-arithmetic kernels (the scalar unit has no
    // floating-point conversion, so converting them in the kernel takes vector instructions)
    float rho_bar_f[MAXS];
    float omega_v_f, omega_d_f;
    int pair_drag;                   // 1: drag frequency per pair (three or more species)
    double omega_pair[MAXS][MAXS];   // symmetric; the diagonal is not used
    int forcing;                     // 0: forcing of the Appendix; 1: the Guo-type variant
    double valence[MAXS];
    double E[3];                     // applied field, acceleration per unit valence
    const double *psi;               // potential on fluid nodes (charged runs)
    double *q;                       // out: charge density on fluid nodes (charged runs)
    double q_rest;                   // sum_s valence_s * rho_bar_s
    const PlaneInfo *planes;         // [nzf] for geometries with walls (null for the box)
    const int32_t *fluid_of_full;    // [nzfull]: fluid plane of a full-lattice plane, -1 = wall
    uint32_t nzfull;                 // planes of the full-lattice arrays
    double *partials;                // out: [species][block] FP64 sums of n - rho_bar
    int stochastic;                  // 16-bit forms: 1 = stochastic rounding, 0 = nearest-even
    int wide;                        // FP32 / 16-bit forms: 1 = density deviation carried in FP64,
                                     // 0 = FP32 collision arithmetic throughout
    uint32_t seed;                   // per-step seed of the rounding hash
    const unsigned long long *step_dev;  // non-null (captured steps): seed from the step count
    unsigned long long round_seed;       // ... here, as the host derives it
    uint32_t block_x, block_y;       // launch shape of stream_collide (0: the default shape)
    TileOrder tiles;                 // filled by launch_stream_collide (charged step)
};

dim3 node_grid(uint32_t nx, uint32_t ny, uint32_t nz, dim3 *block);
// Work-group shape of stream_collide: bx x by threads (bx x by <= STEP_BLOCK), or by default
// rows of up to 256 nodes along x, two rows per work-group, and for a plane narrower than 64
// nodes 512 / nx whole rows per work-group.
dim3 step_grid(uint32_t nx, uint32_t ny, uint32_t nzf, dim3 *block, uint32_t bx = 0, uint32_t by = 0);

// The work-group shape launch_stream_collide uses: the set one (bx_set, by_set), or 0 x 0 for
// step_grid's default, except: one row of up to 256 nodes for FP32 with stochastic rounding
// and at most two species (three waves per SIMD) and for one or two 16-bit species (rows of at
// least 64 nodes), and 128 threads (128 nodes of a row, or 128 / nx whole rows of a narrow
// plane) for three species in 16 bits (three waves per SIMD).
void step_shape(Store st, bool stochastic, int ns, uint32_t nx, uint32_t bx_set, uint32_t by_set, uint32_t *bx,
                uint32_t *by);
hipError_t launch_stream_collide(Store st, int ns, bool slit, bool field, bool charged,
                                 const StepArgs &a, hipStream_t stream);
// Work-groups of the launch launch_stream_collide makes for these arguments (the length of each
// species' row of FP64 mass partials it writes).
uint32_t stream_collide_blocks(Store st, int ns, const StepArgs &a);

// Per-step rounding seed: a splitmix64 finaliser of seed + golden-ratio increment x step,
// folded to 32 bits (step = completed steps + 1).
__host__ __device__ inline uint32_t step_seed(unsigned long long seed, unsigned long long step) {
    unsigned long long z = seed + 0x9e3779b97f4a7c15ull * step;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (uint32_t)(z ^ (z >> 32));
}

// Plain device copy of n16 16-byte elements (16-byte aligned buffers).
hipError_t launch_copy16(const void *src, void *dst, size_t n16, hipStream_t stream);

// *step += 1 (one thread): the step count of captured steps; set_step: *step = value.
hipError_t launch_advance_step(unsigned long long *step, hipStream_t stream);
hipError_t launch_set_step(unsigned long long *step, unsigned long long value, hipStream_t stream);

// Equilibrium of species s from host-layout device arrays n[N_full], u[3][N_full] (u may
// be null), scattered into the slots the first pull reads.
hipError_t launch_init(Store st, bool slit, int s, const StepArgs &a, const double *n,
                       const double *u, hipStream_t stream);

// Pull-gathered pre-collision moments of species s into full-lattice arrays (wall planes
// written as 0); j may be null.
hipError_t launch_moments(Store st, bool slit, int s, const StepArgs &a, double *n, double *j,
                          hipStream_t stream);

// Pull-gathered pre-collision populations (shift added back) of species s, [19][N_full].
hipError_t launch_populations(Store st, bool slit, int s, const StepArgs &a, double *f,
                              hipStream_t stream);

// Charge density q = q_rest + sum_s valence_s (n_s - rho_bar_s) of the pre-collision state
// on fluid nodes.
hipError_t launch_charge(Store st, bool slit, int ns, const StepArgs &a, double *q,
                         hipStream_t stream);

}  // namespace lbmix
