// Internal interface between the C-ABI runtime and the gfx950 kernels of the library.
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

// Arguments of the fused stream-collide launch.  Populations are stored [p][node][species]
// over the fluid nodes only (node = x + nx * (y + ny * zf), zf the fluid plane), in the
// storage type; a stored value is (f_p - w_p rho_bar) * scale_p.
struct StepArgs {
    const void *fin;
    void *fout;
    uint32_t nx, ny, nzf;
    uint32_t N;                      // nx * ny * nzf
    int ns;                          // species count (element stride of the layout)
    double rho_bar[MAXS];            // storage shift per species (0: plain f)
    float scale[MAXS][Q];            // 16-bit forms: power-of-two scale (1 otherwise)
    float inv_scale[MAXS][Q];
    double omega_v, omega_d;
    double valence[MAXS];
    double E[3];                     // applied field, acceleration per unit valence
    const double *psi;               // potential on fluid nodes (charged runs)
    double *q;                       // out: charge density on fluid nodes (charged runs)
    double q_rest;                   // sum_s valence_s * rho_bar_s
    double ghost_lo, ghost_hi;       // 4 pi l_B sigma of the walls z = 0 and z = nz-1
    double *partials;                // out: [species][block] FP64 sums of n - rho_bar
    int stochastic;                  // 16-bit forms: 1 = stochastic rounding, 0 = nearest-even
    uint32_t seed;                   // per-step seed of the rounding hash
};

struct PoissonArgs {
    double *psi;                     // fluid nodes
    const double *q;                 // fluid nodes
    uint32_t nx, ny, nzf;
    uint32_t N;
    int slit;
    double K;                        // 4 pi l_B
    double lump_lo, lump_hi;         // wall charge added to the first / last fluid plane
    const double *bmean;             // device scalar: mean of b over the fluid
    double omega;                    // SOR factor
};

// One level of the multigrid hierarchy for the Poisson operator: cell-centred grid of
// nx * ny * nz cells with per-direction coefficients (1 / H_d^2 for spacing H_d relative to the
// fluid grid); e = correction (the potential itself on level 0), r = right-hand side.
struct MGLevel {
    double *e, *r;
    uint32_t nx, ny, nz;
    double ax, ay, az;
    int periodic_z;              // 1: periodic box, 0: zero-flux planes (slit)
    int fx, fy, fz;              // coarsening factor (1 or 2) towards the next level
};

constexpr int MG_MAX_BOTTOM = 8;
constexpr int MG_BOTTOM_LDS = 4096;   // cells of all bottom levels together (LDS, FP64, e and r)
// The coarse end of the hierarchy, solved by one work-group in LDS: a V-cycle over
// lev[0..n-1]; only lev[0] refers to global memory (its r in, its e out).
struct MGBottom {
    MGLevel lev[MG_MAX_BOTTOM];
    int n;
    int coarse_sweeps;
    const double *coarse_inv;    // dense (A + 1 1^T / m)^-1 of the coarsest level (m cells), or null
};

dim3 node_grid(uint32_t nx, uint32_t ny, uint32_t nz, dim3 *block);
dim3 step_grid(uint32_t nx, uint32_t ny, uint32_t nzf, dim3 *block);

hipError_t launch_stream_collide(Store st, int ns, bool slit, bool field, bool charged,
                                 const StepArgs &a, hipStream_t stream);

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

// Red-black SOR half-sweep of colour 0 or 1.
hipError_t launch_sor(const PoissonArgs &a, int colour, hipStream_t stream);

// Per-block partials of (||b - A psi||^2, ||b||^2, sum psi); nblocks written to *nb.
hipError_t launch_residual(const PoissonArgs &a, double *partials, uint32_t *nb,
                           hipStream_t stream);

// Per-block partials of sum q over the fluid; nblocks written to *nb.
hipError_t launch_qsum(const double *q, uint32_t N, double *partials, uint32_t *nb,
                       hipStream_t stream);

// out[v] = sum_b partials[v * nblocks + b] for v < nv, in a fixed order; then
// out[nv + k] for the post-processing `mode`:
//   mode 0: none;  mode 1: out[nv] = -K (out[0] + lumps) / N   (mean of b);
//   mode 2: out[nv] = out[2] / N                                (mean of psi).
hipError_t launch_finalize(const double *partials, uint32_t nblocks, int nv, double *out,
                           int mode, double K, double lumps, double N, hipStream_t stream);

// Level-0 right-hand side b = -K (q + lump) - mean(b) into r.
hipError_t launch_make_rhs(const PoissonArgs &a, double *r, hipStream_t stream);
// One red-black Gauss-Seidel half-sweep of level L.
hipError_t launch_mg_smooth(const MGLevel &L, int colour, hipStream_t stream);
// Residual of level F restricted (cell average) into the right-hand side of level C; e of
// level C set to 0.
hipError_t launch_mg_restrict(const MGLevel &F, const MGLevel &C, hipStream_t stream);
// e of level F += trilinear interpolation of e of level C.
hipError_t launch_mg_prolong(const MGLevel &F, const MGLevel &C, hipStream_t stream);
// The levels of `b`, solved by one work-group in LDS: V-cycle (2 pre-, 2 post-sweeps) whose
// coarsest level gets b.coarse_sweeps red-black sweeps; e of b.lev[0] starts at 0 and is
// written back to global memory.
hipError_t launch_mg_bottom(const MGBottom &b, hipStream_t stream);
// Warm start from the last three solutions: psi <- psi + p1 - p2, p2 <- p1, p1 <- old psi.
hipError_t launch_extrapolate(double *psi, double *p1, double *p2, uint32_t N, hipStream_t stream);

// psi -= *mean on the fluid nodes.
hipError_t launch_shift(double *psi, uint32_t N, const double *mean, hipStream_t stream);

// Plane sums over x and y of n and j (full-lattice arrays) into out[4][nz].
hipError_t launch_plane_sums(const double *n, const double *j, uint32_t nx, uint32_t ny,
                             uint32_t nz, double *out, hipStream_t stream);

}  // namespace lbmix
