// Internal interface between the C-ABI runtime and the gfx950 Poisson kernels.
// Not installed; the public interface is include/lbmix.h.
#pragma once

#include "lbmix_step.h"

namespace lbmix {

struct PoissonArgs {
    double *psi;                     // fluid nodes
    const double *q;                 // fluid nodes
    uint32_t nx, ny, nzf;
    uint32_t N;
    int slit;                        // 1: walls from `planes` (slit or channel stack)
    const PlaneInfo *planes;         // [nzf] (walls: zero-flux faces, wall charge lumps)
    double K;                        // 4 pi l_B
    const double *bmean;             // device, per channel: mean of -K (q + lump) over it
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
    const PlaneInfo *planes;     // channel stacks (z never coarsened): no z neighbour across a
                                 // wall of this table; null otherwise
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

// Red-black SOR half-sweep of colour 0 or 1.
hipError_t launch_sor(const PoissonArgs &a, int colour, hipStream_t stream);

// Per-block partials of (||b - A psi||^2, ||b||^2, sum psi); nblocks written to *nb.
hipError_t launch_residual(const PoissonArgs &a, double *partials, uint32_t *nb,
                           hipStream_t stream);

// r = b - A psi into r[N], per-block partials of sum r^2; nblocks written to *nb.
hipError_t launch_residual_field(const PoissonArgs &a, double *r, double *partials, uint32_t *nb,
                                 hipStream_t stream);

// Per-block partials of sum q over the fluid; nblocks written to *nb.
hipError_t launch_qsum(const double *q, uint32_t N, double *partials, uint32_t *nb,
                       hipStream_t stream);

// out[z] = sum of v over fluid plane z (nxy nodes per plane), z < nplanes, in a fixed order.
hipError_t launch_plane_sum(const double *v, uint32_t nxy, uint32_t nplanes, double *out, hipStream_t stream);
// Per channel c < nch (planes [first[c], first[c+1])), from the plane sums S_z:
//   mode 0: out[c] = -K (sum_z S_z + nxy sum_z lump_z) / (nxy W_c)   (mean of b);
//   mode 1: out[c] = sum_z S_z / (nxy W_c)                             (mean of psi).
// planes may be null (no lumps).
hipError_t launch_channel_means(const double *plane_sums, const uint32_t *first, uint32_t nch,
                                const PlaneInfo *planes, uint32_t nxy, int mode, double K, double *out,
                                hipStream_t stream);
// psi -= mean[channel of the plane] (planes null: one channel).
hipError_t launch_shift_planes(double *psi, uint32_t nxy, uint32_t N, const PlaneInfo *planes,
                               const double *mean, hipStream_t stream);

// out[v] = sum_b partials[v * nblocks + b] for v < nv, in a fixed order; then
// out[nv + k] for the post-processing `mode`:
//   mode 0: none;  mode 1: out[nv] = -K (out[0] + lumps) / N   (mean of b);
//   mode 2: out[nv] = out[2] / N                                (mean of psi).
hipError_t launch_finalize(const double *partials, uint32_t nblocks, int nv, double *out,
                           int mode, double K, double lumps, double N, hipStream_t stream);

// Level-0 right-hand side b = -K (q + lump) - mean(b) into r (mean per channel).
hipError_t launch_make_rhs(const PoissonArgs &a, double *r, hipStream_t stream);
// One red-black Gauss-Seidel half-sweep of level L.
hipError_t launch_mg_smooth(const MGLevel &L, int colour, hipStream_t stream);
// Residual of level F restricted (cell average) into the right-hand side of level C; e of
// level C set to 0.
hipError_t launch_mg_restrict(const MGLevel &F, const MGLevel &C, hipStream_t stream);
// e of level F += trilinear interpolation of e of level C.
hipError_t launch_mg_prolong(const MGLevel &F, const MGLevel &C, hipStream_t stream);
// Line relaxation along z of a channel-stack level, colour (x + y) mod 2 of the columns:
// launch_mg_line_rhs writes g = (lateral neighbour terms) - r into e of the cells of that
// colour; launch_mg_line_solve then solves the tridiagonal z-system of every line of that colour
// in every channel (planes [first[c], first[c + 1]), c < nch) from both ends towards the
// middle plane W / 2 of a channel of W planes, with the inverse pivots idn[j] of the j-th
// step from either end (one recurrence, shared by the channels) and pmid[c] of the middle
// plane (0 pins the middle plane of a singular line to 0).
hipError_t launch_mg_line_rhs(const MGLevel &L, int colour, hipStream_t stream);
hipError_t launch_mg_line_solve(const MGLevel &L, int colour, const double *idn, const double *pmid,
                                const uint32_t *first, uint32_t nch, hipStream_t stream);
// The levels of `b`, solved by one work-group in LDS: V-cycle (2 pre-, 2 post-sweeps) whose
// coarsest level gets b.coarse_sweeps red-black sweeps; e of b.lev[0] starts at 0 and is
// written back to global memory.
hipError_t launch_mg_bottom(const MGBottom &b, hipStream_t stream);
// Warm start from the last three solutions: psi <- psi + p1 - p2, p2 <- p1, p1 <- old psi.
hipError_t launch_extrapolate(double *psi, double *p1, double *p2, uint32_t N, hipStream_t stream);

// Batched FP64 product C_b[m][n] = sum_k A_b[m][k] B_b[k][n] with element strides (the
// unit stride of C is n).  With rhs set, A holds q and the product takes
// A[m][k] = -rhs_K (q + lump of plane m / rows_per_plane) instead (lumps from planes, which
// may be null), the right-hand side of the Poisson equation formed on the fly.
struct SpecGemm {
    const double *A, *B;
    double *C;
    uint32_t M, N, K, batch;
    size_t sAb, sAm, sAk, sBb, sBk, sBn, sCb, sCm;
    int rhs;
    double rhs_K;
    const PlaneInfo *planes;
    uint32_t rows_per_plane;
};
// a_k_unit: sAk == 1 (else sAm == 1); b_n_unit: sBn == 1 (else sBk == 1); these choose the
// coalesced load pattern only.
hipError_t launch_gemm_f64(const SpecGemm &g, bool a_k_unit, bool b_n_unit, hipStream_t stream);
// Tridiagonal solves along z for every mode (nmodes per plane) and every segment of planes
// [seg[s], seg[s+1]), s < nseg.  Inverse pivots: piv[k][mode] for plane k of a segment
// before its last plane (the same for every segment; as many rows as the longest segment
// less one), piv_end[s][mode] for the last plane of segment s.
hipError_t launch_tridiag_z(const double *b, const double *piv, const double *piv_end, double *out, uint32_t nmodes,
                            const uint32_t *seg, uint32_t nseg, hipStream_t stream);
// Per-plane transform along x and y of planes of at most SPEC_XY_MAX nodes (nx, ny <= 64)
// on the FP64 matrix cores: planes up to 32 x 32 in the registers of one wave each, larger
// ones in LDS (each work-group takes several planes, or half a plane when there are fewer
// planes than compute units).  Forward: out = Ty P Tx^T with P the plane
// of `in`, or, when `q` is given, of b = -K (q + lump_z) (lumps from planes, which may be
// null).  Inverse: out = Ty^T P Tx.
constexpr uint32_t SPEC_XY_MAX = 4096;
constexpr uint32_t SPEC_PAD = 64;    // padded extent of the bases below (row stride SPEC_PAD + 1)
struct SpecXY {
    const double *in, *q;
    double *out;
    const double *tx, *ty;           // nx x nx and ny x ny bases (row k = basis vector k)
    const double *txp, *typ;         // the same zero-padded to 64 rows of stride 65 (required)
    const PlaneInfo *planes;
    double K;
    uint32_t nx, ny, nplanes;
};
hipError_t launch_spec_xy(const SpecXY &a, bool forward, hipStream_t stream);
// Tridiagonal solves as launch_tridiag_z, the columns staged in LDS; `longest` = planes of
// the longest segment, at most TRI_LDS_MAX.  Both forms also remove the segment mean of
// mode 0 from the right-hand side first (the projection onto consistent data of each channel).
constexpr uint32_t TRI_LDS_MAX = 2048;
// They eliminate from both ends of a segment towards its middle plane L / 2, which takes the
// inverse of its condensed diagonal from pmid[s][mode] (0 for the singular mode).
hipError_t launch_tridiag_lds(const double *b, const double *piv, const double *pmid, double *out, uint32_t nmodes,
                              const uint32_t *seg, uint32_t nseg, uint32_t longest, hipStream_t stream);
// The same transforms by fast Fourier transforms, for sequences of a power-of-two length n
// (FFT_MIN <= n <= FFT_MAX) along one axis: the coefficients in the real Fourier basis of
// every sequence (forward), or the sequences from their coefficients (inverse).  Sequence s
// of the batch (s < nseq) lies in plane s / 2^log2pp, at index j = s mod 2^log2pp, and its
// element x at in[plane * s_plane + j * s_seq + x * s_el]; one of s_seq and s_el is 1 (cols:
// s_seq == 1, the sequences of a plane side by side; else s_el == 1, each sequence
// contiguous).  log2pp >= 1.  Forward with rhs: the sequences are those of
// b = -K (q + lump_plane), read from q (lumps from planes, which may be null).  tw holds
// exp(-2 pi i t / n) for t < n as (real, imaginary) pairs.  in and out must not overlap.
constexpr uint32_t FFT_MIN = 8, FFT_MAX = 1024;
struct FftPass {
    const double *in;
    double *out;
    const double *tw;
    uint32_t n, log2n, nseq, log2pp;
    size_t s_plane;
    uint32_t s_seq, s_el;
    int rhs;
    double rhs_K;
    const PlaneInfo *planes;
};
hipError_t launch_fft_pass(const FftPass &f, bool cols, bool inverse, hipStream_t stream);
// a <- -a / (mux[x] + muy[y] + muz[z]), 0 where the sum is 0.
hipError_t launch_spectral_scale(double *a, const double *mux, const double *muy, const double *muz, uint32_t nx,
                                 uint32_t ny, uint32_t N, hipStream_t stream);

// psi -= *mean on the fluid nodes.
hipError_t launch_shift(double *psi, uint32_t N, const double *mean, hipStream_t stream);

// Plane sums over x and y of n and j (full-lattice arrays) into out[4][nz].
hipError_t launch_plane_sums(const double *n, const double *j, uint32_t nx, uint32_t ny,
                             uint32_t nz, double *out, hipStream_t stream);

}  // namespace lbmix
