/*
 * lbmix_oracle.c -- plain, slow FP64 CPU reference of the multicomponent lattice-Boltzmann
 * method with separate time scales for momentum and mass diffusion.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the smoke check
 * and by the CPU-baseline leg of the benchmark, and by nothing else.  It shares no code,
 * table, header or generator with the GPU library; neither includes nor links the other.
 *
 * Source: M. Monteferrante, S. Melchionna, U. Marini Bettolo Marconi, "Lattice Boltzmann
 * Method for mixtures at variable Schmidt number" (arXiv:1507.04891).  Citations below name
 * the section and the equation label of that paper.
 *
 *   Sec. IV (Results), eq. (latboeq): the discrete update
 *       f_p(r + c_p, t + 1) = f_p(r,t) - omega_visc [f_p(r,t) - phi_perp_p(r,t)] + g_p(r,t)
 *   Sec. IV: D3Q19 velocity set, unit time step and lattice spacing.
 *   Appendix, last equation: the orthogonalised equilibrium phi_perp_p.
 *   Appendix, eq. (ourforc): the forcing term g_p.
 *   Sec. II, the equation that defines F^{alpha,drag}/m (after the equal-mass gamma): drag.
 *   Sec. II, eq. (evolution), third term, and eq. (Poisson) with the surface-charge condition
 *       that follows it: electrostatic force, Poisson equation, wall boundary condition.
 *   Sec. III, first equations: n^alpha, u^alpha, barycentric u.
 *
 * Readings where the paper is silent (each one is also applied by the GPU library):
 *   [R1] v_T^2 = 1/3 and Gamma_0p = the D3Q19 weights (1/3, 1/18, 1/36); m = e = 1.
 *   [R2] u^alpha in phi_perp and g is the plain first moment of the pre-collision
 *        populations divided by n^alpha, and u their barycentric average; g has no
 *        (1 - omega/2) factor; n^alpha = 0 gives u^alpha = 0.
 *   [R3] g uses the total force per particle of species alpha, F^alpha = drag + a^alpha,
 *        with the field acceleration a^alpha = z^alpha (E_ext - v_T^2 grad psi~)
 *        (psi~ = e psi / k_B T, so e grad psi / m = v_T^2 grad psi~).
 *   [R3b] The drag is evaluated on the mid-step species velocities u^alpha + a^alpha / 2
 *        (and their barycentric average), i.e. the field forces enter the drag the way a
 *        second-order forcing scheme defines the fluid velocity; the drag itself stays
 *        explicit.  Without this, a state with zero particle flux has u^alpha = -F^alpha/2
 *        before collision, the drag answers it, and every field force is amplified by
 *        1 / (1 - omega_drag / 2): the mobility becomes 1/omega_drag instead of
 *        D / v_T^2 = 1/omega_drag - 1/2, breaking the Boltzmann (Gouy-Chapman) equilibrium
 *        and the Helmholtz-Smoluchowski flow that Sec. III-IV compare against.  Without
 *        field forces (neutral mixtures) nothing changes, so D = v_T^2 (1/omega_drag - 1/2)
 *        of Sec. IV is untouched.
 *   [R4] grad(psi~) by second-order central differences; at a slit wall the ghost value is
 *        psi~(adjacent fluid) + 4 pi l_B sigma, from the surface-charge condition.
 *   [R5] Walls are the solid planes z = 0 and z = nz-1 (half-way bounce-back, at rest).
 *   [R6] Poisson: 7-point finite-volume Laplacian on fluid nodes, periodic in x and y (and z
 *        for the periodic box), zero-flux faces at the walls with the wall charge added to
 *        the first fluid layer; the right-hand side is projected to zero mean and the
 *        solution is gauged to zero mean.
 *   [R7] Ordering: with `lagged` set (the default of the GPU library), the collision at
 *        step t uses the potential solved from q(t-1); before the first step the potential
 *        is solved from q(0).
 *   [R8] Initial populations are the discrete equilibrium of the given n^alpha, u^alpha.
 *
 * Forcing variant (forcing = 1), a second-order scheme of the Guo type: every species moves
 * with v^alpha = u^alpha + F^alpha / 2 in the equilibrium and in the drag, the drag is then
 * implicit in F, F^alpha = a^alpha - omega_drag sum_b (n^b / n)(v^alpha - v^b), and the
 * forcing term is (1 - omega_visc / 2) g_p(F^alpha, v) with v the barycentric average of the
 * v^alpha.  The implicit drag is solved per node as the dense linear system it is.
 *
 * Literal variant (forcing = 2), kept only to pin reading [R3b]: the drag of Sec. II is
 * evaluated on the plain first moments u^alpha of the pre-collision populations (and their
 * barycentric average), everything else as forcing = 0.  Its uniform steady current is
 * (n^+ + n^-) E / omega_drag instead of (D / v_T^2)(n^+ + n^-) E, and its zero-flux profile
 * under a constant force a is n ~ exp(a z / (v_T^2 (1 - omega_drag / 2))) instead of the
 * Boltzmann factor exp(a z / v_T^2).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORA_Q 19
#define ORA_MAXS 8

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* D3Q19 velocities: rest, the 6 axis directions, the 12 face diagonals.  Every moving
 * direction is immediately followed by its opposite. */
static const int CV[ORA_Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Gamma_0p evaluated on D3Q19 [R1]. */
static const double WT[ORA_Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const double VT2 = 1.0 / 3.0; /* v_T^2 [R1] */

static int opposite(int p) {
    if (p == 0) return 0;
    return (p % 2 == 1) ? p + 1 : p - 1;
}

typedef struct {
    int nx, ny, nz;        /* full lattice, wall planes included for the slit */
    int slit;              /* 0: periodic box; 1: solid planes z = 0 and z = nz-1 */
    int ns;                /* number of species */
    double omega_visc;     /* relaxation frequency of the non-hydrodynamic part */
    double omega_drag;     /* drag frequency */
    int valence[ORA_MAXS]; /* z^alpha */
    double bjerrum;        /* l_B; 0 switches the Poisson solve off */
    double sigma_lo;       /* surface charge of the wall z = 0 (per lattice area, units of e) */
    double sigma_hi;       /* surface charge of the wall z = nz-1 */
    double E[3];           /* applied field, as an acceleration per unit valence */
    int poisson;           /* 0: direct spectral solve; 1: red-black SOR */
    int lagged;            /* 1: [R7]; 0: collision at t uses the potential of q(t) */
    double sor_omega;      /* over-relaxation factor */
    double sor_tol;        /* > 0: stop at ||b - A psi||_2 / ||b||_2 <= tol; 0: fixed sweeps */
    int sor_max;           /* sweep cap (fixed count when sor_tol == 0) */
    int sor_check;         /* sweeps between residual evaluations */
    int pair_drag;         /* 1: drag frequency per pair of species from drag_pair */
    double drag_pair[ORA_MAXS * ORA_MAXS]; /* omega^{ab} at [a * ORA_MAXS + b], symmetric */
    int forcing;           /* 0: g with u^alpha, drag on mid-step velocities; 1: the Guo-type variant;
                              2: drag on the plain first moments (literal reading) */
} ora_params;

typedef struct {
    ora_params p;
    long N;          /* nx*ny*nz */
    double *f, *fn;  /* [s][p][N]: pre-collision populations at the current time */
    double *psi;     /* [N]: potential used by the next collision */
    double *q;       /* [N]: charge density of the last moments */
    double *mn, *mj; /* moments work arrays [s][N], [s][3][N] */
    int psi_valid;
    long step;
    int last_sweeps;
    double last_resid;
    int last_status;
} ora_ctx;

static long nidx(const ora_ctx *c, int x, int y, int z) {
    return (long)x + (long)c->p.nx * ((long)y + (long)c->p.ny * (long)z);
}

static int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static int is_wall_plane(const ora_ctx *c, int z) {
    return c->p.slit && (z == 0 || z == c->p.nz - 1);
}

static int charged(const ora_ctx *c) {
    if (!(c->p.bjerrum > 0.0)) return 0;
    for (int s = 0; s < c->p.ns; ++s)
        if (c->p.valence[s] != 0) return 1;
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Per-node pieces, exported so that tests can check them in isolation.                  */

int ora_d3q19(int *c_out, double *w_out, int *opp_out) {
    for (int p = 0; p < ORA_Q; ++p) {
        for (int d = 0; d < 3; ++d) c_out[3 * p + d] = CV[p][d];
        w_out[p] = WT[p];
        opp_out[p] = opposite(p);
    }
    return ORA_Q;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* phi_perp_p, Appendix (last equation), written term by term as printed:
 *   n Gamma_0p { 1 + u^a.c/vT2 + [ 2(u^a.c)(u.c) - 2 vT2 u^a.u - (u.c)^2 + vT2 |u|^2
 *                                  + ((u^a - u).c)^2 - vT2 |u^a - u|^2 ] / (2 vT2^2) } */
void ora_phi_perp(double n, const double *ua, const double *u, double *out) {
    double d[3] = {ua[0] - u[0], ua[1] - u[1], ua[2] - u[2]};
    double uau = dot3(ua, u), uu = dot3(u, u), dd = dot3(d, d);
    for (int p = 0; p < ORA_Q; ++p) {
        double c[3] = {CV[p][0], CV[p][1], CV[p][2]};
        double cua = dot3(ua, c), cu = dot3(u, c), cd = dot3(d, c);
        double bracket = 2.0 * cua * cu - 2.0 * VT2 * uau - cu * cu + VT2 * uu + cd * cd - VT2 * dd;
        out[p] = n * WT[p] * (1.0 + cua / VT2 + bracket / (2.0 * VT2 * VT2));
    }
}

/* g_p, Appendix eq. (ourforc), second line:
 *   n Gamma_0p [ F.c/vT2 + ((F.c)(u.c) - vT2 F.u)/vT2^2 ]                                  */
void ora_forcing(double n, const double *F, const double *u, double *out) {
    double Fu = dot3(F, u);
    for (int p = 0; p < ORA_Q; ++p) {
        double c[3] = {CV[p][0], CV[p][1], CV[p][2]};
        double cF = dot3(F, c), cu = dot3(u, c);
        out[p] = n * WT[p] * (cF / VT2 + (cF * cu - VT2 * Fu) / (VT2 * VT2));
    }
}

/* Drag per unit mass, Sec. II:  F^a = -omega_drag sum_b (n^b / n)(u^a - u^b),
 * n = sum_b n^b [equal masses].  ua is [ns][3]; F is [ns][3]. */
void ora_drag(int ns, const double *n, const double *ua, double omega_drag, double *F) {
    double ntot = 0.0;
    for (int b = 0; b < ns; ++b) ntot += n[b];
    for (int a = 0; a < ns; ++a) {
        for (int d = 0; d < 3; ++d) {
            double acc = 0.0;
            if (ntot != 0.0)
                for (int b = 0; b < ns; ++b) acc += (n[b] / ntot) * (ua[3 * a + d] - ua[3 * b + d]);
            F[3 * a + d] = -omega_drag * acc;
        }
    }
}

/* Drag with one frequency per pair of species (Sec. II: the friction coefficient of the
 * pair (a, b), here for equal masses):  F^a = -sum_b omega^{ab} (n^b / n)(u^a - u^b).
 * omega[a * ld + b] must be symmetric for the pair forces to cancel (third law); the
 * diagonal does not contribute. */
void ora_drag_pair(int ns, const double *n, const double *ua, const double *omega, int ld, double *F) {
    double ntot = 0.0;
    for (int b = 0; b < ns; ++b) ntot += n[b];
    for (int a = 0; a < ns; ++a) {
        for (int d = 0; d < 3; ++d) {
            double acc = 0.0;
            if (ntot != 0.0)
                for (int b = 0; b < ns; ++b)
                    acc += omega[a * ld + b] * (n[b] / ntot) * (ua[3 * a + d] - ua[3 * b + d]);
            F[3 * a + d] = -acc;
        }
    }
}

/* Force of the Guo-type variant: F^a = a^a - omega sum_b (n^b / n)(v^a - v^b) with
 * v^a = u^a + F^a / 2, i.e. per Cartesian component the linear system
 *   sum_b [delta_ab + (omega / 2) M_ab] F^b = a^a - omega sum_b M_ab u^b,
 *   M_ab = delta_ab - n^b / n,
 * solved by Gaussian elimination with partial pivoting.  ua, acc, F are [ns][3]. */
void ora_guo_force(int ns, const double *n, const double *ua, const double *acc, double omega, double *F) {
    double ntot = 0.0;
    for (int b = 0; b < ns; ++b) ntot += n[b];
    for (int d = 0; d < 3; ++d) {
        double A[ORA_MAXS][ORA_MAXS + 1];
        for (int a = 0; a < ns; ++a) {
            double rhs = acc[3 * a + d];
            for (int b = 0; b < ns; ++b) {
                const double M = (a == b ? 1.0 : 0.0) - (ntot != 0.0 ? n[b] / ntot : 0.0);
                A[a][b] = (a == b ? 1.0 : 0.0) + 0.5 * omega * M;
                rhs -= omega * M * ua[3 * b + d];
            }
            A[a][ns] = rhs;
        }
        for (int k = 0; k < ns; ++k) {
            int piv = k;
            for (int r = k + 1; r < ns; ++r)
                if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
            if (piv != k)
                for (int j = 0; j <= ns; ++j) {
                    const double t = A[k][j];
                    A[k][j] = A[piv][j];
                    A[piv][j] = t;
                }
            for (int r = k + 1; r < ns; ++r) {
                const double m = A[r][k] / A[k][k];
                for (int j = k; j <= ns; ++j) A[r][j] -= m * A[k][j];
            }
        }
        for (int a = ns - 1; a >= 0; --a) {
            double v = A[a][ns];
            for (int j = a + 1; j < ns; ++j) v -= A[a][j] * F[3 * j + d];
            F[3 * a + d] = v / A[a][a];
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Poisson equation, eq. (Poisson) with the surface-charge condition [R6].               */

/* Right-hand side on the fluid nodes: b = -4 pi l_B (q + wall charge in the first layer),
 * projected to zero mean.  Wall planes get 0. */
static void poisson_rhs(const ora_ctx *c, const double *q, double *b) {
    const ora_params *P = &c->p;
    double k = 4.0 * M_PI * P->bjerrum;
    double sum = 0.0;
    long nfluid = 0;
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long i = nidx(c, x, y, z);
                if (is_wall_plane(c, z)) {
                    b[i] = 0.0;
                    continue;
                }
                double lump = 0.0;
                if (P->slit && z == 1) lump += P->sigma_lo;
                if (P->slit && z == P->nz - 2) lump += P->sigma_hi;
                b[i] = -k * (q[i] + lump);
                sum += b[i];
                nfluid++;
            }
    double mean = sum / (double)nfluid;
    for (int z = 0; z < P->nz; ++z) {
        if (is_wall_plane(c, z)) continue;
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) b[nidx(c, x, y, z)] -= mean;
    }
}

/* (A psi)(x) = sum over fluid neighbours (psi_nb - psi); in the slit, the neighbour across
 * a wall is absent (zero flux, the wall charge being in the right-hand side). */
static double apply_A(const ora_ctx *c, const double *psi, int x, int y, int z, double *nbsum, int *deg) {
    const ora_params *P = &c->p;
    static const int nb[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    double s = 0.0;
    int d = 0;
    for (int k = 0; k < 6; ++k) {
        int zz = z + nb[k][2];
        if (P->slit) {
            if (is_wall_plane(c, zz)) continue;
        } else {
            zz = wrap(zz, P->nz);
        }
        int xx = wrap(x + nb[k][0], P->nx), yy = wrap(y + nb[k][1], P->ny);
        s += psi[nidx(c, xx, yy, zz)];
        d++;
    }
    if (nbsum) *nbsum = s;
    if (deg) *deg = d;
    return s - (double)d * psi[nidx(c, x, y, z)];
}

static double fluid_mean(const ora_ctx *c, const double *a) {
    double s = 0.0;
    long n = 0;
    for (int z = 0; z < c->p.nz; ++z) {
        if (is_wall_plane(c, z)) continue;
        for (int y = 0; y < c->p.ny; ++y)
            for (int x = 0; x < c->p.nx; ++x) {
                s += a[nidx(c, x, y, z)];
                n++;
            }
    }
    return s / (double)n;
}

static void residual_norms(const ora_ctx *c, const double *b, const double *psi, double *r2, double *b2) {
    double rs = 0.0, bs = 0.0;
    for (int z = 0; z < c->p.nz; ++z) {
        if (is_wall_plane(c, z)) continue;
        for (int y = 0; y < c->p.ny; ++y)
            for (int x = 0; x < c->p.nx; ++x) {
                long i = nidx(c, x, y, z);
                double r = b[i] - apply_A(c, psi, x, y, z, NULL, NULL);
                rs += r * r;
                bs += b[i] * b[i];
            }
    }
    *r2 = rs;
    *b2 = bs;
}

/* One red-black colour: nodes with (x + y + z) mod 2 == colour, z the lattice index. */
static void sor_colour(const ora_ctx *c, const double *b, double *psi, int colour) {
    const ora_params *P = &c->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nz; ++z) {
        if (is_wall_plane(c, z)) continue;
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                if (((x + y + z) & 1) != colour) continue;
                long i = nidx(c, x, y, z);
                double s;
                int d;
                apply_A(c, psi, x, y, z, &s, &d);
                double gs = (s - b[i]) / (double)d;
                psi[i] = psi[i] + P->sor_omega * (gs - psi[i]);
            }
    }
}

/* Orthonormal eigenvectors (columns) and eigenvalues of the 1-D second difference with
 * either periodic wrap or zero-flux ends half-way between nodes.  V is n x n, V[i*n+k]. */
static void eig1d(int n, int neumann, double *V, double *lam) {
    if (neumann) {
        for (int k = 0; k < n; ++k) {
            double ck = (k == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
            lam[k] = 2.0 * cos(M_PI * k / n) - 2.0;
            for (int i = 0; i < n; ++i) V[i * n + k] = ck * cos(M_PI * k * (i + 0.5) / n);
        }
        return;
    }
    /* periodic: constant, then cos/sin pairs, then the alternating mode when n is even */
    for (int i = 0; i < n; ++i) V[i * n + 0] = sqrt(1.0 / n);
    lam[0] = 0.0;
    int col = 1;
    for (int m = 1; 2 * m < n; ++m) {
        double l = 2.0 * cos(2.0 * M_PI * m / n) - 2.0;
        for (int i = 0; i < n; ++i) {
            V[i * n + col] = sqrt(2.0 / n) * cos(2.0 * M_PI * m * i / n);
            V[i * n + col + 1] = sqrt(2.0 / n) * sin(2.0 * M_PI * m * i / n);
        }
        lam[col] = l;
        lam[col + 1] = l;
        col += 2;
    }
    if (n % 2 == 0 && n > 1) {
        for (int i = 0; i < n; ++i) V[i * n + col] = ((i % 2) ? -1.0 : 1.0) * sqrt(1.0 / n);
        lam[col] = -4.0;
    }
}

/* a[z][y][x] on the fluid grid of extents e[0..2].  Along `axis`: a <- V^T a when
 * `transpose` is set (to mode amplitudes), a <- V a otherwise (back to nodes). */
static void apply_axis(double *a, const int *e, int axis, const double *V, int transpose) {
    int n = e[axis];
    long stride = (axis == 0) ? 1 : (axis == 1) ? e[0] : (long)e[0] * e[1];
    long lines = ((long)e[0] * e[1] * e[2]) / n;
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (long l = 0; l < lines; ++l) {
            /* base index of the l-th line along `axis` */
            long base;
            if (axis == 0) base = l * e[0];
            else if (axis == 1) base = (l / e[0]) * (long)e[0] * e[1] + (l % e[0]);
            else base = l;
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) {
                    double m = transpose ? V[k * n + i] : V[i * n + k];
                    s += m * a[base + (long)k * stride];
                }
                tmp[i] = s;
            }
            for (int i = 0; i < n; ++i) a[base + (long)i * stride] = tmp[i];
        }
        free(tmp);
    }
}

/* Direct solve of A psi = b: A is diagonalised by the tensor product of the 1-D bases;
 * the zero mode is dropped, which projects b to zero mean and gauges psi to zero mean. */
static void poisson_direct(const ora_ctx *c, const double *b, double *psi) {
    const ora_params *P = &c->p;
    int z0 = P->slit ? 1 : 0;
    int e[3] = {P->nx, P->ny, P->slit ? P->nz - 2 : P->nz};
    long nf = (long)e[0] * e[1] * e[2];
    double *a = (double *)malloc(sizeof(double) * nf);
    double *V[3], *L[3];
    for (int ax = 0; ax < 3; ++ax) {
        V[ax] = (double *)malloc(sizeof(double) * e[ax] * e[ax]);
        L[ax] = (double *)malloc(sizeof(double) * e[ax]);
        eig1d(e[ax], (ax == 2) && P->slit, V[ax], L[ax]);
    }
    for (int z = 0; z < e[2]; ++z)
        for (int y = 0; y < e[1]; ++y)
            for (int x = 0; x < e[0]; ++x)
                a[x + (long)e[0] * (y + (long)e[1] * z)] = b[nidx(c, x, y, z + z0)];
    for (int ax = 0; ax < 3; ++ax) apply_axis(a, e, ax, V[ax], 1);
    for (int z = 0; z < e[2]; ++z)
        for (int y = 0; y < e[1]; ++y)
            for (int x = 0; x < e[0]; ++x) {
                long i = x + (long)e[0] * (y + (long)e[1] * z);
                double lam = L[0][x] + L[1][y] + L[2][z];
                a[i] = (x == 0 && y == 0 && z == 0) ? 0.0 : a[i] / lam;
            }
    for (int ax = 0; ax < 3; ++ax) apply_axis(a, e, ax, V[ax], 0);
    for (long i = 0; i < c->N; ++i) psi[i] = 0.0;
    for (int z = 0; z < e[2]; ++z)
        for (int y = 0; y < e[1]; ++y)
            for (int x = 0; x < e[0]; ++x)
                psi[nidx(c, x, y, z + z0)] = a[x + (long)e[0] * (y + (long)e[1] * z)];
    for (int ax = 0; ax < 3; ++ax) {
        free(V[ax]);
        free(L[ax]);
    }
    free(a);
}

/* Red-black SOR from the current psi (warm start).  Returns 0, or -5 when the sweep cap
 * was reached before the tolerance.  Afterwards psi is gauged to zero mean. */
static int poisson_sor(ora_ctx *c, const double *b, double *psi) {
    const ora_params *P = &c->p;
    double r2, b2;
    int status = 0, sweeps = 0;
    residual_norms(c, b, psi, &r2, &b2);
    if (b2 == 0.0) {
        for (long i = 0; i < c->N; ++i) psi[i] = 0.0;
        c->last_sweeps = 0;
        c->last_resid = 0.0;
        return 0;
    }
    if (P->sor_tol > 0.0) {
        for (;;) {
            if (sqrt(r2 / b2) <= P->sor_tol) break;
            if (sweeps >= P->sor_max) {
                status = -5;
                break;
            }
            int todo = P->sor_check;
            if (todo > P->sor_max - sweeps) todo = P->sor_max - sweeps;
            for (int s = 0; s < todo; ++s) {
                sor_colour(c, b, psi, 0);
                sor_colour(c, b, psi, 1);
            }
            sweeps += todo;
            residual_norms(c, b, psi, &r2, &b2);
        }
    } else {
        for (int s = 0; s < P->sor_max; ++s) {
            sor_colour(c, b, psi, 0);
            sor_colour(c, b, psi, 1);
        }
        sweeps = P->sor_max;
        residual_norms(c, b, psi, &r2, &b2);
    }
    double m = fluid_mean(c, psi);
    for (int z = 0; z < P->nz; ++z) {
        if (is_wall_plane(c, z)) continue;
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) psi[nidx(c, x, y, z)] -= m;
    }
    c->last_sweeps = sweeps;
    c->last_resid = sqrt(r2 / b2);
    return status;
}

static int solve_potential(ora_ctx *c, const double *q) {
    double *b = (double *)malloc(sizeof(double) * c->N);
    poisson_rhs(c, q, b);
    int st = 0;
    if (c->p.poisson == 0) {
        poisson_direct(c, b, c->psi);
        double r2, b2;
        residual_norms(c, b, c->psi, &r2, &b2);
        c->last_sweeps = 0;
        c->last_resid = (b2 > 0.0) ? sqrt(r2 / b2) : 0.0;
    } else {
        st = poisson_sor(c, b, c->psi);
    }
    free(b);
    c->psi_valid = 1;
    c->last_status = st;
    return st;
}

/* ------------------------------------------------------------------------------------ */
/* Lattice object.                                                                       */

ora_ctx *ora_create(const ora_params *p) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->ns < 1 || p->ns > ORA_MAXS) return NULL;
    if (p->slit && p->nz < 3) return NULL;
    if (p->forcing < 0 || p->forcing > 2) return NULL;
    if (p->forcing != 0 && p->pair_drag) return NULL;
    ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
    c->p = *p;
    c->N = (long)p->nx * p->ny * p->nz;
    size_t nf = (size_t)p->ns * ORA_Q * c->N;
    c->f = (double *)calloc(nf, sizeof(double));
    c->fn = (double *)calloc(nf, sizeof(double));
    c->psi = (double *)calloc(c->N, sizeof(double));
    c->q = (double *)calloc(c->N, sizeof(double));
    c->mn = (double *)calloc((size_t)p->ns * c->N, sizeof(double));
    c->mj = (double *)calloc((size_t)p->ns * 3 * c->N, sizeof(double));
    if (!c->f || !c->fn || !c->psi || !c->q || !c->mn || !c->mj) {
        free(c->f); free(c->fn); free(c->psi); free(c->q); free(c->mn); free(c->mj);
        free(c);
        return NULL;
    }
    return c;
}

void ora_destroy(ora_ctx *c) {
    if (!c) return;
    free(c->f); free(c->fn); free(c->psi); free(c->q); free(c->mn); free(c->mj);
    free(c);
}

/* Equilibrium initial state [R8] of species s from n[N] and u[3][N] (u may be NULL). */
int ora_set_state(ora_ctx *c, int s, const double *n, const double *u) {
    if (s < 0 || s >= c->p.ns) return -1;
    double feq[ORA_Q];
    for (long i = 0; i < c->N; ++i) {
        int z = (int)(i / ((long)c->p.nx * c->p.ny));
        double ua[3] = {0.0, 0.0, 0.0};
        if (u) {
            ua[0] = u[i];
            ua[1] = u[c->N + i];
            ua[2] = u[2 * c->N + i];
        }
        if (is_wall_plane(c, z)) {
            for (int p = 0; p < ORA_Q; ++p) c->f[((long)s * ORA_Q + p) * c->N + i] = 0.0;
            continue;
        }
        ora_phi_perp(n[i], ua, ua, feq);
        for (int p = 0; p < ORA_Q; ++p) c->f[((long)s * ORA_Q + p) * c->N + i] = feq[p];
    }
    c->psi_valid = 0;
    c->step = 0;
    return 0;
}

/* Raw access to the pre-collision populations [p][N] of species s. */
int ora_set_f(ora_ctx *c, int s, const double *f) {
    if (s < 0 || s >= c->p.ns) return -1;
    memcpy(c->f + (size_t)s * ORA_Q * c->N, f, sizeof(double) * ORA_Q * c->N);
    c->psi_valid = 0;
    c->step = 0;
    return 0;
}

int ora_get_f(const ora_ctx *c, int s, double *f) {
    if (s < 0 || s >= c->p.ns) return -1;
    memcpy(f, c->f + (size_t)s * ORA_Q * c->N, sizeof(double) * ORA_Q * c->N);
    return 0;
}

/* Moments of Sec. III at every fluid node: n^a = sum_p f_p, j^a = sum_p f_p c_p. */
static void compute_moments(ora_ctx *c) {
    const ora_params *P = &c->p;
    long N = c->N;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        int z = (int)(i / ((long)P->nx * P->ny));
        double qq = 0.0;
        for (int s = 0; s < P->ns; ++s) {
            double n = 0.0, j[3] = {0.0, 0.0, 0.0};
            if (!is_wall_plane(c, z)) {
                for (int p = 0; p < ORA_Q; ++p) {
                    double f = c->f[((long)s * ORA_Q + p) * N + i];
                    n += f;
                    for (int d = 0; d < 3; ++d) j[d] += f * CV[p][d];
                }
            }
            c->mn[(long)s * N + i] = n;
            for (int d = 0; d < 3; ++d) c->mj[((long)s * 3 + d) * N + i] = j[d];
            qq += P->valence[s] * n;
        }
        c->q[i] = qq;
    }
}

int ora_moments(ora_ctx *c, int s, double *n_out, double *j_out) {
    if (s < 0 || s >= c->p.ns) return -1;
    compute_moments(c);
    if (n_out) memcpy(n_out, c->mn + (size_t)s * c->N, sizeof(double) * c->N);
    if (j_out) memcpy(j_out, c->mj + (size_t)s * 3 * c->N, sizeof(double) * 3 * c->N);
    return 0;
}

/* FP64 totals sum_x n^s(x), in a fixed order. */
int ora_mass_totals(ora_ctx *c, double *out) {
    compute_moments(c);
    for (int s = 0; s < c->p.ns; ++s) {
        double t = 0.0;
        for (long i = 0; i < c->N; ++i) t += c->mn[(long)s * c->N + i];
        out[s] = t;
    }
    return 0;
}

/* grad psi~ at a fluid node [R4]. */
static void grad_psi(const ora_ctx *c, int x, int y, int z, double *g) {
    const ora_params *P = &c->p;
    const double *psi = c->psi;
    double k = 4.0 * M_PI * P->bjerrum;
    g[0] = 0.5 * (psi[nidx(c, wrap(x + 1, P->nx), y, z)] - psi[nidx(c, wrap(x - 1, P->nx), y, z)]);
    g[1] = 0.5 * (psi[nidx(c, x, wrap(y + 1, P->ny), z)] - psi[nidx(c, x, wrap(y - 1, P->ny), z)]);
    double up, dn;
    if (P->slit) {
        double here = psi[nidx(c, x, y, z)];
        up = (z + 1 == P->nz - 1) ? here + k * P->sigma_hi : psi[nidx(c, x, y, z + 1)];
        dn = (z - 1 == 0) ? here + k * P->sigma_lo : psi[nidx(c, x, y, z - 1)];
    } else {
        up = psi[nidx(c, x, y, wrap(z + 1, P->nz))];
        dn = psi[nidx(c, x, y, wrap(z - 1, P->nz))];
    }
    g[2] = 0.5 * (up - dn);
}

/* One time step of eq. (latboeq): collide at every fluid node, push to r + c_p. */
static int one_step(ora_ctx *c) {
    const ora_params *P = &c->p;
    const long N = c->N;
    const int ns = P->ns;
    const int elec = charged(c);
    int status = 0;

    compute_moments(c); /* n^a(t), j^a(t), q(t) */
    if (elec) {
        if (!P->lagged || !c->psi_valid) status = solve_potential(c, c->q);
    } else {
        for (long i = 0; i < N; ++i) c->psi[i] = 0.0;
    }

#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        int x = (int)(i % P->nx);
        int y = (int)((i / P->nx) % P->ny);
        int z = (int)(i / ((long)P->nx * P->ny));
        if (is_wall_plane(c, z)) continue;
        double n[ORA_MAXS], ua[3 * ORA_MAXS], F[3 * ORA_MAXS];
        double ntot = 0.0, u[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < ns; ++s) {
            n[s] = c->mn[(long)s * N + i];
            for (int d = 0; d < 3; ++d)
                ua[3 * s + d] = (n[s] != 0.0) ? c->mj[((long)s * 3 + d) * N + i] / n[s] : 0.0;
            ntot += n[s];
        }
        /* barycentric velocity, sum_a rho^a u^a / rho with equal masses */
        if (ntot != 0.0)
            for (int d = 0; d < 3; ++d) {
                double acc = 0.0;
                for (int s = 0; s < ns; ++s) acc += n[s] * ua[3 * s + d];
                u[d] = acc / ntot;
            }
        /* field acceleration a^a = z^a (E - vT2 grad psi~) [R3] */
        double gp[3] = {0.0, 0.0, 0.0}, acc[3 * ORA_MAXS], umid[3 * ORA_MAXS];
        if (elec) grad_psi(c, x, y, z, gp);
        for (int s = 0; s < ns; ++s)
            for (int d = 0; d < 3; ++d) {
                acc[3 * s + d] = P->valence[s] * (P->E[d] - VT2 * gp[d]);
                umid[3 * s + d] = ua[3 * s + d] + 0.5 * acc[3 * s + d];
            }
        double gscale = 1.0;
        if (P->forcing == 1) {
            /* Guo-type variant: solve F = a - omega (I - 1 w^T)(u + F/2) per component, w_b =
             * n^b / n, then move every species (and the barycentric velocity) half a force
             * step */
            ora_guo_force(ns, n, ua, acc, P->omega_drag, F);
            for (int s = 0; s < ns; ++s)
                for (int d = 0; d < 3; ++d) ua[3 * s + d] += 0.5 * F[3 * s + d];
            for (int d = 0; d < 3; ++d) {
                double sum = 0.0;
                for (int s = 0; s < ns; ++s) sum += n[s] * ua[3 * s + d];
                u[d] = ntot != 0.0 ? sum / ntot : 0.0;
            }
            gscale = 1.0 - 0.5 * P->omega_visc;
        } else {
            /* drag on the mid-step velocities [R3b] (forcing = 2: on the plain first
             * moments), then the total force */
            if (P->pair_drag)
                ora_drag_pair(ns, n, umid, P->drag_pair, ORA_MAXS, F);
            else
                ora_drag(ns, n, P->forcing == 2 ? ua : umid, P->omega_drag, F);
            for (int s = 0; s < ns; ++s)
                for (int d = 0; d < 3; ++d) F[3 * s + d] += acc[3 * s + d];
        }

        for (int s = 0; s < ns; ++s) {
            double phi[ORA_Q], g[ORA_Q];
            ora_phi_perp(n[s], &ua[3 * s], u, phi);
            ora_forcing(n[s], &F[3 * s], u, g);
            for (int p = 0; p < ORA_Q; ++p) {
                double f = c->f[((long)s * ORA_Q + p) * N + i];
                double post = f - P->omega_visc * (f - phi[p]) + gscale * g[p];
                int xd = wrap(x + CV[p][0], P->nx), yd = wrap(y + CV[p][1], P->ny), zd = z + CV[p][2];
                if (P->slit && is_wall_plane(c, zd)) {
                    /* half-way bounce-back: returns to the same node, reversed [R5] */
                    c->fn[((long)s * ORA_Q + opposite(p)) * N + i] = post;
                } else {
                    if (!P->slit) zd = wrap(zd, P->nz);
                    c->fn[((long)s * ORA_Q + p) * N + nidx(c, xd, yd, zd)] = post;
                }
            }
        }
    }
    double *t = c->f;
    c->f = c->fn;
    c->fn = t;

    if (elec && P->lagged) {
        int st = solve_potential(c, c->q); /* q(t), used by step t+1 */
        if (st) status = st;
    }
    c->step++;
    return status;
}

int ora_step(ora_ctx *c, int nsteps) {
    int status = 0;
    for (int k = 0; k < nsteps; ++k) {
        int st = one_step(c);
        if (st) status = st;
    }
    return status;
}

/* Potential the next collision will use (solved from the current state when not yet
 * available), and charge density of the current state. */
int ora_get_psi(ora_ctx *c, double *out) {
    if (charged(c) && !c->psi_valid) {
        compute_moments(c);
        solve_potential(c, c->q);
    }
    memcpy(out, c->psi, sizeof(double) * c->N);
    return 0;
}

int ora_get_q(ora_ctx *c, double *out) {
    compute_moments(c);
    memcpy(out, c->q, sizeof(double) * c->N);
    return 0;
}

/* Stand-alone Poisson solve of the charge q (wall planes ignored) with this lattice's
 * parameters; psi is the warm start for SOR and receives the solution. */
int ora_poisson(ora_ctx *c, const double *q, double *psi, int *sweeps, double *resid) {
    memcpy(c->psi, psi, sizeof(double) * c->N);
    int st = solve_potential(c, q);
    memcpy(psi, c->psi, sizeof(double) * c->N);
    if (sweeps) *sweeps = c->last_sweeps;
    if (resid) *resid = c->last_resid;
    c->psi_valid = 0;
    return st;
}

int ora_stats(const ora_ctx *c, long *step, int *sweeps, double *resid) {
    if (step) *step = c->step;
    if (sweeps) *sweeps = c->last_sweeps;
    if (resid) *resid = c->last_resid;
    return c->last_status;
}
