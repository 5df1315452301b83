/*
 * lbmix.h -- C ABI of the MI355X (gfx950) multicomponent lattice-Boltzmann library.
 *
 * The library advances a mixture of NS species on a D3Q19 lattice with the modified BGK
 * update of Monteferrante, Melchionna and Marini Bettolo Marconi, "Lattice Boltzmann Method
 * for mixtures at variable Schmidt number" (arXiv:1507.04891):
 *
 *   f_p(r + c_p, t + 1) = f_p - omega_visc (f_p - phi_perp_p) + g_p          (Sec. IV, eq. latboeq)
 *
 * phi_perp_p is the orthogonalised equilibrium (last equation of the Appendix), g_p the
 * second-order forcing term (Appendix, eq. ourforc) of the total force on the species: the
 * interspecies drag (Sec. II, F^{alpha,drag}) plus, for charged species, the electrostatic
 * force of the potential that solves the Poisson equation (Sec. II, eq. Poisson) with
 * charged walls (the surface-charge condition that follows it) and an applied field.
 *
 * Conventions (all of them shared with the documentation of every call below):
 *   - lattice units: unit spacing and time step, equal masses m = 1, charge unit e = 1,
 *     k_B T / m = v_T^2 = 1/3;
 *   - node index i = x + nx * (y + ny * z), x fastest; host arrays cover all nz planes,
 *     vector fields are planar [3][nz][ny][nx], populations [19][nz][ny][nx];
 *   - geometry LBMIX_PERIODIC: periodic in x, y, z;  LBMIX_SLIT_Z: periodic in x and y,
 *     the planes z = 0 and z = nz-1 are solid walls at rest (half-way bounce-back, wall
 *     surfaces at z = 1/2 and z = nz - 3/2); LBMIX_CHANNELS: independent slit channels of
 *     their own widths stacked along z (lbmix_create_channels), each with its two wall
 *     planes; wall-plane entries of host arrays are ignored on input and written as 0 on
 *     output;
 *   - D3Q19 order: p = 0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 = (+1,+1,0), (-1,-1,0),
 *     (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1), (-1,0,+1), (0,+1,+1),
 *     (0,-1,-1), (0,+1,-1), (0,-1,+1); weights 1/3, 1/18, 1/36;
 *   - "time t" is the number of completed steps; moments read back are those of the
 *     pre-collision populations at time t;
 *   - readings of the paper applied here: the drag acts on the mid-step species velocities
 *     u^alpha + a^alpha / 2, where a^alpha = z^alpha (E_ext - v_T^2 grad psi~) is the field
 *     acceleration (lbmix_set_forcing selects a Guo-type alternative); grad psi~ by central
 *     differences, ghost value psi~ + 4 pi l_B sigma across a wall; the collision at step t
 *     uses the potential solved from the charge density of step t-1 (before the first step:
 *     of step 0).
 *
 * Status codes: every call returns LBMIX_OK (0) or a negative code; no C++ exception
 * crosses the ABI.  lbmix_last_error() returns a text for the last failure of a context.
 * A context is not thread-safe; distinct contexts are independent.  Device work is issued
 * on the context's HIP stream; calls that return host data synchronise that stream.
 */
#ifndef LBMIX_H
#define LBMIX_H

#ifdef __cplusplus
extern "C" {
#endif

#define LBMIX_Q 19
#define LBMIX_MAX_SPECIES 4

enum lbmix_status {
    LBMIX_OK = 0,
    LBMIX_EINVAL = -1,     /* bad argument; nothing changed */
    LBMIX_ENOMEM = -2,     /* device or host allocation failed */
    LBMIX_EDEVICE = -3,    /* HIP runtime error (no GPU, launch failure, fault) */
    LBMIX_ESTATE = -4,     /* call not allowed in the context's current state */
    LBMIX_ENOCONV = -5,    /* Poisson solve hit its sweep cap before the tolerance */
    LBMIX_ENONFINITE = -6  /* a mass total is NaN or Inf; latched until set_state / load */
};

enum lbmix_geometry { LBMIX_PERIODIC = 0, LBMIX_SLIT_Z = 1, LBMIX_CHANNELS = 2 };

/* Forcing schemes (lbmix_set_forcing). */
enum lbmix_forcing { LBMIX_FORCING_PAPER = 0, LBMIX_FORCING_GUO = 1 };

/* Population storage.  F64 and F32 store f.  The SHIFTED forms store the deviation
 * f_p - w_p rho0 (rho0 = the species' rest density given to lbmix_add_species), in FP32,
 * or in BF16 / FP16 times a power-of-two scale per species and direction; the collision
 * arithmetic is FP64 for F64 and FP32 for all other forms, except that the FP32 forms with
 * stochastic rounding (lbmix_set_rounding) collide in FP64.  Mass totals and the Poisson
 * solve are FP64 in every form. */
enum lbmix_storage {
    LBMIX_F64 = 0,
    LBMIX_F32 = 1,
    LBMIX_F32_SHIFTED = 2,
    LBMIX_BF16_SHIFTED = 3,
    LBMIX_F16_SHIFTED = 4
};

typedef struct lbmix_ctx lbmix_ctx;
typedef struct lbmix_net lbmix_net;

typedef struct {
    long long steps;          /* completed time steps */
    long long poisson_solves; /* Poisson solves so far */
    long long total_sweeps;   /* red-black sweeps so far */
    int last_sweeps;          /* sweeps of the last solve */
    int last_status;          /* LBMIX_OK or LBMIX_ENOCONV for the last solve */
    double last_residual;     /* ||b - A psi||_2 / ||b||_2 after the last solve */
    double fluid_nodes;       /* nx * ny * (nz, or nz - 2 for a slit) */
    double bytes_per_step;    /* algorithmic HBM bytes of one stream-collide launch */
    int block_x, block_y;     /* work-group shape of the stream-collide launch */
} lbmix_stats;

/* Library version, major * 10000 + minor * 100 + patch. */
int lbmix_version(void);

/* Create a lattice of nx * ny * nz nodes (wall planes included for LBMIX_SLIT_Z, which
 * needs nz >= 3).  `storage` is an lbmix_storage.  `hip_stream` is the hipStream_t to issue
 * all device work on (borrowed, never destroyed); NULL is the HIP null stream.
 * No device memory is allocated until the first lbmix_set_state.  Defaults: tau_visc = 1,
 * Schmidt number 1 (tau_drag = tau_visc), no charge, Poisson tolerance 1e-8.
 * Errors: EINVAL for non-positive extents, nz < 3 for a slit, an unknown geometry or
 * storage, a lattice of more than 2^31 - 1 nodes, or a plane of 2^32 / (19 x 4 x element
 * bytes) nodes or more (nx * ny >= 7.06 M for F64, 14.1 M for FP32, 28.3 M for the 16-bit
 * forms: the fused step addresses the 19 populations of a plane with 32-bit offsets). */
int lbmix_create(lbmix_ctx **out, int nx, int ny, int nz, int geometry, int storage,
                 void *hip_stream);

/* Create a stack of `nchannels` slit channels (the charged slit of Sec. IV, many at once):
 * each channel c has nx * ny lateral nodes (periodic), widths[c] >= 1 fluid planes and its
 * own two wall planes, so host arrays cover nz = sum_c (widths[c] + 2) planes, channel c
 * from plane sum_{c' < c} (widths[c'] + 2) (its lower wall) upwards.  Channels share the
 * species, tau_visc, the Bjerrum length, the field and the storage; each has its own drag
 * and wall charges (lbmix_set_channel) and is neutral and gauged on its own.  One fused
 * launch steps all channels; the Poisson solve is any of the three (multigrid in its channel form,
 * see lbmix_set_poisson_method).
 * Errors: as lbmix_create; EINVAL for nchannels < 1 or a width < 1. */
int lbmix_create_channels(lbmix_ctx **out, int nx, int ny, int nchannels, const int *widths,
                          int storage, void *hip_stream);

/* Parameters of channel `channel` of a stack: tau_drag > 1/2 (<= 0: the context's drag, from
 * lbmix_set_tau_drag or lbmix_set_schmidt), and the surface charges of its lower and upper
 * walls in units of e per lattice area.  Defaults: the context's drag, uncharged walls.
 * Errors: EINVAL for a context not made by lbmix_create_channels, a bad index or tau_drag
 * in (0, 1/2]; ESTATE after the first step. */
int lbmix_set_channel(lbmix_ctx *ctx, int channel, double tau_drag, double sigma_lo,
                      double sigma_hi);

/* Add a species with rest density rho0 > 0 (the storage shift of the SHIFTED forms and
 * the reference density of the FP16 scale) and integer valence z^alpha (Sec. II; the
 * ternary electrolyte of Sec. III has z = 0, +1, -1).  Writes its index to *id_out.
 * Errors: ESTATE after the first set_state; EINVAL beyond LBMIX_MAX_SPECIES or rho0 <= 0. */
int lbmix_add_species(lbmix_ctx *ctx, double rho0, int valence, int *id_out);

/* omega_visc = 1 / tau_visc; kinematic viscosity nu = v_T^2 (tau_visc - 1/2) (Sec. IV).
 * Errors: EINVAL unless tau_visc > 1/2; ESTATE after the first step. */
int lbmix_set_tau_visc(lbmix_ctx *ctx, double tau_visc);

/* omega_drag = 1 / tau_drag; mutual diffusivity D = v_T^2 (tau_drag - 1/2) (Sec. IV).
 * Overrides a Schmidt number set before.  Errors: EINVAL unless tau_drag > 1/2; ESTATE
 * after the first step. */
int lbmix_set_tau_drag(lbmix_ctx *ctx, double tau_drag);

/* Schmidt number Sc = nu / D: tau_drag = 1/2 + (tau_visc - 1/2) / Sc (with the Guo-type
 * forcing variant, where D = v_T^2 tau_drag: tau_drag = (tau_visc - 1/2) / Sc), evaluated at
 * the first step.  Errors: EINVAL unless Sc > 0 (lbmix_step: for the Guo-type variant unless
 * tau_visc > 1/2 + Sc / 2, which keeps tau_drag > 1/2); ESTATE after the first step. */
int lbmix_set_schmidt(lbmix_ctx *ctx, double sc);

/* enable != 0: replay each step as a captured HIP graph (the fused step, the direct Poisson
 * solve and the step count from which the stochastic-rounding seed is derived, captured
 * once per buffer parity) when a step needs no host decision: no Poisson solve, or the
 * direct one.  Other steps run as before.  Results are bitwise those of uncaptured steps;
 * the stats residual is then evaluated once per lbmix_step call.  Default 0.  Errors:
 * EINVAL for a null context. */
int lbmix_set_step_graph(lbmix_ctx *ctx, int enable);

/* Time `reps` launches of the fused stream-collide step for each candidate work-group shape
 * (64 to 512 threads: rows of 64, 128, 256 or, in planes at least 512 nodes wide, 512 nodes
 * times 1 to 8 rows; for planes narrower than 64 nodes, whole rows filling 64 to 512 threads)
 * on the current state, twice, and keep the fastest for the following steps if it beats the
 * default shape by more than 1.5 % (lbmix_stats reports the shape in use).  The default
 * shape: rows of up to 256 nodes, two per work-group; one row for one or two 16-bit species
 * and for FP32 with stochastic rounding; 128 threads for three 16-bit species; in planes
 * wider than 256 nodes, rows of the width that leaves the fewest idle lanes.  The state does not advance:
 * the launches write the buffer the next step overwrites.  Results do not depend on the
 * shape.  Call after lbmix_set_state.  Errors: ESTATE without a state; EINVAL for reps < 1. */
int lbmix_autotune(lbmix_ctx *ctx, int reps);

/* Drag with one relaxation time per pair of species (Sec. II: the friction gamma^{ab} of the
 * pair, here for equal masses and any molecular diameters), replacing the single omega_drag:
 *   F^a / m = -sum_b omega^{ab} (n^b / n)(u^a - u^b),  omega^{ab} = 1 / tau[a * ns + b],
 * on the mid-step velocities like the single-frequency drag.  tau is ns x ns row-major with
 * ns the number of species added so far (add every species first); it must be symmetric
 * (to 1e-12 relative: the pair forces then cancel) with off-diagonal entries > 1/2; the
 * diagonal is ignored.  A binary's single pair gives D = v_T^2 (tau^{01} - 1/2).  NULL goes
 * back to the single drag frequency.  A channel stack with a pair matrix takes no per-channel
 * drag.  Errors: EINVAL for fewer than two species, an asymmetric matrix or an entry <= 1/2
 * (lbmix_step: for a species count that changed since, or per-channel drags); ESTATE after
 * the first step. */
int lbmix_set_drag_pairs(lbmix_ctx *ctx, const double *tau_pairs);

/* Forcing scheme of the collision.
 *   LBMIX_FORCING_PAPER (default): the equilibrium phi_perp at the species velocity u^a and
 *     the forcing term g_p of the Appendix (eq. ourforc), with the drag of Sec. II taken on
 *     the mid-step velocities u^a + a^a / 2 (a^a the field acceleration).
 *   LBMIX_FORCING_GUO: a second-order scheme of the Guo type.  Every species moves with
 *     v^a = u^a + F^a / 2 in the equilibrium and in the drag, so the drag is implicit,
 *     F^a = a^a - omega_drag sum_b (n^b / n)(v^a - v^b); it is solved in closed form per
 *     node.  The forcing term is (1 - omega_visc / 2) g_p(F^a, v), v the barycentric mean of
 *     the v^a.  The velocity difference then relaxes by (1 - omega/2) / (1 + omega/2) per
 *     step, which gives D = v_T^2 tau_drag (the continuum expression, instead of
 *     v_T^2 (tau_drag - 1/2)) and an electric mobility tau_drag; the viscosity is unchanged.
 *     D >= v_T^2 / 2 here, so high Schmidt numbers need large viscosities.
 * Errors: EINVAL for an unknown scheme (lbmix_step: for the Guo variant with a pair drag
 * matrix of three or more species); ESTATE after the first step. */
int lbmix_set_forcing(lbmix_ctx *ctx, int scheme);

/* Electrostatics (Sec. II, eq. Poisson and its surface-charge condition): Bjerrum length
 * l_B >= 0 (0: no Poisson solve), surface charges of the walls z = 0 and z = nz-1 in units
 * of e per lattice area (used by LBMIX_SLIT_Z only; channels take theirs from
 * lbmix_set_channel), and the applied field E_ext[3] as an acceleration per unit valence
 * (may be NULL for zero).  A charged run (l_B > 0 and a species with z != 0) needs nx and
 * ny even or 1 (nz too for a periodic box) for the red-black ordering of SOR and multigrid,
 * and neutral channels: |sum z rho0 N + (sigma_lo + sigma_hi) nx ny| of each channel (the
 * whole lattice for the box) must be small against the charge carried by its species
 * (checked at the first step).
 * Errors: EINVAL for l_B < 0; ESTATE after the first step. */
int lbmix_set_electrostatics(lbmix_ctx *ctx, double bjerrum, double sigma_lo,
                             double sigma_hi, const double *E_ext);

/* Poisson solver: red-black SOR (colour (x + y + z) mod 2, colour 0 first), warm-started
 * from the previous potential.  rel_tol > 0: sweep until ||b - A psi||_2 / ||b||_2 <=
 * rel_tol, checking every check_every sweeps, and report ENOCONV from lbmix_step when
 * max_sweeps is reached first; rel_tol == 0: exactly max_sweeps sweeps per solve, never
 * ENOCONV.  omega_sor in (0, 2), or <= 0 for 2 / (1 + sin(pi / L)), L the largest fluid
 * extent.  After each solve psi is shifted to zero mean over the fluid of each channel.
 * The right-hand side b = -4 pi l_B (q + wall charge lumped into the first and last fluid
 * planes) is projected onto zero mean per channel.  Errors: EINVAL
 * for rel_tol < 0, max_sweeps < 1, check_every < 1 or omega_sor >= 2. */
int lbmix_set_poisson(lbmix_ctx *ctx, double rel_tol, int max_sweeps, int check_every,
                      double omega_sor);

/* Poisson solver method: 0 red-black SOR (default); 1 geometric multigrid: cell-centred
 * V-cycles of red-black Gauss-Seidel (one sweep before and after the correction on the
 * finest level, two on coarser ones) over a hierarchy that halves each axis while the
 * colouring stays consistent (coefficients 1 / H^2 per axis, cell-average restriction,
 * linear interpolation; the levels of at most 2048 cells are cycled by one work-group in
 * LDS, the coarsest of at most 64 cells solved exactly), each cycle and its residual replayed
 * as one captured HIP graph.  With multigrid, max_sweeps of
 * lbmix_set_poisson caps (or, with rel_tol == 0, fixes) the number of V-cycles per solve and
 * lbmix_stats counts cycles in place of sweeps.  2 direct: the operator of eq. `Poisson` is
 * diagonalised along x and y by orthonormal real Fourier bases (planes of up to 64 x 64
 * nodes one at a time on the FP64 matrix cores; larger ones by fast Fourier transforms when
 * both extents are powers of two up to 1024, else by batched FP64 products) and solved
 * exactly along z, by a tridiagonal elimination per (x, y) mode and channel in a slit or
 * stack (from both ends towards the middle plane), by a third Fourier basis in a periodic
 * box (fast transforms for more than 64 planes of a power-of-two count); its result is exact to rounding, takes any extents and
 * needs no warm start (rel_tol and max_sweeps do not apply; lbmix_stats counts one sweep
 * per solve and reports the residual of every check_every-th solve).  On a stack of channels
 * (lbmix_create_channels), whose widths are arbitrary, multigrid keeps every plane on every
 * level and halves x and y only, relaxing whole z lines instead of points: a red-black sweep
 * over the columns (colour (x + y) mod 2) solves the tridiagonal z-system of each column in
 * each channel exactly, its lateral neighbours held fixed; V(1,1) cycles down to one column
 * per channel, where the line solve is the exact coarse solve.  SOR and multigrid need even
 * periodic extents (or 1).  Errors: EINVAL for another method, or SOR or multigrid on odd
 * extents once stepping has started (checked by lbmix_step before). */
int lbmix_set_poisson_method(lbmix_ctx *ctx, int method);

/* Warm start of each Poisson solve: 0 the previous potential (default); 1 the
 * extrapolation psi(t-1) + psi(t-2) - psi(t-3), exact for a potential that changes linearly
 * in time plus an oscillation of period two steps (the interdiffusion flux relaxes with the
 * factor 1 - omega_drag per step, which is close to -1 at large Schmidt number).  A plain
 * linear extrapolation 2 psi(t-1) - psi(t-2) triples that oscillation instead.  2 learned:
 * the extrapolation, then psi += alpha s net(r / s, c / s, dpsi_1 / s, dpsi_2 / s, wall mask)
 * with r = b - A psi the residual of the extrapolated guess, s its root mean square, c the
 * coarse-grid solution of A c = r (r restricted down the multigrid hierarchy, the coarse end
 * solved as in a V-cycle, interpolated back without smoothing: the global part of A^-1 r that
 * a few 3 x 3 x 3 layers cannot reach), dpsi_1 = psi(t-1) - psi(t-2), dpsi_2 = psi(t-2) -
 * psi(t-3) and alpha the network's output scale (the network of lbmix_set_warm_start_net;
 * applied once three previous solutions exist).  Applies to SOR and multigrid; the direct
 * solve needs none.
 * Errors: EINVAL for another mode, or 2 without a network. */
int lbmix_set_poisson_warm_start(lbmix_ctx *ctx, int mode);

/* ---- learned warm start ---------------------------------------------------------------
 * A fully convolutional network: `layers` 3 x 3 x 3 convolutions (periodic in x and y; in z
 * periodic, or zero beyond the end planes for a slit), in_channels -> hidden -> ... -> hidden
 * -> 1 channels, bias and ReLU on every layer but the last; FP32 master parameters
 * [layer][cout][cin][27] then [cout], tap k = (dz + 1) 9 + (dy + 1) 3 + (dx + 1).  Every
 * convolution (forward, transposed and weight gradient) rounds its weights and inputs to BF16
 * (nearest-even) and accumulates in FP32 (the layers of 16 or more channel pairs on the BF16
 * matrix cores); Adam updates the FP32 parameters.  It lives on the device current at
 * creation.  The warm start uses in_channels = 5 (scaled residual, its scaled coarse-grid
 * solution, the two last scaled increments of the potential, wall mask). */

/* Create a network, weights uniform in +-sqrt(6 / fan_in) (+-1 / sqrt(fan_in) for the last
 * layer) from a splitmix64 stream of `seed`, biases 0.  Errors: EINVAL for channels outside
 * 1..16 or layers outside 1..16; ENOMEM; EDEVICE. */
int lbmix_net_create(lbmix_net **out, int in_channels, int hidden, int layers, unsigned long long seed);
/* Number of FP32 parameters, or EINVAL for a null network. */
int lbmix_net_num_params(const lbmix_net *net);
/* Copy the parameters out / in (host arrays of lbmix_net_num_params floats); setting them
 * resets the Adam moments.  Errors: EINVAL for null pointers or a non-finite parameter. */
int lbmix_net_get_params(lbmix_net *net, float *params);
int lbmix_net_set_params(lbmix_net *net, const float *params);
/* Gradient of the last lbmix_net_gradient call (host array of lbmix_net_num_params floats). */
int lbmix_net_get_gradient(lbmix_net *net, float *grad);
/* y_dev[nz][ny][nx] = net(x_dev[in_channels][nz][ny][nx]) on the hipStream_t `stream` (NULL:
 * the null stream); device pointers.  z_walls: 1 zero beyond the end planes, 0 periodic.
 * Errors: EINVAL for null pointers or bad extents. */
int lbmix_net_forward(lbmix_net *net, const float *x_dev, float *y_dev, int nx, int ny, int nz, int z_walls,
                      void *stream);
/* lbmix_net_forward for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result, bitwise, but the
 * hidden layers' outputs live in a static device array of 64 MiB that every GPU the library
 * runs on holds until the process ends, so the call allocates nothing.  It needs
 * min(2, layers - 1) x hidden x nx ny nz x 4 bytes of it: up to 524288 nodes with 16 hidden
 * channels.  The caller passes x_dev and y_dev as for lbmix_net_forward, with the network's
 * device current.  All calls on one GPU share the array, so calls that overlap on one GPU
 * (other streams, other threads, other networks) race and must be serialised by the caller.
 * Errors: EINVAL for null pointers, bad extents, a lattice beyond the scratch size (nothing
 * launched) or another device current; EDEVICE. */
int lbmix_net_forward_noalloc(lbmix_net *net, const float *x_dev, float *y_dev, int nx, int ny, int nz,
                              int z_walls, void *stream);
/* Mean-square loss mean((net(x) - t)^2) and its gradient with respect to every parameter by
 * back-propagation (kept on the device for lbmix_net_adam; lbmix_net_get_gradient copies it
 * out).  loss may be NULL (else the call synchronises the stream). */
int lbmix_net_gradient(lbmix_net *net, const float *x_dev, const float *t_dev, int nx, int ny, int nz,
                       int z_walls, double *loss, void *stream);
/* One Adam update with the last gradient: beta1 0.9, beta2 0.999, eps 1e-8, step size lr > 0. */
int lbmix_net_adam(lbmix_net *net, float lr, void *stream);
/* Output scale alpha of the warm start (the correction is alpha s net(...)): scale > 0 sets
 * it; *current (may be NULL) receives the value in use (0: not set, then 1 is used; training
 * sets it from the root mean square of the first target).  Errors: EINVAL. */
int lbmix_net_output_scale(lbmix_net *net, double scale, double *current);
const char *lbmix_net_last_error(const lbmix_net *net);
void lbmix_net_destroy(lbmix_net *net);

/* Network of the learned warm start (borrowed: it must outlive its use; NULL detaches it
 * and falls back to warm start 1).  Errors: EINVAL unless it takes 5 input channels and
 * lives on the lattice's device. */
int lbmix_set_warm_start_net(lbmix_ctx *ctx, lbmix_net *net);
/* Advance the lattice `nsteps` steps with the direct Poisson solve, training `net` on the
 * way: at each step (once three previous solutions exist) the sample is the input of the
 * learned warm start and the target the exact correction (psi - guess) / (alpha s); one Adam step of
 * size lr per sample.  A network without an output scale gets the root mean square of its
 * first target.  losses (may be NULL) receives the loss of every sample.  Errors: EINVAL
 * without charged species, for a bad network or arguments; ESTATE without a state. */
int lbmix_train_warm_start(lbmix_ctx *ctx, lbmix_net *net, int nsteps, float lr, double *losses);

/* Rounding of the stored populations of the FP32 and 16-bit forms: mode 0 rounds to
 * nearest-even (default); mode 1 rounds stochastically, each stored value going up or down
 * with the probabilities that make its expectation exact, the random bits drawn from a
 * counter-based hash of (seed, step, node, direction, species), so runs are reproducible
 * and a restored checkpoint continues bitwise.  Nearest rounding has fixed points: a slow
 * mode whose change per step is below half a unit in the last place of the stored value
 * (relative 2.4e-4 for FP16) stops evolving, and one just above it is biased the same way
 * every step; stochastic rounding removes this bias at the price of noise that averages out
 * over nodes.  For the FP32 forms mode 1 also computes the collision in FP64 (the exact
 * value being rounded must be known beyond FP32).  Errors: EINVAL for another mode, or
 * mode 1 with FP64 storage; ESTATE for a change of mode after the first step. */
int lbmix_set_rounding(lbmix_ctx *ctx, int mode, unsigned long long seed);

/* Arithmetic of the collision in the FP32 and 16-bit storage forms (nearest rounding, and the
 * 16-bit forms with stochastic rounding).  mode 1 (default): the density deviation of each
 * node and species, dn = sum_p (f_p - w_p rho0), and the term w_p omega_visc dn of the update
 * (eq. latboeq with the equilibrium of the Appendix, whose density part is w_p n) are carried
 * beyond FP32 (an FP64 sum; for the 16-bit forms an FP64 combination of exact FP32 sums per
 * weight class), so the deterministic FP32 rounding of w_p omega_visc dn does not bias slow
 * modes; everything else is FP32.  mode 0: FP32 collision arithmetic throughout, FP64 only for
 * the mass totals, the charge density and the Poisson solve.  No effect on FP64 storage or on
 * the FP32 forms with stochastic rounding (FP64 arithmetic).  Errors: EINVAL for another mode;
 * ESTATE for a change of mode after the first step. */
int lbmix_set_arithmetic(lbmix_ctx *ctx, int mode);

/* FP16 storage scale of one species: the bound `rel_range` of |f_p - w_p rho0| / (w_p rho0)
 * the lattice is expected to reach (default 0.1).  The power-of-two scale per direction
 * maps that bound near 2^12, leaving a factor 16 of headroom below the FP16 maximum and
 * about eight binary decades above its normal minimum.  Errors: EINVAL; ESTATE after the
 * first set_state. */
int lbmix_set_storage_range(lbmix_ctx *ctx, int species, double rel_range);

/* Equilibrium initial state of one species at time 0 (re-initialises a running context,
 * resetting its step counter and latched error once every species is set again):
 * f_p = phi_perp_p(n, u^alpha), the pre-collision populations at time 0.  n is a host
 * array [nz][ny][nx] of number densities, u a host array [3][nz][ny][nx] or NULL for
 * rest.  Allocates device memory on the first call (ENOMEM, EDEVICE).  Errors: EINVAL for
 * a bad species index or a NULL n. */
int lbmix_set_state(lbmix_ctx *ctx, int species, const double *n, const double *u);

/* Advance nsteps >= 0 time steps: per step one fused stream-collide launch (pull
 * streaming with bounce-back, moments, drag and field forces, collision, store, charge
 * density and FP64 mass partials) and, for charged runs, one Poisson solve.  Returns
 * ENOCONV if any solve of this call hit its sweep cap (the steps are still taken), ESTATE
 * before every species has a state, the latched code after ENONFINITE, EINVAL for a
 * non-neutral charged system. */
int lbmix_step(lbmix_ctx *ctx, int nsteps);

/* Moments of the pre-collision populations at the current time into host arrays:
 * n_out [nz][ny][nx] number density, j_out [3][nz][ny][nx] momentum density (either may
 * be NULL).  FP64 output whatever the storage.  Synchronises.  Errors: EINVAL, ESTATE. */
int lbmix_get_moments(lbmix_ctx *ctx, int species, double *n_out, double *j_out);

/* Same as lbmix_get_moments into device memory (FP64, same layout, either may be NULL),
 * ordered on the context stream, no synchronisation. */
int lbmix_get_moments_device(lbmix_ctx *ctx, int species, double *n_dev, double *j_dev);

/* Pre-collision populations f_p of one species at the current time, host [19][nz][ny][nx],
 * FP64 (the shift of the SHIFTED forms added back).  Synchronises. */
int lbmix_get_populations(lbmix_ctx *ctx, int species, double *f_out);

/* The potential psi~ = e psi / k_B T the next collision will use (solved now if it is not
 * yet available), host [nz][ny][nx], zero mean over the fluid.  Synchronises. */
int lbmix_get_potential(lbmix_ctx *ctx, double *psi_out);

/* FP64 totals sum_x n^alpha(x) of every species at the current time, host [nspecies],
 * summed in a fixed order (bitwise reproducible).  A non-finite total latches ENONFINITE.
 * Synchronises. */
int lbmix_get_mass_totals(lbmix_ctx *ctx, double *totals);

/* FP64 totals sum_x n^alpha(x) of every species, host [nspecies], of the state the last
 * stream-collide launch read (the populations after streaming, before the collision; streaming
 * moves or reflects every population, so this is the mass of the state before that step),
 * from the per-work-group FP64 partials the fused step writes (continuity, eq. `continuityb`:
 * a mass monitor that needs no extra pass over the populations).  The shifted forms' shift is
 * added back.  With the FP64 carry of the density deviation (lbmix_set_arithmetic mode 1) the
 * FP32 forms sum every stored value in FP64 and the 16-bit forms each weight class in FP32;
 * in mode 0 each node's deviation is an FP32 sum.  Fixed summation order (bitwise
 * reproducible).  Synchronises.  Errors: EINVAL for a null output, ESTATE before the first
 * step; a non-finite total latches ENONFINITE. */
int lbmix_get_step_mass(lbmix_ctx *ctx, double *totals);

/* Plane averages over x and y of the pre-collision moments at the current time, host
 * [nspecies][4][nz]: n, j_x, j_y, j_z per plane (wall planes 0), FP64 in a fixed order.
 * These give the channel observables of Sec. IV: mass flow, electric current and its
 * electro-osmotic part.  Synchronises. */
int lbmix_get_zprofiles(lbmix_ctx *ctx, double *out);

/* Counters of the context. */
int lbmix_get_stats(lbmix_ctx *ctx, lbmix_stats *out);

/* Plain device copy of `bytes` bytes from src to dst (device pointers, 16-byte aligned, bytes
 * a multiple of 16, not overlapping) on the hipStream_t `stream` (NULL: the null stream),
 * with 16-byte non-temporal loads and stores.  It is the copy kernel whose bandwidth the
 * fused step's HBM bandwidth is compared with (each byte read once and written once, as each
 * population is by the step).  Errors: EINVAL for null or misaligned pointers or a size that
 * is not a multiple of 16; EDEVICE for a launch failure. */
int lbmix_device_copy(void *dst, const void *src, unsigned long long bytes, void *stream);

/* Block until all work issued on the context stream has finished. */
int lbmix_sync(lbmix_ctx *ctx);

/* Checkpoint: the stored populations (native storage), potential, step counter and every
 * parameter, with a versioned header.  lbmix_load needs a context created with the same
 * extents, geometry, storage and species; restoring and stepping reproduces an
 * uninterrupted run bitwise.  Errors: EINVAL (mismatch, bad file), ESTATE, EDEVICE. */
int lbmix_save(lbmix_ctx *ctx, const char *path);
int lbmix_load(lbmix_ctx *ctx, const char *path);

/* Text of the last error of this context ("" if none); valid until the next call. */
const char *lbmix_last_error(const lbmix_ctx *ctx);

/* Free the context and its device memory (ctx may be NULL). */
void lbmix_destroy(lbmix_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMIX_H */
