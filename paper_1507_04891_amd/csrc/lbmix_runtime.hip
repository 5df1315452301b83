// Host runtime of the multicomponent lattice-Boltzmann library: the context behind the C ABI
// of include/lbmix.h.  It owns the device memory (double-buffered populations over the
// fluid nodes, stored per plane in blocks of rows of all 19 slots, potential, charge density,
// reduction scratch), maps the physical parameters
// to relaxation frequencies (Sec. IV: nu = v_T^2 (1/omega_visc - 1/2),
// D = v_T^2 (1/omega_drag - 1/2)) and sequences a time step: one fused stream-collide
// launch, then for charged runs the Poisson solve of the new charge density, used by the
// next collision.
#include "lbmix.h"
#include "lbmix_net.h"
#include "lbmix_netobj.h"
#include "lbmix_poisson.h"
#include "lbmix_step.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

using namespace lbmix;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kW[Q] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
constexpr char kMagic[8] = {'L', 'B', 'M', 'X', 'C', 'K', '0', '1'};

}  // namespace

struct lbmix_ctx {
    // lattice
    int nx = 0, ny = 0, nz = 0, nzf = 0, geometry = 0, storage = 0;
    Store st = Store::F64;
    size_t esize = 8;
    uint32_t Nf = 0;
    size_t Nfull = 0;
    bool slit = false;                // walls along z (a slit or a stack of channels)
    // channels along z: a slit is one channel, the periodic box one channel without walls.
    // Fluid width, first fluid plane and first full plane (its lower wall) of each channel,
    // per-channel drag (tau <= 0: the context's) and wall charges.
    int nch = 1;
    std::vector<int> ch_width, ch_first, ch_full;
    std::vector<double> ch_tau_d, ch_sig_lo, ch_sig_hi;
    std::vector<double> ch_total;     // [species][channel]: FP64 totals of the initial densities
    PlaneInfo *d_planes = nullptr;
    int32_t *d_fof = nullptr;         // fluid plane of each full plane (-1: wall)
    uint32_t *d_first = nullptr;      // first fluid plane of each channel, then nzf
    double *d_chan = nullptr;         // per channel: mean of b, then mean of psi
    double *d_psums = nullptr;        // per fluid plane sums
    bool tables_dirty = true;
    int direct_count = 0;             // direct solves (the residual is evaluated every check_every)
    // species and parameters
    int ns = 0;
    double rho0[MAXS] = {};
    int valence[MAXS] = {};
    double host_total[MAXS] = {};     // FP64 sum of the initial densities (neutrality check)
    double rel_range[MAXS] = {};      // FP16 scale: bound of |f - w rho0| / (w rho0)
    double tau_v = 1.0, tau_d = 1.0, sc = 1.0;
    bool drag_from_sc = true;
    int pair_ns = 0;                  // > 0: drag relaxation time per pair of species
    double tau_pair[MAXS][MAXS] = {};
    int forcing = 0;                  // 0: forcing of the Appendix; 1: the Guo-type variant
    double lB = 0.0, sig_lo = 0.0, sig_hi = 0.0, E[3] = {0.0, 0.0, 0.0};
    double sor_tol = 1e-8, sor_omega = -1.0;
    int poisson_method = 0;           // 0 red-black SOR, 1 multigrid, 2 direct (spectral)
    int warm_start = 0;               // 0 previous potential, 1 extrapolation in time, 2 learned
    lbmix_net *ws_net = nullptr;      // borrowed network of the learned warm start
    double *ws_r = nullptr, *ws_guess = nullptr, *ws_scale = nullptr;   // residual, guess, rms (device)
    double *ws_c = nullptr;           // coarse-grid solution of A c = r, prolonged to the fluid
    float *ws_x = nullptr, *ws_y = nullptr, *ws_t = nullptr, *ws_mask = nullptr;
    double *psi_prev = nullptr;       // two previous solutions (warm_start 1)
    int have_prev = 0;
    int mg_last = 0;                  // V-cycles of the last multigrid solve
    int rounding = 0;                 // FP32 and 16-bit forms: 0 nearest-even, 1 stochastic
    int wide = 1;                     // FP32 and 16-bit forms: density deviation carried in FP64
    unsigned long long round_seed = 0;
    int sor_max = 200000, sor_check = 10;
    // device
    hipStream_t stream = nullptr;     // borrowed; nullptr is the HIP null stream
    int device = 0;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    double *psi = nullptr, *q = nullptr;
    double *partials = nullptr;       // per-block partial sums
    size_t partials_cap = 0;
    double *step_partials = nullptr;  // mass partials of the last stream-collide
    uint32_t step_nb = 0;             // capacity in blocks (the largest candidate launch)
    uint32_t part_nb = 0;             // blocks of the last stream-collide launch (0: none yet)
    uint32_t blk_x = 0, blk_y = 0;    // launch shape of stream_collide (0: default)
    double *dred = nullptr;           // device results of reductions (16 doubles)
    double *hred = nullptr;           // pinned host mirror
    double *scratch = nullptr;        // readback staging
    size_t scratch_cap = 0;
    // multigrid: level 0 is (psi, b); coarser levels own their arrays
    std::vector<MGLevel> mg;
    bool mg_lines = false;            // channel stack: lateral coarsening, z-line relaxation
    std::vector<double *> mg_idn, mg_pmid;   // per level: pivots of the z lines
    double *mg_b = nullptr;
    double *mg_cinv = nullptr;        // exact inverse of the coarsest level (<= 64 cells)
    hipStream_t cap_stream = nullptr;  // capture-only stream (graphs replay on `stream`)
    hipGraph_t vgraph = nullptr;
    hipGraphExec_t vexec = nullptr;
    // captured steps (fused step + direct solve), one per buffer parity, and the device step
    // count they derive the rounding seed from
    int use_graph = 0;
    hipGraph_t sgraph[2] = {nullptr, nullptr};
    hipGraphExec_t sexec[2] = {nullptr, nullptr};
    unsigned long long *step_dev = nullptr;
    // direct solve: orthonormal bases of the periodic axes, their eigenvalues, the inverse
    // pivots of the z systems (slit), segment bounds, two work arrays
    double *sp_tx = nullptr, *sp_ty = nullptr, *sp_tz = nullptr, *sp_mu = nullptr;
    double *sp_txp = nullptr, *sp_typ = nullptr;   // x and y bases zero-padded to 64 x 65 (planes up to 64)
    double *sp_fx = nullptr, *sp_fy = nullptr, *sp_fz = nullptr;   // FFT twiddles along x, y, z (power-of-two extents)
    double *sp_piv = nullptr, *sp_piv_end = nullptr, *sp_pmid = nullptr, *sp_a = nullptr, *sp_b = nullptr;
    uint32_t *sp_seg = nullptr;
    float scale[MAXS][Q], inv_scale[MAXS][Q];
    // state
    bool allocated = false, started = false, psi_valid = false;
    bool set[MAXS] = {};
    long long steps = 0, solves = 0, total_sweeps = 0;
    int last_sweeps = 0, last_status = 0;
    double last_resid = 0.0;
    bool resid_on_device = false;     // fixed-sweep solves leave the residual in dred
    int latched = 0;
    std::string err;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip(hipError_t e, const char *what) {
        if (e == hipSuccess) return LBMIX_OK;
        return fail(e == hipErrorOutOfMemory ? LBMIX_ENOMEM : LBMIX_EDEVICE, "%s: %s", what,
                    hipGetErrorString(e));
    }
    bool charged() const {
        if (!(lB > 0.0)) return false;
        for (int s = 0; s < ns; ++s)
            if (valence[s] != 0) return true;
        return false;
    }
    bool field() const { return charged() || E[0] != 0.0 || E[1] != 0.0 || E[2] != 0.0; }
    double omega_drag() const {
        if (pair_ns == 2) return 1.0 / tau_pair[0][1];   // a binary has a single pair
        if (!drag_from_sc) return 1.0 / tau_d;
        // D = nu / Sc with D = v_T^2 (tau_drag - 1/2), or v_T^2 tau_drag for the Guo-type variant
        return forcing == 1 ? sc / (tau_v - 0.5) : 1.0 / (0.5 + (tau_v - 0.5) / sc);
    }
    double sor_w() const {
        if (sor_omega > 0.0) return sor_omega;
        const int L = std::max(nx, std::max(ny, nzf));
        return 2.0 / (1.0 + std::sin(kPi / L));
    }
    double rho_bar(int s) const {
        return (storage == LBMIX_F64 || storage == LBMIX_F32) ? 0.0 : rho0[s];
    }
    uint32_t node_blocks() const {
        dim3 b;
        const dim3 g = node_grid(nx, ny, nzf, &b);
        return g.x * g.y * g.z;
    }
    // candidate launch shapes of stream_collide (bx x by threads, 64..512 threads)
    std::vector<std::pair<uint32_t, uint32_t>> step_shapes() const {
        std::vector<std::pair<uint32_t, uint32_t>> v;
        if (nx >= 64) {
            const uint32_t cap = std::min<uint32_t>(STEP_BLOCK, ((nx + 63) / 64) * 64);
            for (uint32_t bx = 64; bx <= cap; bx *= 2)
                for (uint32_t by = 1; bx * by <= (uint32_t)STEP_BLOCK; by *= 2)
                    if (by <= (uint32_t)ny || by == 1) v.push_back({bx, by});
        } else {
            for (uint32_t t = 64; t <= (uint32_t)STEP_BLOCK; t *= 2) {
                const uint32_t by = std::min<uint32_t>(std::max<uint32_t>(t / nx, 1), ny);
                if (nx * by <= (uint32_t)STEP_BLOCK && (v.empty() || v.back().second != by)) v.push_back({(uint32_t)nx, by});
            }
        }
        return v;
    }
    uint32_t step_blocks() const {   // the most blocks any candidate (or the default) launches
        dim3 b;
        dim3 g = step_grid(nx, ny, nzf, &b);
        uint32_t m = g.x * g.y * g.z;
        for (auto &sh : step_shapes()) {
            g = step_grid(nx, ny, nzf, &b, sh.first, sh.second);
            m = std::max(m, g.x * g.y * g.z);
        }
        for (bool sr : {false, true}) {   // the default shapes of either rounding
            uint32_t bx, by;
            step_shape(st, sr, ns, (uint32_t)nx, 0, 0, &bx, &by);
            g = step_grid(nx, ny, nzf, &b, bx, by);
            m = std::max(m, g.x * g.y * g.z);
        }
        return m;
    }
    StepArgs args() const {
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.fin = f[cur];
        a.fout = f[cur ^ 1];
        a.nx = nx;
        a.ny = ny;
        a.nzf = nzf;
        a.blog = pop_block_log2((uint32_t)nx, (uint32_t)ny, (uint32_t)ns, (uint32_t)esize);
        a.N = (uint32_t)nx << a.blog;
        a.ns = ns;
        a.q_rest = 0.0;
        for (int s = 0; s < MAXS; ++s) {
            a.rho_bar[s] = s < ns ? rho_bar(s) : 0.0;
            a.valence[s] = s < ns ? valence[s] : 0;
            for (int p = 0; p < Q; ++p) {
                a.scale[s][p] = scale[s][p];
                a.inv_scale[s][p] = inv_scale[s][p];
            }
            if (s < ns) a.q_rest += valence[s] * a.rho_bar[s];
            for (int k = 0; k < 3; ++k) {
                const int rep = k == 0 ? 0 : (k == 1 ? 1 : 7);
                a.cw[s][k] = kW[rep] * (double)scale[s][rep];
                a.cwo[s][k] = kW[rep] * (1.0 / tau_v) * (double)scale[s][rep];
                a.cwf[s][k] = (float)a.cw[s][k];
                a.cwof[s][k] = (float)a.cwo[s][k];
                a.inv_scale_k[s][k] = (double)inv_scale[s][rep];
            }
            a.rho_bar_f[s] = (float)a.rho_bar[s];
        }
        a.omega_v = 1.0 / tau_v;
        a.omega_d = omega_drag();
        a.omega_v_f = (float)a.omega_v;
        a.omega_d_f = (float)a.omega_d;
        a.pair_drag = pair_ns >= 3 ? 1 : 0;
        a.forcing = forcing;
        for (int s = 0; s < MAXS; ++s)
            for (int b = 0; b < MAXS; ++b)
                a.omega_pair[s][b] = (pair_ns >= 3 && s < ns && b < ns && s != b) ? 1.0 / tau_pair[s][b] : 0.0;
        for (int d = 0; d < 3; ++d) a.E[d] = E[d];
        a.psi = psi;
        a.q = q;
        a.planes = slit ? d_planes : nullptr;
        a.fluid_of_full = d_fof;
        a.nzfull = (uint32_t)nz;
        a.partials = step_partials;
        a.stochastic = rounding;
        a.wide = wide;
        a.block_x = blk_x;
        a.block_y = blk_y;
        a.seed = step_seed(round_seed, (unsigned long long)(steps + 1));
        a.step_dev = nullptr;
        a.round_seed = round_seed;
        return a;
    }
    PoissonArgs pargs() const {
        PoissonArgs p;
        p.psi = psi;
        p.q = q;
        p.nx = nx;
        p.ny = ny;
        p.nzf = nzf;
        p.N = Nf;
        p.slit = slit ? 1 : 0;
        p.K = 4.0 * kPi * lB;
        p.planes = slit ? d_planes : nullptr;
        p.bmean = d_chan;
        p.omega = sor_w();
        return p;
    }
    void compute_scales() {
        for (int s = 0; s < MAXS; ++s)
            for (int p = 0; p < Q; ++p) {
                float sc_ = 1.0f;
                if (storage == LBMIX_F16_SHIFTED && s < ns) {
                    // largest |f - w rho0| expected: w rho0 rel_range; map it near 2^12 so
                    // FP16 keeps 11 significant bits over eight more binary decades
                    const double dmax = kW[p] * rho0[s] * rel_range[s];
                    const int e = (int)std::floor(std::log2(4096.0 / dmax));
                    sc_ = std::ldexp(1.0f, std::max(-60, std::min(60, e)));
                }
                scale[s][p] = sc_;
                inv_scale[s][p] = 1.0f / sc_;
            }
    }
};

namespace {

// Captured graphs hold their arguments by value; drop them when these change.
void drop_graph(lbmix_ctx *c) {
    if (c->vexec) (void)hipGraphExecDestroy(c->vexec);
    if (c->vgraph) (void)hipGraphDestroy(c->vgraph);
    c->vexec = nullptr;
    c->vgraph = nullptr;
    for (int k = 0; k < 2; ++k) {
        if (c->sexec[k]) (void)hipGraphExecDestroy(c->sexec[k]);
        if (c->sgraph[k]) (void)hipGraphDestroy(c->sgraph[k]);
        c->sexec[k] = nullptr;
        c->sgraph[k] = nullptr;
    }
}

int ensure_scratch(lbmix_ctx *c, size_t bytes) {
    if (c->scratch_cap >= bytes) return LBMIX_OK;
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_cap = 0;
    int rc = c->hip(hipMalloc((void **)&c->scratch, bytes), "hipMalloc(readback scratch)");
    if (rc) return rc;
    c->scratch_cap = bytes;
    return LBMIX_OK;
}

int allocate(lbmix_ctx *c) {
    if (c->allocated) return LBMIX_OK;
    int rc = c->hip(hipGetDevice(&c->device), "hipGetDevice");
    if (rc) return rc;
    const size_t pop = (size_t)c->ns * Q * c->Nf * c->esize;
    for (int k = 0; k < 2; ++k) {
        rc = c->hip(hipMalloc(&c->f[k], pop), "hipMalloc(populations)");
        if (rc) return rc;
        rc = c->hip(hipMemsetAsync(c->f[k], 0, pop, c->stream), "hipMemset(populations)");
        if (rc) return rc;
    }
    const uint32_t nb = c->node_blocks();
    const uint32_t qb = (c->Nf + BLOCK - 1) / BLOCK;
    c->step_nb = c->step_blocks();
    c->partials_cap = (size_t)4 * std::max(nb, qb);
    rc = c->hip(hipMalloc((void **)&c->partials, c->partials_cap * sizeof(double)), "hipMalloc(partials)");
    if (rc) return rc;
    rc = c->hip(hipMalloc((void **)&c->step_partials, (size_t)MAXS * c->step_nb * sizeof(double)), "hipMalloc(partials)");
    if (rc) return rc;
    rc = c->hip(hipMemsetAsync(c->step_partials, 0, (size_t)MAXS * c->step_nb * sizeof(double), c->stream), "hipMemset");
    if (rc) return rc;
    rc = c->hip(hipMalloc((void **)&c->dred, 16 * sizeof(double)), "hipMalloc(reduction)");
    if (rc) return rc;
    rc = c->hip(hipMemsetAsync(c->dred, 0, 16 * sizeof(double), c->stream), "hipMemset");
    if (rc) return rc;
    rc = c->hip(hipHostMalloc((void **)&c->hred, 16 * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    if (rc) return rc;
    c->allocated = true;
    return LBMIX_OK;
}

int ensure_field_buffers(lbmix_ctx *c) {
    if (c->psi) return LBMIX_OK;
    int rc = c->hip(hipMalloc((void **)&c->psi, (size_t)c->Nf * sizeof(double)), "hipMalloc(psi)");
    if (rc) return rc;
    rc = c->hip(hipMalloc((void **)&c->q, (size_t)c->Nf * sizeof(double)), "hipMalloc(q)");
    if (rc) return rc;
    rc = c->hip(hipMemsetAsync(c->psi, 0, (size_t)c->Nf * sizeof(double), c->stream), "hipMemset(psi)");
    if (rc) return rc;
    return c->hip(hipMemsetAsync(c->q, 0, (size_t)c->Nf * sizeof(double), c->stream), "hipMemset(q)");
}

double channel_omega_drag(const lbmix_ctx *c, int ch) {
    const double t = c->ch_tau_d.empty() ? 0.0 : c->ch_tau_d[ch];
    return t > 0.0 ? 1.0 / t : c->omega_drag();
}

// Per-plane and per-channel device tables from the current parameters (after every change).
int ensure_tables(lbmix_ctx *c) {
    if (!c->tables_dirty) return LBMIX_OK;
    int rc;
    if (!c->d_fof) {
        if ((rc = c->hip(hipMalloc((void **)&c->d_planes, (size_t)c->nzf * sizeof(PlaneInfo)), "hipMalloc(tables)")) ||
            (rc = c->hip(hipMalloc((void **)&c->d_fof, (size_t)c->nz * sizeof(int32_t)), "hipMalloc(tables)")) ||
            (rc = c->hip(hipMalloc((void **)&c->d_first, (size_t)(c->nch + 1) * sizeof(uint32_t)), "hipMalloc(tables)")) ||
            (rc = c->hip(hipMalloc((void **)&c->d_chan, (size_t)2 * c->nch * sizeof(double)), "hipMalloc(tables)")) ||
            (rc = c->hip(hipMalloc((void **)&c->d_psums, (size_t)c->nzf * sizeof(double)), "hipMalloc(tables)")))
            return rc;
    }
    std::vector<PlaneInfo> pl(c->nzf);
    std::vector<int32_t> fof(c->nz, -1);
    std::vector<uint32_t> first(c->nch + 1);
    const double K = 4.0 * kPi * c->lB;
    for (int ch = 0; ch < c->nch; ++ch) {
        first[ch] = (uint32_t)c->ch_first[ch];
        const int W = c->ch_width[ch];
        for (int k = 0; k < W; ++k) {
            const int zf = c->ch_first[ch] + k;
            const int zfull = c->slit ? c->ch_full[ch] + 1 + k : zf;
            PlaneInfo &P = pl[zf];
            std::memset(&P, 0, sizeof P);
            P.omega_d = channel_omega_drag(c, ch);
            P.chan = (uint32_t)ch;
            P.zfull = (uint32_t)zfull;
            P.zloc = (uint32_t)(c->slit ? k + 1 : k);
            if (c->slit) {
                if (k == 0) { P.walls |= 1u; P.ghost_lo = K * c->ch_sig_lo[ch]; P.lump += c->ch_sig_lo[ch]; }
                if (k == W - 1) { P.walls |= 2u; P.ghost_hi = K * c->ch_sig_hi[ch]; P.lump += c->ch_sig_hi[ch]; }
            }
            fof[zfull] = zf;
        }
    }
    first[c->nch] = (uint32_t)c->nzf;
    // the tables may be read by work still queued on the stream
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    if ((rc = c->hip(hipMemcpy(c->d_planes, pl.data(), pl.size() * sizeof(PlaneInfo), hipMemcpyHostToDevice), "copy tables")) ||
        (rc = c->hip(hipMemcpy(c->d_fof, fof.data(), fof.size() * sizeof(int32_t), hipMemcpyHostToDevice), "copy tables")) ||
        (rc = c->hip(hipMemcpy(c->d_first, first.data(), first.size() * sizeof(uint32_t), hipMemcpyHostToDevice), "copy tables")))
        return rc;
    c->tables_dirty = false;
    drop_graph(c);
    return LBMIX_OK;
}

// Per-channel means of v over the fluid into d_chan[off .. off + nch): mode 0 = mean of
// b = -K (q + lump), mode 1 = plain mean.
int channel_means(lbmix_ctx *c, const double *v, int mode, int off) {
    const uint32_t nxy = (uint32_t)c->nx * c->ny;
    int rc = c->hip(launch_plane_sum(v, nxy, (uint32_t)c->nzf, c->d_psums, c->stream), "plane_sum");
    if (rc) return rc;
    return c->hip(launch_channel_means(c->d_psums, c->d_first, (uint32_t)c->nch, c->slit ? c->d_planes : nullptr, nxy,
                                       mode, 4.0 * kPi * c->lB, c->d_chan + off, c->stream),
                  "channel_means");
}

int fetch(lbmix_ctx *c, int count) {
    int rc = c->hip(hipMemcpyAsync(c->hred, c->dred, count * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                    "hipMemcpy(reduction)");
    if (rc) return rc;
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

// dred[0] = sum q, dred[1] = mean b; dred[4..7] = (r2, b2, sum psi, mean psi).
int residual(lbmix_ctx *c, const PoissonArgs &pa) {
    uint32_t nb = 0;
    int rc = c->hip(launch_residual(pa, c->partials, &nb, c->stream), "residual");
    if (rc) return rc;
    return c->hip(launch_finalize(c->partials, nb, 3, c->dred + 4, 2, 0.0, 0.0, (double)c->Nf, c->stream),
                  "finalize(residual)");
}

// ---- multigrid -------------------------------------------------------------------------

// sweeps before / after the coarse-grid correction: one on the finest level (the costly
// one), two on the coarser grid levels
constexpr int kPre0 = 1, kPost0 = 1, kPre = 2, kPost = 2;

// One stream-collide launch; remembers how many work-groups wrote mass partials.
hipError_t collide(lbmix_ctx *c, const StepArgs &a, bool field, bool charged, hipStream_t st) {
    c->part_nb = stream_collide_blocks(c->st, c->ns, a);
    return launch_stream_collide(c->st, c->ns, c->slit, field, charged, a, st);
}

// Pivots of the z-line systems of a channel-stack level, (Ld + az n_z) e - az (e_up + e_down)
// = g with Ld its lateral diagonal, eliminated from both ends of a channel towards its middle
// plane mid = W / 2: one recurrence from an end, shared by every channel and both ends (idn[k],
// k < longest - 1), and the middle plane of each channel (pmid[c]; 0 where the line is
// singular, which pins that plane).
int mg_line_pivots(lbmix_ctx *c, const MGLevel &L) {
    const double Ld = (L.nx > 1 ? 2.0 * L.ax : 0.0) + (L.ny > 1 ? 2.0 * L.ay : 0.0), az = L.az;
    int longest = 1;
    for (int w : c->ch_width) longest = std::max(longest, w);
    std::vector<double> denom(std::max(longest - 1, 1), 1.0), idn(denom.size(), 0.0), last(c->nch, 0.0);
    for (int k = 0; k + 1 < longest; ++k) {
        denom[k] = k == 0 ? Ld + az : (Ld + 2.0 * az) - az * az / denom[k - 1];
        idn[k] = 1.0 / denom[k];
    }
    for (int ch = 0; ch < c->nch; ++ch) {
        const int W = c->ch_width[ch], mid = W / 2;
        double d = Ld;
        if (mid >= 1) d += az - az * az * idn[mid - 1];
        if (mid + 1 < W) d += az - az * az * idn[W - 2 - mid];
        last[ch] = d > 1e-12 * (Ld + 2.0 * az) ? 1.0 / d : 0.0;
    }
    double *di = nullptr, *dl = nullptr;
    int rc;
    if ((rc = c->hip(hipMalloc((void **)&di, idn.size() * sizeof(double)), "hipMalloc(mg)"))) return rc;
    c->mg_idn.push_back(di);
    if ((rc = c->hip(hipMalloc((void **)&dl, last.size() * sizeof(double)), "hipMalloc(mg)"))) return rc;
    c->mg_pmid.push_back(dl);
    if ((rc = c->hip(hipMemcpy(di, idn.data(), idn.size() * sizeof(double), hipMemcpyHostToDevice), "copy pivots")))
        return rc;
    return c->hip(hipMemcpy(dl, last.data(), last.size() * sizeof(double), hipMemcpyHostToDevice), "copy pivots");
}

int mg_build(lbmix_ctx *c) {
    if (!c->mg.empty()) return LBMIX_OK;
    int rc = c->hip(hipMalloc((void **)&c->mg_b, (size_t)c->Nf * sizeof(double)), "hipMalloc(mg)");
    if (rc) return rc;
    // a stack of channels of any widths keeps every plane on every level and coarsens x and y
    // only, relaxing whole z lines of each channel (their systems are solved exactly), down to
    // one column per channel, where the line solve is the exact coarse solve
    c->mg_lines = c->nch > 1;
    MGLevel L{};
    L.e = c->psi;
    L.r = c->mg_b;
    L.nx = c->nx;
    L.ny = c->ny;
    L.nz = c->nzf;
    L.ax = L.ay = L.az = 1.0;
    L.periodic_z = c->slit ? 0 : 1;
    L.planes = c->mg_lines ? c->d_planes : nullptr;
    double hx = 1.0, hy = 1.0, hz = 1.0;
    for (;;) {
        // a periodic axis halves while the red-black colouring stays consistent (even size
        // after halving, or one cell); a zero-flux axis halves while its size is even
        auto per_ok = [](uint32_t n) { return n >= 2 && n % 2 == 0 && ((n / 2) % 2 == 0 || n == 2); };
        auto neu_ok = [](uint32_t n) { return n >= 2 && n % 2 == 0; };
        L.fx = per_ok(L.nx) ? 2 : 1;
        L.fy = per_ok(L.ny) ? 2 : 1;
        L.fz = (!c->mg_lines && (L.periodic_z ? per_ok(L.nz) : neu_ok(L.nz))) ? 2 : 1;
        const bool last = (L.fx == 1 && L.fy == 1 && L.fz == 1) ||
                          (!c->mg_lines && (size_t)L.nx * L.ny * L.nz <= 64);
        if (last) L.fx = L.fy = L.fz = 1;
        if (c->mg_lines && (rc = mg_line_pivots(c, L))) return rc;
        c->mg.push_back(L);
        if (last) break;
        MGLevel C{};
        C.nx = L.nx / L.fx;
        C.ny = L.ny / L.fy;
        C.nz = L.nz / L.fz;
        hx *= L.fx;
        hy *= L.fy;
        hz *= L.fz;
        C.ax = 1.0 / (hx * hx);
        C.ay = 1.0 / (hy * hy);
        C.az = 1.0 / (hz * hz);
        C.periodic_z = L.periodic_z;
        C.planes = L.planes;
        const size_t n = (size_t)C.nx * C.ny * C.nz;
        if ((rc = c->hip(hipMalloc((void **)&C.e, n * sizeof(double)), "hipMalloc(mg)"))) return rc;
        if ((rc = c->hip(hipMalloc((void **)&C.r, n * sizeof(double)), "hipMalloc(mg)"))) return rc;
        L = C;
    }
    // exact coarsest solve: invert A + 1 1^T / m (A: the level's operator, m <= 64 cells) by
    // Gauss-Jordan elimination with partial pivoting in FP64
    const MGLevel &B = c->mg.back();
    const int m = (int)(B.nx * B.ny * B.nz);
    if (!c->mg_lines && c->mg.size() >= 2 && m <= 64) {
        std::vector<double> A((size_t)m * m, 0.0), I((size_t)m * m, 0.0);
        auto id = [&](int x, int y, int z) { return (z * (int)B.ny + y) * (int)B.nx + x; };
        for (int z = 0; z < (int)B.nz; ++z)
            for (int y = 0; y < (int)B.ny; ++y)
                for (int x = 0; x < (int)B.nx; ++x) {
                    const int i = id(x, y, z);
                    auto link = [&](int j, double a) { A[(size_t)i * m + j] += a; A[(size_t)i * m + i] -= a; };
                    if (B.nx > 1) {
                        link(id((x + 1) % B.nx, y, z), B.ax);
                        link(id((x + B.nx - 1) % B.nx, y, z), B.ax);
                    }
                    if (B.ny > 1) {
                        link(id(x, (y + 1) % B.ny, z), B.ay);
                        link(id(x, (y + B.ny - 1) % B.ny, z), B.ay);
                    }
                    if (B.nz > 1) {
                        if (B.periodic_z) {
                            link(id(x, y, (z + 1) % B.nz), B.az);
                            link(id(x, y, (z + B.nz - 1) % B.nz), B.az);
                        } else {
                            if (z + 1 < (int)B.nz) link(id(x, y, z + 1), B.az);
                            if (z > 0) link(id(x, y, z - 1), B.az);
                        }
                    }
                }
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[(size_t)i * m + j] += 1.0 / m;
            I[(size_t)i * m + i] = 1.0;
        }
        bool ok = true;
        for (int col = 0; col < m && ok; ++col) {
            int piv = col;
            for (int r = col + 1; r < m; ++r)
                if (std::fabs(A[(size_t)r * m + col]) > std::fabs(A[(size_t)piv * m + col])) piv = r;
            if (std::fabs(A[(size_t)piv * m + col]) < 1e-12) { ok = false; break; }
            for (int j = 0; j < m; ++j) {
                std::swap(A[(size_t)col * m + j], A[(size_t)piv * m + j]);
                std::swap(I[(size_t)col * m + j], I[(size_t)piv * m + j]);
            }
            const double d = A[(size_t)col * m + col];
            for (int j = 0; j < m; ++j) {
                A[(size_t)col * m + j] /= d;
                I[(size_t)col * m + j] /= d;
            }
            for (int r = 0; r < m; ++r) {
                if (r == col) continue;
                const double f = A[(size_t)r * m + col];
                if (f == 0.0) continue;
                for (int j = 0; j < m; ++j) {
                    A[(size_t)r * m + j] -= f * A[(size_t)col * m + j];
                    I[(size_t)r * m + j] -= f * I[(size_t)col * m + j];
                }
            }
        }
        if (ok) {
            if ((rc = c->hip(hipMalloc((void **)&c->mg_cinv, (size_t)m * m * sizeof(double)), "hipMalloc(mg)")))
                return rc;
            if ((rc = c->hip(hipMemcpy(c->mg_cinv, I.data(), (size_t)m * m * sizeof(double), hipMemcpyHostToDevice),
                             "copy coarse inverse")))
                return rc;
        }
    }
    return LBMIX_OK;
}

// One V(2,2) cycle on level 0 (psi, b), then the residual norms of the result.  The levels
// from the first one of at most kBottomCells cells down are solved by one work-group in LDS
// (their cells together must fit MG_BOTTOM_LDS).
constexpr size_t kBottomCells = 2048;

// One V(1,1) cycle of z-line red-black relaxation on a channel stack, then the residual norms.
int mg_line_vcycle(lbmix_ctx *c, const PoissonArgs &pa, hipStream_t st) {
    const int nl = (int)c->mg.size();
    int rc;
    auto sweep = [&](int l) -> int {
        for (int col = 0; col < 2; ++col) {
            int r = c->hip(launch_mg_line_rhs(c->mg[l], col, st), "mg_line_rhs");
            if (r) return r;
            if ((r = c->hip(launch_mg_line_solve(c->mg[l], col, c->mg_idn[l], c->mg_pmid[l], c->d_first,
                                                 (uint32_t)c->nch, st),
                            "mg_line_solve")))
                return r;
        }
        return LBMIX_OK;
    };
    for (int l = 0; l + 1 < nl; ++l) {
        if ((rc = sweep(l))) return rc;
        if ((rc = c->hip(launch_mg_restrict(c->mg[l], c->mg[l + 1], st), "mg_restrict"))) return rc;
    }
    // coarsest level: one column per channel is solved exactly by its line solve; a level that
    // could not be coarsened that far gets repeated sweeps
    const MGLevel &B = c->mg[nl - 1];
    const int count = (B.nx == 1 && B.ny == 1) ? 1 : std::max(4, 2 * (int)std::max(B.nx, B.ny));
    for (int k = 0; k < count; ++k)
        if ((rc = sweep(nl - 1))) return rc;
    for (int l = nl - 2; l >= 0; --l) {
        if ((rc = c->hip(launch_mg_prolong(c->mg[l], c->mg[l + 1], st), "mg_prolong"))) return rc;
        if ((rc = sweep(l))) return rc;
    }
    uint32_t nb = 0;
    if ((rc = c->hip(launch_residual(pa, c->partials, &nb, st), "residual"))) return rc;
    return c->hip(launch_finalize(c->partials, nb, 3, c->dred + 4, 2, 0.0, 0.0, (double)c->Nf, st),
                  "finalize(residual)");
}

int mg_vcycle(lbmix_ctx *c, const PoissonArgs &pa, hipStream_t st) {
    if (c->mg_lines) return mg_line_vcycle(c, pa, st);
    const int nl = (int)c->mg.size();
    // levels [0, lb) run as grid kernels, levels [lb, nl) inside one work-group; a hierarchy
    // of one level (no axis could be halved) is plain red-black Gauss-Seidel
    int lb = nl;
    for (int l = 1; l < nl; ++l)
        if ((size_t)c->mg[l].nx * c->mg[l].ny * c->mg[l].nz <= kBottomCells) { lb = l; break; }
    auto bottom_fits = [&](int from) {
        size_t cells = 0;
        for (int l = from; l < nl; ++l) cells += (size_t)c->mg[l].nx * c->mg[l].ny * c->mg[l].nz;
        return nl - from <= MG_MAX_BOTTOM && cells <= (size_t)MG_BOTTOM_LDS;
    };
    while (lb < nl && !bottom_fits(lb)) ++lb;   // a bottom that does not fit stays on the grid
    int rc;
    for (int l = 0; l < lb; ++l) {
        for (int k = 0; k < (l == 0 ? kPre0 : kPre); ++k)
            for (int col = 0; col < 2; ++col)
                if ((rc = c->hip(launch_mg_smooth(c->mg[l], col, st), "mg_smooth"))) return rc;
        if (l + 1 < nl && (rc = c->hip(launch_mg_restrict(c->mg[l], c->mg[l + 1], st), "mg_restrict")))
            return rc;
    }
    if (lb == nl) {   // no bottom solve: the coarsest grid level gets many sweeps
        const MGLevel &B = c->mg[nl - 1];
        const int sweeps = nl == 1 ? 0 : std::max(20, 4 * (int)std::max(B.nx, std::max(B.ny, B.nz)));
        for (int k = 0; k < sweeps; ++k)
            for (int col = 0; col < 2; ++col)
                if ((rc = c->hip(launch_mg_smooth(B, col, st), "mg_smooth"))) return rc;
    }
    if (lb < nl) {
        MGBottom bb{};
        bb.n = nl - lb;
        for (int l = lb; l < nl; ++l) bb.lev[l - lb] = c->mg[l];
        const MGLevel &B = c->mg[nl - 1];
        bb.coarse_sweeps = std::max(20, 4 * (int)std::max(B.nx, std::max(B.ny, B.nz)));
        bb.coarse_inv = c->mg_cinv;
        if ((rc = c->hip(launch_mg_bottom(bb, st), "mg_bottom"))) return rc;
    }
    for (int l = lb - 1; l >= 0; --l) {
        if (l + 1 < nl && (rc = c->hip(launch_mg_prolong(c->mg[l], c->mg[l + 1], st), "mg_prolong"))) return rc;
        for (int k = 0; k < (l == 0 ? kPost0 : kPost); ++k)
            for (int col = 0; col < 2; ++col)
                if ((rc = c->hip(launch_mg_smooth(c->mg[l], col, st), "mg_smooth"))) return rc;
    }
    uint32_t nb = 0;
    if ((rc = c->hip(launch_residual(pa, c->partials, &nb, st), "residual"))) return rc;
    return c->hip(launch_finalize(c->partials, nb, 3, c->dred + 4, 2, 0.0, 0.0, (double)c->Nf, st),
                  "finalize(residual)");
}

// The V-cycle and its residual as one graph, captured once and replayed on the context stream.
int mg_cycle(lbmix_ctx *c, const PoissonArgs &pa) {
    int rc;
    if (!c->vexec) {
        if (!c->cap_stream &&
            (rc = c->hip(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate")))
            return rc;
        if ((rc = c->hip(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "capture")))
            return rc;
        const int r1 = mg_vcycle(c, pa, c->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (r1) {
            if (g) (void)hipGraphDestroy(g);
            return r1;
        }
        if ((rc = c->hip(e, "hipStreamEndCapture"))) return rc;
        c->vgraph = g;
        if ((rc = c->hip(hipGraphInstantiate(&c->vexec, c->vgraph, nullptr, nullptr, 0), "hipGraphInstantiate")))
            return rc;
    }
    return c->hip(hipGraphLaunch(c->vexec, c->stream), "hipGraphLaunch");
}

// ---- direct solve -----------------------------------------------------------------------

// Orthonormal real Fourier basis of a periodic axis of n nodes, row k = basis vector k
// (frequency (k + 1) / 2), and the eigenvalues 4 sin^2(pi freq / n) of minus the 1-D
// second difference.
void periodic_basis(int n, std::vector<double> &T, std::vector<double> &mu) {
    T.assign((size_t)n * n, 0.0);
    mu.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        const int freq = (k + 1) / 2;
        const bool nyquist = (2 * freq == n);
        const bool sine = (k % 2 == 0) && k > 0 && !nyquist;
        const double norm = (k == 0 || nyquist) ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
        for (int x = 0; x < n; ++x) {
            const double ang = 2.0 * kPi * (double)(((long long)freq * x) % n) / n;
            T[(size_t)k * n + x] = norm * (sine ? std::sin(ang) : std::cos(ang));
        }
        const double sn = std::sin(kPi * freq / n);
        mu[k] = 4.0 * sn * sn;
    }
}

// Extents the FFT passes take (powers of two), and their twiddles exp(-2 pi i t / n), t < n,
// as (real, imaginary) pairs.
bool fft_extent(int n) { return n >= (int)FFT_MIN && n <= (int)FFT_MAX && (n & (n - 1)) == 0; }
std::vector<double> fft_twiddles(int n) {
    std::vector<double> w(2 * (size_t)n);
    for (int t = 0; t < n; ++t) {
        const double ang = 2.0 * kPi * t / n;
        w[2 * t] = std::cos(ang);
        w[2 * t + 1] = -std::sin(ang);
    }
    return w;
}
int log2_exact(uint32_t n) {
    int l = 0;
    while ((1u << l) < n) ++l;
    return l;
}

int upload(lbmix_ctx *c, double **dst, const std::vector<double> &v) {
    int rc = c->hip(hipMalloc((void **)dst, v.size() * sizeof(double)), "hipMalloc(direct solve)");
    if (rc) return rc;
    return c->hip(hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice), "copy(direct solve)");
}

int spec_build(lbmix_ctx *c) {
    if (c->sp_a) return LBMIX_OK;
    std::vector<double> tx, ty, tz, mux, muy, muz;
    periodic_basis(c->nx, tx, mux);
    periodic_basis(c->ny, ty, muy);
    int rc;
    if ((rc = upload(c, &c->sp_tx, tx)) || (rc = upload(c, &c->sp_ty, ty))) return rc;
    // FFT passes replace the products along x and y for planes larger than 64 x 64 with both
    // extents powers of two, and along z in a periodic box of more than 64 planes
    if (fft_extent(c->nx) && fft_extent(c->ny) && !(c->nx <= 64 && c->ny <= 64))
        if ((rc = upload(c, &c->sp_fx, fft_twiddles(c->nx))) || (rc = upload(c, &c->sp_fy, fft_twiddles(c->ny))))
            return rc;
    if (!c->slit && c->nzf > 64 && fft_extent(c->nzf) && (rc = upload(c, &c->sp_fz, fft_twiddles(c->nzf)))) return rc;
    if (c->nx <= (int)SPEC_PAD && c->ny <= (int)SPEC_PAD) {
        auto pad = [](const std::vector<double> &b, int n) {
            std::vector<double> p((size_t)SPEC_PAD * (SPEC_PAD + 1), 0.0);
            for (int r = 0; r < n; ++r)
                for (int k = 0; k < n; ++k) p[(size_t)r * (SPEC_PAD + 1) + k] = b[(size_t)r * n + k];
            return p;
        };
        if ((rc = upload(c, &c->sp_txp, pad(tx, c->nx))) || (rc = upload(c, &c->sp_typ, pad(ty, c->ny)))) return rc;
    }
    std::vector<double> mu(mux);
    mu.insert(mu.end(), muy.begin(), muy.end());
    if (c->slit) {
        // zero-flux z in every channel: rows of the z system carry diagonal -(2 + mu),
        // -(1 + mu) on the two end planes of the channel (-mu for a single plane).  The
        // inverse pivots before the last plane are those of one recurrence from the first
        // plane, shared by every channel; each channel has its own last pivot.
        const size_t nm = (size_t)c->nx * c->ny;
        int longest = 1;
        for (int w : c->ch_width) longest = std::max(longest, w);
        std::vector<double> piv(nm * (size_t)std::max(longest - 1, 1), 0.0), piv_end(nm * c->nch), pmid(nm * c->nch);
        for (int my = 0; my < c->ny; ++my)
            for (int mx = 0; mx < c->nx; ++mx) {
                const size_t m = (size_t)my * c->nx + mx;
                const double mxy = mux[mx] + muy[my];
                double prev = 0.0;
                for (int k = 0; k + 1 < longest; ++k) {
                    prev = 1.0 / (-(2.0 + mxy) + (k == 0 ? 1.0 : 0.0) - prev);
                    piv[(size_t)k * nm + m] = prev;
                }
                for (int ch = 0; ch < c->nch; ++ch) {
                    const int W = c->ch_width[ch];
                    const double before = W > 1 ? piv[(size_t)(W - 2) * nm + m] : 0.0;
                    const double d = -(2.0 + mxy) + 1.0 + (W == 1 ? 1.0 : 0.0);
                    piv_end[(size_t)ch * nm + m] = m == 0 ? 0.0 : 1.0 / (d - before);
                    // middle plane h = W / 2 of the elimination from both ends: its diagonal
                    // less the pivots of its two neighbours (pivot W - 2 - h from the bottom)
                    const int h = W / 2;
                    const double dh = -(2.0 + mxy) + (h == 0 ? 1.0 : 0.0) + (h == W - 1 ? 1.0 : 0.0);
                    const double above = h >= 1 ? piv[(size_t)(h - 1) * nm + m] : 0.0;
                    const double below = h + 1 < W ? piv[(size_t)(W - 2 - h) * nm + m] : 0.0;
                    pmid[(size_t)ch * nm + m] = m == 0 ? 0.0 : 1.0 / (dh - above - below);
                }
            }
        if ((rc = upload(c, &c->sp_piv, piv)) || (rc = upload(c, &c->sp_piv_end, piv_end)) ||
            (rc = upload(c, &c->sp_pmid, pmid)))
            return rc;
        std::vector<uint32_t> seg(c->nch + 1);
        for (int ch = 0; ch <= c->nch; ++ch) seg[ch] = ch < c->nch ? (uint32_t)c->ch_first[ch] : (uint32_t)c->nzf;
        if ((rc = c->hip(hipMalloc((void **)&c->sp_seg, seg.size() * sizeof(uint32_t)), "hipMalloc(direct solve)")))
            return rc;
        if ((rc = c->hip(hipMemcpy(c->sp_seg, seg.data(), seg.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
                         "copy(direct solve)")))
            return rc;
    } else {
        periodic_basis(c->nzf, tz, muz);
        if ((rc = upload(c, &c->sp_tz, tz))) return rc;
        mu.insert(mu.end(), muz.begin(), muz.end());
    }
    if ((rc = upload(c, &c->sp_mu, mu))) return rc;
    const size_t bytes = (size_t)c->Nf * sizeof(double);
    if ((rc = c->hip(hipMalloc((void **)&c->sp_b, bytes), "hipMalloc(direct solve)"))) return rc;
    return c->hip(hipMalloc((void **)&c->sp_a, bytes), "hipMalloc(direct solve)");
}

// Transforms along x (rows of nx), y (per plane) and z (whole array) into `out`;
// inverse = the transposed basis.
int spec_x(lbmix_ctx *c, const double *in, double *out, bool inverse, bool from_q = false) {
    SpecGemm g{};
    g.A = in; g.C = out; g.B = c->sp_tx;
    if (from_q) {   // in = q: the product forms b = -K (q + lump) as it loads it
        g.rhs = 1;
        g.rhs_K = 4.0 * kPi * c->lB;
        g.planes = c->slit ? c->d_planes : nullptr;
        g.rows_per_plane = (uint32_t)c->ny;
    }
    g.M = (uint32_t)c->ny * c->nzf; g.N = c->nx; g.K = c->nx; g.batch = 1;
    g.sAm = c->nx; g.sAk = 1; g.sCm = c->nx;
    // forward: C[m][k] = sum_x A[m][x] T[k][x];  inverse: C[m][x] = sum_k A[m][k] T[k][x]
    if (inverse) { g.sBk = c->nx; g.sBn = 1; } else { g.sBk = 1; g.sBn = c->nx; }
    return c->hip(launch_gemm_f64(g, true, inverse, c->stream), "gemm(x)");
}
int spec_left(lbmix_ctx *c, const double *T, uint32_t n, uint32_t inner, uint32_t batch, const double *in,
              double *out, bool inverse, const char *what) {
    SpecGemm g{};
    g.A = T; g.B = in; g.C = out;
    g.M = n; g.N = inner; g.K = n; g.batch = batch;
    // forward: C[k][i] = sum_j T[k][j] B[j][i];  inverse: C[j][i] = sum_k T[k][j] B[k][i]
    if (inverse) { g.sAm = 1; g.sAk = n; } else { g.sAm = n; g.sAk = 1; }
    g.sBb = g.sCb = (size_t)n * inner;
    g.sBk = inner; g.sBn = 1; g.sCm = inner;
    return c->hip(launch_gemm_f64(g, !inverse, true, c->stream), what);
}

// Transform along x (rows, from q when `from_q`) or y (columns of each plane) by the FFT pass.
int fft_x(lbmix_ctx *c, const double *in, double *out, bool inverse, bool from_q = false) {
    FftPass f{};
    f.in = in; f.out = out; f.tw = c->sp_fx;
    f.n = (uint32_t)c->nx; f.log2n = (uint32_t)log2_exact(f.n);
    f.nseq = (uint32_t)c->ny * c->nzf; f.log2pp = (uint32_t)log2_exact((uint32_t)c->ny);
    f.s_plane = (size_t)c->nx * c->ny; f.s_seq = (uint32_t)c->nx; f.s_el = 1;
    if (from_q) {
        f.rhs = 1;
        f.rhs_K = 4.0 * kPi * c->lB;
        f.planes = c->slit ? c->d_planes : nullptr;
    }
    return c->hip(launch_fft_pass(f, false, inverse, c->stream), "fft(x)");
}
int fft_y(lbmix_ctx *c, const double *in, double *out, bool inverse) {
    FftPass f{};
    f.in = in; f.out = out; f.tw = c->sp_fy;
    f.n = (uint32_t)c->ny; f.log2n = (uint32_t)log2_exact(f.n);
    f.nseq = (uint32_t)c->nx * c->nzf; f.log2pp = (uint32_t)log2_exact((uint32_t)c->nx);
    f.s_plane = (size_t)c->nx * c->ny; f.s_seq = 1; f.s_el = (uint32_t)c->nx;
    return c->hip(launch_fft_pass(f, true, inverse, c->stream), "fft(y)");
}
int fft_z(lbmix_ctx *c, const double *in, double *out, bool inverse) {   // periodic box
    FftPass f{};
    const uint32_t nxy = (uint32_t)c->nx * c->ny;
    f.in = in; f.out = out; f.tw = c->sp_fz;
    f.n = (uint32_t)c->nzf; f.log2n = (uint32_t)log2_exact(f.n);
    f.nseq = nxy; f.log2pp = (uint32_t)log2_exact(nxy);
    f.s_plane = 0; f.s_seq = 1; f.s_el = nxy;
    return c->hip(launch_fft_pass(f, true, inverse, c->stream), "fft(z)");
}

// The direct solve.  Planes of at most 64 x 64 nodes are transformed per plane (in
// registers up to 32 x 32, in LDS above); larger planes by FFT passes along x and y when
// both extents are powers of two, else by the batched products.  Each reads q and forms
// b = -K (q + lump) as it loads it.  The projection onto zero channel mean acts
// on the constant mode only and is applied there: by the z elimination of a slit or stack,
// by the spectral scale of a periodic box.
int spec_solve(lbmix_ctx *c, const PoissonArgs &pa) {
    int rc;
    if ((rc = spec_build(c))) return rc;
    const uint32_t nxy = (uint32_t)c->nx * c->ny;
    double *a = c->sp_a, *b = c->sp_b;
    const bool in_lds = c->nx <= 64 && c->ny <= 64;
    SpecXY xy{};
    xy.tx = c->sp_tx; xy.ty = c->sp_ty; xy.txp = c->sp_txp; xy.typ = c->sp_typ;
    xy.planes = c->slit ? c->d_planes : nullptr;
    xy.K = 4.0 * kPi * c->lB; xy.nx = c->nx; xy.ny = c->ny; xy.nplanes = c->nzf;
    if (in_lds) {
        xy.q = c->q; xy.in = nullptr; xy.out = a;
        if ((rc = c->hip(launch_spec_xy(xy, true, c->stream), "spec_xy"))) return rc;
    } else if (c->sp_fx) {
        if ((rc = fft_x(c, c->q, b, false, true)) || (rc = fft_y(c, b, a, false))) return rc;
    } else {
        // b = -K (q + lump) formed by the x product as it loads q; its projection onto zero
        // channel mean acts on the constant mode only, which the z solve projects
        if ((rc = spec_x(c, c->q, b, false, true))) return rc;
        if ((rc = spec_left(c, c->sp_ty, c->ny, c->nx, c->nzf, b, a, false, "gemm(y)"))) return rc;
    }
    if (c->slit) {
        int longest = 0;
        for (int w : c->ch_width) longest = std::max(longest, w);
        if (longest <= (int)TRI_LDS_MAX)
            rc = c->hip(launch_tridiag_lds(a, c->sp_piv, c->sp_pmid, b, nxy, c->sp_seg, c->nch, (uint32_t)longest,
                                           c->stream),
                        "tridiag_lds");
        else
            rc = c->hip(launch_tridiag_z(a, c->sp_piv, c->sp_piv_end, b, nxy, c->sp_seg, c->nch, c->stream), "tridiag_z");
        if (rc) return rc;
    } else {
        if ((rc = c->sp_fz ? fft_z(c, a, b, false) : spec_left(c, c->sp_tz, c->nzf, nxy, 1, a, b, false, "gemm(z)")))
            return rc;
        if ((rc = c->hip(launch_spectral_scale(b, c->sp_mu, c->sp_mu + c->nx, c->sp_mu + c->nx + c->ny, c->nx,
                                               c->ny, c->Nf, c->stream), "spectral_scale")))
            return rc;
        if ((rc = c->sp_fz ? fft_z(c, b, a, true) : spec_left(c, c->sp_tz, c->nzf, nxy, 1, b, a, true, "gemm(z)")))
            return rc;
        std::swap(a, b);
    }
    if (in_lds) {
        xy.q = nullptr; xy.in = b; xy.out = c->psi;
        return c->hip(launch_spec_xy(xy, false, c->stream), "spec_xy");
    }
    if (c->sp_fx) {
        if ((rc = fft_y(c, b, a, true))) return rc;
        return fft_x(c, a, c->psi, true);
    }
    if ((rc = spec_left(c, c->sp_ty, c->ny, c->nx, c->nzf, b, a, true, "gemm(y)"))) return rc;
    return spec_x(c, a, c->psi, true);
}

// Warm start psi(t-1) + psi(t-2) - psi(t-3) once three solutions exist (exact for a linear
// trend plus a period-two oscillation in time); before that, the previous potential.
int extrapolated_guess(lbmix_ctx *c) {
    int rc;
    const size_t bytes = (size_t)c->Nf * sizeof(double);
    if (!c->psi_prev) {
        if ((rc = c->hip(hipMalloc((void **)&c->psi_prev, 2 * bytes), "hipMalloc(psi_prev)"))) return rc;
        c->have_prev = 0;
    }
    double *p1 = c->psi_prev, *p2 = c->psi_prev + c->Nf;
    if (c->have_prev >= 2) return c->hip(launch_extrapolate(c->psi, p1, p2, c->Nf, c->stream), "extrapolate");
    // history not complete: shift it, keep the previous potential as the guess
    if (c->have_prev == 1 &&
        (rc = c->hip(hipMemcpyAsync(p2, p1, bytes, hipMemcpyDeviceToDevice, c->stream), "copy psi")))
        return rc;
    if ((rc = c->hip(hipMemcpyAsync(p1, c->psi, bytes, hipMemcpyDeviceToDevice, c->stream), "copy psi"))) return rc;
    c->have_prev++;
    return LBMIX_OK;
}

int ensure_ws_buffers(lbmix_ctx *c) {
    if (c->ws_r) return LBMIX_OK;
    const size_t N = c->Nf;
    int rc;
    if ((rc = c->hip(hipMalloc((void **)&c->ws_r, N * sizeof(double)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_c, N * sizeof(double)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_guess, N * sizeof(double)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_scale, sizeof(double)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_x, WS_CHANNELS * N * sizeof(float)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_y, N * sizeof(float)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_t, N * sizeof(float)), "hipMalloc(warm start)")) ||
        (rc = c->hip(hipMalloc((void **)&c->ws_mask, (size_t)c->nzf * sizeof(float)), "hipMalloc(warm start)")))
        return rc;
    std::vector<float> mask(c->nzf, 0.0f);   // second input channel: planes next to a wall
    if (c->slit)
        for (int ch = 0; ch < c->nch; ++ch) {
            mask[c->ch_first[ch]] = 1.0f;
            mask[c->ch_first[ch] + c->ch_width[ch] - 1] = 1.0f;
        }
    return c->hip(hipMemcpy(c->ws_mask, mask.data(), mask.size() * sizeof(float), hipMemcpyHostToDevice),
                  "copy mask");
}

// The coarse-grid part of A^-1 r for the network's input, which a 3 x 3 x 3 network of a few
// layers cannot form itself (the inverse of the operator is global): r restricted down the
// multigrid hierarchy, the coarse end solved as in a V-cycle, the result interpolated back to
// the fluid nodes without smoothing on the way up (into ws_c).
int coarse_correction(lbmix_ctx *c) {
    int rc;
    if ((rc = mg_build(c))) return rc;
    const int nl = (int)c->mg.size();
    if ((rc = c->hip(hipMemsetAsync(c->ws_c, 0, (size_t)c->Nf * sizeof(double), c->stream), "hipMemset(ws_c)")))
        return rc;
    if (nl < 2) return LBMIX_OK;
    std::vector<MGLevel> lev(c->mg);
    lev[0].e = c->ws_c;
    lev[0].r = c->ws_r;
    // the levels from lb down are solved together in one work-group (as in the V-cycle); a
    // channel stack relaxes z lines down to one column per channel, where that is exact
    int lb = nl;
    if (!c->mg_lines) {
        for (int l = 1; l < nl; ++l)
            if ((size_t)lev[l].nx * lev[l].ny * lev[l].nz <= kBottomCells) { lb = l; break; }
        size_t cells = 0;
        for (int l = lb; l < nl; ++l) cells += (size_t)lev[l].nx * lev[l].ny * lev[l].nz;
        if (lb < nl && (nl - lb > MG_MAX_BOTTOM || cells > (size_t)MG_BOTTOM_LDS)) lb = nl;
    }
    const int top = lb < nl ? lb : nl - 1;   // the first level not on the way down
    for (int l = 0; l < top; ++l)
        if ((rc = c->hip(launch_mg_restrict(lev[l], lev[l + 1], c->stream), "mg_restrict"))) return rc;
    if (lb < nl) {
        MGBottom bb{};
        bb.n = nl - lb;
        for (int l = lb; l < nl; ++l) bb.lev[l - lb] = lev[l];
        const MGLevel &B = lev[nl - 1];
        bb.coarse_sweeps = std::max(20, 4 * (int)std::max(B.nx, std::max(B.ny, B.nz)));
        bb.coarse_inv = c->mg_cinv;
        if ((rc = c->hip(launch_mg_bottom(bb, c->stream), "mg_bottom"))) return rc;
    } else {
        const MGLevel &B = lev[nl - 1];
        const bool exact = c->mg_lines && B.nx == 1 && B.ny == 1;
        const int count = exact ? 1 : std::max(20, 4 * (int)std::max(B.nx, std::max(B.ny, B.nz)));
        for (int k = 0; k < count; ++k)
            for (int col = 0; col < 2; ++col) {
                if (c->mg_lines) {
                    if ((rc = c->hip(launch_mg_line_rhs(B, col, c->stream), "mg_line_rhs")) ||
                        (rc = c->hip(launch_mg_line_solve(B, col, c->mg_idn[nl - 1], c->mg_pmid[nl - 1], c->d_first,
                                                          (uint32_t)c->nch, c->stream),
                                     "mg_line_solve")))
                        return rc;
                } else if ((rc = c->hip(launch_mg_smooth(B, col, c->stream), "mg_smooth"))) {
                    return rc;
                }
            }
    }
    for (int l = top - 1; l >= 0; --l)
        if ((rc = c->hip(launch_mg_prolong(lev[l], lev[l + 1], c->stream), "mg_prolong"))) return rc;
    return LBMIX_OK;
}

// Network input after the extrapolation (history complete): the residual of the guess, its
// coarse-grid solution, the last two increments of the potential (psi(t-1) - psi(t-2),
// psi(t-2) - psi(t-3) = guess - psi(t-1)), all over s = rms(r), and the wall mask.
int net_sample_input(lbmix_ctx *c, const PoissonArgs &pa) {
    int rc = ensure_ws_buffers(c);
    if (rc) return rc;
    uint32_t nb = 0;
    if ((rc = c->hip(launch_residual_field(pa, c->ws_r, c->partials, &nb, c->stream), "residual_field")) ||
        (rc = c->hip(launch_finalize(c->partials, nb, 1, c->ws_scale, 0, 0.0, 0.0, 1.0, c->stream), "finalize")) ||
        (rc = c->hip(launch_finish_scale(c->ws_scale, c->Nf, c->stream), "finish_scale")) ||
        (rc = coarse_correction(c)))
        return rc;
    return c->hip(launch_net_input(c->ws_r, c->ws_c, c->psi_prev, c->psi_prev + c->Nf, c->psi, c->ws_scale, c->ws_x,
                                   (uint32_t)c->nx * c->ny, (uint32_t)c->nzf, c->ws_mask, c->stream),
                  "net_input");
}

// Learned warm start: psi += s net(r / s, mask) on top of the extrapolated guess.
int learned_correction(lbmix_ctx *c, const PoissonArgs &pa) {
    int rc = net_sample_input(c, pa);
    if (rc) return rc;
    if ((rc = net_forward(c->ws_net, c->ws_x, c->ws_y, c->nx, c->ny, c->nzf, c->slit ? 1 : 0, c->stream)))
        return c->fail(rc, "warm-start network: %s", lbmix_net_last_error(c->ws_net));
    const double alpha = net_output_scale(c->ws_net) > 0.0 ? net_output_scale(c->ws_net) : 1.0;
    return c->hip(launch_add_correction(c->psi, c->ws_y, c->ws_scale, alpha, c->Nf, c->stream), "add_correction");
}

// Poisson solve of the charge in c->q into c->psi (warm start), then zero-mean gauge.
int finish_zero_rhs(lbmix_ctx *c) {   // b == 0: the solution is psi = 0
    int rc = c->hip(hipMemsetAsync(c->psi, 0, (size_t)c->Nf * sizeof(double), c->stream), "hipMemset(psi)");
    if (rc) return rc;
    c->last_resid = 0.0;
    c->last_sweeps = 0;
    c->last_status = LBMIX_OK;
    c->resid_on_device = false;
    c->solves++;
    c->psi_valid = true;
    return LBMIX_OK;
}

// Relative residual from the norms in dred[4..5] (fetched), or -1 when b == 0.
double fetched_residual(lbmix_ctx *c) {
    const double r2 = c->hred[4], b2 = c->hred[5];
    return b2 == 0.0 ? -1.0 : std::sqrt(r2 / b2);
}

int solve(lbmix_ctx *c) {
    int rc = LBMIX_OK;
    const PoissonArgs pa = c->pargs();
    if (c->poisson_method == 2) {
        // direct: exact to rounding, the gauge is part of it; the residual norms of every
        // check_every-th solve stay on the device for the stats
        if ((rc = spec_solve(c, pa))) return rc;
        if (c->direct_count++ % c->sor_check == 0) {
            if ((rc = channel_means(c, c->q, 0, 0)) || (rc = residual(c, pa))) return rc;
            c->resid_on_device = true;
        }
        c->last_sweeps = 1;
        c->last_status = LBMIX_OK;
        c->total_sweeps += 1;
        c->solves++;
        c->psi_valid = true;
        return LBMIX_OK;
    }
    if ((rc = channel_means(c, c->q, 0, 0))) return rc;
    if (c->warm_start >= 1 && c->psi_valid) {
        const bool history = c->have_prev >= 2;   // the extrapolation below is the full one
        if ((rc = extrapolated_guess(c))) return rc;
        if (c->warm_start == 2 && history && (rc = learned_correction(c, pa))) return rc;
    }
    int work = 0, status = LBMIX_OK;
    if (c->poisson_method == 1) {
        // multigrid: each V-cycle is one graph replay that also leaves the residual norms of
        // its result in dred[4..7]; the first (previous count - 1) cycles run without reading
        // them back, since they are expected to be needed
        if ((rc = mg_build(c))) return rc;
        if ((rc = c->hip(launch_make_rhs(pa, c->mg_b, c->stream), "make_rhs"))) return rc;
        if (c->sor_tol > 0.0) {
            const int blind = std::min(std::max(0, c->mg_last - 1), c->sor_max);
            double res;
            if (blind == 0) {
                if ((rc = residual(c, pa)) || (rc = fetch(c, 8))) return rc;
            } else {
                for (int k = 0; k < blind; ++k)
                    if ((rc = mg_cycle(c, pa))) return rc;
                work = blind;
                if ((rc = fetch(c, 8))) return rc;
            }
            res = fetched_residual(c);
            if (res < 0.0) return finish_zero_rhs(c);
            while (res > c->sor_tol) {
                if (work >= c->sor_max) {
                    status = LBMIX_ENOCONV;
                    break;
                }
                if ((rc = mg_cycle(c, pa)) || (rc = fetch(c, 8))) return rc;
                ++work;
                res = fetched_residual(c);
            }
            c->last_resid = res;
            c->mg_last = work;
            c->resid_on_device = false;
        } else {
            for (int k = 0; k < c->sor_max; ++k)
                if ((rc = mg_cycle(c, pa))) return rc;
            work = c->sor_max;
            c->resid_on_device = true;
        }
    } else {
        auto sweeps = [&](int count) -> int {
            for (int k = 0; k < count; ++k) {
                int r = c->hip(launch_sor(pa, 0, c->stream), "sor(red)");
                if (r) return r;
                if ((r = c->hip(launch_sor(pa, 1, c->stream), "sor(black)"))) return r;
            }
            return LBMIX_OK;
        };
        if (c->sor_tol > 0.0) {
            for (;;) {
                if ((rc = residual(c, pa)) || (rc = fetch(c, 8))) return rc;
                const double res = fetched_residual(c);
                if (res < 0.0) return finish_zero_rhs(c);
                c->last_resid = res;
                if (res <= c->sor_tol) break;
                if (work >= c->sor_max) {
                    status = LBMIX_ENOCONV;
                    break;
                }
                const int todo = std::min(c->sor_check, c->sor_max - work);
                if ((rc = sweeps(todo))) return rc;
                work += todo;
            }
            c->resid_on_device = false;
        } else {
            if ((rc = sweeps(c->sor_max))) return rc;
            work = c->sor_max;
            if ((rc = residual(c, pa))) return rc;
            c->resid_on_device = true;
        }
    }
    // zero-mean gauge per channel
    if ((rc = channel_means(c, c->psi, 1, c->nch))) return rc;
    rc = c->hip(launch_shift_planes(c->psi, (uint32_t)c->nx * c->ny, c->Nf, c->slit ? c->d_planes : nullptr,
                                    c->d_chan + c->nch, c->stream),
                "shift(psi)");
    if (rc) return rc;
    c->last_sweeps = work;
    c->last_status = status;
    c->total_sweeps += work;
    c->solves++;
    c->psi_valid = true;
    return status;
}

// A step needs no host decision when there is no Poisson solve or it is the direct one.
bool step_capturable(const lbmix_ctx *c) { return !c->charged() || c->poisson_method == 2; }

// Capture the step that reads buffer `par`: fused step, direct solve, step count + 1.
int capture_step(lbmix_ctx *c, int par) {
    int rc;
    if (!c->cap_stream &&
        (rc = c->hip(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate")))
        return rc;
    if (!c->step_dev && (rc = c->hip(hipMalloc((void **)&c->step_dev, sizeof(unsigned long long)), "hipMalloc(step)")))
        return rc;
    const bool charged = c->charged(), field = c->field();
    if (charged && (rc = spec_build(c))) return rc;   // allocations stay out of the capture
    const int save_cur = c->cur;
    hipStream_t save = c->stream;
    c->cur = par;
    c->stream = c->cap_stream;
    if ((rc = c->hip(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "capture"))) {
        c->cur = save_cur;
        c->stream = save;
        return rc;
    }
    StepArgs a = c->args();
    a.step_dev = c->step_dev;
    int r1 = c->hip(collide(c, a, field, charged, c->cap_stream), "stream_collide");
    if (!r1 && charged) {
        c->cur = par ^ 1;   // the solve sees the state the step writes (q is written by the step)
        r1 = spec_solve(c, c->pargs());
    }
    if (!r1) r1 = c->hip(launch_advance_step(c->step_dev, c->cap_stream), "advance_step");
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->cur = save_cur;
    c->stream = save;
    if (r1) {
        if (g) (void)hipGraphDestroy(g);
        return r1;
    }
    if ((rc = c->hip(e, "hipStreamEndCapture"))) return rc;
    c->sgraph[par] = g;
    return c->hip(hipGraphInstantiate(&c->sexec[par], g, nullptr, nullptr, 0), "hipGraphInstantiate");
}

int initial_potential(lbmix_ctx *c) {
    int rc = ensure_field_buffers(c);
    if (rc) return rc;
    const StepArgs a = c->args();
    rc = c->hip(launch_charge(c->st, c->slit, c->ns, a, c->q, c->stream), "charge");
    if (rc) return rc;
    rc = solve(c);
    return rc == LBMIX_ENOCONV ? LBMIX_OK : rc;
}

int check_ready(lbmix_ctx *c) {
    if (!c) return LBMIX_EINVAL;
    if (c->ns == 0) return c->fail(LBMIX_ESTATE, "no species");
    for (int s = 0; s < c->ns; ++s)
        if (!c->set[s]) return c->fail(LBMIX_ESTATE, "species %d has no state (lbmix_set_state)", s);
    return LBMIX_OK;
}

bool redblack_extents(const lbmix_ctx *c) {
    auto bad_extent = [](int n) { return n > 1 && (n % 2) != 0; };
    return !(bad_extent(c->nx) || bad_extent(c->ny) || (!c->slit && bad_extent(c->nz)));   // walls cut z
}

int validate_start(lbmix_ctx *c) {
    if (c->pair_ns && c->pair_ns != c->ns)
        return c->fail(LBMIX_EINVAL, "the pair drag matrix was set for %d species, the lattice has %d", c->pair_ns, c->ns);
    if (c->forcing == 1 && c->pair_ns >= 3)
        return c->fail(LBMIX_EINVAL, "the Guo-type forcing variant has one drag frequency; it excludes a pair drag matrix");
    bool context_drag_used = false;   // by a channel without a drag of its own
    for (int ch = 0; ch < c->nch; ++ch) context_drag_used = context_drag_used || !(c->ch_tau_d[ch] > 0.0);
    if (c->forcing == 1 && c->pair_ns == 0 && c->drag_from_sc && context_drag_used && !(c->omega_drag() < 2.0))
        return c->fail(LBMIX_EINVAL, "with the Guo-type variant, Sc = %g needs tau_visc > 1/2 + Sc / 2", c->sc);
    for (int ch = 0; c->pair_ns && ch < c->nch; ++ch)
        if (c->ch_tau_d[ch] > 0.0)
            return c->fail(LBMIX_EINVAL, "channel %d has its own drag; a pair drag matrix applies to all channels", ch);
    if (!c->charged()) return LBMIX_OK;
    if (c->poisson_method != 2 && !redblack_extents(c))
        return c->fail(LBMIX_EINVAL, "charged runs need even periodic extents (or 1) for red-black SOR and "
                                     "multigrid (the direct solve takes any)");
    const double area = (double)c->nx * c->ny;
    for (int ch = 0; ch < c->nch; ++ch) {   // every channel is neutral on its own
        double qtot = 0.0, scale = 0.0;
        for (int s = 0; s < c->ns; ++s) {
            const double t = c->ch_total[(size_t)s * c->nch + ch];
            qtot += c->valence[s] * t;
            scale += std::fabs((double)c->valence[s]) * t;
        }
        const double lo = c->slit ? c->ch_sig_lo[ch] : 0.0, hi = c->slit ? c->ch_sig_hi[ch] : 0.0;
        const double wall = (lo + hi) * area;
        scale = std::max(scale, (std::fabs(lo) + std::fabs(hi)) * area);
        if (std::fabs(qtot + wall) > 1e-9 * scale)
            return c->fail(LBMIX_EINVAL, "channel %d is not neutral: fluid charge %.17g, wall charge %.17g", ch, qtot,
                           wall);
    }
    return LBMIX_OK;
}

struct Guard {   // make the context's device current for the duration of a call
    int prev = -1;
    explicit Guard(const lbmix_ctx *c) {
        if (c && c->allocated && hipGetDevice(&prev) == hipSuccess && prev != c->device)
            (void)hipSetDevice(c->device);
        else
            prev = -1;
    }
    ~Guard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Header {
    char magic[8];
    int32_t version, nx, ny, nz, geometry, storage, ns, nch, valence[MAXS];
    double rho0[MAXS], rel_range[MAXS], host_total[MAXS];
    double tau_v, tau_d, sc;
    int32_t drag_from_sc, sor_max, sor_check, psi_valid, rounding, poisson_method;
    uint64_t round_seed;
    double lB, sig_lo, sig_hi, E[3], sor_tol, sor_omega;
    int64_t steps;
    int32_t pair_ns, forcing;
    double tau_pair[MAXS * MAXS];
    int32_t wide, pad;
};

}  // namespace

// =======================================================================================
// C ABI

extern "C" {

int lbmix_version(void) { return 10000; }

}  // extern "C"

namespace {

// Context of nx * ny lateral nodes and channels of the given fluid widths along z (walls
// around each), or one periodic box of widths[0] planes.
int create_ctx(lbmix_ctx **out, int nx, int ny, int geometry, const std::vector<int> &widths, int storage,
               void *hip_stream) {
    if (!out) return LBMIX_EINVAL;
    *out = nullptr;
    if (nx < 1 || ny < 1 || widths.empty()) return LBMIX_EINVAL;
    if (storage < LBMIX_F64 || storage > LBMIX_F16_SHIFTED) return LBMIX_EINVAL;
    const bool walls = geometry != LBMIX_PERIODIC;
    double nz = 0, nzf = 0;
    for (int w : widths) {
        if (w < 1) return LBMIX_EINVAL;
        nz += w + (walls ? 2 : 0);
        nzf += w;
    }
    if ((double)nx * ny * nz > 2147483647.0) return LBMIX_EINVAL;
    // the fused step addresses the populations of a plane (all slots) with 32-bit byte offsets
    const double ebytes = storage == LBMIX_F64 ? 8.0 : (storage <= LBMIX_F32_SHIFTED ? 4.0 : 2.0);
    if ((double)nx * ny * Q * MAXS * ebytes >= 4294967296.0) return LBMIX_EINVAL;
    lbmix_ctx *c = new (std::nothrow) lbmix_ctx();
    if (!c) return LBMIX_ENOMEM;
    c->nx = nx;
    c->ny = ny;
    c->nz = (int)nz;
    c->nzf = (int)nzf;
    c->geometry = geometry;
    c->slit = walls;
    c->nch = (int)widths.size();
    c->ch_width = widths;
    int f = 0, full = 0;
    for (int w : widths) {
        c->ch_first.push_back(f);
        c->ch_full.push_back(full);
        f += w;
        full += w + (walls ? 2 : 0);
    }
    c->ch_tau_d.assign(c->nch, 0.0);
    c->ch_sig_lo.assign(c->nch, 0.0);
    c->ch_sig_hi.assign(c->nch, 0.0);
    c->ch_total.assign((size_t)MAXS * c->nch, 0.0);
    c->storage = storage;
    switch (storage) {
        case LBMIX_F64: c->st = Store::F64; c->esize = 8; break;
        case LBMIX_F32:
        case LBMIX_F32_SHIFTED: c->st = Store::F32; c->esize = 4; break;
        case LBMIX_BF16_SHIFTED: c->st = Store::BF16; c->esize = 2; break;
        default: c->st = Store::F16; c->esize = 2; break;
    }
    c->Nf = (uint32_t)((size_t)nx * ny * c->nzf);
    c->Nfull = (size_t)nx * ny * c->nz;
    c->stream = static_cast<hipStream_t>(hip_stream);
    for (int s = 0; s < MAXS; ++s) c->rel_range[s] = 0.1;
    c->compute_scales();
    *out = c;
    return LBMIX_OK;
}

}  // namespace

extern "C" {

int lbmix_create(lbmix_ctx **out, int nx, int ny, int nz, int geometry, int storage, void *hip_stream) {
    if (out) *out = nullptr;
    if (geometry != LBMIX_PERIODIC && geometry != LBMIX_SLIT_Z) return LBMIX_EINVAL;
    if (nz < (geometry == LBMIX_SLIT_Z ? 3 : 1)) return LBMIX_EINVAL;
    return create_ctx(out, nx, ny, geometry, {geometry == LBMIX_SLIT_Z ? nz - 2 : nz}, storage, hip_stream);
}

int lbmix_create_channels(lbmix_ctx **out, int nx, int ny, int nchannels, const int *widths, int storage,
                          void *hip_stream) {
    if (out) *out = nullptr;
    if (nchannels < 1 || !widths) return LBMIX_EINVAL;
    return create_ctx(out, nx, ny, LBMIX_CHANNELS, std::vector<int>(widths, widths + nchannels), storage,
                      hip_stream);
}

int lbmix_set_channel(lbmix_ctx *c, int channel, double tau_drag, double sigma_lo, double sigma_hi) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (c->geometry != LBMIX_CHANNELS) return c->fail(LBMIX_EINVAL, "not a channel stack (lbmix_create_channels)");
    if (channel < 0 || channel >= c->nch) return c->fail(LBMIX_EINVAL, "bad channel index");
    if (!std::isfinite(tau_drag) || (tau_drag > 0.0 && !(tau_drag > 0.5)) || !std::isfinite(sigma_lo) ||
        !std::isfinite(sigma_hi))
        return c->fail(LBMIX_EINVAL, "bad channel parameters (tau_drag > 1/2, or <= 0 for the context's)");
    c->ch_tau_d[channel] = tau_drag > 0.0 ? tau_drag : 0.0;
    c->ch_sig_lo[channel] = sigma_lo;
    c->ch_sig_hi[channel] = sigma_hi;
    c->tables_dirty = true;
    c->psi_valid = false;
    return LBMIX_OK;
}

int lbmix_add_species(lbmix_ctx *c, double rho0, int valence, int *id_out) {
    if (!c) return LBMIX_EINVAL;
    if (c->allocated) return c->fail(LBMIX_ESTATE, "species must be added before the first set_state");
    if (c->ns >= MAXS) return c->fail(LBMIX_EINVAL, "at most %d species", MAXS);
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) return c->fail(LBMIX_EINVAL, "rho0 must be positive");
    c->rho0[c->ns] = rho0;
    c->valence[c->ns] = valence;
    if (id_out) *id_out = c->ns;
    c->ns++;
    c->compute_scales();
    return LBMIX_OK;
}

int lbmix_set_tau_visc(lbmix_ctx *c, double tau) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (!(tau > 0.5) || !std::isfinite(tau)) return c->fail(LBMIX_EINVAL, "tau_visc must exceed 1/2");
    c->tau_v = tau;
    c->tables_dirty = true;
    return LBMIX_OK;
}

int lbmix_set_tau_drag(lbmix_ctx *c, double tau) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (!(tau > 0.5) || !std::isfinite(tau)) return c->fail(LBMIX_EINVAL, "tau_drag must exceed 1/2");
    c->tau_d = tau;
    c->drag_from_sc = false;
    c->tables_dirty = true;
    return LBMIX_OK;
}

int lbmix_set_schmidt(lbmix_ctx *c, double sc) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (!(sc > 0.0) || !std::isfinite(sc)) return c->fail(LBMIX_EINVAL, "Schmidt number must be positive");
    c->sc = sc;
    c->drag_from_sc = true;
    c->tables_dirty = true;
    return LBMIX_OK;
}

int lbmix_set_drag_pairs(lbmix_ctx *c, const double *tau) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (!tau) {
        c->pair_ns = 0;
        c->tables_dirty = true;
        return LBMIX_OK;
    }
    const int ns = c->ns;
    if (ns < 2) return c->fail(LBMIX_EINVAL, "a pair drag matrix needs at least two species");
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            if (a == b) continue;
            const double t = tau[a * ns + b], u = tau[b * ns + a];
            if (!std::isfinite(t) || !(t > 0.5) || std::fabs(t - u) > 1e-12 * std::fabs(t))
                return c->fail(LBMIX_EINVAL, "pair drag times must be symmetric and exceed 1/2 (pair %d, %d)", a, b);
        }
    for (int a = 0; a < MAXS; ++a)
        for (int b = 0; b < MAXS; ++b) c->tau_pair[a][b] = (a < ns && b < ns) ? tau[a * ns + b] : 0.0;
    c->pair_ns = ns;
    c->tables_dirty = true;
    return LBMIX_OK;
}

int lbmix_set_forcing(lbmix_ctx *c, int scheme) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (scheme != LBMIX_FORCING_PAPER && scheme != LBMIX_FORCING_GUO)
        return c->fail(LBMIX_EINVAL, "unknown forcing scheme %d", scheme);
    c->forcing = scheme;
    return LBMIX_OK;
}

int lbmix_set_electrostatics(lbmix_ctx *c, double bjerrum, double sigma_lo, double sigma_hi, const double *E) {
    if (!c) return LBMIX_EINVAL;
    if (c->started) return c->fail(LBMIX_ESTATE, "parameters are fixed once stepping has started");
    if (!(bjerrum >= 0.0) || !std::isfinite(bjerrum) || !std::isfinite(sigma_lo) || !std::isfinite(sigma_hi))
        return c->fail(LBMIX_EINVAL, "bad electrostatic parameters");
    if (E)
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(E[d])) return c->fail(LBMIX_EINVAL, "bad field");
    drop_graph(c);
    c->lB = bjerrum;
    c->sig_lo = sigma_lo;
    c->sig_hi = sigma_hi;
    if (c->geometry == LBMIX_SLIT_Z) {
        c->ch_sig_lo[0] = sigma_lo;
        c->ch_sig_hi[0] = sigma_hi;
    }
    c->tables_dirty = true;
    for (int d = 0; d < 3; ++d) c->E[d] = E ? E[d] : 0.0;
    c->psi_valid = false;
    return LBMIX_OK;
}

int lbmix_set_poisson(lbmix_ctx *c, double rel_tol, int max_sweeps, int check_every, double omega_sor) {
    if (!c) return LBMIX_EINVAL;
    if (!(rel_tol >= 0.0) || max_sweeps < 1 || check_every < 1 || !(omega_sor < 2.0))
        return c->fail(LBMIX_EINVAL, "bad Poisson parameters");
    drop_graph(c);
    c->sor_tol = rel_tol;
    c->sor_max = max_sweeps;
    c->sor_check = check_every;
    c->sor_omega = omega_sor;
    return LBMIX_OK;
}

int lbmix_set_poisson_method(lbmix_ctx *c, int method) {
    if (!c) return LBMIX_EINVAL;
    if (method < 0 || method > 2) return c->fail(LBMIX_EINVAL, "Poisson method is 0 (SOR), 1 (multigrid) or 2 (direct)");
    if (c->started && method != 2 && c->charged() && !redblack_extents(c))
        return c->fail(LBMIX_EINVAL, "SOR and multigrid need even periodic extents (or 1)");
    drop_graph(c);
    c->poisson_method = method;
    return LBMIX_OK;
}

int lbmix_set_poisson_warm_start(lbmix_ctx *c, int mode) {
    if (!c) return LBMIX_EINVAL;
    if (mode < 0 || mode > 2)
        return c->fail(LBMIX_EINVAL, "warm start is 0 (previous), 1 (extrapolated) or 2 (learned)");
    if (mode == 2 && !c->ws_net) return c->fail(LBMIX_EINVAL, "the learned warm start needs lbmix_set_warm_start_net");
    c->warm_start = mode;
    c->have_prev = 0;
    return LBMIX_OK;
}

int lbmix_set_warm_start_net(lbmix_ctx *c, lbmix_net *net) {
    if (!c) return LBMIX_EINVAL;
    if (net && net_in_channels(net) != WS_CHANNELS)
        return c->fail(LBMIX_EINVAL, "the warm-start network takes %d input channels", WS_CHANNELS);
    if (net && c->allocated && net_device(net) != c->device)
        return c->fail(LBMIX_EINVAL, "the network lives on device %d, the lattice on %d", net_device(net), c->device);
    if (!net && c->warm_start == 2) c->warm_start = 1;
    c->ws_net = net;
    return LBMIX_OK;
}

int lbmix_train_warm_start(lbmix_ctx *c, lbmix_net *net, int nsteps, float lr, double *losses) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!net || net_in_channels(net) != WS_CHANNELS || nsteps < 0 || !(lr > 0.0f))
        return c->fail(LBMIX_EINVAL, "training needs a %d-channel network, nsteps >= 0 and lr > 0", WS_CHANNELS);
    if (!c->charged()) return c->fail(LBMIX_EINVAL, "no charged species: there is no Poisson solve to learn");
    if (c->latched) return c->fail(c->latched, "context latched an earlier error (%d)", c->latched);
    Guard g(c);
    if ((rc = ensure_tables(c))) return rc;
    if (!c->started) {
        if ((rc = validate_start(c))) return rc;
        c->started = true;
    }
    if (!c->psi_valid && (rc = initial_potential(c))) return rc;
    const bool field = c->field();
    for (int k = 0; k < nsteps; ++k) {
        const StepArgs a = c->args();
        if ((rc = c->hip(collide(c, a, field, true, c->stream), "stream_collide")))
            return rc;
        c->cur ^= 1;
        c->steps++;
        // sample: the residual of the extrapolated guess and the exact correction to it (once
        // the history is complete; before that the step only solves)
        const PoissonArgs pa = c->pargs();
        const bool history = c->have_prev >= 2;
        if ((rc = channel_means(c, c->q, 0, 0)) || (rc = extrapolated_guess(c))) return rc;
        if (!history) {
            if ((rc = spec_solve(c, pa))) return rc;
            c->solves++;
            c->total_sweeps++;
            if (losses) losses[k] = 0.0;
            continue;
        }
        if ((rc = net_sample_input(c, pa))) return rc;
        if ((rc = c->hip(hipMemcpyAsync(c->ws_guess, c->psi, (size_t)c->Nf * sizeof(double), hipMemcpyDeviceToDevice,
                                        c->stream),
                         "copy guess")))
            return rc;
        if ((rc = spec_solve(c, pa))) return rc;
        c->solves++;
        c->total_sweeps++;
        c->last_sweeps = 1;
        if (!(net_output_scale(net) > 0.0)) {
            // output scale of a fresh network: the root mean square of its first target
            double rms = 0.0;
            if ((rc = c->hip(launch_correction_target(c->psi, c->ws_guess, c->ws_scale, 1.0, c->ws_t, c->Nf, c->stream),
                             "correction_target")))
                return rc;
            if ((rc = net_rms(net, c->ws_t, c->Nf, &rms, c->stream))) return c->fail(rc, "%s", lbmix_net_last_error(net));
            net_set_output_scale(net, rms > 0.0 ? rms : 1.0);
        }
        if ((rc = c->hip(launch_correction_target(c->psi, c->ws_guess, c->ws_scale, net_output_scale(net), c->ws_t,
                                                  c->Nf, c->stream),
                         "correction_target")))
            return rc;
        double loss = 0.0;
        if ((rc = net_gradient(net, c->ws_x, c->ws_t, c->nx, c->ny, c->nzf, c->slit ? 1 : 0, losses ? &loss : nullptr,
                               c->stream)) ||
            (rc = net_adam(net, lr, c->stream)))
            return c->fail(rc, "training: %s", lbmix_net_last_error(net));
        if (losses) losses[k] = loss;
    }
    return LBMIX_OK;
}

int lbmix_set_rounding(lbmix_ctx *c, int mode, unsigned long long seed) {
    if (!c) return LBMIX_EINVAL;
    if (mode != 0 && mode != 1) return c->fail(LBMIX_EINVAL, "rounding mode is 0 or 1");
    if (mode == 1 && c->storage == LBMIX_F64)
        return c->fail(LBMIX_EINVAL, "stochastic rounding applies to the FP32 and 16-bit storage forms");
    if (c->started && mode != c->rounding)
        return c->fail(LBMIX_ESTATE, "the rounding mode is fixed once stepping has started");
    c->rounding = mode;
    c->round_seed = seed;
    return LBMIX_OK;
}

int lbmix_set_arithmetic(lbmix_ctx *c, int mode) {
    if (!c) return LBMIX_EINVAL;
    if (mode != 0 && mode != 1) return c->fail(LBMIX_EINVAL, "arithmetic mode is 0 or 1");
    if (c->started && mode != c->wide)
        return c->fail(LBMIX_ESTATE, "the arithmetic mode is fixed once stepping has started");
    c->wide = mode;
    return LBMIX_OK;
}

int lbmix_set_storage_range(lbmix_ctx *c, int species, double rel_range) {
    if (!c) return LBMIX_EINVAL;
    if (c->allocated) return c->fail(LBMIX_ESTATE, "the storage range is fixed at the first set_state");
    if (species < 0 || species >= c->ns || !(rel_range > 0.0) || !std::isfinite(rel_range))
        return c->fail(LBMIX_EINVAL, "bad species or range");
    c->rel_range[species] = rel_range;
    c->compute_scales();
    return LBMIX_OK;
}

int lbmix_set_state(lbmix_ctx *c, int s, const double *n, const double *u) {
    if (!c) return LBMIX_EINVAL;
    if (s < 0 || s >= c->ns || !n) return c->fail(LBMIX_EINVAL, "bad species index or null density");
    int rc = allocate(c);
    if (rc) return rc;
    Guard g(c);
    if ((rc = ensure_tables(c))) return rc;
    double tot = 0.0;
    const size_t plane = (size_t)c->nx * c->ny;
    for (int ch = 0; ch < c->nch; ++ch) {   // channel totals in plane order
        double t = 0.0;
        for (int k = 0; k < c->ch_width[ch]; ++k) {
            const size_t z = (size_t)(c->slit ? c->ch_full[ch] + 1 + k : c->ch_first[ch] + k);
            for (size_t i = 0; i < plane; ++i) t += n[z * plane + i];
        }
        c->ch_total[(size_t)s * c->nch + ch] = t;
        tot += t;
    }
    double *dn = nullptr, *du = nullptr;
    rc = c->hip(hipMalloc((void **)&dn, c->Nfull * sizeof(double)), "hipMalloc(staging)");
    if (rc) return rc;
    if (u) {
        rc = c->hip(hipMalloc((void **)&du, 3 * c->Nfull * sizeof(double)), "hipMalloc(staging)");
        if (rc) { (void)hipFree(dn); return rc; }
    }
    rc = c->hip(hipMemcpyAsync(dn, n, c->Nfull * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy n");
    if (!rc && u)
        rc = c->hip(hipMemcpyAsync(du, u, 3 * c->Nfull * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy u");
    if (!rc) {
        StepArgs a = c->args();
        a.fout = c->f[c->cur];
        rc = c->hip(launch_init(c->st, c->slit, s, a, dn, du, c->stream), "init_equilibrium");
    }
    if (!rc) rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    (void)hipFree(dn);
    if (du) (void)hipFree(du);
    if (rc) return rc;
    c->host_total[s] = tot;
    c->have_prev = 0;
    c->mg_last = 0;
    c->set[s] = true;
    c->started = false;
    c->psi_valid = false;
    c->steps = 0;
    c->latched = 0;
    return LBMIX_OK;
}

int lbmix_step(lbmix_ctx *c, int nsteps) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (nsteps < 0) return c->fail(LBMIX_EINVAL, "negative step count");
    if (c->latched) return c->fail(c->latched, "context latched an earlier error (%d)", c->latched);
    Guard g(c);
    if ((rc = ensure_tables(c))) return rc;
    if (!c->started) {
        if ((rc = validate_start(c))) return rc;
        c->started = true;
    }
    const bool charged = c->charged();
    if (charged && !c->psi_valid) {
        if ((rc = initial_potential(c))) return rc;
    }
    int status = LBMIX_OK;
    const bool field = c->field();
    if (c->use_graph && step_capturable(c) && nsteps > 0) {
        for (int par = 0; par < 2; ++par)
            if (!c->sexec[par] && (rc = capture_step(c, par))) return rc;
        if ((rc = c->hip(launch_set_step(c->step_dev, (unsigned long long)c->steps, c->stream), "set_step"))) return rc;
        for (int k = 0; k < nsteps; ++k) {
            if ((rc = c->hip(hipGraphLaunch(c->sexec[c->cur], c->stream), "hipGraphLaunch"))) return rc;
            c->cur ^= 1;
            c->steps++;
            if (charged) {
                c->solves++;
                c->total_sweeps++;
                c->last_sweeps = 1;
                c->last_status = LBMIX_OK;
                c->direct_count++;
            }
        }
        if (charged) {   // the residual of the last solve, for the stats
            const PoissonArgs pa = c->pargs();
            if ((rc = channel_means(c, c->q, 0, 0)) || (rc = residual(c, pa))) return rc;
            c->resid_on_device = true;
        }
        return LBMIX_OK;
    }
    for (int k = 0; k < nsteps; ++k) {
        const StepArgs a = c->args();
        rc = c->hip(collide(c, a, field, charged, c->stream), "stream_collide");
        if (rc) return rc;
        c->cur ^= 1;
        c->steps++;
        if (charged) {
            rc = solve(c);
            if (rc == LBMIX_ENOCONV)
                status = LBMIX_ENOCONV;
            else if (rc)
                return rc;
        }
    }
    if (status == LBMIX_ENOCONV)
        return c->fail(LBMIX_ENOCONV, "Poisson solve reached %d sweeps at residual %.3e", c->sor_max, c->last_resid);
    return LBMIX_OK;
}

int lbmix_set_step_graph(lbmix_ctx *c, int enable) {
    if (!c) return LBMIX_EINVAL;
    c->use_graph = enable ? 1 : 0;
    return LBMIX_OK;
}

int lbmix_autotune(lbmix_ctx *c, int reps) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (reps < 1) return c->fail(LBMIX_EINVAL, "reps must be positive");
    if (c->latched) return c->fail(c->latched, "context latched an earlier error (%d)", c->latched);
    Guard g(c);
    if ((rc = ensure_tables(c))) return rc;
    const bool charged = c->charged(), field = c->field();
    if (charged && (rc = ensure_field_buffers(c))) return rc;
    hipEvent_t e0, e1;
    if ((rc = c->hip(hipEventCreate(&e0), "hipEventCreate"))) return rc;
    if ((rc = c->hip(hipEventCreate(&e1), "hipEventCreate"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    // the launches read the current state and write the other buffer, which the next step
    // overwrites: the state does not advance.  Two sweeps over the candidates, the best time
    // of each kept; a candidate replaces the default shape only when it is faster by more
    // than 1.5 % (launch times of a bandwidth-bound kernel vary by about that much)
    std::vector<std::pair<uint32_t, uint32_t>> cand = c->step_shapes();
    cand.insert(cand.begin(), {0u, 0u});
    std::vector<float> best_ms(cand.size(), -1.0f);
    for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
        for (size_t i = 0; i < cand.size() && !rc; ++i) {
            StepArgs a = c->args();
            a.block_x = cand[i].first;
            a.block_y = cand[i].second;
            rc = c->hip(collide(c, a, field, charged, c->stream), "stream_collide");
            if (!rc) rc = c->hip(hipEventRecord(e0, c->stream), "hipEventRecord");
            for (int k = 0; !rc && k < reps; ++k)
                rc = c->hip(collide(c, a, field, charged, c->stream),
                            "stream_collide");
            if (!rc) rc = c->hip(hipEventRecord(e1, c->stream), "hipEventRecord");
            if (!rc) rc = c->hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            if (!rc) rc = c->hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (!rc && (best_ms[i] < 0.0f || ms < best_ms[i])) best_ms[i] = ms;
        }
    }
    uint32_t bx = 0, by = 0;
    float best = best_ms[0];
    for (size_t i = 1; i < cand.size(); ++i)
        if (best_ms[i] >= 0.0f && best_ms[i] < 0.985f * best_ms[0] && best_ms[i] < best) {
            best = best_ms[i];
            bx = cand[i].first;
            by = cand[i].second;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (bx != c->blk_x || by != c->blk_y) drop_graph(c);   // captured steps hold the launch shape
    c->blk_x = bx;
    c->blk_y = by;
    return LBMIX_OK;
}

int lbmix_get_moments_device(lbmix_ctx *c, int s, double *n_dev, double *j_dev) {
    int rc = check_ready(c);
    if (rc) return rc;
    {
        Guard g0(c);
        if ((rc = ensure_tables(c))) return rc;
    }
    if (s < 0 || s >= c->ns) return c->fail(LBMIX_EINVAL, "bad species index");
    Guard g(c);
    const StepArgs a = c->args();
    if (!n_dev) {
        if (!j_dev) return LBMIX_OK;
        if ((rc = ensure_scratch(c, c->Nfull * sizeof(double)))) return rc;
        n_dev = c->scratch;
    }
    return c->hip(launch_moments(c->st, c->slit, s, a, n_dev, j_dev, c->stream), "moments");
}

int lbmix_get_moments(lbmix_ctx *c, int s, double *n_out, double *j_out) {
    int rc = check_ready(c);
    if (rc) return rc;
    {
        Guard g0(c);
        if ((rc = ensure_tables(c))) return rc;
    }
    if (s < 0 || s >= c->ns) return c->fail(LBMIX_EINVAL, "bad species index");
    Guard g(c);
    if ((rc = ensure_scratch(c, 4 * c->Nfull * sizeof(double)))) return rc;
    double *dn = c->scratch, *dj = c->scratch + c->Nfull;
    const StepArgs a = c->args();
    if ((rc = c->hip(launch_moments(c->st, c->slit, s, a, dn, dj, c->stream), "moments"))) return rc;
    if (n_out && (rc = c->hip(hipMemcpyAsync(n_out, dn, c->Nfull * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy n")))
        return rc;
    if (j_out && (rc = c->hip(hipMemcpyAsync(j_out, dj, 3 * c->Nfull * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy j")))
        return rc;
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

int lbmix_get_populations(lbmix_ctx *c, int s, double *f_out) {
    int rc = check_ready(c);
    if (rc) return rc;
    {
        Guard g0(c);
        if ((rc = ensure_tables(c))) return rc;
    }
    if (s < 0 || s >= c->ns || !f_out) return c->fail(LBMIX_EINVAL, "bad species index or null output");
    Guard g(c);
    if ((rc = ensure_scratch(c, (size_t)Q * c->Nfull * sizeof(double)))) return rc;
    const StepArgs a = c->args();
    if ((rc = c->hip(launch_populations(c->st, c->slit, s, a, c->scratch, c->stream), "populations"))) return rc;
    if ((rc = c->hip(hipMemcpyAsync(f_out, c->scratch, (size_t)Q * c->Nfull * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy f")))
        return rc;
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

int lbmix_get_potential(lbmix_ctx *c, double *psi_out) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!psi_out) return c->fail(LBMIX_EINVAL, "null output");
    Guard g(c);
    std::memset(psi_out, 0, c->Nfull * sizeof(double));
    if (!c->charged()) return LBMIX_OK;
    if ((rc = ensure_tables(c))) return rc;
    if (!c->psi_valid) {
        if (!c->started) {
            if ((rc = validate_start(c))) return rc;
        }
        if ((rc = initial_potential(c))) return rc;
    }
    const size_t plane = (size_t)c->nx * c->ny;
    for (int ch = 0; ch < c->nch; ++ch) {   // each channel's fluid planes into place
        const size_t zf = (size_t)c->ch_first[ch], zfull = (size_t)(c->slit ? c->ch_full[ch] + 1 : c->ch_first[ch]);
        if ((rc = c->hip(hipMemcpyAsync(psi_out + zfull * plane, c->psi + zf * plane,
                                        (size_t)c->ch_width[ch] * plane * sizeof(double), hipMemcpyDeviceToHost,
                                        c->stream),
                         "copy psi")))
            return rc;
    }
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

int lbmix_get_mass_totals(lbmix_ctx *c, double *totals) {
    int rc = check_ready(c);
    if (rc) return rc;
    {
        Guard g0(c);
        if ((rc = ensure_tables(c))) return rc;
    }
    if (!totals) return c->fail(LBMIX_EINVAL, "null output");
    Guard g(c);
    if ((rc = ensure_scratch(c, c->Nfull * sizeof(double)))) return rc;
    const StepArgs a = c->args();
    for (int s = 0; s < c->ns; ++s) {
        uint32_t nb = 0;
        if ((rc = c->hip(launch_moments(c->st, c->slit, s, a, c->scratch, nullptr, c->stream), "moments"))) return rc;
        if ((rc = c->hip(launch_qsum(c->scratch, (uint32_t)c->Nfull, c->partials, &nb, c->stream), "sum"))) return rc;
        if ((rc = c->hip(launch_finalize(c->partials, nb, 1, c->dred + 8 + s, 0, 0, 0, 1, c->stream), "finalize")))
            return rc;
    }
    if ((rc = c->hip(hipMemcpyAsync(c->hred, c->dred + 8, c->ns * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy")))
        return rc;
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    bool finite = true;
    for (int s = 0; s < c->ns; ++s) {
        totals[s] = c->hred[s];
        finite = finite && std::isfinite(totals[s]);
    }
    if (!finite) {
        c->latched = LBMIX_ENONFINITE;
        return c->fail(LBMIX_ENONFINITE, "non-finite mass total");
    }
    return LBMIX_OK;
}

int lbmix_get_step_mass(lbmix_ctx *c, double *totals) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!totals) return c->fail(LBMIX_EINVAL, "null output");
    if (c->part_nb == 0) return c->fail(LBMIX_ESTATE, "no step has run");
    Guard g(c);
    if ((rc = c->hip(launch_finalize(c->step_partials, c->part_nb, c->ns, c->dred + 8, 0, 0, 0, 1, c->stream),
                     "finalize")))
        return rc;
    if ((rc = c->hip(hipMemcpyAsync(c->hred, c->dred + 8, c->ns * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy")))
        return rc;
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    bool finite = true;
    for (int s = 0; s < c->ns; ++s) {
        totals[s] = c->hred[s] + c->rho_bar(s) * (double)c->Nf;
        finite = finite && std::isfinite(totals[s]);
    }
    if (!finite) {
        c->latched = LBMIX_ENONFINITE;
        return c->fail(LBMIX_ENONFINITE, "non-finite mass total");
    }
    return LBMIX_OK;
}

int lbmix_get_zprofiles(lbmix_ctx *c, double *out) {
    int rc = check_ready(c);
    if (rc) return rc;
    {
        Guard g0(c);
        if ((rc = ensure_tables(c))) return rc;
    }
    if (!out) return c->fail(LBMIX_EINVAL, "null output");
    Guard g(c);
    if ((rc = ensure_scratch(c, (4 * c->Nfull + 4 * (size_t)c->nz * MAXS) * sizeof(double)))) return rc;
    double *dn = c->scratch, *dj = c->scratch + c->Nfull, *dp = c->scratch + 4 * c->Nfull;
    const StepArgs a = c->args();
    for (int s = 0; s < c->ns; ++s) {
        if ((rc = c->hip(launch_moments(c->st, c->slit, s, a, dn, dj, c->stream), "moments"))) return rc;
        if ((rc = c->hip(launch_plane_sums(dn, dj, c->nx, c->ny, c->nz, dp + (size_t)s * 4 * c->nz, c->stream), "plane sums")))
            return rc;
    }
    if ((rc = c->hip(hipMemcpyAsync(out, dp, (size_t)c->ns * 4 * c->nz * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy")))
        return rc;
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    const double area = (double)c->nx * c->ny;
    for (size_t i = 0; i < (size_t)c->ns * 4 * c->nz; ++i) out[i] /= area;
    return LBMIX_OK;
}

int lbmix_get_stats(lbmix_ctx *c, lbmix_stats *out) {
    if (!c || !out) return LBMIX_EINVAL;
    Guard g(c);
    if (c->allocated && c->resid_on_device) {
        int rc = fetch(c, 8);
        if (rc) return rc;
        c->last_resid = c->hred[5] > 0.0 ? std::sqrt(c->hred[4] / c->hred[5]) : 0.0;
        c->resid_on_device = false;
    }
    out->steps = c->steps;
    out->poisson_solves = c->solves;
    out->total_sweeps = c->total_sweeps;
    out->last_sweeps = c->last_sweeps;
    out->last_status = c->last_status;
    out->last_residual = c->last_resid;
    out->fluid_nodes = (double)c->Nf;
    out->bytes_per_step = 2.0 * Q * c->ns * (double)c->esize * c->Nf;
    dim3 b;
    uint32_t bx, by;
    step_shape(c->st, c->rounding != 0, c->ns, (uint32_t)c->nx, c->blk_x, c->blk_y, &bx, &by);
    (void)step_grid(c->nx, c->ny, c->nzf, &b, bx, by);
    out->block_x = (int)b.x;
    out->block_y = (int)b.y;
    return LBMIX_OK;
}

int lbmix_device_copy(void *dst, const void *src, unsigned long long bytes, void *stream) {
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return LBMIX_EINVAL;
    if (bytes == 0) return LBMIX_OK;
    const hipError_t e = launch_copy16(src, dst, (size_t)(bytes / 16), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LBMIX_OK : LBMIX_EDEVICE;
}

int lbmix_sync(lbmix_ctx *c) {
    if (!c) return LBMIX_EINVAL;
    if (!c->allocated) return LBMIX_OK;
    Guard g(c);
    return c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

int lbmix_save(lbmix_ctx *c, const char *path) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!path) return c->fail(LBMIX_EINVAL, "null path");
    Guard g(c);
    Header h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kMagic, 8);
    h.version = 7;   // 7: populations in blocks of rows of all slots per plane
    h.nx = c->nx; h.ny = c->ny; h.nz = c->nz; h.geometry = c->geometry; h.storage = c->storage; h.ns = c->ns;
    h.nch = c->nch;
    h.pair_ns = c->pair_ns;
    h.forcing = c->forcing;
    h.wide = c->wide;
    h.pad = 0;
    for (int a = 0; a < MAXS; ++a)
        for (int b = 0; b < MAXS; ++b) h.tau_pair[a * MAXS + b] = c->tau_pair[a][b];
    for (int s = 0; s < MAXS; ++s) {
        h.valence[s] = c->valence[s];
        h.rho0[s] = c->rho0[s];
        h.rel_range[s] = c->rel_range[s];
        h.host_total[s] = c->host_total[s];
    }
    h.tau_v = c->tau_v; h.tau_d = c->tau_d; h.sc = c->sc; h.drag_from_sc = c->drag_from_sc;
    h.sor_max = c->sor_max; h.sor_check = c->sor_check; h.psi_valid = c->psi_valid && c->psi;
    h.rounding = c->rounding; h.round_seed = c->round_seed; h.poisson_method = c->poisson_method;
    h.lB = c->lB; h.sig_lo = c->sig_lo; h.sig_hi = c->sig_hi;
    for (int d = 0; d < 3; ++d) h.E[d] = c->E[d];
    h.sor_tol = c->sor_tol; h.sor_omega = c->sor_omega; h.steps = c->steps;
    const size_t pop = (size_t)c->ns * Q * c->Nf * c->esize;
    std::vector<char> buf(pop);
    if ((rc = c->hip(hipMemcpyAsync(buf.data(), c->f[c->cur], pop, hipMemcpyDeviceToHost, c->stream), "copy f"))) return rc;
    std::vector<double> ps(h.psi_valid ? c->Nf : 0);
    if (h.psi_valid &&
        (rc = c->hip(hipMemcpyAsync(ps.data(), c->psi, c->Nf * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy psi")))
        return rc;
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    // per channel: width, drag, wall charges, initial totals of every species
    std::vector<double> chan;
    for (int ch = 0; ch < c->nch; ++ch) {
        chan.push_back(c->ch_width[ch]);
        chan.push_back(c->ch_tau_d[ch]);
        chan.push_back(c->ch_sig_lo[ch]);
        chan.push_back(c->ch_sig_hi[ch]);
        for (int s = 0; s < MAXS; ++s) chan.push_back(c->ch_total[(size_t)s * c->nch + ch]);
    }
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return c->fail(LBMIX_EINVAL, "cannot open %s", path);
    bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1 &&
              std::fwrite(chan.data(), sizeof(double), chan.size(), fp) == chan.size() &&
              std::fwrite(buf.data(), 1, pop, fp) == pop;
    if (ok && h.psi_valid) ok = std::fwrite(ps.data(), sizeof(double), ps.size(), fp) == ps.size();
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? LBMIX_OK : c->fail(LBMIX_EINVAL, "write to %s failed", path);
}

int lbmix_load(lbmix_ctx *c, const char *path) {
    if (!c || !path) return LBMIX_EINVAL;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return c->fail(LBMIX_EINVAL, "cannot open %s", path);
    Header h;
    bool ok = std::fread(&h, sizeof h, 1, fp) == 1 && std::memcmp(h.magic, kMagic, 8) == 0 && h.version == 7;
    ok = ok && h.nx == c->nx && h.ny == c->ny && h.nz == c->nz && h.geometry == c->geometry &&
         h.storage == c->storage && h.ns == c->ns && h.nch == c->nch;
    constexpr int kPerChan = 4 + MAXS;
    std::vector<double> chan(ok ? (size_t)kPerChan * c->nch : 0);
    ok = ok && std::fread(chan.data(), sizeof(double), chan.size(), fp) == chan.size();
    for (int ch = 0; ok && ch < c->nch; ++ch) ok = (int)chan[(size_t)kPerChan * ch] == c->ch_width[ch];
    for (int s = 0; ok && s < c->ns; ++s) ok = h.valence[s] == c->valence[s] && h.rho0[s] == c->rho0[s];
    if (!ok) {
        std::fclose(fp);
        return c->fail(LBMIX_EINVAL, "%s: not a checkpoint of this lattice", path);
    }
    const size_t pop = (size_t)c->ns * Q * c->Nf * c->esize;
    std::vector<char> buf(pop);
    std::vector<double> ps(h.psi_valid ? c->Nf : 0);
    ok = std::fread(buf.data(), 1, pop, fp) == pop;
    if (ok && h.psi_valid) ok = std::fread(ps.data(), sizeof(double), ps.size(), fp) == ps.size();
    std::fclose(fp);
    if (!ok) return c->fail(LBMIX_EINVAL, "%s: truncated checkpoint", path);
    int rc = allocate(c);
    if (rc) return rc;
    Guard g(c);
    for (int s = 0; s < MAXS; ++s) {
        c->rel_range[s] = h.rel_range[s];
        c->host_total[s] = h.host_total[s];
    }
    c->compute_scales();
    c->tau_v = h.tau_v; c->tau_d = h.tau_d; c->sc = h.sc; c->drag_from_sc = h.drag_from_sc != 0;
    c->sor_max = h.sor_max; c->sor_check = h.sor_check; c->sor_tol = h.sor_tol; c->sor_omega = h.sor_omega;
    c->rounding = h.rounding; c->round_seed = h.round_seed; c->poisson_method = h.poisson_method;
    c->lB = h.lB; c->sig_lo = h.sig_lo; c->sig_hi = h.sig_hi;
    for (int d = 0; d < 3; ++d) c->E[d] = h.E[d];
    c->pair_ns = h.pair_ns;
    c->forcing = h.forcing;
    c->wide = h.wide;
    for (int a = 0; a < MAXS; ++a)
        for (int b = 0; b < MAXS; ++b) c->tau_pair[a][b] = h.tau_pair[a * MAXS + b];
    for (int ch = 0; ch < c->nch; ++ch) {
        const double *v = chan.data() + (size_t)kPerChan * ch;
        c->ch_tau_d[ch] = v[1];
        c->ch_sig_lo[ch] = v[2];
        c->ch_sig_hi[ch] = v[3];
        for (int s = 0; s < MAXS; ++s) c->ch_total[(size_t)s * c->nch + ch] = v[4 + s];
    }
    c->tables_dirty = true;
    drop_graph(c);
    if ((rc = ensure_tables(c))) return rc;
    if ((rc = c->hip(hipMemcpyAsync(c->f[c->cur], buf.data(), pop, hipMemcpyHostToDevice, c->stream), "copy f"))) return rc;
    if (h.psi_valid) {
        if ((rc = ensure_field_buffers(c))) return rc;
        if ((rc = c->hip(hipMemcpyAsync(c->psi, ps.data(), c->Nf * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy psi")))
            return rc;
    }
    if ((rc = c->hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize"))) return rc;
    for (int s = 0; s < c->ns; ++s) c->set[s] = true;
    c->psi_valid = h.psi_valid != 0;
    c->steps = h.steps;
    c->started = h.steps > 0;
    c->latched = 0;
    return LBMIX_OK;
}

const char *lbmix_last_error(const lbmix_ctx *c) { return c ? c->err.c_str() : "null context"; }

void lbmix_destroy(lbmix_ctx *c) {
    if (!c) return;
    if (c->allocated) {
        Guard g(c);
        (void)hipStreamSynchronize(c->stream);
        for (int k = 0; k < 2; ++k)
            if (c->f[k]) (void)hipFree(c->f[k]);
        if (c->psi) (void)hipFree(c->psi);
        if (c->q) (void)hipFree(c->q);
        if (c->partials) (void)hipFree(c->partials);
        if (c->step_partials) (void)hipFree(c->step_partials);
        if (c->dred) (void)hipFree(c->dred);
        if (c->hred) (void)hipHostFree(c->hred);
        if (c->scratch) (void)hipFree(c->scratch);
        drop_graph(c);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->mg_b) (void)hipFree(c->mg_b);
        if (c->mg_cinv) (void)hipFree(c->mg_cinv);
        if (c->psi_prev) (void)hipFree(c->psi_prev);
        for (void *p : {(void *)c->ws_r, (void *)c->ws_c, (void *)c->ws_guess, (void *)c->ws_scale, (void *)c->ws_x, (void *)c->ws_y,
                        (void *)c->ws_t, (void *)c->ws_mask})
            if (p) (void)hipFree(p);
        for (double *p : {c->sp_tx, c->sp_ty, c->sp_txp, c->sp_typ, c->sp_tz, c->sp_mu, c->sp_piv, c->sp_piv_end, c->sp_pmid,
                          c->sp_a, c->sp_b, c->sp_fx, c->sp_fy, c->sp_fz})
            if (p) (void)hipFree(p);
        if (c->sp_seg) (void)hipFree(c->sp_seg);
        if (c->step_dev) (void)hipFree(c->step_dev);
        for (void *p : {(void *)c->d_planes, (void *)c->d_fof, (void *)c->d_first, (void *)c->d_chan,
                        (void *)c->d_psums})
            if (p) (void)hipFree(p);
        for (double *p : c->mg_idn) (void)hipFree(p);
        for (double *p : c->mg_pmid) (void)hipFree(p);
        for (size_t l = 1; l < c->mg.size(); ++l) {
            (void)hipFree(c->mg[l].e);
            (void)hipFree(c->mg[l].r);
        }
    }
    delete c;
}

}  // extern "C"
