// gfx950 kernels of the Poisson solvers (eq. Poisson with the surface-charge condition of
// Sec. II): the operator, its right-hand side and residual, red-black SOR, geometric
// multigrid, the direct solve by real Fourier bases and tridiagonal eliminations, and the
// deterministic reductions shared with the observables.
#include "lbmix_poisson.h"
#include "lbmix_device.h"

namespace lbmix {

// ---------------------------------------------------------------------------------------
// Poisson: 7-point finite-volume operator on fluid nodes (eq. Poisson, Sec. II), periodic in
// x, y (and z for the box); no neighbour across a wall, whose charge sits in the first
// fluid layer.  b = -K (q + lump) - mean(b), the mean taken per channel (each channel of a
// stack is an independent problem).

struct Stencil {
    double sum;
    int deg;
};

__device__ inline Stencil neighbours(const PoissonArgs &a, const double *psi, uint32_t x, uint32_t y,
                                     uint32_t z) {
    const uint32_t xm = x == 0 ? a.nx - 1 : x - 1, xp = x + 1 == a.nx ? 0 : x + 1;
    const uint32_t ym = y == 0 ? a.ny - 1 : y - 1, yp = y + 1 == a.ny ? 0 : y + 1;
    const uint32_t row = (z * a.ny + y) * a.nx;
    double s = psi[row + xp];
    s += psi[row + xm];
    s += psi[(z * a.ny + yp) * a.nx + x];
    s += psi[(z * a.ny + ym) * a.nx + x];
    int deg = 4;
    if (a.slit) {
        const uint32_t walls = a.planes[z].walls;
        if (!(walls & 2u)) { s += psi[((z + 1) * a.ny + y) * a.nx + x]; ++deg; }
        if (!(walls & 1u)) { s += psi[((z - 1) * a.ny + y) * a.nx + x]; ++deg; }
    } else {
        const uint32_t zp = z + 1 == a.nzf ? 0 : z + 1, zm = z == 0 ? a.nzf - 1 : z - 1;
        s += psi[(zp * a.ny + y) * a.nx + x];
        s += psi[(zm * a.ny + y) * a.nx + x];
        deg = 6;
    }
    return {s, deg};
}

__device__ inline double rhs(const PoissonArgs &a, uint32_t i, uint32_t z) {
    if (a.slit) return -a.K * (a.q[i] + a.planes[z].lump) - a.bmean[a.planes[z].chan];
    return -a.K * a.q[i] - a.bmean[0];
}

// One thread per node of the colour: thread t of plane z takes row y = t / nxh and the node
// x = 2 (t mod nxh) + ((y + zc + colour) mod 2) of that row's colour, nxh = ceil(nx / 2).  The
// nodes of a colour are independent, so the order does not change the result.  (One thread
// per node with the other colour's threads returning took 8.9 us per half-sweep on the
// 64 x 64 x 128 slit: 8192 one-wave work-groups, half of each wave idle.)
__global__ __launch_bounds__(BLOCK) void sor_half(const PoissonArgs a, int colour) {
    const uint32_t nxh = (a.nx + 1) / 2;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nxh * a.ny) return;
    const uint32_t y = t / nxh, z = blockIdx.y;
    const uint32_t zc = a.slit ? a.planes[z].zloc : z;   // colour by the channel's own lattice
    const uint32_t x = 2 * (t - y * nxh) + ((y + zc + (uint32_t)colour) & 1u);
    if (x >= a.nx) return;
    const uint32_t i = (z * a.ny + y) * a.nx + x;
    const Stencil st = neighbours(a, a.psi, x, y, z);
    const double b = rhs(a, i, z);
    const double gs = (st.sum - b) / (double)st.deg;
    a.psi[i] = a.psi[i] + a.omega * (gs - a.psi[i]);
}

constexpr uint32_t RES_PLANES = 8;   // fluid planes per work-group of the residual kernel

// One thread per node of a plane (256 per work-group) and RES_PLANES planes.
__global__ __launch_bounds__(BLOCK) void residual(const PoissonArgs a, double *partials) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (t < a.nx * a.ny) {
        const uint32_t y = t / a.nx, x = t - y * a.nx;
        const uint32_t z1 = min(a.nzf, (blockIdx.y + 1) * RES_PLANES);
#pragma unroll 4
        for (uint32_t z = blockIdx.y * RES_PLANES; z < z1; ++z) {
            const uint32_t i = (z * a.ny + y) * a.nx + x;
            const Stencil st = neighbours(a, a.psi, x, y, z);
            const double b = rhs(a, i, z);
            const double r = b - (st.sum - st.deg * a.psi[i]);
            v[0] += r * r;
            v[1] += b * b;
            v[2] += a.psi[i];
        }
    }
    block_sum_store<3>(v, partials, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y);
}

// r = b - A psi on every fluid node, and per-block partial sums of r^2.
__global__ __launch_bounds__(BLOCK) void residual_field(const PoissonArgs a, double *r, double *partials) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (x < a.nx) {
        const uint32_t y = blockIdx.y, z = blockIdx.z;
        const uint32_t i = (z * a.ny + y) * a.nx + x;
        const Stencil st = neighbours(a, a.psi, x, y, z);
        const double ri = rhs(a, i, z) - (st.sum - st.deg * a.psi[i]);
        r[i] = ri;
        v[0] = ri * ri;
    }
    const uint32_t bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum_store<1>(v, partials, gridDim.x * gridDim.y * gridDim.z, bid);
}

__global__ __launch_bounds__(BLOCK) void qsum(const double *q, uint32_t N, double *partials) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {i < N ? q[i] : 0.0};
    block_sum_store<1>(v, partials, gridDim.x, blockIdx.x);
}

// Sum of one fluid plane per work-group (fixed order).
__global__ __launch_bounds__(BLOCK) void plane_sum(const double *v, uint32_t nxy, double *out) {
    __shared__ double red[BLOCK];
    const double *p = v + (size_t)blockIdx.x * nxy;
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < nxy; i += BLOCK) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// One thread per channel: the plane sums of the channel in order.
__global__ __launch_bounds__(BLOCK) void channel_means(const double *ps, const uint32_t *first, uint32_t nch,
                                                      const PlaneInfo *planes, uint32_t nxy, int mode, double K,
                                                      double *out) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    double s = 0.0, lump = 0.0;
    for (uint32_t z = first[c]; z < first[c + 1]; ++z) {
        s += ps[z];
        if (planes) lump += planes[z].lump;
    }
    const double n = (double)nxy * (double)(first[c + 1] - first[c]);
    out[c] = mode == 0 ? -K * (s + (double)nxy * lump) / n : s / n;
}

__global__ __launch_bounds__(BLOCK) void shift_planes(double *psi, uint32_t nxy, uint32_t N, const PlaneInfo *planes,
                                                     const double *mean) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    psi[i] -= mean[planes ? planes[i / nxy].chan : 0u];
}

constexpr int FIN_BLOCK = 1024;

__global__ __launch_bounds__(FIN_BLOCK) void finalize(const double *partials, uint32_t nb, int nv, double *out,
                                                     int mode, double K, double lumps, double N) {
    __shared__ double red[FIN_BLOCK];
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (uint32_t b = threadIdx.x; b < nb; b += FIN_BLOCK) s += partials[(size_t)v * nb + b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = FIN_BLOCK / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == 1) out[nv] = -K * (out[0] + lumps) / N;
        if (mode == 2) out[nv] = out[2] / N;
    }
}

__global__ __launch_bounds__(BLOCK) void make_rhs(const PoissonArgs a, double *r) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const uint32_t i = (blockIdx.z * a.ny + blockIdx.y) * a.nx + x;
    r[i] = rhs(a, i, blockIdx.z);
}

// ---------------------------------------------------------------------------------------
// Geometric multigrid for the same operator (cell-centred, V-cycles).  On a level with
// spacings H_d the equation reads sum_d a_d (e_{+d} + e_{-d} - 2 e) = r, a_d = 1 / H_d^2, with
// periodic x, y, periodic or zero-flux z (a missing neighbour drops its term).

struct MGNb {
    double sum, diag;
};

__device__ inline MGNb mg_nb(const MGLevel &L, const double *e, uint32_t x, uint32_t y, uint32_t z) {
    double s = 0.0, dg = 0.0;
    if (L.nx > 1) {
        const uint32_t xm = x == 0 ? L.nx - 1 : x - 1, xp = x + 1 == L.nx ? 0 : x + 1;
        s += L.ax * (e[(z * L.ny + y) * L.nx + xp] + e[(z * L.ny + y) * L.nx + xm]);
        dg += 2.0 * L.ax;
    }
    if (L.ny > 1) {
        const uint32_t ym = y == 0 ? L.ny - 1 : y - 1, yp = y + 1 == L.ny ? 0 : y + 1;
        s += L.ay * (e[(z * L.ny + yp) * L.nx + x] + e[(z * L.ny + ym) * L.nx + x]);
        dg += 2.0 * L.ay;
    }
    if (L.planes) {   // a stack of channels: no neighbour across a wall
        const uint32_t w = L.planes[z].walls;
        if (!(w & 2u)) { s += L.az * e[((z + 1) * L.ny + y) * L.nx + x]; dg += L.az; }
        if (!(w & 1u)) { s += L.az * e[((z - 1) * L.ny + y) * L.nx + x]; dg += L.az; }
    } else if (L.nz > 1) {
        if (L.periodic_z) {
            const uint32_t zm = z == 0 ? L.nz - 1 : z - 1, zp = z + 1 == L.nz ? 0 : z + 1;
            s += L.az * (e[(zp * L.ny + y) * L.nx + x] + e[(zm * L.ny + y) * L.nx + x]);
            dg += 2.0 * L.az;
        } else {
            if (z + 1 < L.nz) { s += L.az * e[((z + 1) * L.ny + y) * L.nx + x]; dg += L.az; }
            if (z > 0) { s += L.az * e[((z - 1) * L.ny + y) * L.nx + x]; dg += L.az; }
        }
    }
    return {s, dg};
}

// One thread per cell of the colour (x + y + z) mod 2, mapped as in sor_half.
__global__ __launch_bounds__(BLOCK) void mg_smooth(const MGLevel L, int colour) {
    const uint32_t nxh = (L.nx + 1) / 2;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nxh * L.ny) return;
    const uint32_t y = t / nxh, z = blockIdx.y;
    const uint32_t x = 2 * (t - y * nxh) + ((y + z + (uint32_t)colour) & 1u);
    if (x >= L.nx) return;
    const uint32_t i = (z * L.ny + y) * L.nx + x;
    const MGNb nb = mg_nb(L, L.e, x, y, z);
    if (nb.diag > 0.0) L.e[i] = (nb.sum - L.r[i]) / nb.diag;
}

// Line relaxation along z for channel stacks, whose channels may be of any width: the z
// lines of the columns of one colour (x + y) mod 2 are solved exactly, their lateral
// neighbours (the other colour) held fixed.  First the right-hand sides g = (lateral terms) - r
// of the line equations (Ld + az n_z) e - az (e_up + e_down) = g, written over e (the line's
// own values are not needed), then one thread per line and channel eliminates and substitutes.
// (one thread per cell of the colour: rows of even length hold nx / 2 of them)
__global__ __launch_bounds__(BLOCK) void mg_line_rhs(const MGLevel L, int colour) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t rowcells = (L.nx % 2 == 0) ? L.nx / 2 : L.nx;
    if (t >= rowcells * L.ny * L.nz) return;
    const uint32_t row = t / rowcells, y = row % L.ny, z = row / L.ny;
    const uint32_t x = (L.nx % 2 == 0) ? 2 * (t % rowcells) + ((y + (uint32_t)colour) & 1u) : t % rowcells;
    if (((x + y) & 1u) != (uint32_t)colour) return;
    double s = 0.0;
    if (L.nx > 1) {
        const uint32_t xm = x == 0 ? L.nx - 1 : x - 1, xp = x + 1 == L.nx ? 0 : x + 1;
        s += L.ax * (L.e[(z * L.ny + y) * L.nx + xp] + L.e[(z * L.ny + y) * L.nx + xm]);
    }
    if (L.ny > 1) {
        const uint32_t ym = y == 0 ? L.ny - 1 : y - 1, yp = y + 1 == L.ny ? 0 : y + 1;
        s += L.ay * (L.e[(z * L.ny + yp) * L.nx + x] + L.e[(z * L.ny + ym) * L.nx + x]);
    }
    const uint32_t i = (z * L.ny + y) * L.nx + x;
    L.e[i] = s - L.r[i];
}

constexpr uint32_t LINE_CHUNK = 8;   // planes whose loads a line thread keeps in flight together

// Two threads per line, in the same work-group (threads h and h + LINE_HALF): the first
// eliminates from the channel's first plane towards its middle plane mid = W / 2, the second
// from its last plane (the rows are symmetric, so both take the pivots idn[j] of the j-th step
// from their end); the first then solves the middle plane from both sides (pivot pmid[c]; 0
// pins the middle plane of a singular line to 0), and both substitute back outwards.  Half
// the serial steps of an elimination from one end.
constexpr uint32_t LINE_HALF = BLOCK / 2;

__global__ __launch_bounds__(BLOCK) void mg_line_solve(const MGLevel L, int colour, const double *idn,
                                                      const double *pmid, const uint32_t *first, uint32_t nch) {
    // line u is the u-th column of the colour (rows of even length hold nx / 2 of them)
    const uint32_t ncol = L.nx * L.ny;
    const uint32_t rowcols = (L.nx % 2 == 0) ? L.nx / 2 : L.nx;
    const bool bottom = threadIdx.x >= LINE_HALF;
    const uint32_t u = blockIdx.x * LINE_HALF + threadIdx.x % LINE_HALF;
    const uint32_t c = blockIdx.y;   // uniform: the whole work-group is in one channel
    if (c >= nch) return;
    const uint32_t y = u / rowcols;
    const uint32_t x = (L.nx % 2 == 0) ? 2 * (u % rowcols) + ((y + (uint32_t)colour) & 1u) : u % rowcols;
    const bool act = u < rowcols * L.ny && ((x + y) & 1u) == (uint32_t)colour;
    const uint32_t W = first[c + 1] - first[c];   // >= 1, uniform
    const uint32_t mid = W / 2;
    const uint32_t steps = bottom ? W - 1 - mid : mid;
    double *e = L.e + (size_t)first[c] * ncol + (act ? y * L.nx + x : 0);
    auto at = [&](uint32_t j) -> size_t { return (size_t)(bottom ? W - 1 - j : j) * ncol; };   // j-th step
    const double az = L.az;
    if (act) {   // elimination towards the middle: d_j = (g_j + az d_{j-1}) idn[j]
        double d = 0.0;
        uint32_t j = 0;
        for (; j + LINE_CHUNK <= steps; j += LINE_CHUNK) {
            double g[LINE_CHUNK];
#pragma unroll
            for (uint32_t q = 0; q < LINE_CHUNK; ++q) g[q] = e[at(j + q)];
#pragma unroll
            for (uint32_t q = 0; q < LINE_CHUNK; ++q) {
                d = (g[q] + az * d) * idn[j + q];
                e[at(j + q)] = d;
            }
        }
        for (; j < steps; ++j) {
            d = (e[at(j)] + az * d) * idn[j];
            e[at(j)] = d;
        }
    }
    __syncthreads();
    if (act && !bottom) {   // the middle plane from both neighbours
        const double up = mid >= 1 ? e[(size_t)(mid - 1) * ncol] : 0.0;
        const double down = mid + 1 < W ? e[(size_t)(mid + 1) * ncol] : 0.0;
        e[(size_t)mid * ncol] = (e[(size_t)mid * ncol] + az * (up + down)) * pmid[c];
    }
    __syncthreads();
    if (act) {   // back substitution outwards: x_j = d_j + az idn[j] x_{j+1}
        double v = e[(size_t)mid * ncol];
        int j = (int)steps - 1;
        for (; j + 1 >= (int)LINE_CHUNK; j -= (int)LINE_CHUNK) {
            double dv[LINE_CHUNK];
#pragma unroll
            for (uint32_t q = 0; q < LINE_CHUNK; ++q) dv[q] = e[at((uint32_t)(j - (int)q))];
#pragma unroll
            for (uint32_t q = 0; q < LINE_CHUNK; ++q) {
                v = dv[q] + az * idn[j - (int)q] * v;
                e[at((uint32_t)(j - (int)q))] = v;
            }
        }
        for (; j >= 0; --j) {
            v = e[at((uint32_t)j)] + az * idn[j] * v;
            e[at((uint32_t)j)] = v;
        }
    }
}

// one thread per coarse cell: average of the fine residuals of its children
// (one thread per cell over the whole level, so that narrow levels leave no lanes idle)
__global__ __launch_bounds__(BLOCK) void mg_restrict(const MGLevel F, const MGLevel C) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C.nx * C.ny * C.nz) return;
    const uint32_t X = c % C.nx, Y = (c / C.nx) % C.ny, Z = c / (C.nx * C.ny);
    double acc = 0.0;
    for (int k = 0; k < F.fz; ++k)
        for (int j = 0; j < F.fy; ++j)
            for (int i = 0; i < F.fx; ++i) {
                const uint32_t x = X * F.fx + i, y = Y * F.fy + j, z = Z * F.fz + k;
                const uint32_t fi = (z * F.ny + y) * F.nx + x;
                const MGNb nb = mg_nb(F, F.e, x, y, z);
                acc += F.r[fi] - (nb.sum - nb.diag * F.e[fi]);
            }
    const uint32_t ci = (Z * C.ny + Y) * C.nx + X;
    C.r[ci] = acc / double(F.fx * F.fy * F.fz);
    C.e[ci] = 0.0;
}

// cell-centred linear interpolation along each coarsened axis: weights 3/4 (own coarse
// cell) and 1/4 (the coarse neighbour on the side of the fine cell); a zero-flux boundary
// reflects (the neighbour is the cell itself), a periodic one wraps
__device__ inline void lin1(uint32_t f, int factor, uint32_t nc, bool periodic, uint32_t &c0, uint32_t &c1,
                            double &w0) {
    if (factor == 1) { c0 = c1 = f; w0 = 1.0; return; }
    c0 = f >> 1;
    const bool lo = (f & 1u) == 0;
    if (lo) c1 = c0 == 0 ? (periodic ? nc - 1 : 0) : c0 - 1;
    else c1 = c0 + 1 == nc ? (periodic ? 0 : c0) : c0 + 1;
    w0 = 0.75;
}

__global__ __launch_bounds__(BLOCK) void mg_prolong(const MGLevel F, const MGLevel C) {
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F.nx * F.ny * F.nz) return;
    const uint32_t x = f % F.nx, y = (f / F.nx) % F.ny, z = f / (F.nx * F.ny);
    uint32_t xa, xb, ya, yb, za, zb;
    double wx, wy, wz;
    lin1(x, F.fx, C.nx, true, xa, xb, wx);
    lin1(y, F.fy, C.ny, true, ya, yb, wy);
    lin1(z, F.fz, C.nz, F.periodic_z != 0, za, zb, wz);
    const double *e = C.e;
    auto at = [&](uint32_t i, uint32_t j, uint32_t k) { return e[(k * C.ny + j) * C.nx + i]; };
    const double v = wz * (wy * (wx * at(xa, ya, za) + (1 - wx) * at(xb, ya, za)) +
                           (1 - wy) * (wx * at(xa, yb, za) + (1 - wx) * at(xb, yb, za))) +
                     (1 - wz) * (wy * (wx * at(xa, ya, zb) + (1 - wx) * at(xb, ya, zb)) +
                                 (1 - wy) * (wx * at(xa, yb, zb) + (1 - wx) * at(xb, yb, zb)));
    F.e[(z * F.ny + y) * F.nx + x] += v;
}

// The coarse end of the hierarchy in one work-group: every sweep, restriction and
// interpolation of the small levels is a loop over cells with barriers between phases.
__device__ void blk_smooth(const MGLevel &L, int colour) {
    const uint32_t n = L.nx * L.ny * L.nz;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
        if (((x + y + z) & 1u) != (uint32_t)colour) continue;
        const MGNb nb = mg_nb(L, L.e, x, y, z);
        if (nb.diag > 0.0) L.e[i] = (nb.sum - L.r[i]) / nb.diag;
    }
    __syncthreads();
}

// View of bottom level l in LDS (offsets from the sizes of the levels above it); built from
// the kernel arguments on demand, so no level table is indexed at run time in private memory.
__device__ inline MGLevel bottom_view(const MGBottom &b, int l, double *se, double *sr) {
    uint32_t off = 0;
    for (int k = 0; k < l; ++k) off += b.lev[k].nx * b.lev[k].ny * b.lev[k].nz;
    MGLevel v = b.lev[l];
    v.e = se + off;
    v.r = sr + off;
    return v;
}

__global__ __launch_bounds__(1024) void mg_bottom(const MGBottom b) {
    __shared__ double se[MG_BOTTOM_LDS], sr[MG_BOTTOM_LDS];
    {
        const uint32_t n0 = b.lev[0].nx * b.lev[0].ny * b.lev[0].nz;
        for (uint32_t i = threadIdx.x; i < n0; i += blockDim.x) {
            se[i] = 0.0;
            sr[i] = b.lev[0].r[i];
        }
        __syncthreads();
    }
    for (int l = 0; l < b.n; ++l) {
        const MGLevel L = bottom_view(b, l, se, sr);
        if (l > 0) {   // restrict the residual of level l-1 into level l, e = 0
            const MGLevel F = bottom_view(b, l - 1, se, sr);
            const uint32_t n = L.nx * L.ny * L.nz;
            for (uint32_t ci = threadIdx.x; ci < n; ci += blockDim.x) {
                const uint32_t X = ci % L.nx, Y = (ci / L.nx) % L.ny, Z = ci / (L.nx * L.ny);
                double acc = 0.0;
                for (int k = 0; k < F.fz; ++k)
                    for (int j = 0; j < F.fy; ++j)
                        for (int i = 0; i < F.fx; ++i) {
                            const uint32_t x = X * F.fx + i, y = Y * F.fy + j, z = Z * F.fz + k;
                            const uint32_t fi = (z * F.ny + y) * F.nx + x;
                            const MGNb nb = mg_nb(F, F.e, x, y, z);
                            acc += F.r[fi] - (nb.sum - nb.diag * F.e[fi]);
                        }
                L.r[ci] = acc / double(F.fx * F.fy * F.fz);
                L.e[ci] = 0.0;
            }
            __syncthreads();
        }
        if (l == b.n - 1 && b.coarse_inv) {
            // exact coarsest solve: (A + 1 1^T / m) e = r gives the zero-mean solution of a
            // consistent r (and absorbs the rounding of its mean)
            const uint32_t m = L.nx * L.ny * L.nz;
            double acc = 0.0;
            if (threadIdx.x < m)
                for (uint32_t j = 0; j < m; ++j) acc += b.coarse_inv[threadIdx.x * m + j] * L.r[j];
            __syncthreads();
            if (threadIdx.x < m) L.e[threadIdx.x] = acc;
            __syncthreads();
            continue;
        }
        const int sweeps = (l == b.n - 1) ? b.coarse_sweeps : 2;
        for (int k = 0; k < sweeps; ++k) {
            blk_smooth(L, 0);
            blk_smooth(L, 1);
        }
    }
    for (int l = b.n - 2; l >= 0; --l) {
        const MGLevel F = bottom_view(b, l, se, sr), C = bottom_view(b, l + 1, se, sr);
        const uint32_t n = F.nx * F.ny * F.nz;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t x = i % F.nx, y = (i / F.nx) % F.ny, z = i / (F.nx * F.ny);
            uint32_t xa, xb, ya, yb, za, zb;
            double wx, wy, wz;
            lin1(x, F.fx, C.nx, true, xa, xb, wx);
            lin1(y, F.fy, C.ny, true, ya, yb, wy);
            lin1(z, F.fz, C.nz, F.periodic_z != 0, za, zb, wz);
            auto at = [&](uint32_t ii, uint32_t jj, uint32_t kk) { return C.e[(kk * C.ny + jj) * C.nx + ii]; };
            F.e[i] += wz * (wy * (wx * at(xa, ya, za) + (1 - wx) * at(xb, ya, za)) +
                            (1 - wy) * (wx * at(xa, yb, za) + (1 - wx) * at(xb, yb, za))) +
                      (1 - wz) * (wy * (wx * at(xa, ya, zb) + (1 - wx) * at(xb, ya, zb)) +
                                  (1 - wy) * (wx * at(xa, yb, zb) + (1 - wx) * at(xb, yb, zb)));
        }
        __syncthreads();
        for (int k = 0; k < 2; ++k) {
            blk_smooth(F, 0);
            blk_smooth(F, 1);
        }
    }
    const uint32_t n0 = b.lev[0].nx * b.lev[0].ny * b.lev[0].nz;
    for (uint32_t i = threadIdx.x; i < n0; i += blockDim.x) b.lev[0].e[i] = se[i];
}

// psi <- psi + p1 - p2 (p1, p2 = the two previous solutions), then p2 <- p1, p1 <- psi_old:
// exact for a linear trend plus an oscillation of period two steps
__global__ __launch_bounds__(BLOCK) void extrapolate(double *psi, double *p1, double *p2, uint32_t N) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double a = psi[i], b = p1[i];
    psi[i] = a + b - p2[i];
    p2[i] = b;
    p1[i] = a;
}

__global__ __launch_bounds__(BLOCK) void shift(double *psi, uint32_t N, const double *mean) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) psi[i] -= *mean;
}

// ---- direct Poisson solve ----------------------------------------------------------------
// The 7-point operator separates: along a periodic axis of n nodes it is diagonal in the
// orthonormal real Fourier basis (1/sqrt(n); sqrt(2/n) cos, sqrt(2/n) sin of 2 pi k x / n;
// (-1)^x / sqrt(n) for even n) with eigenvalue -4 sin^2(pi k / n).  The transforms are small
// batched products C_b = A_b B_b in FP64; the zero-flux z direction of a slit is solved by
// one tridiagonal system per transformed (x, y) mode.

// FP64 matrix cores, v_mfma_f64_16x16x4f64: lane l holds A(i, k) and B(k, j) with
// i, j = l mod 16 and k = l / 16 of its 16 x 4 and 4 x 16 fragments, and the result rows
// l / 16 + 4 r, r < 4, of column l mod 16 (checked on the GPU with a one-wave probe).
typedef double f64x4 __attribute__((ext_vector_type(4)));

// C_b[m][n] = sum_k A_b[m][k] B_b[k][n]; 64 x 64 output tile per work-group of 256 threads,
// k in steps of 16 through LDS, each wave a 32 x 32 block on the FP64 matrix cores.  AK1: the
// unit stride of A is its k index (else its m index); BN1: the unit stride of B is its n
// index (else its k index), so that consecutive threads load consecutive addresses.
constexpr int GT = 64, GK = 16;

template <bool AK1, bool BN1>
__global__ __launch_bounds__(256) void gemm_f64(const SpecGemm g) {
    __shared__ double As[GK][GT + 1], Bs[GK][GT + 1];
    const uint32_t m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const double *A = g.A + (size_t)blockIdx.z * g.sAb;
    const double *B = g.B + (size_t)blockIdx.z * g.sBb;
    double *C = g.C + (size_t)blockIdx.z * g.sCb;
    const uint32_t t = threadIdx.x;
    const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    // with BN1 the next k step's tile is read into registers while the current one is
    // multiplied (the other layout measured slower that way, so it reads each tile in turn)
    constexpr bool PIPE = BN1;
    double ra[4], rb[4];
    auto fetch = [&](uint32_t k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t e = t + 256 * i;
            const uint32_t ak = AK1 ? e % GK : e / GT, am = AK1 ? e / GK : e % GT;
            const uint32_t m = m0 + am, ka = k0 + ak;
            double av = 0.0;
            if (m < g.M && ka < g.K) {
                av = A[(size_t)m * g.sAm + (size_t)ka * g.sAk];
                if (g.rhs) av = -g.rhs_K * (av + (g.planes ? g.planes[m / g.rows_per_plane].lump : 0.0));
            }
            ra[i] = av;
            const uint32_t bk = BN1 ? e / GT : e % GK, bn = BN1 ? e % GT : e / GK;
            const uint32_t n = n0 + bn, kb = k0 + bk;
            rb[i] = (n < g.N && kb < g.K) ? B[(size_t)kb * g.sBk + (size_t)n * g.sBn] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t e = t + 256 * i;
            As[AK1 ? e % GK : e / GT][AK1 ? e / GK : e % GT] = ra[i];
            Bs[BN1 ? e / GT : e % GK][BN1 ? e % GT : e / GK] = rb[i];
        }
    };
    if (PIPE) {
        fetch(0);
        stage();
        __syncthreads();
    }
    for (uint32_t k0 = 0; k0 < g.K; k0 += GK) {
        const bool more = k0 + GK < g.K;
        if (!PIPE) {
            fetch(k0);
            stage();
            __syncthreads();
        } else if (more) {
            fetch(k0 + GK);
        }
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int k = 4 * ks + lk;
            const double a0 = As[k][r0 + li], a1 = As[k][r0 + 16 + li];
            const double b0 = Bs[k][c0 + li], b1 = Bs[k][c0 + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        if (PIPE && more) {
            stage();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t m = m0 + r0 + 16 * i + lk + 4 * r;
            if (m >= g.M) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t n = n0 + c0 + 16 * j + li;
                if (n < g.N) C[(size_t)m * g.sCm + n] = acc[i][j][r];
            }
        }
}

// One thread per (mode, segment): rows psi_{z-1} - (2 + mu) psi_z + psi_{z+1} = b_z of a
// segment of planes with zero-flux ends, by elimination with the precomputed inverse
// pivots p_k = 1 / (d_k - p_{k-1}) of plane k of the segment.  Every segment shares the
// pivots before its last plane (piv, [k][mode]); only the last differs (piv_end,
// [segment][mode]).  The singular mode (mu = 0, index 0) has its last pivot stored as 0,
// which fixes psi = 0 on the segment's last plane; its segment mean is removed afterwards.
__device__ __forceinline__ double seg_pivot(const double *piv, const double *piv_end, uint32_t k, uint32_t L,
                                            uint32_t s, uint32_t mode, uint32_t nmodes) {
    return k + 1 == L ? piv_end[(size_t)s * nmodes + mode] : piv[(size_t)k * nmodes + mode];
}

// Pivots of the elimination from both ends of a segment towards its middle plane m = L / 2:
// plane k < m takes the pivot of plane k from the top, plane k > m that of plane L - 1 - k
// (the same recurrence from the bottom, since the rows are symmetric), and the middle plane
// the inverse of its condensed diagonal, pmid[segment][mode] (0 for the singular mode, which
// fixes psi = 0 on the middle plane).
__device__ __forceinline__ double twoway_pivot(const double *piv, const double *pmid, uint32_t k, uint32_t L,
                                               uint32_t s, uint32_t mode, uint32_t nmodes) {
    const uint32_t m = L / 2;
    return k == m ? pmid[(size_t)s * nmodes + mode] : piv[(size_t)(k < m ? k : L - 1 - k) * nmodes + mode];
}

__global__ __launch_bounds__(64) void tridiag_z(const double *b, const double *piv, const double *piv_end,
                                                double *out, uint32_t nmodes, const uint32_t *seg) {
    const uint32_t mode = blockIdx.x * 64 + threadIdx.x;
    if (mode >= nmodes) return;
    const uint32_t z0 = seg[blockIdx.y], z1 = seg[blockIdx.y + 1];
    double bm = 0.0;   // mode 0: project the right-hand side onto zero segment mean
    if (mode == 0) {
        for (uint32_t z = z0; z < z1; ++z) bm += b[(size_t)z * nmodes];
        bm /= double(z1 - z0);
    }
    double r = 0.0;
#pragma unroll 8
    for (uint32_t z = z0; z < z1; ++z) {
        const size_t i = (size_t)z * nmodes + mode;
        r = (b[i] - bm - r) * seg_pivot(piv, piv_end, z - z0, z1 - z0, blockIdx.y, mode, nmodes);
        out[i] = r;
    }
    double x = 0.0;
#pragma unroll 8
    for (uint32_t z = z1; z-- > z0;) {
        const size_t i = (size_t)z * nmodes + mode;
        x = out[i] - seg_pivot(piv, piv_end, z - z0, z1 - z0, blockIdx.y, mode, nmodes) * x;
        out[i] = x;
    }
    if (mode == 0) {
        double sum = 0.0;
        for (uint32_t z = z0; z < z1; ++z) sum += out[(size_t)z * nmodes];
        const double mean = sum / double(z1 - z0);
        for (uint32_t z = z0; z < z1; ++z) out[(size_t)z * nmodes] -= mean;
    }
}

// The same eliminations with the columns staged in LDS: one work-group of 256 threads per
// MODES modes of one segment of at most LMAX planes (MODES * LMAX <= 8192).  All threads stage the right-hand side
// and pivots with coalesced loads, issued sixteen at a time; 2 MODES threads run the
// recurrences from LDS, from both ends of the segment; all threads write the result back.
// The work-group holding mode 0 removes its segment mean before and after the elimination
// with all threads.
constexpr uint32_t TRI_CELLS = 8192;

// LDS layout of the columns of one segment folded at its middle plane mid = L / 2: row j
// holds plane j in columns 0 .. MODES - 1 (j < mid) and plane L - 1 - j in columns MODES ..
// 2 MODES - 1 (j < L - 1 - mid); the middle plane sits after the rows, at offset `cells`.
// The elimination from the top and the one from the bottom then walk the same rows.
template <uint32_t MODES>
__device__ __forceinline__ uint32_t folded(uint32_t z, uint32_t m, uint32_t L, uint32_t cells) {
    const uint32_t mid = L / 2;
    return z < mid ? z * 2 * MODES + m : z > mid ? (L - 1 - z) * 2 * MODES + MODES + m : cells + m;
}

// Mean over planes z < L of mode 0 in the folded layout, by all 256 threads in a fixed
// order; every thread receives it.
template <uint32_t MODES, uint32_t CELLS>
__device__ double column0_mean(const double *s, uint32_t L, double *red) {
    const uint32_t t = threadIdx.x;
    double v = 0.0;
    for (uint32_t z = t; z < L; z += 256) v += s[folded<MODES>(z, 0, L, CELLS)];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    const double m = ((red[0] + red[1]) + (red[2] + red[3])) / double(L);
    __syncthreads();
    return m;
}

template <uint32_t MODES, uint32_t LMAX>
__global__ __launch_bounds__(256) void tridiag_lds(const double *b, const double *piv, const double *pmid,
                                                   double *out, uint32_t nmodes, const uint32_t *seg) {
    constexpr uint32_t CELLS = MODES * LMAX;   // segments of at most LMAX planes
    static_assert(CELLS <= TRI_CELLS, "LDS");
    constexpr uint32_t RS = 2 * MODES;   // row stride of the folded layout
    __shared__ double sb[CELLS + MODES], sp[CELLS + MODES];
    __shared__ double red[4];
    const uint32_t m0 = blockIdx.x * MODES;
    const uint32_t z0 = seg[blockIdx.y], L = seg[blockIdx.y + 1] - z0;
    const uint32_t t = threadIdx.x, cells = L * MODES;
    for (uint32_t k0 = 0; k0 < cells; k0 += 256 * 16) {
        double vb[16], vp[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t k = k0 + u * 256 + t, z = k / MODES, m = k % MODES;
            const bool in = k < cells && m0 + m < nmodes;
            const size_t i = (size_t)(z0 + z) * nmodes + m0 + m;
            vb[u] = in ? b[i] : 0.0;
            vp[u] = in ? twoway_pivot(piv, pmid, z, L, blockIdx.y, m0 + m, nmodes) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t k = k0 + u * 256 + t;
            if (k < cells) {
                const uint32_t f = folded<MODES>(k / MODES, k % MODES, L, CELLS);
                sb[f] = vb[u];
                sp[f] = vp[u];
            }
        }
    }
    __syncthreads();
    if (m0 == 0) {   // mode 0: project onto zero segment mean
        const double bm = column0_mean<MODES, CELLS>(sb, L, red);
        for (uint32_t z = t; z < L; z += 256) sb[folded<MODES>(z, 0, L, CELLS)] -= bm;
        __syncthreads();
    }
    // Elimination from both ends towards the middle plane mid: thread c < MODES sweeps down
    // over planes 0 .. mid - 1 of mode c, thread MODES + c up over planes L - 1 .. mid + 1,
    // both along the rows of the folded layout with r_k = (b_k - r_prev) p_k; then the middle
    // plane is solved from its two neighbours, and both threads substitute back outwards,
    // x_k = r_k - p_k x_(next).
    const uint32_t mid = L / 2, c = t % MODES;
    const bool top = t < MODES, act = t < RS && m0 + c < nmodes;
    const uint32_t steps = top ? mid : L - 1 - mid;
    if (act) {
        double r = 0.0;
#pragma unroll 8
        for (uint32_t j = 0; j < steps; ++j) {
            r = (sb[j * RS + t] - r) * sp[j * RS + t];
            sb[j * RS + t] = r;
        }
    }
    __syncthreads();
    if (top && act) {
        const double up = mid >= 1 ? sb[(mid - 1) * RS + t] : 0.0;
        const double down = mid + 1 < L ? sb[(L - 2 - mid) * RS + MODES + t] : 0.0;
        sb[CELLS + t] = (sb[CELLS + t] - up - down) * sp[CELLS + t];
    }
    __syncthreads();
    if (act) {
        double x = sb[CELLS + c];
#pragma unroll 8
        for (uint32_t j = steps; j-- > 0;) {
            x = sb[j * RS + t] - sp[j * RS + t] * x;
            sb[j * RS + t] = x;
        }
    }
    __syncthreads();
    if (m0 == 0) {   // and gauge it to zero segment mean
        const double mean = column0_mean<MODES, CELLS>(sb, L, red);
        for (uint32_t z = t; z < L; z += 256) sb[folded<MODES>(z, 0, L, CELLS)] -= mean;
        __syncthreads();
    }
    for (uint32_t k = t; k < cells; k += 256) {
        const uint32_t z = k / MODES, m = k % MODES;
        if (m0 + m < nmodes) out[(size_t)(z0 + z) * nmodes + m0 + m] = sb[folded<MODES>(z, m, L, CELLS)];
    }
}

// C(r, c) = sum_k A(r, k) B(k, c) for r < RN, c < CN (multiples of 32), k < KN, with
// A(r, k) = A[r ar + k ak], B(k, c) = B[k bk + c bc] and C(r, c) = C[r ldc + c] (operands in
// LDS or device memory), on the FP64 matrix cores.  Each wave takes 32 x 32 blocks of four
// 16 x 16 tiles, so that every operand fragment feeds two products.

template <int RN, int CN, int KN>
__device__ void mfma_product(const double *A, int ar, int ak, const double *B, int bk, int bc, double *C, int ldc) {
    constexpr int NBR = RN / 32, NBC = CN / 32;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int nwaves = blockDim.x >> 6;
    for (int blk = threadIdx.x >> 6; blk < NBR * NBC; blk += nwaves) {
        const int r0 = (blk / NBC) * 32, c0 = (blk % NBC) * 32;
        f64x4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k = 0; k < KN; k += 4) {
            const int kk = k + lk;
            const double a0 = A[(r0 + li) * ar + kk * ak], a1 = A[(r0 + 16 + li) * ar + kk * ak];
            const double b0 = B[kk * bk + (c0 + li) * bc], b1 = B[kk * bk + (c0 + 16 + li) * bc];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) C[(r0 + 16 * i + lk + 4 * r) * ldc + c0 + 16 * j + li] = acc[i][j][r];
    }
}

// Transform of planes along x and y staged in LDS, zero-padded to PM x PM (PM = 64: 256
// threads, 67 KB of LDS; planes up to 32 x 32 take the register form spec_xy32 instead).  A
// work-group transforms the planes z = blockIdx.x, blockIdx.x + gridDim.x, ...; the
// matrix-core steps read the bases from their zero-padded copies in device memory, which
// stay in the caches.
template <bool FWD, int PM>
__global__ __launch_bounds__(PM == 64 ? 256 : 64) void spec_xy(const SpecXY a) {
    constexpr int LD = PM + 1;              // row stride of the LDS arrays
    constexpr int BLD = SPEC_PAD + 1;       // row stride of the padded bases
    __shared__ double P[PM * LD], R[PM * LD];
    const double *Tx = a.txp, *Ty = a.typ;   // read by the matrix-core steps from the caches
    const int nx = a.nx, ny = a.ny;
    // planes zero-padded to PM x PM (the padding contributes nothing); all loads of a thread
    // are issued before its LDS stores, in batches of eight elements
    constexpr int NT = PM == 64 ? 256 : 64, PER = PM * PM / NT, BATCH = 8;
    const bool from_q = FWD && a.q;
    const double *src = from_q ? a.q : a.in;
    for (uint32_t z = blockIdx.x; z < a.nplanes; z += gridDim.x) {
        const size_t base = (size_t)z * nx * ny;
        const double lump = (from_q && a.planes) ? a.planes[z].lump : 0.0;
#pragma unroll
        for (int b0 = 0; b0 < PER; b0 += BATCH) {
            double vp[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                const int k = threadIdx.x + (b0 + u) * NT, r = k / PM, c = k % PM;
                vp[u] = (r < ny && c < nx) ? src[base + r * nx + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                const int k = threadIdx.x + (b0 + u) * NT, r = k / PM, c = k % PM;
                P[r * LD + c] = (from_q && r < ny && c < nx) ? -a.K * (vp[u] + lump) : vp[u];
            }
        }
        __syncthreads();
        if (FWD) {
            // R[y][kx] = sum_x P[y][x] Tx[kx][x];  P[ky][kx] = sum_y Ty[ky][y] R[y][kx]
            mfma_product<PM, PM, PM>(P, LD, 1, Tx, 1, BLD, R, LD);
            __syncthreads();
            mfma_product<PM, PM, PM>(Ty, BLD, 1, R, LD, 1, P, LD);
        } else {
            // R[y][kx] = sum_ky Ty[ky][y] P[ky][kx];  P[y][x] = sum_kx R[y][kx] Tx[kx][x]
            mfma_product<PM, PM, PM>(Ty, 1, BLD, P, LD, 1, R, LD);
            __syncthreads();
            mfma_product<PM, PM, PM>(R, LD, 1, Tx, BLD, 1, P, LD);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nx * ny; k += blockDim.x) a.out[base + k] = P[(k / nx) * LD + k % nx];
        __syncthreads();   // P is restaged for the next plane
    }
}

// Transform of planes up to 32 x 32 by one wave each, held in registers: no LDS and no
// barrier.  Both directions take x first and then y, so that the result of the first
// product, in the accumulator layout of v_mfma_f64_16x16x4f64 (register r of lane l holds
// row 4 r + l / 16 of column l mod 16 of its 16 x 16 tile), is already the second product's
// B operand of k-step r (rows 4 r + l / 16 at lane l).
//   forward: R = P Tx^T, out = Ty R;   inverse: R = P Tx, out = Ty^T R.
// The two basis operands (16 values per lane each) are loaded once per wave from the
// zero-padded copies.  Loading the next plane ahead of the current plane's products, at two
// waves per SIMD, was no faster than three waves per SIMD without it.
template <bool FWD>
__global__ __launch_bounds__(64, 3) void spec_xy32(const SpecXY a) {   // three waves per SIMD
    constexpr int BLD = SPEC_PAD + 1;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int nx = a.nx, ny = a.ny;
    double b1[2][8], a2[2][8];   // [tile][k-step]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            // B1(k, j): forward Tx[j][k], inverse Tx[k][j];  A2(i, k): forward Ty[i][k], inverse Ty[k][i]
            const int j = 16 * t + li, k = 4 * s + lk;
            b1[t][s] = FWD ? a.txp[j * BLD + k] : a.txp[k * BLD + j];
            a2[t][s] = FWD ? a.typ[j * BLD + k] : a.typ[k * BLD + j];
        }
    const bool from_q = FWD && a.q;
    const double *src = from_q ? a.q : a.in;
    // A1(i, k) = plane[16 t + i][4 s + k], zero outside the plane
    auto load = [&](uint32_t z, double (&p)[2][8]) {
        const size_t base = (size_t)z * nx * ny;
        const double lump = (from_q && a.planes) ? a.planes[z].lump : 0.0;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int r = 16 * t + li, c = 4 * s + lk;
                const bool in = r < ny && c < nx;
                const double v = in ? src[base + r * nx + c] : 0.0;
                p[t][s] = (from_q && in) ? -a.K * (v + lump) : v;
            }
    };
    uint32_t z = blockIdx.x;
    if (z >= a.nplanes) return;
    double p[2][8];
    load(z, p);
    for (; z < a.nplanes; z += gridDim.x) {
        const uint32_t zn = z + gridDim.x;
        f64x4 c1[2][2], c2[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) c1[i][j] = c2[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    c1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[i][s], b1[j][s], c1[i][j], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    c2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i][s], c1[s / 4][j][s % 4], c2[i][j], 0, 0, 0);
        const size_t base = (size_t)z * nx * ny;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * i + 4 * r + lk, col = 16 * j + li;
                    if (row < ny && col < nx) a.out[base + row * nx + col] = c2[i][j][r];
                }
        if (zn < a.nplanes) load(zn, p);
    }
}

// One block of 16 TI x 16 TJ of a product on the FP64 matrix cores, C(r0 + r, c0 + c) =
// sum_k A(r, k) B(k, c) over KN, with the operand fragments of k-step ks supplied by
// fa(ks, i) (row 16 i + lane mod 16, column 4 ks + lane / 16) and fb(ks, j) (row 4 ks +
// lane / 16, column 16 j + lane mod 16).
template <int KN, int TI, int TJ, class FA, class FB>
__device__ __forceinline__ void mfma_block(FA fa, FB fb, double *C, int ldc, int r0, int c0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    f64x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KN / 4; ++ks) {
        double av[TI], bv[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) av[i] = fa(ks, i);
#pragma unroll
        for (int j = 0; j < TJ; ++j) bv[j] = fb(ks, j);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) C[(r0 + 16 * i + lk + 4 * r) * ldc + c0 + 16 * j + li] = acc[i][j][r];
}

// Half of the transform of one plane up to 64 x 64 per work-group, for lattices with fewer
// planes than compute units: the forward transform splits the output columns kx, the inverse
// the output rows y, and each half needs the whole plane, staged in LDS.  Each product of a
// half (64 x 32 or 32 x 64) is split over the four waves in blocks of 16 x 32 or 32 x 16;
// their basis fragments are read from the zero-padded copies into registers at the start,
// together with the plane, so the matrix-core steps wait on LDS only.
template <bool FWD>
__global__ __launch_bounds__(256) void spec_xy_half(const SpecXY a) {
    constexpr int PM = 64, LD = PM + 1, HM = 32, NT = 256, BATCH = 8, KS = PM / 4;
    static_assert(PM == (int)SPEC_PAD, "padded bases");
    __shared__ double P[PM * LD], R[PM * (HM + 1)];
    const int nx = a.nx, ny = a.ny;
    const uint32_t z = blockIdx.x >> 1;
    const int h = blockIdx.x & 1;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const size_t base = (size_t)z * nx * ny;
    // basis fragments of this wave's blocks: f1 for the first product, f2 for the second
    //   forward: f1[ks][j] = Tx[32 h + 16 j + li][4 ks + lk], f2[ks] = Ty[16 w + li][4 ks + lk]
    //   inverse: f1[ks][i] = Ty[4 ks + lk][32 h + 16 i + li], f2[ks] = Tx[4 ks + lk][16 w + li]
    double f1[KS][2], f2[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lk;
#pragma unroll
        for (int u = 0; u < 2; ++u)
            f1[ks][u] = FWD ? a.txp[(HM * h + 16 * u + li) * LD + k] : a.typ[k * LD + HM * h + 16 * u + li];
        f2[ks] = FWD ? a.typ[(16 * w + li) * LD + k] : a.txp[k * LD + 16 * w + li];
    }
    const bool from_q = FWD && a.q;
    const double *src = from_q ? a.q : a.in;
    const double lump = (from_q && a.planes) ? a.planes[z].lump : 0.0;
#pragma unroll
    for (int b0 = 0; b0 < PM * PM / NT; b0 += BATCH) {
        double vp[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int k = threadIdx.x + (b0 + u) * NT, r = k / PM, c = k % PM;
            vp[u] = (r < ny && c < nx) ? src[base + r * nx + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int k = threadIdx.x + (b0 + u) * NT, r = k / PM, c = k % PM;
            P[r * LD + c] = (from_q && r < ny && c < nx) ? -a.K * (vp[u] + lump) : vp[u];
        }
    }
    __syncthreads();
    if (FWD) {
        // R[y][kx'] = sum_x P[y][x] Tx[32 h + kx'][x]  (rows 16 w of R by wave w)
        mfma_block<PM, 1, 2>([&](int ks, int) { return P[(16 * w + li) * LD + 4 * ks + lk]; },
                             [&](int ks, int j) { return f1[ks][j]; }, R, HM + 1, 16 * w, 0);
        __syncthreads();
        // P[ky][kx'] = sum_y Ty[ky][y] R[y][kx']  (rows 16 w)
        mfma_block<PM, 1, 2>([&](int ks, int) { return f2[ks]; },
                             [&](int ks, int j) { return R[(4 * ks + lk) * (HM + 1) + 16 * j + li]; }, P, LD, 16 * w,
                             0);
        __syncthreads();
        for (int k = threadIdx.x; k < PM * HM; k += NT) {
            const int ky = k / HM, kx = HM * h + k % HM;
            if (ky < ny && kx < nx) a.out[base + ky * nx + kx] = P[ky * LD + k % HM];
        }
    } else {
        // R[y'][kx] = sum_ky Ty[ky][32 h + y'] P[ky][kx]  (columns 16 w of R by wave w)
        mfma_block<PM, 2, 1>([&](int ks, int i) { return f1[ks][i]; },
                             [&](int ks, int) { return P[(4 * ks + lk) * LD + 16 * w + li]; }, R, LD, 0, 16 * w);
        __syncthreads();
        // P[y'][x] = sum_kx R[y'][kx] Tx[kx][x]  (columns 16 w)
        mfma_block<PM, 2, 1>([&](int ks, int i) { return R[(16 * i + li) * LD + 4 * ks + lk]; },
                             [&](int ks, int) { return f2[ks]; }, P, LD, 0, 16 * w);
        __syncthreads();
        for (int k = threadIdx.x; k < HM * PM; k += NT) {
            const int y = HM * h + k / PM, x = k % PM;
            if (y < ny && x < nx) a.out[base + y * nx + x] = P[(k / PM) * LD + x];
        }
    }
}

// ---- the transforms by fast Fourier transforms (power-of-two extents) ---------------------
// Two real sequences a and b of length n are transformed together as z = a + i b.  With
// Z[f] = sum_x z[x] exp(-2 pi i f x / n), their spectra are A[f] = (Z[f] + conj Z[n - f]) / 2
// and B[f] = (Z[f] - conj Z[n - f]) / 2i, and a sequence's coefficients in the real Fourier
// basis are A[0] / sqrt(n), sqrt(2/n) Re A[f] (cosine of frequency f, 0 < f < n/2),
// -sqrt(2/n) Im A[f] (sine) and A[n/2] / sqrt(n) (the alternating vector).  The inverse
// builds the Hermitian spectra A and B from the coefficients, W = A + i B, and takes
// a + i b = conj(DFT(conj W)) / n.
// The DFT runs as Stockham (self-sorting) passes of radix 8, and one of radix 2 or 4 when
// log2 n is not a multiple of 3.  A pass of radix R after passes whose radices multiply to
// p maps, for i < n/R and k = i mod p, the R values u_j = X[i + j n/R] exp(-2 pi i j k / (R p))
// through an R-point DFT U to Y[(i - k) R + k + j p] = U_j; after the last pass Y is the DFT
// in natural order.  A pass reads every value into registers before the work-group's barrier
// and writes after it, so one LDS buffer serves as X and Y.  About 5 log2 n flops per value
// against 2n for the product with the dense basis, and three LDS round trips for n = 128
// where radix-2 stages take seven.  In LDS, value x of pair c sits at c (n + n/8 + 1) + x + x/8
// (fft_at) and twiddle m at m + m/8: the strides of 8 values of the first pass and of n values
// across pairs then fall on different banks.
constexpr uint32_t FFT_BLOCK = 256;
constexpr uint32_t FFT_SPAN = 1024;   // complex values of a work-group (2^10): FFT_SPAN / n pairs of sequences
constexpr uint32_t FFT_LDS = FFT_SPAN + FFT_SPAN / 8 + FFT_SPAN / FFT_MIN;   // with the padding
__device__ __forceinline__ uint32_t fft_at(uint32_t c, uint32_t x, uint32_t S) { return c * S + x + (x >> 3); }
__device__ __forceinline__ uint32_t tw_at(uint32_t m) { return m + (m >> 3); }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }   // a (-i)

// In-register DFTs (exponent sign -) of 2, 4 and 8 points.
__device__ __forceinline__ void dft(double2 (&u)[2]) {
    const double2 a = u[0];
    u[0] = cadd(a, u[1]);
    u[1] = csub(a, u[1]);
}
__device__ __forceinline__ void dft(double2 (&u)[4]) {
    const double2 t0 = cadd(u[0], u[2]), t1 = csub(u[0], u[2]), t2 = cadd(u[1], u[3]), t3 = mul_mi(csub(u[1], u[3]));
    u[0] = cadd(t0, t2);
    u[2] = csub(t0, t2);
    u[1] = cadd(t1, t3);
    u[3] = csub(t1, t3);
}
__device__ __forceinline__ void dft(double2 (&u)[8]) {
    double2 e[4] = {u[0], u[2], u[4], u[6]}, o[4] = {u[1], u[3], u[5], u[7]};
    dft(e);
    dft(o);
    constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
    o[1] = make_double2((o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h);    // exp(-i pi / 4)
    o[2] = mul_mi(o[2]);                                                    // exp(-i pi / 2)
    o[3] = make_double2((o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h);   // exp(-3 i pi / 4)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u[k] = cadd(e[k], o[k]);
        u[k + 4] = csub(e[k], o[k]);
    }
}

// One radix-R pass over the FFT_SPAN / n sequences of length n = 2^L in B (pair stride S),
// after passes whose radices multiply to p = 2^lp; tw[tw_at(m)] = exp(-2 pi i m / n), m < n.
template <int R>
__device__ __forceinline__ void fft_radix(double2 *B, const double2 *tw, uint32_t t, uint32_t L, uint32_t lp,
                                          uint32_t S) {
    constexpr uint32_t LR = R == 8 ? 3 : R == 4 ? 2 : 1;
    constexpr uint32_t NBF = FFT_SPAN / R, PER = (NBF + FFT_BLOCK - 1) / FFT_BLOCK;
    const uint32_t lm = L - LR, pm = (1u << lp) - 1;   // n / R = 2^lm butterflies per sequence
    double2 u[PER][R];
    uint32_t dst[PER];
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t e = t + q * FFT_BLOCK;
        if (e >= NBF) continue;
        const uint32_t c = e >> lm, i = e & ((1u << lm) - 1), k = i & pm;
        u[q][0] = B[fft_at(c, i, S)];
#pragma unroll
        for (int j = 1; j < R; ++j) u[q][j] = cmul(B[fft_at(c, i + (j << lm), S)], tw[tw_at((j * k) << (lm - lp))]);
        dft(u[q]);
        dst[q] = (c << 16) | (((i - k) << LR) + k);   // pair, position of output 0
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        if (t + q * FFT_BLOCK >= NBF) continue;
#pragma unroll
        for (int j = 0; j < R; ++j) B[fft_at(dst[q] >> 16, (dst[q] & 0xffffu) + (j << lp), S)] = u[q][j];
    }
    __syncthreads();
}

template <bool COLS, bool INV>
__global__ __launch_bounds__(FFT_BLOCK) void fft_pass(const FftPass f) {
    // per thread: NE elements in and out, NC complex values of the pre and post steps; each
    // step reads all of its values before the barrier and writes after it
    constexpr uint32_t NE = 2 * FFT_SPAN / FFT_BLOCK, NC = FFT_SPAN / FFT_BLOCK;
    __shared__ double2 buf[FFT_LDS];
    extern __shared__ double2 tw[];   // n twiddles (padded)
    const uint32_t t = threadIdx.x, n = f.n, L = f.log2n, half = n >> 1, S = n + (n >> 3) + 1;
    const uint32_t nreal = 2 * (FFT_SPAN >> L);   // real sequences of this work-group (pairs of them)
    const uint32_t s0 = blockIdx.x * nreal;
    const uint32_t ppm = (1u << f.log2pp) - 1;
    // element e of the work-group's block of nreal x n values: its sequence r and position x,
    // consecutive e along the unit stride in memory
    auto where = [&](uint32_t e, uint32_t &r, uint32_t &x) {
        if (COLS) {   // nreal = 2^(11 - L)
            r = e & (nreal - 1);
            x = e >> (11 - L);
        } else {
            r = e >> L;
            x = e & (n - 1);
        }
    };
    auto addr = [&](uint32_t s, uint32_t x) -> size_t {
        return (size_t)(s >> f.log2pp) * f.s_plane + (size_t)(s & ppm) * f.s_seq + (size_t)x * f.s_el;
    };
    auto slot = [&](uint32_t r, uint32_t x) -> double * {   // sequence r's part of pair r / 2
        return reinterpret_cast<double *>(&buf[fft_at(r >> 1, x, S)]) + (r & 1);
    };
    {
        // sequences past the batch read the last one (a valid address) and load 0
        double v[NE], lump[NE];
#pragma unroll
        for (uint32_t u = 0; u < NE; ++u) {
            uint32_t r, x;
            where(t + u * FFT_BLOCK, r, x);
            v[u] = f.in[addr(min(s0 + r, f.nseq - 1), x)];
        }
        if (f.rhs && f.planes) {
#pragma unroll
            for (uint32_t u = 0; u < NE; ++u) {
                uint32_t r, x;
                where(t + u * FFT_BLOCK, r, x);
                lump[u] = f.planes[min(s0 + r, f.nseq - 1) >> f.log2pp].lump;
            }
        } else {
#pragma unroll
            for (uint32_t u = 0; u < NE; ++u) lump[u] = 0.0;
        }
        for (uint32_t i = t; i < n; i += FFT_BLOCK) tw[tw_at(i)] = make_double2(f.tw[2 * i], f.tw[2 * i + 1]);
#pragma unroll
        for (uint32_t u = 0; u < NE; ++u) {
            uint32_t r, x;
            where(t + u * FFT_BLOCK, r, x);
            const double b = f.rhs ? -f.rhs_K * (v[u] + lump[u]) : v[u];
            *slot(r, x) = s0 + r < f.nseq ? b : 0.0;
        }
    }
    __syncthreads();
    if (INV) {   // conj W from the coefficients of each pair
        const double rn = sqrt((double)n), rh = sqrt(0.5 * (double)n);
        double2 w[NC];
#pragma unroll
        for (uint32_t u = 0; u < NC; ++u) {
            const uint32_t e = t + u * FFT_BLOCK, c = e >> L, fq = e & (n - 1);
            double ar, ai = 0.0, br, bi = 0.0;   // A[fq], B[fq]
            if (fq == 0) {
                const double2 c0 = buf[fft_at(c, 0, S)];
                ar = c0.x * rn;
                br = c0.y * rn;
            } else if (fq == half) {
                const double2 cn = buf[fft_at(c, n - 1, S)];
                ar = cn.x * rn;
                br = cn.y * rn;
            } else {   // A[g] = sqrt(n/2) (c[2g-1] - i c[2g]), A[n-g] = conj A[g]
                const uint32_t g = fq < half ? fq : n - fq;
                const double sg = fq < half ? -rh : rh;
                const double2 cc = buf[fft_at(c, 2 * g - 1, S)], cs = buf[fft_at(c, 2 * g, S)];
                ar = rh * cc.x;
                ai = sg * cs.x;
                br = rh * cc.y;
                bi = sg * cs.y;
            }
            w[u] = make_double2(ar - bi, -(ai + br));   // conj(A + i B)
        }
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < NC; ++u) {
            const uint32_t e = t + u * FFT_BLOCK;
            buf[fft_at(e >> L, e & (n - 1), S)] = w[u];
        }
        __syncthreads();
    }
    uint32_t lp = 0;
    for (; lp + 3 <= L; lp += 3) fft_radix<8>(buf, tw, t, L, lp, S);
    if (L - lp == 2) fft_radix<4>(buf, tw, t, L, lp, S);
    else if (L - lp == 1) fft_radix<2>(buf, tw, t, L, lp, S);
    if (!INV) {   // the coefficients of each pair from Z
        const double r1 = 1.0 / sqrt((double)n), r2 = sqrt(2.0 / (double)n);
        double2 o[NC];
#pragma unroll
        for (uint32_t u = 0; u < NC; ++u) {
            const uint32_t e = t + u * FFT_BLOCK, c = e >> L, k = e & (n - 1), fq = (k + 1) >> 1;
            const double2 zf = buf[fft_at(c, fq, S)], zm = buf[fft_at(c, (n - fq) & (n - 1), S)];
            const double are = 0.5 * (zf.x + zm.x), aim = 0.5 * (zf.y - zm.y);
            const double bre = 0.5 * (zf.y + zm.y), bim = 0.5 * (zm.x - zf.x);
            if (k == 0 || 2 * fq == n)
                o[u] = make_double2(are * r1, bre * r1);
            else if (k & 1)
                o[u] = make_double2(are * r2, bre * r2);
            else
                o[u] = make_double2(-aim * r2, -bim * r2);
        }
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < NC; ++u) {
            const uint32_t e = t + u * FFT_BLOCK;
            buf[fft_at(e >> L, e & (n - 1), S)] = o[u];
        }
        __syncthreads();
    }
    const double inv_n = 1.0 / (double)n;
    double o[NE];
#pragma unroll
    for (uint32_t u = 0; u < NE; ++u) {
        uint32_t r, x;
        where(t + u * FFT_BLOCK, r, x);
        const double y = *slot(r, x);
        o[u] = INV ? ((r & 1) ? -y * inv_n : y * inv_n) : y;
    }
#pragma unroll
    for (uint32_t u = 0; u < NE; ++u) {
        uint32_t r, x;
        where(t + u * FFT_BLOCK, r, x);
        const uint32_t s = s0 + r;
        if (s < f.nseq) f.out[addr(s, x)] = o[u];
    }
}

// a <- -a / (mu_x + mu_y + mu_z) in the transformed basis of a periodic box (0 for the
// constant mode)
__global__ __launch_bounds__(BLOCK) void spectral_scale(double *a, const double *mux, const double *muy,
                                                        const double *muz, uint32_t nx, uint32_t ny, uint32_t N) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    const double mu = mux[x] + muy[y] + muz[z];
    a[i] = mu > 0.0 ? -a[i] / mu : 0.0;
}

__global__ __launch_bounds__(BLOCK) void plane_sums(const double *n, const double *j, uint32_t nx, uint32_t ny,
                                                   uint32_t nz, double *out) {
    __shared__ double red[4][BLOCK];
    const uint32_t z = blockIdx.x;
    const size_t plane = (size_t)nx * ny, Nfull = plane * nz;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t k = threadIdx.x; k < plane; k += BLOCK) {
        const size_t i = z * plane + k;
        s[0] += n[i];
        s[1] += j[i];
        s[2] += j[Nfull + i];
        s[3] += j[2 * Nfull + i];
    }
    for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[(size_t)threadIdx.x * nz + z] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------------------
// Launchers.

hipError_t launch_sor(const PoissonArgs &a, int colour, hipStream_t stream) {
    const uint32_t per_plane = (a.nx + 1) / 2 * a.ny;
    const dim3 g((per_plane + BLOCK - 1) / BLOCK, a.nzf);
    hipLaunchKernelGGL(sor_half, g, dim3(BLOCK), 0, stream, a, colour);
    return hipGetLastError();
}

hipError_t launch_residual(const PoissonArgs &a, double *partials, uint32_t *nb, hipStream_t stream) {
    const dim3 g((a.nx * a.ny + BLOCK - 1) / BLOCK, (a.nzf + RES_PLANES - 1) / RES_PLANES);
    *nb = g.x * g.y;
    hipLaunchKernelGGL(residual, g, dim3(BLOCK), 0, stream, a, partials);
    return hipGetLastError();
}

hipError_t launch_residual_field(const PoissonArgs &a, double *r, double *partials, uint32_t *nb, hipStream_t stream) {
    dim3 b;
    const dim3 g = node_grid(a.nx, a.ny, a.nzf, &b);
    *nb = g.x * g.y * g.z;
    hipLaunchKernelGGL(residual_field, g, b, 0, stream, a, r, partials);
    return hipGetLastError();
}

hipError_t launch_qsum(const double *q, uint32_t N, double *partials, uint32_t *nb, hipStream_t stream) {
    *nb = (N + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(qsum, dim3(*nb), dim3(BLOCK), 0, stream, q, N, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, uint32_t nblocks, int nv, double *out, int mode, double K,
                           double lumps, double N, hipStream_t stream) {
    hipLaunchKernelGGL(finalize, dim3(1), dim3(FIN_BLOCK), 0, stream, partials, nblocks, nv, out, mode, K, lumps, N);
    return hipGetLastError();
}

hipError_t launch_make_rhs(const PoissonArgs &a, double *r, hipStream_t stream) {
    dim3 b;
    const dim3 g = node_grid(a.nx, a.ny, a.nzf, &b);
    hipLaunchKernelGGL(make_rhs, g, b, 0, stream, a, r);
    return hipGetLastError();
}
hipError_t launch_mg_smooth(const MGLevel &L, int colour, hipStream_t stream) {
    const uint32_t per_plane = (L.nx + 1) / 2 * L.ny;
    const dim3 g((per_plane + BLOCK - 1) / BLOCK, L.nz);
    hipLaunchKernelGGL(mg_smooth, g, dim3(BLOCK), 0, stream, L, colour);
    return hipGetLastError();
}
hipError_t launch_mg_restrict(const MGLevel &F, const MGLevel &C, hipStream_t stream) {
    const uint32_t n = C.nx * C.ny * C.nz;
    hipLaunchKernelGGL(mg_restrict, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, F, C);
    return hipGetLastError();
}
hipError_t launch_mg_prolong(const MGLevel &F, const MGLevel &C, hipStream_t stream) {
    const uint32_t n = F.nx * F.ny * F.nz;
    hipLaunchKernelGGL(mg_prolong, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, F, C);
    return hipGetLastError();
}
hipError_t launch_mg_line_rhs(const MGLevel &L, int colour, hipStream_t stream) {
    const uint32_t n = ((L.nx % 2 == 0) ? L.nx / 2 : L.nx) * L.ny * L.nz;
    hipLaunchKernelGGL(mg_line_rhs, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, L, colour);
    return hipGetLastError();
}
hipError_t launch_mg_line_solve(const MGLevel &L, int colour, const double *idn, const double *pmid,
                                const uint32_t *first, uint32_t nch, hipStream_t stream) {
    const uint32_t ncol = ((L.nx % 2 == 0) ? L.nx / 2 : L.nx) * L.ny;   // columns of one colour
    hipLaunchKernelGGL(mg_line_solve, dim3((ncol + LINE_HALF - 1) / LINE_HALF, nch), dim3(BLOCK), 0, stream, L, colour,
                       idn, pmid, first, nch);
    return hipGetLastError();
}
hipError_t launch_mg_bottom(const MGBottom &b, hipStream_t stream) {
    hipLaunchKernelGGL(mg_bottom, dim3(1), dim3(1024), 0, stream, b);
    return hipGetLastError();
}
hipError_t launch_extrapolate(double *psi, double *p1, double *p2, uint32_t N, hipStream_t stream) {
    hipLaunchKernelGGL(extrapolate, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, psi, p1, p2, N);
    return hipGetLastError();
}

hipError_t launch_shift(double *psi, uint32_t N, const double *mean, hipStream_t stream) {
    hipLaunchKernelGGL(shift, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, psi, N, mean);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(const SpecGemm &g, bool a_k_unit, bool b_n_unit, hipStream_t stream) {
    const dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, g.batch);
    if (a_k_unit && b_n_unit)
        hipLaunchKernelGGL((gemm_f64<true, true>), grid, dim3(256), 0, stream, g);
    else if (a_k_unit)
        hipLaunchKernelGGL((gemm_f64<true, false>), grid, dim3(256), 0, stream, g);
    else if (b_n_unit)
        hipLaunchKernelGGL((gemm_f64<false, true>), grid, dim3(256), 0, stream, g);
    else
        hipLaunchKernelGGL((gemm_f64<false, false>), grid, dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_plane_sum(const double *v, uint32_t nxy, uint32_t nplanes, double *out, hipStream_t stream) {
    hipLaunchKernelGGL(plane_sum, dim3(nplanes), dim3(BLOCK), 0, stream, v, nxy, out);
    return hipGetLastError();
}

hipError_t launch_channel_means(const double *plane_sums, const uint32_t *first, uint32_t nch,
                                const PlaneInfo *planes, uint32_t nxy, int mode, double K, double *out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(channel_means, dim3((nch + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, plane_sums, first, nch,
                       planes, nxy, mode, K, out);
    return hipGetLastError();
}

hipError_t launch_shift_planes(double *psi, uint32_t nxy, uint32_t N, const PlaneInfo *planes, const double *mean,
                               hipStream_t stream) {
    hipLaunchKernelGGL(shift_planes, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, psi, nxy, N, planes, mean);
    return hipGetLastError();
}

hipError_t launch_spec_xy(const SpecXY &a, bool forward, hipStream_t stream) {
    if (a.nx > 64 || a.ny > 64) return hipErrorInvalidValue;
    const bool small = a.nx <= 32 && a.ny <= 32;
    if (!small && a.nplanes <= 256 && a.txp && a.typ) {   // too few planes to give every compute unit a whole one
        if (forward)
            hipLaunchKernelGGL((spec_xy_half<true>), dim3(2 * a.nplanes), dim3(256), 0, stream, a);
        else
            hipLaunchKernelGGL((spec_xy_half<false>), dim3(2 * a.nplanes), dim3(256), 0, stream, a);
        return hipGetLastError();
    }
    if (!a.txp || !a.typ) return hipErrorInvalidValue;
    // as many work-groups as fit on the chip at once: twelve one-wave work-groups per compute
    // unit for the register transform (three per SIMD), two for the 64-wide one (LDS-bound)
    const uint32_t fit = small ? 12 * 256 : 2 * 256;
    const dim3 g(a.nplanes < fit ? a.nplanes : fit);
    if (small) {
        if (forward)
            hipLaunchKernelGGL((spec_xy32<true>), g, dim3(64), 0, stream, a);
        else
            hipLaunchKernelGGL((spec_xy32<false>), g, dim3(64), 0, stream, a);
    } else {
        if (forward)
            hipLaunchKernelGGL((spec_xy<true, 64>), g, dim3(256), 0, stream, a);
        else
            hipLaunchKernelGGL((spec_xy<false, 64>), g, dim3(256), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_fft_pass(const FftPass &f, bool cols, bool inverse, hipStream_t stream) {
    if (f.n < FFT_MIN || f.n > FFT_MAX || (1u << f.log2n) != f.n || f.log2pp < 1 || f.log2pp > 31 || !f.tw)
        return hipErrorInvalidValue;
    if (cols ? f.s_seq != 1 : f.s_el != 1) return hipErrorInvalidValue;
    const uint32_t nreal = 2 * (FFT_SPAN >> f.log2n);
    const dim3 g((f.nseq + nreal - 1) / nreal);
    const size_t lds = (size_t)(f.n + f.n / 8) * sizeof(double2);
    if (cols) {
        if (inverse) hipLaunchKernelGGL((fft_pass<true, true>), g, dim3(FFT_BLOCK), lds, stream, f);
        else hipLaunchKernelGGL((fft_pass<true, false>), g, dim3(FFT_BLOCK), lds, stream, f);
    } else {
        if (inverse) hipLaunchKernelGGL((fft_pass<false, true>), g, dim3(FFT_BLOCK), lds, stream, f);
        else hipLaunchKernelGGL((fft_pass<false, false>), g, dim3(FFT_BLOCK), lds, stream, f);
    }
    return hipGetLastError();
}

hipError_t launch_tridiag_lds(const double *b, const double *piv, const double *pmid, double *out, uint32_t nmodes,
                              const uint32_t *seg, uint32_t nseg, uint32_t longest, hipStream_t stream) {
    if (longest > TRI_LDS_MAX) return hipErrorInvalidValue;
    // Up to 256 planes: 16 modes per work-group, 64 KB of LDS, so two work-groups share a
    // compute unit and one stages its columns while the other runs its recurrences (on 64
    // stacked channels of 32 x 32 planes, 71-76 us against 81 with 8 modes and 97 with 32).
    // Longer segments: fewer modes per work-group in 128 KB of LDS.
    const dim3 blk(256);
    if (longest <= 256)
        hipLaunchKernelGGL((tridiag_lds<16, 256>), dim3((nmodes + 15) / 16, nseg), blk, 0, stream, b, piv, pmid, out,
                           nmodes, seg);
    else if (longest <= 1024)
        hipLaunchKernelGGL((tridiag_lds<8, 1024>), dim3((nmodes + 7) / 8, nseg), blk, 0, stream, b, piv, pmid, out,
                           nmodes, seg);
    else
        hipLaunchKernelGGL((tridiag_lds<4, 2048>), dim3((nmodes + 3) / 4, nseg), blk, 0, stream, b, piv, pmid, out,
                           nmodes, seg);
    return hipGetLastError();
}

hipError_t launch_tridiag_z(const double *b, const double *piv, const double *piv_end, double *out, uint32_t nmodes,
                            const uint32_t *seg, uint32_t nseg, hipStream_t stream) {
    hipLaunchKernelGGL(tridiag_z, dim3((nmodes + 63) / 64, nseg), dim3(64), 0, stream, b, piv, piv_end, out, nmodes,
                       seg);
    return hipGetLastError();
}

hipError_t launch_spectral_scale(double *a, const double *mux, const double *muy, const double *muz, uint32_t nx,
                                 uint32_t ny, uint32_t N, hipStream_t stream) {
    hipLaunchKernelGGL(spectral_scale, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, stream, a, mux, muy, muz, nx,
                       ny, N);
    return hipGetLastError();
}

hipError_t launch_plane_sums(const double *n, const double *j, uint32_t nx, uint32_t ny, uint32_t nz,
                             double *out, hipStream_t stream) {
    hipLaunchKernelGGL(plane_sums, dim3(nz), dim3(BLOCK), 0, stream, n, j, nx, ny, nz, out);
    return hipGetLastError();
}

}  // namespace lbmix
