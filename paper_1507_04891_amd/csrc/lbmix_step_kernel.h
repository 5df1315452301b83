// gfx950 kernels of the multicomponent lattice-Boltzmann library.
//
// The hot kernel is stream_collide: one thread per fluid node, all species' populations in
// registers, pull streaming (each stored value is read exactly once, each output written
// once, both coalesced along x), the moments of Sec. III, the drag of Sec. II and the field
// force, and the collision of eq. (latboeq), Sec. IV, with the equilibrium of the Appendix
// (phi_perp_p, which equals the second-order equilibrium at the species velocity) and the
// forcing g_p of eq. (ourforc).  The step is bound by HBM bandwidth (about 3 flop per byte
// in FP32), so there are no matrix-core contractions; the design goals are coalesced
// streams, no re-reads, and no LDS round trips.
//
// Work-group shape: 256 threads along x (fewer when nx < 256) times two rows, so z and every
// bounce-back decision are uniform per work-group (y too per wave when nx >= 64), and the
// x-shifted loads of a row stay in one work-group (and one L2).  Planes with walls (a slit,
// or a stack of channels) read their wall flags and channel parameters from a per-plane
// table.  Populations are interleaved by species, so each direction is one non-temporal
// vector load and one vector store of all species.  All arithmetic is done on deviations
// d_p = f_p - w_p rho_bar, which makes the shifted storage forms exact in their range and
// costs nothing for the plain ones (rho_bar = 0).
//
// This internal header holds the kernel template and its dispatch; each storage form is
// instantiated in a translation unit of its own.  Not installed.
#pragma once

#include "lbmix_step.h"
#include "lbmix_device.h"

#include <hip/hip_fp16.h>

namespace lbmix {

// ---------------------------------------------------------------------------------------
// D3Q19 (order documented in include/lbmix.h).

__host__ __device__ constexpr int cx(int p) {
    constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[p];
}
__host__ __device__ constexpr int cy(int p) {
    constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[p];
}
__host__ __device__ constexpr int cz(int p) {
    constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[p];
}
__host__ __device__ constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }
template <class C>
__host__ __device__ constexpr C wgt(int p) {
    return p == 0 ? C(1) / C(3) : (p < 7 ? C(1) / C(18) : C(1) / C(36));
}

// ---------------------------------------------------------------------------------------
// Storage codecs.  C is the arithmetic type, S the stored element; a stored element is
// (f - w rho_bar) * scale.

struct BF16 {};
struct F16 {};
struct F32X {};   // FP32 storage with FP64 arithmetic, for stochastic rounding of the stores

template <class T> struct Codec;
template <> struct Codec<double> {
    using C = double;
    using S = double;
    static constexpr bool kRounds = false;
    static constexpr bool kWideSum = true;   // density deviation summed in FP64
    __device__ static C decode(S v, float) { return v; }
    template <bool SR = false>
    __device__ static S encode(C v, float, uint32_t = 0) { return v; }
};
template <> struct Codec<float> {
    using C = float;
    using S = float;
    static constexpr bool kRounds = false;
    static constexpr bool kWideSum = true;   // density deviation summed in FP64
    __device__ static C decode(S v, float) { return v; }
    template <bool SR = false>
    __device__ static S encode(C v, float, uint32_t = 0) { return v; }
};
// Counter-based 32-bit hash (the "lowbias32" integer mixer: xor-shift / multiply rounds
// with the published constants 0x7feb352d and 0x846ca68b).  It seeds, once per node and
// step, a Marsaglia xorshift32 stream (shifts 13, 17, 5) that supplies the random bits of
// stochastic rounding: one 32-bit draw per direction, its high and low halves for the two
// species of a pair.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// bfloat16: upper half of an IEEE binary32, nearest-even written out.
__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    const bool special = (u & 0x7f800000u) == 0x7f800000u;      // Inf, NaN (kept, NaN quiet)
    const uint32_t r = special ? (u | ((u & 0x007fffffu) ? 0x00400000u : 0u)) : u + 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(r >> 16);
}
// Stochastic rounding: gfx950's v_cvt_sr_bf16_f32 / v_cvt_sr_f16_f32 add the high bits of a
// random 32-bit operand below the kept mantissa and truncate, so the magnitude goes up with
// probability equal to the dropped fraction and the expected stored value is the exact one
// (checked on the device: mean error below 0.003 unit in the last place over 65536 draws,
// binary16 subnormals included; only the operand's high bits are used).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint16_t f32_to_bf16_sr(float f, uint32_t rnd) {
    bf16x2 t = {};
    t = __builtin_amdgcn_cvt_sr_bf16_f32(t, f, rnd, false);
    return __builtin_bit_cast(uint16_t, t[0]);
}
__device__ inline uint16_t f32_to_f16_sr(float f, uint32_t rnd) {
    f16x2 t = {};
    t = __builtin_amdgcn_cvt_sr_f16_f32(t, f, rnd, false);
    return __builtin_bit_cast(uint16_t, t[0]);
}

template <> struct Codec<BF16> {
    using C = float;
    using S = uint16_t;
    static constexpr bool kRounds = true;
    static constexpr bool kWideSum = false;  // density deviation summed in FP32
    __device__ static C decode(S v, float inv) { return __uint_as_float(uint32_t(v) << 16) * inv; }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) {
        if constexpr (SR) return f32_to_bf16_sr(v * sc, rnd);
        else return f32_to_bf16_rne(v * sc);
    }
};
template <> struct Codec<F16> {
    using C = float;
    using S = uint16_t;
    static constexpr bool kRounds = true;
    static constexpr bool kWideSum = true;   // density deviation summed in FP64
    __device__ static C decode(S v, float inv) { return __half2float(__ushort_as_half(v)) * inv; }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) {
        if constexpr (SR) return f32_to_f16_sr(v * sc, rnd);
        else return __half_as_ushort(__float2half_rn(v * sc));   // IEEE nearest-even
    }
};

// FP32 storage, stochastically rounded from FP64 arithmetic: the nearest FP32 value f of v and
// its neighbour g on the side of v are chosen with probabilities that make the expected stored
// value v (to 2^-17 of a unit in the last place: 16 random bits, the high half of rnd).  The
// residual v - f and the spacing g - f are exact in FP64.
__device__ inline float f64_to_f32_sr(double v, uint32_t rnd) {
    const float f = float(v);
    const double r = v - double(f);
    if (r == 0.0 || !isfinite(f)) return f;
    const uint32_t bits = __float_as_uint(f);
    uint32_t gb;
    if (f == 0.0f)
        gb = r > 0.0 ? 1u : 0x80000001u;                       // smallest subnormal, sign of r
    else
        gb = ((f > 0.0f) == (r > 0.0)) ? bits + 1u : bits - 1u;   // away from / toward zero
    const float g = __uint_as_float(gb);
    const double s = fabs(double(g) - double(f));
    const double u = (double(rnd >> 16) + 0.5) * (1.0 / 65536.0);
    return fabs(r) > u * s ? g : f;
}

template <> struct Codec<F32X> {
    using C = double;
    using S = float;
    static constexpr bool kRounds = true;
    static constexpr bool kWideSum = true;
    __device__ static C decode(S v, float inv) { return double(v) * double(inv); }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) {
        if constexpr (SR) return f64_to_f32_sr(v * double(sc), rnd);
        else return float(v * double(sc));
    }
};

// Species-interleaved layout: the NS values of one direction at one node are contiguous,
// element (s, p, node) at ((p * N) + node) * NS + s.  One vector access per direction and
// node; non-temporal, since each element is touched once per step.  Three-element vectors
// are only used where the ISA access has exactly their size (FP32: dwordx3).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x3 __attribute__((ext_vector_type(3), aligned(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

template <class S, int NS> struct VecIO {
    __device__ static void load(const S *p, S (&o)[NS]) {
#pragma unroll
        for (int s = 0; s < NS; ++s) o[s] = __builtin_nontemporal_load(p + s);
    }
    __device__ static void store(S *p, const S (&v)[NS]) {
#pragma unroll
        for (int s = 0; s < NS; ++s) __builtin_nontemporal_store(v[s], p + s);
    }
};
template <class S, class V, int NS> struct VecIOv {
    __device__ static void load(const S *p, S (&o)[NS]) {
        const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
        for (int s = 0; s < NS; ++s) o[s] = v[s];
    }
    __device__ static void store(S *p, const S (&o)[NS]) {
        V v;
#pragma unroll
        for (int s = 0; s < NS; ++s) v[s] = o[s];
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    }
};
template <> struct VecIO<float, 2> : VecIOv<float, f32x2, 2> {};
template <> struct VecIO<float, 3> : VecIOv<float, f32x3, 3> {};
template <> struct VecIO<float, 4> : VecIOv<float, f32x4, 4> {};
template <> struct VecIO<double, 2> : VecIOv<double, f64x2, 2> {};
template <> struct VecIO<double, 4> : VecIOv<double, f64x4, 4> {};
template <> struct VecIO<uint16_t, 2> : VecIOv<uint16_t, u16x2, 2> {};
template <> struct VecIO<uint16_t, 4> : VecIOv<uint16_t, u16x4, 4> {};

__device__ __forceinline__ size_t elem(int arr, uint32_t node, uint32_t N, int ns) {
    return ((size_t)arr * N + node) * ns;
}

// The elements of direction slot arr at node plane + inplane in the fused step's layout: the
// address of the plane in the slot (uniform per work-group, formed on the scalar unit) plus a
// 32-bit byte offset within the plane (a plane of a slot holds less than 4 GiB).
template <int NS, class S>
__device__ __forceinline__ S *slot(S *base, int arr, uint32_t plane, uint32_t inplane, uint32_t N) {
    S *start = base + ((size_t)arr * N + plane) * NS;
    using B = std::conditional_t<std::is_const_v<S>, const char, char>;
    return reinterpret_cast<S *>(reinterpret_cast<B *>(start) + (uint32_t)(inplane * (NS * sizeof(S))));
}

// ---------------------------------------------------------------------------------------
// Pull addressing shared by every kernel that reads a pre-collision state: the value of
// direction p at node (x, y, z) comes from slot (p, node - c_p), or from slot (opp(p),
// node) when node - c_p is a wall (half-way bounce-back at rest).

struct Pull {
    uint32_t xs, xm, xp;       // x, x-1, x+1 with periodic wrap (per lane)
    uint32_t r0, rm, rp;       // node offsets y nx of the rows y, y-1, y+1 (wrapped)
    uint32_t p0, pm, pp;       // node offsets z nx ny of the planes z, z-1, z+1 (wrapped; uniform)
    uint32_t y, z;
    bool bb_lo, bb_hi;         // z - 1 / z + 1 is a wall (slit)

    __device__ Pull(uint32_t x, uint32_t y_, uint32_t z_, uint32_t nx, uint32_t ny, uint32_t nzf,
                    uint32_t walls)
        : xs(x), y(y_), z(z_) {
        xm = (x == 0) ? nx - 1 : x - 1;
        xp = (x + 1 == nx) ? 0 : x + 1;
        r0 = y * nx;
        rm = (y == 0) ? (ny - 1) * nx : r0 - nx;
        rp = (y + 1 == ny) ? 0 : r0 + nx;
        const uint32_t plane = nx * ny;
        p0 = z * plane;
        pm = (z == 0) ? (nzf - 1) * plane : p0 - plane;
        pp = (z + 1 == nzf) ? 0 : p0 + plane;
        bb_lo = (walls & 1u) != 0;
        bb_hi = (walls & 2u) != 0;
    }
    __device__ uint32_t own() const { return p0 + r0 + xs; }
    __device__ uint32_t own_inplane() const { return r0 + xs; }
    // slot direction, plane offset (uniform) and in-plane offset (per lane) of the value that
    // direction p pulls
    template <int p>
    __device__ void src(int &arr, uint32_t &plane, uint32_t &inplane) const {
        constexpr int X = cx(p), Y = cy(p), Z = cz(p);
        const bool bb = (Z == 1 && bb_lo) || (Z == -1 && bb_hi);
        const uint32_t sx = X == 1 ? xm : (X == -1 ? xp : xs);
        const uint32_t sy = Y == 1 ? rm : (Y == -1 ? rp : r0);
        const uint32_t sz = Z == 1 ? pm : (Z == -1 ? pp : p0);
        arr = bb ? opp(p) : p;
        plane = bb ? p0 : sz;
        inplane = bb ? r0 + xs : sy + sx;
    }
    // ... and as one node index
    template <int p>
    __device__ void src(int &arr, uint32_t &node) const {
        uint32_t plane, inplane;
        src<p>(arr, plane, inplane);
        node = plane + inplane;
    }
};

// ---------------------------------------------------------------------------------------
// The fused step.

// Drag models of stream_collide.
enum : int {
    kDragOne = 0,    // one frequency, drag on mid-step velocities u_s + a_s / 2
    kDragPair = 1,   // one frequency per pair of species, on the same velocities
    kDragGuo = 2,    // one frequency, second-order (Guo-type) forcing
};

template <int NS, class T, bool SLIT, bool FIELD, bool CHARGED, int DRAG>
__global__ __launch_bounds__(STEP_BLOCK) void stream_collide(const StepArgs a) {
    using CD = Codec<T>;
    using C = typename CD::C;
    using S = typename CD::S;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y * blockDim.y + threadIdx.y;   // uniform per wave if nx >= 64
    const bool active = x < a.nx && y < a.ny;
    const uint32_t z = blockIdx.z;
    const uint32_t walls = SLIT ? a.planes[z].walls : 0u;   // uniform per work-group
    const Pull pl(x < a.nx ? x : 0, y < a.ny ? y : 0, z, a.nx, a.ny, a.nzf, walls);
    const uint32_t own = pl.own();
    const uint32_t own_in = pl.own_inplane();
    const S *fin = static_cast<const S *>(a.fin);
    S *fout = static_cast<S *>(a.fout);

    // 1. pull streaming with bounce-back: one vector load of all species per direction
    C d[NS][Q];
    static_for<Q>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        int arr;
        uint32_t plane, inplane;
        pl.template src<p>(arr, plane, inplane);
        S raw[NS];
        VecIO<S, NS>::load(slot<NS>(fin, arr, plane, inplane, a.N), raw);
#pragma unroll
        for (int s = 0; s < NS; ++s) d[s][p] = CD::decode(raw[s], a.inv_scale[s][arr]);
    });

    // 2. moments (Sec. III): n = rho_bar + sum d, j = sum d c.  The density deviation is also
    //    summed in FP64 (dnh): with deviations stored, the update of a direction is
    //    w dn + (flux and force terms), and FP32 rounding at the scale of w dn would be about
    //    1 % of the per-step change of a slow diffusion mode at Sc = 100.  That rounding is
    //    deterministic, so it biases slow modes where stochastic rounding of the stored values
    //    only adds noise that averages out: with FP32 sums the spread of the FP16 form's
    //    electro-osmotic mobility over rounding seeds grows by 40 %.  BF16 storage is the
    //    exception: its own rounding noise is 8 times FP16's and the FP32 sum leaves its
    //    spread unchanged, so it keeps the FP32 sum.
    C dn[NS], jx[NS], jy[NS], jz[NS], n[NS];
    double dnh[NS];
    C ntot = 0, sjx = 0, sjy = 0, sjz = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        C m0 = 0, mx = 0, my = 0, mz = 0;
        double m0h = 0.0;
        static_for<Q>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            m0 += d[s][p];
            if constexpr (CD::kWideSum) m0h += double(d[s][p]);
            if constexpr (cx(p) == 1) mx += d[s][p];
            if constexpr (cx(p) == -1) mx -= d[s][p];
            if constexpr (cy(p) == 1) my += d[s][p];
            if constexpr (cy(p) == -1) my -= d[s][p];
            if constexpr (cz(p) == 1) mz += d[s][p];
            if constexpr (cz(p) == -1) mz -= d[s][p];
        });
        dn[s] = m0;
        dnh[s] = CD::kWideSum ? m0h : double(m0);
        jx[s] = mx;
        jy[s] = my;
        jz[s] = mz;
        n[s] = C(a.rho_bar[s]) + m0;
        ntot += n[s];
        sjx += mx;
        sjy += my;
        sjz += mz;
    }
    const C inv_ntot = ntot != C(0) ? C(1) / ntot : C(0);
    C ux = sjx * inv_ntot, uy = sjy * inv_ntot, uz = sjz * inv_ntot;   // barycentric

    // 3. field acceleration a_s = z_s (E - cs2 grad psi) and its charge-weighted mean
    C fx = 0, fy = 0, fz = 0, qn = 0;
    if constexpr (FIELD) {
        double gx = 0.0, gy = 0.0, gz = 0.0;
        if constexpr (CHARGED) {
            const double *psi = a.psi;
            const uint32_t row = pl.p0 + pl.r0;
            const double here = psi[row + pl.xs];
            gx = 0.5 * (psi[row + pl.xp] - psi[row + pl.xm]);
            gy = 0.5 * (psi[pl.p0 + pl.rp + pl.xs] - psi[pl.p0 + pl.rm + pl.xs]);
            const double up = (SLIT && pl.bb_hi) ? here + a.planes[z].ghost_hi : psi[pl.pp + pl.r0 + pl.xs];
            const double dw = (SLIT && pl.bb_lo) ? here + a.planes[z].ghost_lo : psi[pl.pm + pl.r0 + pl.xs];
            gz = 0.5 * (up - dw);
        }
        constexpr double cs2 = 1.0 / 3.0;
        fx = C(a.E[0] - cs2 * gx);
        fy = C(a.E[1] - cs2 * gy);
        fz = C(a.E[2] - cs2 * gz);
#pragma unroll
        for (int s = 0; s < NS; ++s) qn += C(a.valence[s]) * n[s];
    }
    if constexpr (CHARGED) {
        if (active) {
            double qq = a.q_rest;
#pragma unroll
            for (int s = 0; s < NS; ++s) qq += a.valence[s] * dnh[s];
            a.q[own] = qq;
        }
    }

    // 4. forces per species: drag on mid-step velocities plus the field force,
    //    F_s = -od (u_s + a_s/2 - (u + sum n a / 2 ntot)) + a_s (or per pair, or the
    //    Guo-type variant), then the coefficients of the collision that are common to
    //    every direction
    const C ov = C(a.omega_v), od = C(SLIT ? a.planes[z].omega_d : a.omega_d);
    C uax[NS], uay[NS], uaz[NS], Fx[NS], Fy[NS], Fz[NS], base[NS], ov45[NS], n9[NS], n3[NS];
    C bhi[NS][3], blo[NS][3];   // w ov dn (FP64) split hi + lo for the three weight classes
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const C inv_n = n[s] != C(0) ? C(1) / n[s] : C(0);
        uax[s] = jx[s] * inv_n;
        uay[s] = jy[s] * inv_n;
        uaz[s] = jz[s] * inv_n;
        if constexpr (DRAG == kDragOne) {
            Fx[s] = -od * (uax[s] - ux);
            Fy[s] = -od * (uay[s] - uy);
            Fz[s] = -od * (uaz[s] - uz);
            if constexpr (FIELD) {
                const C k = C(a.valence[s]) * (C(1) - C(0.5) * od) + C(0.5) * od * qn * inv_ntot;
                Fx[s] += k * fx;
                Fy[s] += k * fy;
                Fz[s] += k * fz;
            }
        }
    }
    if constexpr (DRAG == kDragPair) {
        // one drag frequency per pair (Sec. II, equal masses), on the mid-step velocities
        // v_b = u_b + a_b / 2:  F_s = a_s - sum_b omega_sb (n_b / n)(v_s - v_b)
        C vx[NS], vy[NS], vz[NS];
#pragma unroll
        for (int b = 0; b < NS; ++b) {
            const C h = FIELD ? C(0.5) * C(a.valence[b]) : C(0);
            vx[b] = uax[b] + h * fx;
            vy[b] = uay[b] + h * fy;
            vz[b] = uaz[b] + h * fz;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            C gx = 0, gy = 0, gz = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                if (b == s) continue;
                const C w = C(a.omega_pair[s][b]) * n[b] * inv_ntot;
                gx += w * (vx[s] - vx[b]);
                gy += w * (vy[s] - vy[b]);
                gz += w * (vz[s] - vz[b]);
            }
            const C zs = FIELD ? C(a.valence[s]) : C(0);
            Fx[s] = zs * fx - gx;
            Fy[s] = zs * fy - gy;
            Fz[s] = zs * fz - gz;
        }
    }
    if constexpr (DRAG == kDragGuo) {
        // Guo-type variant: every species moves with v_s = u_s + F_s / 2 in the equilibrium and
        // in the drag, F_s = a_s - od sum_b (n_b / n)(v_s - v_b).  The drag operator is a
        // projector, so this implicit system has the closed form
        //   F_s = abar + [(a_s - abar) - od (u_s - u)] / (1 + od / 2),  abar = sum_b n_b a_b / n;
        // the barycentric velocity becomes u + abar / 2 and the forcing term is scaled by
        // 1 - ov / 2.
        const C r = C(1) / (C(1) + C(0.5) * od);
        const C kbar = FIELD ? qn * inv_ntot : C(0);   // abar = kbar (fx, fy, fz)
        const C gs = C(1) - C(0.5) * ov;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C ka = FIELD ? (C(a.valence[s]) - kbar) * r + kbar : C(0);
            const C Gx = ka * fx - r * od * (uax[s] - ux);
            const C Gy = ka * fy - r * od * (uay[s] - uy);
            const C Gz = ka * fz - r * od * (uaz[s] - uz);
            uax[s] += C(0.5) * Gx;
            uay[s] += C(0.5) * Gy;
            uaz[s] += C(0.5) * Gz;
            Fx[s] = gs * Gx;
            Fy[s] = gs * Gy;
            Fz[s] = gs * Gz;
        }
        ux += C(0.5) * kbar * fx;
        uy += C(0.5) * kbar * fy;
        uz += C(0.5) * kbar * fz;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const C uu = uax[s] * uax[s] + uay[s] * uay[s] + uaz[s] * uaz[s];
        const C Fu = Fx[s] * ux + Fy[s] * uy + Fz[s] * uz;
        // f*_p = [(1 - ov) d_p + w (base + ov45 (c.u_s)^2 + n9 (c.F)(c.u)) +- w n3 (ov c.u_s + c.F)]
        //        + w ov dn, the last term in FP64, added as hi + lo: (t + lo) + hi rounds like the
        //        FP64 sum (t is far below the scale of hi, or carries its own FP32 rounding)
        base[s] = -C(1.5) * ov * n[s] * uu - C(3) * n[s] * Fu;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double big = wgt<double>(k == 0 ? 0 : (k == 1 ? 1 : 7)) * a.omega_v * dnh[s];
            bhi[s][k] = C(big);
            blo[s][k] = CD::kWideSum ? C(big - double(bhi[s][k])) : C(0);
        }
        ov45[s] = C(4.5) * ov * n[s];
        n9[s] = C(9) * n[s];
        n3[s] = C(3) * n[s];
    }

    // 5. collision and store, one direction pair at a time, all species per vector store.
    //    Stochastic rounding (16-bit forms) draws 32 random bits per direction from a
    //    per-node xorshift stream, 16 bits per species of each pair.
    const C keep = C(1) - ov;
    auto collide_store = [&](auto sr_tag) {
        constexpr bool SR = decltype(sr_tag)::value;
        const uint32_t seed = a.step_dev ? step_seed(a.round_seed, *a.step_dev + 1ull) : a.seed;
        uint32_t rs = SR ? (mix32(own ^ seed) | 1u) : 0u;
        auto rbits = [&](int s) -> uint32_t {     // the conversions use the high bits
            if constexpr (!SR) return 0u;
            if ((s & 1) == 0) rs = xorshift32(rs);
            return (s & 1) ? (rs << 16) : rs;
        };
        auto plus_dn = [&](C v, int s, int cls) -> C {   // + w ov dn (hi + lo with the FP64 sum)
            if constexpr (CD::kWideSum)
                return (v + blo[s][cls]) + bhi[s][cls];
            else
                return v + bhi[s][cls];
        };
        S o0[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s)
            o0[s] = CD::template encode<SR>(plus_dn(keep * d[s][0] + wgt<C>(0) * base[s], s, 0),
                                            a.scale[s][0], rbits(s));
        VecIO<S, NS>::store(slot<NS>(fout, 0, pl.p0, own_in, a.N), o0);
        static_for<9>([&](auto kc) {
            constexpr int p = 2 * decltype(kc)::value + 1;   // 1, 3, ..., 17
            constexpr int pb = p + 1;
            constexpr C w = wgt<C>(p);
            constexpr int cls = p < 7 ? 1 : 2;
            S op[NS], ob[NS];
            C vp[NS], vb[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const C cu = C(cx(p)) * uax[s] + C(cy(p)) * uay[s] + C(cz(p)) * uaz[s];
                const C cub = C(cx(p)) * ux + C(cy(p)) * uy + C(cz(p)) * uz;
                const C cF = C(cx(p)) * Fx[s] + C(cy(p)) * Fy[s] + C(cz(p)) * Fz[s];
                const C sym = w * (base[s] + ov45[s] * cu * cu + n9[s] * cF * cub);
                const C anti = w * n3[s] * (ov * cu + cF);
                vp[s] = plus_dn(keep * d[s][p] + sym + anti, s, cls);
                vb[s] = plus_dn(keep * d[s][pb] + sym - anti, s, cls);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) op[s] = CD::template encode<SR>(vp[s], a.scale[s][p], rbits(s));
#pragma unroll
            for (int s = 0; s < NS; ++s) ob[s] = CD::template encode<SR>(vb[s], a.scale[s][pb], rbits(s));
            VecIO<S, NS>::store(slot<NS>(fout, p, pl.p0, own_in, a.N), op);
            VecIO<S, NS>::store(slot<NS>(fout, pb, pl.p0, own_in, a.N), ob);
        });
    };
    if (active) {
        if (CD::kRounds && a.stochastic)
            collide_store(std::integral_constant<bool, CD::kRounds>{});
        else
            collide_store(std::false_type{});
    }

    // 7. FP64 mass partials of this work-group
    double v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = active ? dnh[s] : 0.0;
    const uint32_t bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const uint32_t nb = gridDim.x * gridDim.y * gridDim.z;
    block_sum_store<NS>(v, a.partials, nb, bid);
}


// ---------------------------------------------------------------------------------------
// Dispatch over species count, geometry, field and drag model.

template <int NS, class T, bool SLIT, int DRAG>
static hipError_t sc_fields(bool field, bool charged, const StepArgs &a, dim3 g, dim3 b, hipStream_t st) {
    if (charged)
        hipLaunchKernelGGL((stream_collide<NS, T, SLIT, true, true, DRAG>), g, b, 0, st, a);
    else if (field)
        hipLaunchKernelGGL((stream_collide<NS, T, SLIT, true, false, DRAG>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((stream_collide<NS, T, SLIT, false, false, DRAG>), g, b, 0, st, a);
    return hipGetLastError();
}

template <int NS, class T>
static hipError_t sc_geom(bool slit, bool field, bool charged, const StepArgs &a, dim3 g, dim3 b, hipStream_t st) {
    if (a.forcing == 1)
        return slit ? sc_fields<NS, T, true, kDragGuo>(field, charged, a, g, b, st)
                    : sc_fields<NS, T, false, kDragGuo>(field, charged, a, g, b, st);
    // pair frequencies only matter with three or more species (a binary has one pair)
    if constexpr (NS >= 3) {
        if (a.pair_drag)
            return slit ? sc_fields<NS, T, true, kDragPair>(field, charged, a, g, b, st)
                        : sc_fields<NS, T, false, kDragPair>(field, charged, a, g, b, st);
    }
    return slit ? sc_fields<NS, T, true, kDragOne>(field, charged, a, g, b, st)
                : sc_fields<NS, T, false, kDragOne>(field, charged, a, g, b, st);
}

// Launch of stream_collide for storage form T on grid g, work-group b (instantiated once per
// storage form, each in a translation unit of its own).
template <class T>
hipError_t stream_collide_store(int ns, bool slit, bool field, bool charged, const StepArgs &a, dim3 g, dim3 b,
                                hipStream_t st) {
    switch (ns) {
        case 1: return sc_geom<1, T>(slit, field, charged, a, g, b, st);
        case 2: return sc_geom<2, T>(slit, field, charged, a, g, b, st);
        case 3: return sc_geom<3, T>(slit, field, charged, a, g, b, st);
        case 4: return sc_geom<4, T>(slit, field, charged, a, g, b, st);
        default: return hipErrorInvalidValue;
    }
}

#define LBMIX_STEP_STORE(T)                                                                              \
    template hipError_t stream_collide_store<T>(int, bool, bool, bool, const StepArgs &, dim3, dim3, hipStream_t)
extern LBMIX_STEP_STORE(double);
extern LBMIX_STEP_STORE(float);
extern LBMIX_STEP_STORE(BF16);
extern LBMIX_STEP_STORE(F16);
extern LBMIX_STEP_STORE(F32X);

}  // namespace lbmix
