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
// c_p . (x, y, z) with the zero components left out: IEEE arithmetic does not fold a product
// by zero away (0 * inf is NaN), so the plain three-term form costs instructions that compute
// nothing.  A D3Q19 direction has one or two non-zero components, so the result takes at most
// one addition and is the same number.
template <int P, class C>
__device__ __forceinline__ C cdot(C x, C y, C z) {
    constexpr int X = cx(P), Y = cy(P), Z = cz(P);
    static_assert(X != 0 || Y != 0 || Z != 0, "rest direction");
    C r = C(0);
    bool first = true;
    auto add = [&](int c, C v) {
        r = first ? (c > 0 ? v : -v) : (c > 0 ? r + v : r - v);
        first = false;
    };
    if constexpr (X != 0) add(X, x);
    if constexpr (Y != 0) add(Y, y);
    if constexpr (Z != 0) add(Z, z);
    return r;
}
template <class C>
__host__ __device__ constexpr C wgt(int p) {
    return p == 0 ? C(1) / C(3) : (p < 7 ? C(1) / C(18) : C(1) / C(36));
}

// ---------------------------------------------------------------------------------------
// Storage codecs.  C is the arithmetic type, S the stored element; a stored element is
// (f - w rho_bar) * scale.  raw / put convert between S and C in stored units (the fused
// step works in those); decode / encode apply the scale too (the other kernels).
//   kScaled: the stored values carry a power-of-two scale per species and weight class;
//   kWide: how the fused step carries the density deviation beyond C when asked to:
//     0 C is FP64 already; 1 an FP64 sum of every population; 2 an FP64 combination of the
//     three per-class FP32 sums, which are exact for 16-bit values of similar magnitude;
//   kHold: the fused step keeps the loaded values as S and converts them where they are used;
//   kMinWaves: waves per SIMD the fused step's register budget must allow.

struct BF16 {};
struct F16 {};
struct F32X {};   // FP32 storage with FP64 arithmetic, for stochastic rounding of the stores

template <class T> struct Codec;
template <> struct Codec<double> {
    using C = double;
    using S = double;
    static constexpr bool kRounds = false;
    static constexpr bool kScaled = false;
    static constexpr bool kPacked = false;
    static constexpr int kWide = 0;
    static constexpr bool kHold = false;
    static constexpr int kMinWaves = 1;
    __device__ static C raw(S v) { return v; }
    template <bool SR = false>
    __device__ static S put(C v, uint32_t = 0) { return v; }
    __device__ static C decode(S v, float) { return v; }
    template <bool SR = false>
    __device__ static S encode(C v, float, uint32_t = 0) { return v; }
};
template <> struct Codec<float> {
    using C = float;
    using S = float;
    static constexpr bool kRounds = false;
    static constexpr bool kScaled = false;
    static constexpr bool kPacked = false;
    static constexpr int kWide = 1;
    static constexpr bool kHold = false;
    static constexpr int kMinWaves = 1;
    __device__ static C raw(S v) { return v; }
    template <bool SR = false>
    __device__ static S put(C v, uint32_t = 0) { return v; }
    __device__ static C decode(S v, float) { return v; }
    template <bool SR = false>
    __device__ static S encode(C v, float, uint32_t = 0) { return v; }
};
// Counter-based 32-bit hash (the "lowbias32" integer mixer: xor-shift / multiply rounds
// with the published constants 0x7feb352d and 0x846ca68b) of the node and step seeds the high
// half, and the node index mixed with the step seed the low half, of a Marsaglia xorshift64
// stream per node and step (shifts 13, 7, 17, a full-period triple of his
// "Xorshift RNGs") that supplies the random bits of stochastic rounding: each 64-bit draw gives
// the 32-bit words of two directions (its high, then its low half), and a word's high and low
// halves go to the two species of a pair.  The 64-bit shifts are single instructions on
// gfx950, so a word costs half the instructions of a 32-bit xorshift draw.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint64_t xorshift64(uint64_t x) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
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
// binary16 subnormals included; only the operand's high bits are used).  Each conversion
// writes one half of a 32-bit register and keeps the other, so a species pair is converted
// straight into the packed word that is stored.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
// (only the low half is kept, so the register starts as a live value: no clearing move)
__device__ inline uint16_t f32_to_bf16_sr(float f, uint32_t rnd) {
    bf16x2 t = __builtin_bit_cast(bf16x2, f);
    t = __builtin_amdgcn_cvt_sr_bf16_f32(t, f, rnd, false);
    return __builtin_bit_cast(uint16_t, t[0]);
}
__device__ inline uint16_t f32_to_f16_sr(float f, uint32_t rnd) {
    f16x2 t = __builtin_bit_cast(f16x2, f);
    t = __builtin_amdgcn_cvt_sr_f16_f32(t, f, rnd, false);
    return __builtin_bit_cast(uint16_t, t[0]);
}

template <> struct Codec<BF16> {
    using C = float;
    using S = uint16_t;
    static constexpr bool kRounds = true;
    static constexpr bool kScaled = false;
    static constexpr bool kPacked = true;
    static constexpr int kWide = 2;
    static constexpr bool kHold = false;
    static constexpr int kMinWaves = 1;
    __device__ static C raw(S v) { return __uint_as_float(uint32_t(v) << 16); }
    template <bool SR = false>
    __device__ static S put(C v, uint32_t rnd = 0) {
        if constexpr (SR) return f32_to_bf16_sr(v, rnd);
        else return f32_to_bf16_rne(v);
    }
    // stochastically rounded pair (lo, hi) in one word
    __device__ static u16x2 put_pair_sr(C lo, C hi, uint32_t rlo, uint32_t rhi) {
        // both halves are written, so the register starts as any live value (no clearing move)
        bf16x2 t = __builtin_bit_cast(bf16x2, lo);
        t = __builtin_amdgcn_cvt_sr_bf16_f32(t, lo, rlo, false);
        t = __builtin_amdgcn_cvt_sr_bf16_f32(t, hi, rhi, true);
        return __builtin_bit_cast(u16x2, t);
    }
    __device__ static C decode(S v, float inv) { return raw(v) * inv; }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) { return put<SR>(v * sc, rnd); }
};
template <> struct Codec<F16> {
    using C = float;
    using S = uint16_t;
    static constexpr bool kRounds = true;
    static constexpr bool kScaled = true;
    static constexpr bool kPacked = true;
    static constexpr int kWide = 2;
    static constexpr bool kHold = false;
    static constexpr int kMinWaves = 1;
    __device__ static C raw(S v) { return __half2float(__ushort_as_half(v)); }
    template <bool SR = false>
    __device__ static S put(C v, uint32_t rnd = 0) {
        if constexpr (SR) return f32_to_f16_sr(v, rnd);
        else return __half_as_ushort(__float2half_rn(v));   // IEEE nearest-even
    }
    __device__ static u16x2 put_pair_sr(C lo, C hi, uint32_t rlo, uint32_t rhi) {
        // both halves are written, so the register starts as any live value (no clearing move)
        f16x2 t = __builtin_bit_cast(f16x2, lo);
        t = __builtin_amdgcn_cvt_sr_f16_f32(t, lo, rlo, false);
        t = __builtin_amdgcn_cvt_sr_f16_f32(t, hi, rhi, true);
        return __builtin_bit_cast(u16x2, t);
    }
    __device__ static C decode(S v, float inv) { return raw(v) * inv; }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) { return put<SR>(v * sc, rnd); }
};

// FP32 storage, stochastically rounded from FP64 arithmetic, on the bit pattern of v: the 29
// mantissa bits that FP32 drops are the fraction of the gap from |v| truncated to FP32 to the
// next FP32 magnitude.  Adding 16 random bits (and half a step) at their top and truncating
// them rounds the magnitude up with probability equal to that fraction, to 2^-17 of a unit in
// the last place (the high half of rnd); a carry into the exponent gives the next binade's
// first value, and the truncated value converts to FP32 exactly.  Below FP32's normal range
// the conversion rounds to nearest; non-finite values are kept.  (Choosing between f and its
// neighbour by comparing the FP64 residual with a random fraction of the spacing took about
// 20 vector instructions per value, this about 7.)
__host__ __device__ inline float f64_to_f32_sr(double v, uint32_t rnd) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    b += (unsigned long long)(((rnd >> 16) << 13) + 4096u);
    b &= ~((1ull << 29) - 1ull);
    const float f = float(__builtin_bit_cast(double, b));
    return __builtin_isfinite(v) ? f : float(v);
}

template <> struct Codec<F32X> {
    using C = double;
    using S = float;
    static constexpr bool kRounds = true;
    static constexpr bool kScaled = false;
    static constexpr bool kPacked = false;
    static constexpr int kWide = 0;
    // hold the loaded FP32 values and convert them at each use (the FP64 copies would take twice
    // the registers), and ask for three waves per SIMD (at most 168 VGPRs: 166 for two species
    // without spilling; four waves would spill)
    static constexpr bool kHold = true;
    static constexpr int kMinWaves = 3;
    __device__ static C raw(S v) { return double(v); }
    template <bool SR = false>
    __device__ static S put(C v, uint32_t rnd = 0) {
        if constexpr (SR) return f64_to_f32_sr(v, rnd);
        else return float(v);
    }
    __device__ static C decode(S v, float inv) { return double(v) * double(inv); }
    template <bool SR = false>
    __device__ static S encode(C v, float sc, uint32_t rnd = 0) { return put<SR>(v * double(sc), rnd); }
};

// The stochastically rounded pair of a packed codec (instantiated only for those).
template <class CD>
__device__ __forceinline__ u16x2 put_pair_sr(float lo, float hi, uint32_t rlo, uint32_t rhi) {
    return CD::put_pair_sr(lo, hi, rlo, rhi);
}

// Species-interleaved layout: the NS values of one direction at one node are contiguous,
// element (s, p, node) at ((p * N) + node) * NS + s.  One vector access per direction and
// node; non-temporal, since each element is touched once per step.  Three-element vectors
// are only used where the ISA access has exactly their size (FP32: dwordx3).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x3 __attribute__((ext_vector_type(3), aligned(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

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

// Three species in 2-byte elements would make 6-byte records that no single access fits, so
// that layout is split within each block of a slot: the block's 3 N elements hold species 0
// and 1 interleaved as above with NS = 2 (one 4-byte access per direction and node), then
// species 2 (one 2-byte access).  Both accesses of a direction share the plane's address.
template <class S, int NS>
constexpr bool kSplit = sizeof(S) == 2 && NS == 3;

// Element index of species s in slot arr at the population offsets plane + inplane (Pull::src),
// blk the block part of inplane, N the slot stride (nodes of a block of one slot), for ns
// species of element type S.  In the split 16-bit layout a block of one slot holds 3 N
// elements: the pairs of species 0 and 1 (2 N), then species 2 (N).
template <class S>
__host__ __device__ __forceinline__ size_t elem_at(int s, int arr, uint32_t plane, uint32_t inplane, uint32_t blk, uint32_t N,
                                          int ns) {
    if (sizeof(S) == 2 && ns == 3) {
        const size_t base = ((size_t)arr * N + plane) * 3;
        return s < 2 ? base + blk + 2 * (size_t)inplane + s : base + 2 * (size_t)blk + 2 * (size_t)N + inplane;
    }
    return ((size_t)arr * N + plane + inplane) * ns + s;
}

// The elements of direction slot arr at the population offsets plane + inplane: the address of
// the plane and the slot's place in it (uniform per work-group, formed on the scalar unit)
// plus a 32-bit byte offset within the plane (the populations of a plane hold less than 4 GiB).
template <int NS, class S>
__device__ __forceinline__ S *slot(S *base, int arr, uint32_t plane, uint32_t inplane, uint32_t N) {
    S *start = base + ((size_t)arr * N + plane) * NS;
    using B = std::conditional_t<std::is_const_v<S>, const char, char>;
    return reinterpret_cast<S *>(reinterpret_cast<B *>(start) + (uint32_t)(inplane * (NS * sizeof(S))));
}

// The same for a byte offset already formed within the plane.  The empty asm makes the offset
// a fresh 32-bit value where the access is, so the access keeps the scalar-base form (a
// 64-bit scalar address plus the 32-bit lane offset) instead of a 64-bit vector address.  The
// caller's variable itself is renewed (passed by reference), so the next access takes the new
// value and no register copy of the old one is needed.
template <int NS, class S>
__device__ __forceinline__ S *slot_at(S *base, int arr, uint32_t plane, uint32_t &byte_off, uint32_t N) {
    S *start = base + ((size_t)arr * N + plane) * NS;
    asm volatile("" : "+v"(byte_off));
    using B = std::conditional_t<std::is_const_v<S>, const char, char>;
    return reinterpret_cast<S *>(reinterpret_cast<B *>(start) + byte_off);
}

// An element at a 32-bit byte offset from a uniform address (loads), and the same with the
// offset renewed as in slot_at (stores).
template <class S>
__device__ __forceinline__ S *byte_at(S *start, uint32_t byte_off) {
    using B = std::conditional_t<std::is_const_v<S>, const char, char>;
    return reinterpret_cast<S *>(reinterpret_cast<B *>(start) + byte_off);
}
template <class S>
__device__ __forceinline__ S *byte_at_fresh(S *start, uint32_t &byte_off) {
    asm volatile("" : "+v"(byte_off));
    return byte_at(start, byte_off);
}

// ---------------------------------------------------------------------------------------
// Pull addressing shared by every kernel that reads a pre-collision state: the value of
// direction p at node (x, y, z) comes from slot (p, node - c_p), or from slot (opp(p),
// node) when node - c_p is a wall (half-way bounce-back at rest).
//
// The populations of a fluid plane are stored together, in blocks of B = 2^blog rows (B
// divides ny; pop_block_log2 makes a slot's block about 32 KB): block y / B of plane z holds
// the 19 slots one after another, each B rows of nx nodes.  The value of slot p at (x, y, z) is at the node offset z 19 nx ny (the plane) +
// p B nx (the slot) + (y / B) 19 B nx + (y mod B) nx + x (the row and the node), times the
// species per element.  A work-group's 19 read and 19 write streams then lie within a few
// hundred kilobytes of each other instead of 19 slot arrays apart, which the memory system
// serves faster (the same loads and stores without arithmetic: 5.85 against 5.42 TB/s at 256^3,
// with blocks of 8 rows against whole slot arrays; the step itself 0.827 against 0.896 ms).
struct Pull {
    uint32_t xs, xm, xp;       // x, x-1, x+1 with periodic wrap (per lane)
    uint32_t r0, rm, rp;       // node index parts y nx of the rows y, y-1, y+1 (wrapped)
    uint32_t p0, pm, pp;       // node index parts z nx ny of the planes z, z-1, z+1 (wrapped; uniform)
    uint32_t w0, wm, wp;       // population row offsets of the rows y, y-1, y+1
    uint32_t k0, km, kp;       // ... their block parts (y / B) 19 B nx
    uint32_t q0, qm, qp;       // population plane offsets of the planes z, z-1, z+1 (uniform)
    uint32_t y, z;
    bool bb_lo, bb_hi;         // z - 1 / z + 1 is a wall (slit)

    __host__ __device__ Pull(uint32_t x, uint32_t y_, uint32_t z_, uint32_t nx, uint32_t ny, uint32_t nzf,
                             uint32_t walls, uint32_t blog)
        : xs(x), y(y_), z(z_) {
        xm = (x == 0) ? nx - 1 : x - 1;
        xp = (x + 1 == nx) ? 0 : x + 1;
        const uint32_t ym = (y == 0) ? ny - 1 : y - 1, yq = (y + 1 == ny) ? 0 : y + 1;
        r0 = y * nx;
        rm = ym * nx;
        rp = yq * nx;
        const uint32_t plane = nx * ny;
        p0 = z * plane;
        pm = (z == 0) ? (nzf - 1) * plane : p0 - plane;
        pp = (z + 1 == nzf) ? 0 : p0 + plane;
        const uint32_t bmask = (1u << blog) - 1, bnodes = ((uint32_t)Q << blog) * nx;
        k0 = (y >> blog) * bnodes;
        km = (ym >> blog) * bnodes;
        kp = (yq >> blog) * bnodes;
        w0 = k0 + (y & bmask) * nx;
        wm = km + (ym & bmask) * nx;
        wp = kp + (yq & bmask) * nx;
        const uint32_t qplane = (uint32_t)Q * plane;
        q0 = z * qplane;
        qm = (z == 0) ? (nzf - 1) * qplane : q0 - qplane;
        qp = (z + 1 == nzf) ? 0 : q0 + qplane;
        bb_lo = (walls & 1u) != 0;
        bb_hi = (walls & 2u) != 0;
    }
    // node index (the potential, the charge, the rounding streams)
    __host__ __device__ uint32_t own() const { return p0 + r0 + xs; }
    // population offsets of this node's own values: in-plane offset and its block part
    __host__ __device__ uint32_t own_inplane() const { return w0 + xs; }
    __host__ __device__ uint32_t own_blk() const { return k0; }
    // slot direction, population plane offset (uniform), in-plane offset (per lane) and its
    // block part of the value that direction p pulls
    template <int p>
    __host__ __device__ void src(int &arr, uint32_t &plane, uint32_t &inplane, uint32_t &blk) const {
        constexpr int X = cx(p), Y = cy(p), Z = cz(p);
        const bool bb = (Z == 1 && bb_lo) || (Z == -1 && bb_hi);
        const uint32_t sx = X == 1 ? xm : (X == -1 ? xp : xs);
        const uint32_t sy = Y == 1 ? wm : (Y == -1 ? wp : w0);
        const uint32_t sk = Y == 1 ? km : (Y == -1 ? kp : k0);
        const uint32_t sz = Z == 1 ? qm : (Z == -1 ? qp : q0);
        arr = bb ? opp(p) : p;
        plane = bb ? q0 : sz;
        inplane = bb ? w0 + xs : sy + sx;
        blk = bb ? k0 : sk;
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

// 1 / x, or 0 where x is 0 (a species or mixture with no particles has no velocity).  The
// issue-bound 16-bit forms (FAST): the hardware reciprocal refined by one Newton step (within
// one unit in the last place, where the IEEE division takes four times the instructions);
// otherwise the division.
template <class C, bool FAST>
__device__ __forceinline__ C recip_or_zero(C x) {
    if constexpr (FAST && sizeof(C) == 4) {
        const float r0 = __builtin_amdgcn_rcpf(x);
        const float r = fmaf(r0, fmaf(-x, r0, 1.0f), r0);
        return x != 0.0f ? r : 0.0f;
    } else {
        return x != C(0) ? C(1) / x : C(0);
    }
}

// Weight class of direction p: 0 rest, 1 the axis directions, 2 the face diagonals.  A
// class shares the lattice weight and, in the scaled storage forms, the storage scale.
__host__ __device__ constexpr int wclass(int p) { return p == 0 ? 0 : (p < 7 ? 1 : 2); }
constexpr int kClassRep[3] = {0, 1, 7};   // a direction of each class

// A value made opaque to the compiler where it is used, so a conversion of it is redone there
// instead of being kept alive in registers from an earlier use.
template <class V>
__device__ __forceinline__ V fresh(V x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Waves per SIMD the register budget of stream_collide must allow: the codec's request for one
// or two species (three or four species need more registers than it allows).
template <int NS, class T>
constexpr int step_min_waves() {
    return (NS <= 2) ? Codec<T>::kMinWaves : 1;
}

template <int NS, class T, bool SLIT, bool FIELD, bool CHARGED, int DRAG>
__global__ __launch_bounds__(STEP_BLOCK) __attribute__((amdgpu_waves_per_eu(step_min_waves<NS, T>())))
void stream_collide(const StepArgs a) {
    using CD = Codec<T>;
    using C = typename CD::C;
    using S = typename CD::S;
    using H = std::conditional_t<CD::kHold, S, C>;   // how the loaded values are held
    // tile of this work-group: dispatch order, or for the charged step (which reads the potential
    // around each node) bands of rows per XCD
    uint32_t tx = blockIdx.x, ty = blockIdx.y;
    if constexpr (CHARGED)
        if (a.tiles.band) xcd_tile(blockIdx.x, blockIdx.y, a.tiles, gridDim.x, tx, ty);
    const uint32_t x = tx * blockDim.x + threadIdx.x;
    const uint32_t y = ty * blockDim.y + threadIdx.y;   // uniform per wave if nx >= 64
    const bool active = x < a.nx && y < a.ny;
    const uint32_t z = blockIdx.z;
    const uint32_t walls = SLIT ? a.planes[z].walls : 0u;   // uniform per work-group
    const Pull pl(x < a.nx ? x : 0, y < a.ny ? y : 0, z, a.nx, a.ny, a.nzf, walls, a.blog);
    const uint32_t own = pl.own();
    const uint32_t own_in = pl.own_inplane();
    const uint32_t n4 = a.N * 4u;   // bytes of a block's pairs in the split 16-bit layout
    const S *fin = static_cast<const S *>(a.fin);
    S *fout = static_cast<S *>(a.fout);
    // FP64 carry of the density deviation (uniform; see step 2)
    const bool wide = CD::kWide != 0 && a.wide != 0;

    // inverse storage scale of each species and weight class (1 in the unscaled forms)
    auto isc = [&](int s, int k) -> C { return CD::kScaled ? C(a.inv_scale[s][kClassRep[k]]) : C(1); };
    auto iscd = [&](int s, int k) -> double { return CD::kScaled ? a.inv_scale_k[s][k] : 1.0; };
    // a parameter in the arithmetic type (FP32 kernels take the host's FP32 copy)
    auto par = [](double d, float f) -> C {
        if constexpr (sizeof(C) == sizeof(float)) return f;
        else return C(d);
    };

    // 1. pull streaming with bounce-back: one vector load of all species per direction; the
    //    values stay in stored units (h = d * scale)
    H h[NS][Q];
    static_for<Q>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        int arr;
        uint32_t plane, inplane, blk;
        pl.template src<p>(arr, plane, inplane, blk);
        S raw[NS];
        if constexpr (kSplit<S, NS>) {
            const S *block = fin + ((size_t)arr * a.N + plane) * 3;
            S pair[2];
            VecIO<S, 2>::load(byte_at(block, inplane * 4u + blk * 2u), pair);
            raw[0] = pair[0];
            raw[1] = pair[1];
            raw[2] = __builtin_nontemporal_load(byte_at(block, n4 + inplane * 2u + blk * 4u));
        } else {
            VecIO<S, NS>::load(slot<NS>(fin, arr, plane, inplane, a.N), raw);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if constexpr (CD::kHold) h[s][p] = raw[s];
            else h[s][p] = CD::raw(raw[s]);
        }
    });
    // a loaded value in arithmetic precision where the collision uses it
    auto hc = [&](int s, int p) -> C {
        if constexpr (CD::kHold) return CD::raw(fresh(h[s][p]));
        else return h[s][p];
    };

    // 2. moments (Sec. III): n = rho_bar + dn, dn = sum d, j = sum d c; in the 16-bit forms per
    //    weight class (the classes share a storage scale, so each class sum is scaled once,
    //    and the sums take fewer instructions, which these issue-bound forms need).  The density
    //    deviation is also carried in FP64 (dnh) unless the FP32 form is asked for: with
    //    deviations stored, the update of a direction is w dn + (flux and force terms), and
    //    FP32 rounding at the scale of w dn is deterministic, where stochastic rounding of the
    //    stored values only adds noise that averages out, so it would bias slow modes (about 1 %
    //    of the per-step change of a slow diffusion mode at Sc = 100).  The 16-bit forms get dnh
    //    from the three FP32 class sums, which hold their 8- or 11-bit values exactly unless the
    //    values of a class span more than 2^13 (FP16) or 2^16 (BF16).
    C dn[NS], jx[NS], jy[NS], jz[NS], n[NS];
    double dnh[NS];
    C ntot = 0, sjx = 0, sjy = 0, sjz = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const H *v = h[s];
        if constexpr (!CD::kScaled && !CD::kPacked) {
            // FP32 and FP64 storage (bound by HBM, not by instruction issue): one pass over the
            // directions as they arrive, the FP64 carry alongside
            C m0 = 0, mx = 0, my = 0, mz = 0;
            double m0h = 0.0;
            static_for<Q>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                const C vp = CD::raw(v[p]);
                m0 += vp;
                if constexpr (CD::kWide == 1) m0h += double(v[p]);
                if constexpr (cx(p) == 1) mx += vp;
                if constexpr (cx(p) == -1) mx -= vp;
                if constexpr (cy(p) == 1) my += vp;
                if constexpr (cy(p) == -1) my -= vp;
                if constexpr (cz(p) == 1) mz += vp;
                if constexpr (cz(p) == -1) mz -= vp;
            });
            dn[s] = m0;
            jx[s] = mx;
            jy[s] = my;
            jz[s] = mz;
            dnh[s] = (CD::kWide == 1 && wide) ? m0h : double(m0);
            n[s] = par(a.rho_bar[s], a.rho_bar_f[s]) + dn[s];
            ntot += n[s];
            sjx += jx[s];
            sjy += jy[s];
            sjz += jz[s];
            continue;
        }
        const C m1 = ((v[1] + v[2]) + (v[3] + v[4])) + (v[5] + v[6]);
        const C m2 = (((v[7] + v[8]) + (v[9] + v[10])) + ((v[11] + v[12]) + (v[13] + v[14]))) +
                     ((v[15] + v[16]) + (v[17] + v[18]));
        const C d78 = v[7] - v[8], d910 = v[9] - v[10], d1112 = v[11] - v[12];
        const C d1314 = v[13] - v[14], d1516 = v[15] - v[16], d1718 = v[17] - v[18];
        const C x2 = (d78 + d910) + (d1112 + d1314);
        const C y2 = (d78 - d910) + (d1516 + d1718);
        const C z2 = (d1112 - d1314) + (d1516 - d1718);
        if constexpr (CD::kScaled) {
            dn[s] = (v[0] * isc(s, 0) + m1 * isc(s, 1)) + m2 * isc(s, 2);
            jx[s] = (v[1] - v[2]) * isc(s, 1) + x2 * isc(s, 2);
            jy[s] = (v[3] - v[4]) * isc(s, 1) + y2 * isc(s, 2);
            jz[s] = (v[5] - v[6]) * isc(s, 1) + z2 * isc(s, 2);
        } else {
            dn[s] = (v[0] + m1) + m2;
            jx[s] = (v[1] - v[2]) + x2;
            jy[s] = (v[3] - v[4]) + y2;
            jz[s] = (v[5] - v[6]) + z2;
        }
        dnh[s] = double(dn[s]);
        if constexpr (CD::kWide == 2) {
            if (wide)
                dnh[s] = (double(v[0]) * iscd(s, 0) + double(m1) * iscd(s, 1)) + double(m2) * iscd(s, 2);
        }
        n[s] = par(a.rho_bar[s], a.rho_bar_f[s]) + dn[s];
        ntot += n[s];
        sjx += jx[s];
        sjy += jy[s];
        sjz += jz[s];
    }
    const C inv_ntot = recip_or_zero<C, CD::kPacked>(ntot);
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
    const C ov = par(a.omega_v, a.omega_v_f), od = SLIT ? C(a.planes[z].omega_d) : par(a.omega_d, a.omega_d_f);
    C uax[NS], uay[NS], uaz[NS], Fx[NS], Fy[NS], Fz[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const C inv_n = recip_or_zero<C, CD::kPacked>(n[s]);
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
            const C hb = FIELD ? C(0.5) * C(a.valence[b]) : C(0);
            vx[b] = uax[b] + hb * fx;
            vy[b] = uay[b] + hb * fy;
            vz[b] = uaz[b] + hb * fz;
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

    // Collision coefficients per species and weight class k, in stored units (W_k = w_k x the
    // class's storage scale):
    //   f*_p = (1 - ov) d_p + W_k [base + 4.5 ov n (c.u_s)^2 + 9 n (c.F)(c.u)]
    //          +- 3 W_k n (ov c.u_s + c.F) + W_k ov dn
    // With the FP64 carry the last term is split hi + lo (hi its FP32 rounding, lo the rest).
    //   The 16-bit forms (bound by instruction issue) take the weight into per-class
    //   coefficients here and fold the whole term into the symmetric part, B_k + lo + hi, once
    //   per class: that saves an add per direction and species, and over 8 rounding streams the
    //   diffusivity at Sc = 100 came out the same as with hi added last (the stored value is
    //   rounded to 11 or 8 bits afterwards).  The others (bound by HBM, stored in FP32) add lo
    //   and then hi last, so the stored value rounds like the FP64 sum, and multiply by the
    //   constant weight where a direction is collided, which keeps this block, and the time
    //   before a wave's first store, short.
    constexpr bool kF64 = sizeof(C) == 8;
    constexpr bool kPre = CD::kPacked;
    C B[NS][3], O[NS][3], N9[NS][3], M3[NS][3], bhi[NS][3], blo[NS][3];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const C uu = uax[s] * uax[s] + uay[s] * uay[s] + uaz[s] * uaz[s];
        const C Fu = Fx[s] * ux + Fy[s] * uy + Fz[s] * uz;
        const C base = -C(1.5) * ov * n[s] * uu - C(3) * n[s] * Fu;
        const C t45 = C(4.5) * ov * n[s], t9 = C(9) * n[s], t3 = C(3) * n[s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const C W = kPre ? (kF64 ? C(a.cw[s][k]) : C(a.cwf[s][k])) : C(1);   // w_k scale_k
            B[s][k] = W * base;
            O[s][k] = W * t45;
            N9[s][k] = W * t9;
            M3[s][k] = W * t3;
            blo[s][k] = C(0);
            if (wide) {
                const double big = a.cwo[s][k] * dnh[s];                  // w_k ov scale_k dn
                bhi[s][k] = C(big);
                blo[s][k] = C(big - double(bhi[s][k]));
            } else {
                bhi[s][k] = (kF64 ? C(a.cwo[s][k]) : C(a.cwof[s][k])) * dn[s];
            }
            if constexpr (kPre) B[s][k] = (B[s][k] + blo[s][k]) + bhi[s][k];
        }
    }

    // 5. collision and store, one direction pair at a time, all species per vector store.
    //    Stochastic rounding takes 32 random bits per direction and species pair from a
    //    per-node xorshift64 stream, 16 bits per species.
    const C keep = C(1) - ov;
    auto collide_store = [&](auto sr_tag) {
        constexpr bool SR = decltype(sr_tag)::value;
        const uint32_t seed = a.step_dev ? step_seed(a.round_seed, *a.step_dev + 1ull) : a.seed;
        uint64_t rs = SR ? ((uint64_t(mix32(own ^ seed)) << 32) | uint64_t(own ^ (seed * 0x9e3779b9u)) | 1ull)
                         : 0ull;
        uint32_t word = 0u, spare = 0u;
        bool have_spare = false;
        // byte offsets of this node in a plane of the output (the second for the separate
        // third-species array of the split 16-bit layout)
        uint32_t soff = own_in * (uint32_t)((kSplit<S, NS> ? 2 : NS) * sizeof(S)) + (kSplit<S, NS> ? pl.own_blk() * 2u : 0u);
        uint32_t soff1 = n4 + own_in * (uint32_t)sizeof(S) + pl.own_blk() * 4u;
        auto rbits = [&](int s) -> uint32_t {     // the conversions use the high bits
            if constexpr (!SR) return 0u;
            if ((s & 1) == 0) {
                if (have_spare) {
                    word = spare;
                } else {
                    rs = xorshift64(rs);
                    word = uint32_t(rs >> 32);
                    spare = uint32_t(rs);
                }
                have_spare = !have_spare;
            }
            return (s & 1) ? (word << 16) : word;
        };
        // encode the values of direction P and store them with one vector store
        auto put_all = [&](auto pc, const C (&v)[NS]) {
            constexpr int p = decltype(pc)::value;
            S o[NS];
            if constexpr (SR && CD::kPacked && NS >= 2) {   // pairs into packed words, an odd last one alone
#pragma unroll
                for (int s = 0; s + 1 < NS; s += 2) {
                    const uint32_t r0 = rbits(s), r1 = rbits(s + 1);
                    const u16x2 pr = put_pair_sr<CD>(v[s], v[s + 1], r0, r1);
                    o[s] = pr[0];
                    o[s + 1] = pr[1];
                }
                if constexpr (NS % 2 == 1) o[NS - 1] = CD::template put<SR>(v[NS - 1], rbits(NS - 1));
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) o[s] = CD::template put<SR>(v[s], rbits(s));
            }
            if constexpr (kSplit<S, NS>) {
                const S pair[2] = {o[0], o[1]};
                S *block = fout + ((size_t)p * a.N + pl.q0) * 3;
                VecIO<S, 2>::store(byte_at_fresh(block, soff), pair);
                __builtin_nontemporal_store(o[2], byte_at_fresh(block, soff1));
            } else {
                VecIO<S, NS>::store(slot_at<NS>(fout, p, pl.q0, soff, a.N), o);
            }
        };
        {
            C v0[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if constexpr (kPre)
                    v0[s] = keep * hc(s, 0) + B[s][0];
                else
                    v0[s] = ((keep * hc(s, 0) + wgt<C>(0) * B[s][0]) + blo[s][0]) + bhi[s][0];
            }
            put_all(std::integral_constant<int, 0>{}, v0);
        }
        static_for<9>([&](auto kc) {
            constexpr int p = 2 * decltype(kc)::value + 1;   // 1, 3, ..., 17
            constexpr int pb = p + 1;
            constexpr int k = wclass(p);
            const C cub = cdot<p>(ux, uy, uz);
            C vp[NS], vb[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const C cu = cdot<p>(uax[s], uay[s], uaz[s]);
                const C cF = cdot<p>(Fx[s], Fy[s], Fz[s]);
                if constexpr (kPre) {
                    const C sym = (B[s][k] + O[s][k] * (cu * cu)) + N9[s][k] * (cF * cub);
                    const C anti = M3[s][k] * (ov * cu + cF);
                    vp[s] = (keep * hc(s, p) + sym) + anti;
                    vb[s] = (keep * hc(s, pb) + sym) - anti;
                } else {
                    constexpr C w = wgt<C>(p);
                    const C sym = w * (B[s][k] + O[s][k] * cu * cu + N9[s][k] * cF * cub);
                    const C anti = w * M3[s][k] * (ov * cu + cF);
                    vp[s] = (((keep * hc(s, p) + sym) + anti) + blo[s][k]) + bhi[s][k];
                    vb[s] = (((keep * hc(s, pb) + sym) - anti) + blo[s][k]) + bhi[s][k];
                }
            }
            put_all(std::integral_constant<int, p>{}, vp);
            put_all(std::integral_constant<int, pb>{}, vb);
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
    block_sum_store_dpp<NS>(v, a.partials, nb, bid);
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
