// gfx950 kernels around the fused step: the initial equilibrium, gathers of the
// pre-collision state, the charge density, the step counter of captured steps, and the
// launchers.  The fused step itself is in lbmix_step_kernel.h.
#include "lbmix_step_kernel.h"

namespace lbmix {

// ---------------------------------------------------------------------------------------
// Initial equilibrium, scattered to the slots of the first pull.

template <class T, bool SLIT>
__global__ __launch_bounds__(BLOCK) void init_equilibrium(const StepArgs a, int s, const double *nf,
                                                         const double *uf) {
    using CD = Codec<T>;
    using S = typename CD::S;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const Pull pl(x, blockIdx.y, blockIdx.z, a.nx, a.ny, a.nzf, SLIT ? a.planes[blockIdx.z].walls : 0u, a.blog);
    const size_t Nfull = (size_t)a.nx * a.ny * a.nzfull;
    const size_t fi = ((size_t)(SLIT ? a.planes[pl.z].zfull : pl.z) * a.ny + pl.y) * a.nx + x;
    const double n = nf[fi];
    const double ux = uf ? uf[fi] : 0.0, uy = uf ? uf[Nfull + fi] : 0.0, uz = uf ? uf[2 * Nfull + fi] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double dn = n - a.rho_bar[s];
    S *f = static_cast<S *>(a.fout);
    static_for<Q>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        const double cu = cx(p) * ux + cy(p) * uy + cz(p) * uz;
        const double dev = wgt<double>(p) * (dn + n * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        int arr;
        uint32_t plane, inplane, blk;
        pl.template src<p>(arr, plane, inplane, blk);
        f[elem_at<S>(s, arr, plane, inplane, blk, a.N, a.ns)] =
            CD::template encode<false>(typename CD::C(dev), a.scale[s][arr]);
    });
}

// Gathers of the pre-collision state at the current time.
template <class T, bool SLIT, int MODE>   // MODE 0: moments, 1: populations
__global__ __launch_bounds__(BLOCK) void gather(const StepArgs a, int s, double *out0, double *out1) {
    using CD = Codec<T>;
    using S = typename CD::S;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const uint32_t zfull = blockIdx.z;
    const size_t Nfull = (size_t)a.nx * a.ny * a.nzfull;
    const size_t fi = ((size_t)zfull * a.ny + blockIdx.y) * a.nx + x;
    const int32_t zf = SLIT ? a.fluid_of_full[zfull] : (int32_t)zfull;
    if (zf < 0) {
        if constexpr (MODE == 0) {
            out0[fi] = 0.0;
            if (out1) out1[fi] = out1[Nfull + fi] = out1[2 * Nfull + fi] = 0.0;
        } else {
            for (int p = 0; p < Q; ++p) out0[(size_t)p * Nfull + fi] = 0.0;
        }
        return;
    }
    const Pull pl(x, blockIdx.y, (uint32_t)zf, a.nx, a.ny, a.nzf, SLIT ? a.planes[zf].walls : 0u, a.blog);
    const S *fin = static_cast<const S *>(a.fin);
    double m0 = 0, mx = 0, my = 0, mz = 0;
    static_for<Q>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        int arr;
        uint32_t plane, inplane, blk;
        pl.template src<p>(arr, plane, inplane, blk);
        const double dv =
            double(CD::decode(fin[elem_at<S>(s, arr, plane, inplane, blk, a.N, a.ns)], a.inv_scale[s][arr]));
        if constexpr (MODE == 1) {
            out0[(size_t)p * Nfull + fi] = dv + wgt<double>(p) * a.rho_bar[s];
        } else {
            m0 += dv;
            mx += cx(p) * dv;
            my += cy(p) * dv;
            mz += cz(p) * dv;
        }
    });
    if constexpr (MODE == 0) {
        out0[fi] = a.rho_bar[s] + m0;
        if (out1) {
            out1[fi] = mx;
            out1[Nfull + fi] = my;
            out1[2 * Nfull + fi] = mz;
        }
    }
}

template <class T, bool SLIT>
__global__ __launch_bounds__(BLOCK) void charge(const StepArgs a, int ns, double *q) {
    using CD = Codec<T>;
    using S = typename CD::S;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const Pull pl(x, blockIdx.y, blockIdx.z, a.nx, a.ny, a.nzf, SLIT ? a.planes[blockIdx.z].walls : 0u, a.blog);
    const S *fin = static_cast<const S *>(a.fin);
    double qq = a.q_rest;
    for (int s = 0; s < ns; ++s) {
        double m0 = 0.0;
        static_for<Q>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            int arr;
            uint32_t plane, inplane, blk;
            pl.template src<p>(arr, plane, inplane, blk);
            m0 += double(CD::decode(fin[elem_at<S>(s, arr, plane, inplane, blk, a.N, a.ns)], a.inv_scale[s][arr]));
        });
        qq += a.valence[s] * m0;
    }
    q[pl.own()] = qq;
}

// ---------------------------------------------------------------------------------------
// Launchers.

dim3 node_grid(uint32_t nx, uint32_t ny, uint32_t nz, dim3 *block) {
    uint32_t bx = ((nx + 63) / 64) * 64;
    if (bx > BLOCK) bx = BLOCK;
    *block = dim3(bx, 1, 1);
    return dim3((nx + bx - 1) / bx, ny, nz);
}

// Width of a work-group's rows for a plane nx >= 64 nodes wide, at most cap (a multiple of
// 64): 256 where it divides nx (measured best for 256^3 and 512^3), else the widest multiple
// of 64 that leaves the fewest idle lanes at the end of a row (a row of 320 nodes in one
// work-group of 320, not in 256 + 256 with 192 idle).
static uint32_t row_width(uint32_t nx, uint32_t cap) {
    if (cap >= 256 && nx % 256 == 0) return 256;
    uint32_t best = 64, waste = ~0u;
    for (uint32_t w = 64; w <= cap; w += 64) {
        const uint32_t idle = (nx + w - 1) / w * w - nx;
        if (idle <= waste) {
            best = w;
            waste = idle;
        }
    }
    return best;
}

dim3 step_grid(uint32_t nx, uint32_t ny, uint32_t nzf, dim3 *block, uint32_t bx, uint32_t by) {
    if (bx > 0 && by > 0 && bx * by <= (uint32_t)STEP_BLOCK) {
        *block = dim3(bx, by, 1);
        return dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nzf);
    }
    if (nx < 64) {   // narrow plane: whole rows, as many as fill the work-group
        bx = nx;
        by = STEP_BLOCK / nx;
        if (by > ny) by = ny;
    } else if (nx <= (uint32_t)BLOCK) {
        bx = ((nx + 63) / 64) * 64;
        by = STEP_BLOCK / BLOCK;   // rows per work-group (two rows of 256 measured best)
    } else {
        bx = row_width(nx, STEP_BLOCK);
        by = STEP_BLOCK / bx;
    }
    *block = dim3(bx, by, 1);
    return dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nzf);
}

void step_shape(Store st, bool stochastic, int ns, uint32_t nx, uint32_t bx_set, uint32_t by_set, uint32_t *bx,
                uint32_t *by) {
    *bx = bx_set;
    *by = by_set;
    if (bx_set != 0) return;
    // FP32 with stochastic rounding (FP64 arithmetic, 135-143 VGPRs for one or two species): three
    // waves per SIMD need work-groups of one row (four waves, one per SIMD)
    if (st == Store::F32 && stochastic && ns <= 2 && nx >= 64) {
        *bx = nx <= (uint32_t)BLOCK ? ((nx + 63) / 64) * 64 : row_width(nx, BLOCK);
        *by = 1;
    }
    // one or two 16-bit species (at most 128 VGPRs: four waves per SIMD): one row of up to 256
    // nodes per work-group instead of two; as many waves fit, and a work-group's last wave
    // (whose mass partial the others wait for) holds fewer (measured: 512^3 f16s 3.86 -> 3.62
    // ms per step, 256^3 0.445 -> 0.441)
    if ((st == Store::F16 || st == Store::BF16) && ns <= 2 && nx >= 64) {
        *bx = nx <= (uint32_t)BLOCK ? ((nx + 63) / 64) * 64 : row_width(nx, STEP_BLOCK);
        *by = 1;
    }
    // three 16-bit species (149 VGPRs: three waves per SIMD): 128-thread work-groups, six per
    // CU, where one 512-thread work-group leaves a third of the wave slots empty (measured: the
    // 64 batched channels 0.78 -> 0.62 ms per step, the 128 x 128 x 258 slit 0.371 -> 0.362;
    // the autotuner picks the same shapes there and two rows of 64 for the 64 x 64 x 130 slit)
    if ((st == Store::F16 || st == Store::BF16) && ns == 3) {
        if (nx >= 64) {
            *bx = nx > 64 ? 128u : 64u;
            *by = 128 / *bx;
        } else {
            *bx = nx;
            *by = 128 / nx > 0 ? 128 / nx : 1;
        }
    }
}

uint32_t stream_collide_blocks(Store st, int ns, const StepArgs &a) {
    dim3 b;
    uint32_t bx, by;
    step_shape(st, a.stochastic != 0, ns, a.nx, a.block_x, a.block_y, &bx, &by);
    const dim3 g = step_grid(a.nx, a.ny, a.nzf, &b, bx, by);
    return g.x * g.y * g.z;
}

hipError_t launch_stream_collide(Store st, int ns, bool slit, bool field, bool charged, const StepArgs &a,
                                 hipStream_t stream) {
    dim3 b;
    uint32_t bx, by;
    step_shape(st, a.stochastic != 0, ns, a.nx, a.block_x, a.block_y, &bx, &by);
    const dim3 g = step_grid(a.nx, a.ny, a.nzf, &b, bx, by);
    StepArgs t = a;
    t.tiles = tile_order(g.x, g.y);
    switch (st) {
        case Store::F64: return stream_collide_store<double>(ns, slit, field, charged, t, g, b, stream);
        case Store::F32:
            return t.stochastic ? stream_collide_store<F32X>(ns, slit, field, charged, t, g, b, stream)
                                : stream_collide_store<float>(ns, slit, field, charged, t, g, b, stream);
        case Store::BF16: return stream_collide_store<BF16>(ns, slit, field, charged, t, g, b, stream);
        case Store::F16: return stream_collide_store<F16>(ns, slit, field, charged, t, g, b, stream);
    }
    return hipErrorInvalidValue;
}

// Dispatch of the per-storage, per-geometry helper kernels.
template <template <class, bool> class K, class... A>
static hipError_t by_store(Store st, bool slit, A &&...args) {
    switch (st) {
        case Store::F64: return slit ? K<double, true>::go(args...) : K<double, false>::go(args...);
        case Store::F32: return slit ? K<float, true>::go(args...) : K<float, false>::go(args...);
        case Store::BF16: return slit ? K<BF16, true>::go(args...) : K<BF16, false>::go(args...);
        case Store::F16: return slit ? K<F16, true>::go(args...) : K<F16, false>::go(args...);
    }
    return hipErrorInvalidValue;
}

template <class T, bool SLIT> struct InitK {
    static hipError_t go(int s, const StepArgs &a, const double *n, const double *u, hipStream_t st) {
        dim3 b;
        const dim3 g = node_grid(a.nx, a.ny, a.nzf, &b);
        hipLaunchKernelGGL((init_equilibrium<T, SLIT>), g, b, 0, st, a, s, n, u);
        return hipGetLastError();
    }
};
template <class T, bool SLIT> struct MomK {
    static hipError_t go(int s, const StepArgs &a, double *n, double *j, hipStream_t st) {
        dim3 b;
        const dim3 g = node_grid(a.nx, a.ny, a.nzfull, &b);
        hipLaunchKernelGGL((gather<T, SLIT, 0>), g, b, 0, st, a, s, n, j);
        return hipGetLastError();
    }
};
template <class T, bool SLIT> struct PopK {
    static hipError_t go(int s, const StepArgs &a, double *f, hipStream_t st) {
        dim3 b;
        const dim3 g = node_grid(a.nx, a.ny, a.nzfull, &b);
        hipLaunchKernelGGL((gather<T, SLIT, 1>), g, b, 0, st, a, s, f, (double *)nullptr);
        return hipGetLastError();
    }
};
template <class T, bool SLIT> struct ChargeK {
    static hipError_t go(int ns, const StepArgs &a, double *q, hipStream_t st) {
        dim3 b;
        const dim3 g = node_grid(a.nx, a.ny, a.nzf, &b);
        hipLaunchKernelGGL((charge<T, SLIT>), g, b, 0, st, a, ns, q);
        return hipGetLastError();
    }
};

__global__ void advance_step(unsigned long long *step) {
    if (threadIdx.x == 0) *step += 1ull;
}

__global__ void set_step(unsigned long long *step, unsigned long long value) {
    if (threadIdx.x == 0) *step = value;
}

hipError_t launch_advance_step(unsigned long long *step, hipStream_t stream) {
    hipLaunchKernelGGL(advance_step, dim3(1), dim3(64), 0, stream, step);
    return hipGetLastError();
}

hipError_t launch_set_step(unsigned long long *step, unsigned long long value, hipStream_t stream) {
    hipLaunchKernelGGL(set_step, dim3(1), dim3(64), 0, stream, step, value);
    return hipGetLastError();
}

// Plain device copy, 16-byte non-temporal loads and stores: each work-group copies 256
// contiguous elements, one per thread.  Measured on one MI355X for 2 GiB: 6.41 TB/s, against
// 6.00 and 6.17 with two and four elements per thread (all loads issued before the stores),
// 4.10 with eight, 5.39-5.52 for grid-stride loops and 5.64 with plain (temporal) accesses;
// reading alone reached 6.93 TB/s and writing alone 6.04.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t COPY_PER_THREAD = 1;
__global__ __launch_bounds__(BLOCK) void copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n) {
    const size_t base = (size_t)blockIdx.x * (BLOCK * COPY_PER_THREAD) + threadIdx.x;
    u32x4 v[COPY_PER_THREAD];
#pragma unroll
    for (uint32_t k = 0; k < COPY_PER_THREAD; ++k) {
        const size_t i = base + (size_t)BLOCK * k;
        if (i < n) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (uint32_t k = 0; k < COPY_PER_THREAD; ++k) {
        const size_t i = base + (size_t)BLOCK * k;
        if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
}

hipError_t launch_copy16(const void *src, void *dst, size_t n16, hipStream_t stream) {
    const size_t per_block = (size_t)BLOCK * COPY_PER_THREAD;
    const size_t blocks = (n16 + per_block - 1) / per_block;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy16, dim3((uint32_t)blocks), dim3(BLOCK), 0, stream, static_cast<const u32x4 *>(src),
                       static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_init(Store st, bool slit, int s, const StepArgs &a, const double *n, const double *u,
                       hipStream_t stream) {
    return by_store<InitK>(st, slit, s, a, n, u, stream);
}
hipError_t launch_moments(Store st, bool slit, int s, const StepArgs &a, double *n, double *j,
                          hipStream_t stream) {
    return by_store<MomK>(st, slit, s, a, n, j, stream);
}
hipError_t launch_populations(Store st, bool slit, int s, const StepArgs &a, double *f, hipStream_t stream) {
    return by_store<PopK>(st, slit, s, a, f, stream);
}
hipError_t launch_charge(Store st, bool slit, int ns, const StepArgs &a, double *q, hipStream_t stream) {
    return by_store<ChargeK>(st, slit, ns, a, q, stream);
}

}  // namespace lbmix
