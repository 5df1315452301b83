// Device helpers shared by the kernels of the library (not a public interface).
#pragma once

#include "lbmix_step.h"

#include <type_traits>

namespace lbmix {

template <int P, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (P > 0) {
        static_for<P - 1>(f);
        f(std::integral_constant<int, P - 1>{});
    }
}

// Deterministic work-group sum of NV doubles (fixed shuffle tree, fixed wave order).
template <int NV>
__device__ void block_sum_store(double (&v)[NV], double *partials, uint32_t nblocks, uint32_t bid) {
    __shared__ double red[NV][STEP_BLOCK / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        v[k] = t;
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;     // blockDim.x is a multiple of 64
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0)
        for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[tid][w];
        partials[(size_t)tid * nblocks + bid] = s;
    }
}

// Sum of a double over the 64 lanes of a wave, complete in lane 63, by data-parallel-primitive
// moves: shifts by 1, 2, 4 and 8 lanes within each row of 16 (lanes without a source add 0),
// then lane 15 of each row added into the next row and lane 31 into the upper half.  Each
// step moves the two 32-bit halves and adds in FP64 (fixed order, so the result is the same
// on every run).  It takes 18 vector instructions where a shuffle tree takes about 40 and 12
// permutes through the LDS crossbar.
__device__ __forceinline__ double wave_sum_to_lane63(double v) {
    auto step = [](double t, auto ctrl, auto rows) -> double {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, t);
        const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, decltype(ctrl)::value, decltype(rows)::value,
                                                0xf, true);
        const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), decltype(ctrl)::value,
                                                decltype(rows)::value, 0xf, true);
        return t + __builtin_bit_cast(double, ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
    };
    v = step(v, std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xf>{});   // row_shr:1
    v = step(v, std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xf>{});   // row_shr:2
    v = step(v, std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xf>{});   // row_shr:4
    v = step(v, std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xf>{});   // row_shr:8
    v = step(v, std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xa>{});   // row_bcast:15
    v = step(v, std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xc>{});   // row_bcast:31
    return v;
}

// block_sum_store with the wave sums of wave_sum_to_lane63 (the fused step: issue-bound).  A
// work-group that ends in a partial wave (rows of a plane narrower than 64 nodes) has no lane
// 63 there, so it sums all its threads' values from LDS in thread order instead.
template <int NV>
__device__ void block_sum_store_dpp(const double (&v)[NV], double *partials, uint32_t nblocks, uint32_t bid) {
    __shared__ double red[NV][STEP_BLOCK];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nt = blockDim.x * blockDim.y;
    if (nt & 63) {   // uniform
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][tid] = v[k];
        __syncthreads();
        if (tid < NV) {
            double s = 0.0;
            for (int i = 0; i < nt; ++i) s += red[tid][i];
            partials[(size_t)tid * nblocks + bid] = s;
        }
        return;
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double t = wave_sum_to_lane63(v[k]);
        if (lane == 63) red[k][wave] = t;
    }
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
        for (int w = 0; w < (nt >> 6); ++w) s += red[tid][w];
        partials[(size_t)tid * nblocks + bid] = s;
    }
}

}  // namespace lbmix
