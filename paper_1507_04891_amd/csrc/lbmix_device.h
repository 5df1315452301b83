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

}  // namespace lbmix
