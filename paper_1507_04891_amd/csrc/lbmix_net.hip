// gfx950 kernels of the learned warm start of the Poisson solve: 3 x 3 x 3 convolutions with
// bias and ReLU (forward, transposed for the input gradient, weight gradient), mean-square
// loss, Adam, and the glue between the FP64 potential and the network.  The network works on
// lattices of a few hundred thousand nodes with at most 16 channels.  Every convolution takes
// its weights and its inputs rounded to BF16 (nearest-even) and accumulates in FP32; the
// master parameters, the activations in memory and Adam stay FP32.  Convolutions with at
// least 16 channel pairs run on the BF16 matrix cores (channels zero-padded to 16); smaller
// ones use one thread per node that accumulates every output channel, with the weights of the
// layer in LDS (read by all lanes at once).
#include "lbmix_net.h"

namespace lbmix {

namespace {

// Neighbour of node (x, y, z) at tap k, or -1 beyond a zero-padded z end.
__device__ __forceinline__ int64_t tap(int k, uint32_t x, uint32_t y, uint32_t z, uint32_t nx, uint32_t ny,
                                       uint32_t nz, int zwalls) {
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    const uint32_t xx = dx < 0 ? (x == 0 ? nx - 1 : x - 1) : (dx > 0 ? (x + 1 == nx ? 0 : x + 1) : x);
    const uint32_t yy = dy < 0 ? (y == 0 ? ny - 1 : y - 1) : (dy > 0 ? (y + 1 == ny ? 0 : y + 1) : y);
    int64_t zz = (int64_t)z + dz;
    if (zz < 0 || zz >= (int64_t)nz) {
        if (zwalls) return -1;
        zz = zz < 0 ? nz - 1 : 0;
    }
    return ((int64_t)zz * ny + yy) * nx + xx;
}

}  // namespace

constexpr int NET_BLOCK = 256;

// FP32 value rounded to BF16 (nearest-even) and back: the operands of every product.
__device__ __forceinline__ float bf16r(float v) { return (float)(__bf16)v; }
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(NET_BLOCK) void conv3(const ConvArgs a) {
    __shared__ float sw[NET_MAXC * NET_MAXC * NET_K];
    __shared__ float sb[NET_MAXC];
    const int nw = a.cout * a.cin * NET_K;
    for (int i = threadIdx.x; i < nw; i += NET_BLOCK) sw[i] = bf16r(a.w[i]);
    if ((int)threadIdx.x < a.cout) sb[threadIdx.x] = a.b ? a.b[threadIdx.x] : 0.0f;
    __syncthreads();
    const uint32_t v = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (v >= a.N) return;
    const uint32_t x = v % a.nx, y = (v / a.nx) % a.ny, z = v / (a.nx * a.ny);
    float acc[NET_MAXC];
#pragma unroll
    for (int co = 0; co < NET_MAXC; ++co) acc[co] = co < a.cout ? sb[co] : 0.0f;
    for (int k = 0; k < NET_K; ++k) {
        const int64_t nb = tap(k, x, y, z, a.nx, a.ny, a.nz, a.zwalls);
        if (nb < 0) continue;
        for (int ci = 0; ci < a.cin; ++ci) {
            const float xv = bf16r(a.x[(size_t)ci * a.N + nb]);
            const float *wk = sw + ci * NET_K + k;
#pragma unroll
            for (int co = 0; co < NET_MAXC; ++co)
                if (co < a.cout) acc[co] = fmaf(wk[co * a.cin * NET_K], xv, acc[co]);
        }
    }
    for (int co = 0; co < a.cout; ++co) {
        const float r = acc[co];
        a.y[(size_t)co * a.N + v] = (a.relu && r < 0.0f) ? 0.0f : r;
    }
}

// The same convolution on the BF16 matrix cores, channels zero-padded to 16: a dense
// contraction y[co][v] = sum_{k, ci} w[co][ci][k] x[ci][v + offset_k] with K = 27 x 16.
// Each wave computes tiles of 16 consecutive nodes (one 16 x 16 v_mfma_f32_16x16x16_bf16
// output, rows co, columns the nodes) in 27 steps, one per tap k, each over all 16 channels:
// lane l supplies w[co = l mod 16][ci = 4 (l / 16) + q][k], q < 4, from LDS and
// x[ci = 4 (l / 16) + q][neighbour of node l mod 16], both as four BF16 values.  The output
// rows 4 (l / 16) + r, r < 4, of column l mod 16 come back in the lane (FP32).
typedef float f32x4m __attribute__((ext_vector_type(4)));
constexpr int MFMA_C = 16;

__global__ __launch_bounds__(NET_BLOCK) void conv3_mfma(const ConvArgs a) {
    __shared__ bf16x4 sw[MFMA_C * NET_K * 4];   // [co][k][g]: channels 4 g .. 4 g + 3, zero beyond cout, cin
    for (int i = threadIdx.x; i < MFMA_C * NET_K * 4; i += NET_BLOCK) {
        const int co = i / (NET_K * 4), k = (i / 4) % NET_K, g = i % 4;
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ci = 4 * g + q;
            v[q] = (__bf16)((co < a.cout && ci < a.cin) ? a.w[(co * a.cin + ci) * NET_K + k] : 0.0f);
        }
        sw[i] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const uint32_t ntiles = (a.N + 15) / 16;
    const uint32_t wave = blockIdx.x * (NET_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (NET_BLOCK / 64);
    float bias[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = (a.b && 4 * lk + r < a.cout) ? a.b[4 * lk + r] : 0.0f;
    for (uint32_t t = wave; t < ntiles; t += nwaves) {
        const uint32_t v = t * 16 + li;           // the node of this lane's column
        const bool live = v < a.N;
        const uint32_t vv = live ? v : 0;
        const uint32_t x = vv % a.nx, y = (vv / a.nx) % a.ny, z = vv / (a.nx * a.ny);
        f32x4m acc = {bias[0], bias[1], bias[2], bias[3]};
#pragma unroll 3
        for (int k = 0; k < NET_K; ++k) {
            const int64_t nb = live ? tap(k, x, y, z, a.nx, a.ny, a.nz, a.zwalls) : -1;
            bf16x4 bx;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ci = 4 * lk + q;
                bx[q] = (__bf16)((nb >= 0 && ci < a.cin) ? a.x[(size_t)ci * a.N + nb] : 0.0f);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, sw[(li * NET_K + k) * 4 + lk]),
                                                            __builtin_bit_cast(s16x4, bx), acc, 0, 0, 0);
        }
        if (live) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float o = acc[r];
                if (4 * lk + r < a.cout) a.y[(size_t)(4 * lk + r) * a.N + v] = (a.relu && o < 0.0f) ? 0.0f : o;
            }
        }
    }
}

// Weight gradients on the BF16 matrix cores, channels zero-padded to 16: for every tap k the
// 16 x 16 product gw_k[co][ci] = sum_v g[co][v] x[ci][v + offset_k] is a contraction over
// nodes.  Each wave takes WG_CHUNK consecutive nodes, 16 per step (lane l: nodes 4 (l / 16) + q,
// q < 4, of the step, channel l mod 16 of both operands, as BF16), and keeps the 27 tap
// products in its registers (FP32), plus a 28th with x = 1 whose column 0 is the bias gradient
// sum_v g[co][v]; the per-wave partial products go to part[wave][k][co][ci] and are summed in
// FP64, in a fixed order, by conv3_wgrad_sum.
constexpr uint32_t WG_CHUNK = 256;
constexpr int WG_SLOTS = NET_K + 1;   // 27 taps and the bias

__global__ __launch_bounds__(NET_BLOCK) void conv3_wgrad_mfma(const ConvArgs a, const float *g, float *part) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const uint32_t wave = blockIdx.x * (NET_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t v_begin = wave * WG_CHUNK;
    f32x4m acc[WG_SLOTS];
#pragma unroll
    for (int k = 0; k < WG_SLOTS; ++k) acc[k] = f32x4m{0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t v0 = v_begin; v0 < v_begin + WG_CHUNK && v0 < a.N; v0 += 16) {
        uint32_t px[4], py[4], pz[4];
        bool live[4];
        bf16x4 gv, one;   // A: g[co = li][node 4 lk + q]
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t v = v0 + 4 * lk + q;
            live[q] = v < a.N;
            const uint32_t vv = live[q] ? v : 0;
            px[q] = vv % a.nx;
            py[q] = (vv / a.nx) % a.ny;
            pz[q] = vv / (a.nx * a.ny);
            gv[q] = (__bf16)((live[q] && li < a.cout) ? g[(size_t)li * a.N + v] : 0.0f);
            one[q] = (__bf16)(live[q] ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int k = 0; k < NET_K; ++k) {
            bf16x4 xv;   // B: x[ci = li] at the neighbours of the same nodes
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t nb = live[q] ? tap(k, px[q], py[q], pz[q], a.nx, a.ny, a.nz, a.zwalls) : -1;
                xv[q] = (__bf16)((nb >= 0 && li < a.cin) ? a.x[(size_t)li * a.N + nb] : 0.0f);
            }
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, gv),
                                                               __builtin_bit_cast(s16x4, xv), acc[k], 0, 0, 0);
        }
        acc[NET_K] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, gv),
                                                               __builtin_bit_cast(s16x4, one), acc[NET_K], 0, 0, 0);
    }
    float *out = part + (size_t)wave * WG_SLOTS * MFMA_C * MFMA_C;
#pragma unroll
    for (int k = 0; k < WG_SLOTS; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(k * MFMA_C + 4 * lk + r) * MFMA_C + li] = acc[k][r];
}

// gw[co][ci][k] = sum over waves of part[wave][k][co][ci], and gb[co] from the bias slot
// (column 0): one work-group per weight, FP64, strided per thread and then a fixed tree.
__global__ __launch_bounds__(NET_BLOCK) void conv3_wgrad_sum(const float *part, uint32_t nwaves, int cout, int cin,
                                                              float *gw, float *gb) {
    __shared__ double red[NET_BLOCK];
    const uint32_t i = blockIdx.x;   // (slot, co, ci)
    double s = 0.0;
    for (uint32_t w = threadIdx.x; w < nwaves; w += NET_BLOCK) s += (double)part[(size_t)w * WG_SLOTS * MFMA_C * MFMA_C + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = NET_BLOCK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int k = (int)(i / (MFMA_C * MFMA_C)), co = (int)(i / MFMA_C) % MFMA_C, ci = (int)(i % MFMA_C);
        if (k < NET_K && co < cout && ci < cin)
            gw[(co * cin + ci) * NET_K + k] = (float)red[0];
        else if (k == NET_K && ci == 0 && co < cout)
            gb[co] = (float)red[0];
    }
}

__global__ void flip_weights(const float *w, float *wt, int cout, int cin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * cin * NET_K) return;
    const int co = i / (cin * NET_K), ci = (i / NET_K) % cin, k = i % NET_K;
    wt[(ci * cout + co) * NET_K + (NET_K - 1 - k)] = w[i];
}

__global__ __launch_bounds__(NET_BLOCK) void relu_mask(float *g, const float *y, uint32_t n) {
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (i < n && !(y[i] > 0.0f)) g[i] = 0.0f;
}

// One work-group per weight (co, ci, k), or per bias when k == NET_K: the sum over all nodes
// of the BF16-rounded operands in a fixed order (strided per thread, then a tree), accumulated
// in FP64.
__global__ __launch_bounds__(NET_BLOCK) void conv3_wgrad(const ConvArgs a, const float *g, float *gw, float *gb) {
    __shared__ double red[NET_BLOCK];
    const int idx = blockIdx.x;
    const int per_co = a.cin * NET_K + 1;
    const int co = idx / per_co, r = idx % per_co;
    const bool bias = r == a.cin * NET_K;
    const int ci = bias ? 0 : r / NET_K, k = bias ? 0 : r % NET_K;
    const float *gc = g + (size_t)co * a.N;
    const float *xc = a.x + (size_t)ci * a.N;
    double s = 0.0;
    for (uint32_t v = threadIdx.x; v < a.N; v += NET_BLOCK) {
        if (bias) {
            s += bf16r(gc[v]);
        } else {
            const uint32_t x = v % a.nx, y = (v / a.nx) % a.ny, z = v / (a.nx * a.ny);
            const int64_t nb = tap(k, x, y, z, a.nx, a.ny, a.nz, a.zwalls);
            if (nb >= 0) s += (double)bf16r(gc[v]) * (double)bf16r(xc[nb]);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = NET_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (bias)
            gb[co] = (float)red[0];
        else
            gw[(co * a.cin + ci) * NET_K + k] = (float)red[0];
    }
}

__global__ __launch_bounds__(NET_BLOCK) void mse(const float *y, const float *t, float *g, uint32_t n,
                                                 double *partials) {
    __shared__ double red[NET_BLOCK];
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        d = (double)y[i] - (double)t[i];
        g[i] = (float)(2.0 * d / (double)n);
    }
    red[threadIdx.x] = d * d;
    __syncthreads();
    for (int w = NET_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NET_BLOCK) void adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2) {
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void finish_scale(double *s, uint32_t N) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double r = sqrt(*s / (double)N);
        *s = r > 0.0 ? r : 1.0;
    }
}

__global__ __launch_bounds__(NET_BLOCK) void net_input(const double *r, const double *coarse, const double *p1,
                                                       const double *p2, const double *guess, const double *scale,
                                                       float *x, uint32_t nxy, uint32_t nzf, const float *mask) {
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    const uint32_t N = nxy * nzf;
    if (i >= N) return;
    const double inv = 1.0 / *scale, a = p1[i];
    x[i] = (float)(r[i] * inv);
    x[N + i] = (float)(coarse[i] * inv);
    x[2 * N + i] = (float)((a - p2[i]) * inv);
    x[3 * N + i] = (float)((guess[i] - a) * inv);
    x[4 * N + i] = mask ? mask[i / nxy] : 0.0f;
}

__global__ __launch_bounds__(NET_BLOCK) void add_correction(double *psi, const float *y, const double *scale,
                                                            double alpha, uint32_t N) {
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (i < N) psi[i] += alpha * *scale * (double)y[i];
}

__global__ __launch_bounds__(NET_BLOCK) void correction_target(const double *psi, const double *guess,
                                                               const double *scale, double alpha, float *t,
                                                               uint32_t N) {
    const uint32_t i = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (i < N) t[i] = (float)((psi[i] - guess[i]) / (alpha * *scale));
}

// ---------------------------------------------------------------------------------------
// Launchers.

static dim3 grid_of(uint32_t n) { return dim3((n + NET_BLOCK - 1) / NET_BLOCK); }

hipError_t launch_conv3(const ConvArgs &a, hipStream_t stream) {
    if (a.cin < 1 || a.cin > NET_MAXC || a.cout < 1 || a.cout > NET_MAXC) return hipErrorInvalidValue;
    if (a.cin * a.cout >= 16) {   // the 4 -> 16, 16 -> 16 and 16 -> 1 layers
        // four 16-node tiles per work-group and pass; about two passes per wave
        const uint32_t tiles = (a.N + 15) / 16;
        uint32_t blocks = (tiles + 7) / 8;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(conv3_mfma, dim3(blocks), dim3(NET_BLOCK), 0, stream, a);
    } else {
        hipLaunchKernelGGL(conv3, grid_of(a.N), dim3(NET_BLOCK), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_flip_weights(const float *w, float *wt, int cout, int cin, hipStream_t stream) {
    hipLaunchKernelGGL(flip_weights, grid_of((uint32_t)(cout * cin * NET_K)), dim3(NET_BLOCK), 0, stream, w, wt, cout,
                       cin);
    return hipGetLastError();
}

hipError_t launch_relu_mask(float *g, const float *y, uint32_t n, hipStream_t stream) {
    hipLaunchKernelGGL(relu_mask, grid_of(n), dim3(NET_BLOCK), 0, stream, g, y, n);
    return hipGetLastError();
}

size_t conv3_wgrad_workspace(uint32_t N) {
    const size_t waves = (N + WG_CHUNK - 1) / WG_CHUNK;
    return ((waves + 3) / 4) * 4 * WG_SLOTS * MFMA_C * MFMA_C;
}

hipError_t launch_conv3_wgrad(const ConvArgs &a, const float *g, float *gw, float *gb, float *part,
                              hipStream_t stream) {
    if (a.cin * a.cout >= 16 && part) {
        const uint32_t blocks = (a.N + WG_CHUNK * 4 - 1) / (WG_CHUNK * 4);   // four waves each
        hipLaunchKernelGGL(conv3_wgrad_mfma, dim3(blocks), dim3(NET_BLOCK), 0, stream, a, g, part);
        hipLaunchKernelGGL(conv3_wgrad_sum, dim3(WG_SLOTS * MFMA_C * MFMA_C), dim3(NET_BLOCK), 0, stream, part,
                           blocks * 4, a.cout, a.cin, gw, gb);
        return hipGetLastError();
    }
    const uint32_t blocks = (uint32_t)(a.cout * (a.cin * NET_K + 1));
    hipLaunchKernelGGL(conv3_wgrad, dim3(blocks), dim3(NET_BLOCK), 0, stream, a, g, gw, gb);
    return hipGetLastError();
}

hipError_t launch_mse(const float *y, const float *t, float *g, uint32_t n, double *partials, uint32_t *nb,
                      hipStream_t stream) {
    *nb = grid_of(n).x;
    hipLaunchKernelGGL(mse, grid_of(n), dim3(NET_BLOCK), 0, stream, y, t, g, n, partials);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr, float beta1, float beta2,
                       float eps, int step, hipStream_t stream) {
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam, grid_of(n), dim3(NET_BLOCK), 0, stream, p, g, m, v, n, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_finish_scale(double *scale, uint32_t N, hipStream_t stream) {
    hipLaunchKernelGGL(finish_scale, dim3(1), dim3(64), 0, stream, scale, N);
    return hipGetLastError();
}

hipError_t launch_net_input(const double *r, const double *coarse, const double *p1, const double *p2,
                            const double *guess, const double *scale, float *x, uint32_t nxy, uint32_t nzf,
                            const float *plane_mask, hipStream_t stream) {
    hipLaunchKernelGGL(net_input, grid_of(nxy * nzf), dim3(NET_BLOCK), 0, stream, r, coarse, p1, p2, guess, scale, x,
                       nxy, nzf, plane_mask);
    return hipGetLastError();
}

hipError_t launch_add_correction(double *psi, const float *y, const double *scale, double alpha, uint32_t N,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(add_correction, grid_of(N), dim3(NET_BLOCK), 0, stream, psi, y, scale, alpha, N);
    return hipGetLastError();
}

hipError_t launch_correction_target(const double *psi, const double *guess, const double *scale, double alpha, float *t,
                                    uint32_t N, hipStream_t stream) {
    hipLaunchKernelGGL(correction_target, grid_of(N), dim3(NET_BLOCK), 0, stream, psi, guess, scale, alpha, t, N);
    return hipGetLastError();
}

}  // namespace lbmix
