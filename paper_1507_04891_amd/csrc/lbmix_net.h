// Internal interface of the gfx950 kernels of the learned warm start: a fully convolutional
// network of 3 x 3 x 3 convolutions over a lattice of nx * ny * nz nodes (periodic in x and
// y; in z periodic, or zero beyond the first and last plane for a slit), FP32 activations
// stored [channel][node], node = x + nx (y + ny z).  Not installed; the public interface is
// include/lbmix.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbmix {

constexpr int NET_MAXC = 16;   // channels per layer at most
constexpr int NET_K = 27;      // taps of a 3 x 3 x 3 kernel, k = (dz + 1) 9 + (dy + 1) 3 + (dx + 1)

struct ConvArgs {
    const float *x;        // [cin][N]
    float *y;              // [cout][N]
    const float *w;        // [cout][cin][27]
    const float *b;        // [cout] (may be null)
    uint32_t nx, ny, nz, N;
    int cin, cout;
    int zwalls;            // 1: zero beyond the planes z = 0 and z = nz - 1; 0: periodic
    int relu;              // 1: y = max(0, conv)
};

// y[co][v] = b[co] + sum_ci sum_k w[co][ci][k] x[ci][v + offset_k], then ReLU if asked.
hipError_t launch_conv3(const ConvArgs &a, hipStream_t stream);

// Weights of the transposed convolution: wt[ci][co][k] = w[co][ci][26 - k].
hipError_t launch_flip_weights(const float *w, float *wt, int cout, int cin, hipStream_t stream);

// g[i] *= (y[i] > 0) over n values (derivative of the ReLU whose output is y).
hipError_t launch_relu_mask(float *g, const float *y, uint32_t n, hipStream_t stream);

// gw[co][ci][k] = sum_v g[co][v] x[ci][v + offset_k]; gb[co] = sum_v g[co][v] (fixed order).
// 16 -> 16 layers run on the matrix cores with per-wave partial products in `part`
// (conv3_wgrad_workspace(N) floats; null: the general kernel).
size_t conv3_wgrad_workspace(uint32_t N);
hipError_t launch_conv3_wgrad(const ConvArgs &a, const float *g, float *gw, float *gb, float *part,
                              hipStream_t stream);

// Mean-square loss over n values: g = 2 (y - t) / n, partial sums of (y - t)^2 per block
// into partials (nblocks written to *nb).
hipError_t launch_mse(const float *y, const float *t, float *g, uint32_t n, double *partials, uint32_t *nb,
                      hipStream_t stream);

// One Adam update of n parameters with bias-corrected moments; step >= 1.
hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr, float beta1,
                       float beta2, float eps, int step, hipStream_t stream);

// Warm-start glue on fluid nodes (double potential, float network data), s = *scale:
//   finish_scale: *scale <- sqrt(*scale / N) (the root mean square of r from its square sum;
//                 1 if that is 0);
//   net_input: x0 = r / s, x1 = c / s (c: the coarse-grid solution of A c = r, prolonged),
//              x2 = (p1 - p2) / s, x3 = (guess - p1) / s, x4 = plane_mask[plane] (1 next to a
//              wall, else 0), with p1, p2 the two previous potentials;
//   add_correction: psi[i] += alpha s y[i];
//   correction_target: t[i] = (psi[i] - guess[i]) / (alpha s)  (alpha: output scale).
hipError_t launch_finish_scale(double *scale, uint32_t N, hipStream_t stream);
constexpr int WS_CHANNELS = 5;   // input channels of the warm-start network
hipError_t launch_net_input(const double *r, const double *coarse, const double *p1, const double *p2,
                            const double *guess, const double *scale, float *x, uint32_t nxy, uint32_t nzf,
                            const float *plane_mask, hipStream_t stream);
hipError_t launch_add_correction(double *psi, const float *y, const double *scale, double alpha, uint32_t N,
                                 hipStream_t stream);
hipError_t launch_correction_target(const double *psi, const double *guess, const double *scale, double alpha, float *t,
                                    uint32_t N, hipStream_t stream);

}  // namespace lbmix
