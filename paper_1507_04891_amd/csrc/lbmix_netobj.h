// Internal hooks of the network object (lbmix_net of include/lbmix.h) used by the lattice
// runtime for the learned warm start and its training.  Status codes are LBMIX_*.
#pragma once

#include "lbmix.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbmix {

int net_in_channels(const lbmix_net *net);
int net_device(const lbmix_net *net);
// y[N] = net(x[cin][N]) on `stream`.
int net_forward(lbmix_net *net, const float *x, float *y, uint32_t nx, uint32_t ny, uint32_t nz, int zwalls,
                hipStream_t stream);
// Forward, mean-square loss against t[N] and back-propagation; the gradients stay on the
// device for net_adam.  *loss (if not null) receives the loss (synchronises the stream).
int net_gradient(lbmix_net *net, const float *x, const float *t, uint32_t nx, uint32_t ny, uint32_t nz, int zwalls,
                 double *loss, hipStream_t stream);
int net_adam(lbmix_net *net, float lr, hipStream_t stream);
// Output scale alpha of the warm start (0: not set yet).
double net_output_scale(const lbmix_net *net);
void net_set_output_scale(lbmix_net *net, double alpha);
// Root mean square of t[N] (synchronises the stream).
int net_rms(lbmix_net *net, const float *t, uint32_t N, double *rms, hipStream_t stream);

}  // namespace lbmix
