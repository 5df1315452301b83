// The network object of the learned warm start: parameters, Adam state and activation
// workspace on the device, the forward pass, back-propagation of a mean-square loss and the
// Adam update, behind the lbmix_net_* calls of include/lbmix.h.
#include "lbmix.h"
#include "lbmix_net.h"
#include "lbmix_netobj.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace lbmix;

namespace {

// Activation scratch of lbmix_net_forward_noalloc: the outputs of the hidden layers, in two
// buffers used in turn, held in a static device array instead of allocated memory.  Each GPU
// the library runs on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only stands in for the symbol): the device address
// comes from hipGetSymbolAddress, once per device, and is kept in scratch_addr.
constexpr size_t NET_SCRATCH_BYTES = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[NET_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_addr[MAX_DEVICES] = {};

}  // namespace

struct lbmix_net {
    std::vector<int> ch;              // channels at each layer boundary: cin, hidden..., 1
    std::vector<size_t> woff, boff;   // parameter offsets of each layer's weights and bias
    size_t nparams = 0;
    int device = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // parameters, gradients, moments
    int adam_steps = 0;
    double out_scale = 0.0;           // warm start: correction = alpha s y (0: not set)
    // workspace for lattices of up to cap nodes
    size_t cap = 0;
    float *act = nullptr;             // outputs of every layer, [layer][ch][N]
    float *gb[2] = {nullptr, nullptr};   // gradients of activations (max channels x N)
    float *wt = nullptr;              // transposed weights of one layer
    double *partials = nullptr, *dloss = nullptr;
    float *wpart = nullptr;           // per-wave partial weight gradients
    std::string err;

    int layers() const { return (int)ch.size() - 1; }
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
        return fail(e == hipErrorOutOfMemory ? LBMIX_ENOMEM : LBMIX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    size_t act_offset(int l, size_t N) const {   // output of layer l
        size_t o = 0;
        for (int k = 1; k <= l; ++k) o += (size_t)ch[k] * N;
        return o;
    }
    int workspace(size_t N) {
        if (N <= cap) return LBMIX_OK;
        for (float *q : {act, gb[0], gb[1], wt}) if (q) (void)hipFree(q);
        if (partials) (void)hipFree(partials);
        if (dloss) (void)hipFree(dloss);
        if (wpart) (void)hipFree(wpart);
        act = gb[0] = gb[1] = wt = nullptr;
        partials = dloss = nullptr;
        wpart = nullptr;
        cap = 0;
        size_t tot = 0;
        int cmax = 0;
        for (int k = 1; k < (int)ch.size(); ++k) tot += (size_t)ch[k];
        for (int c : ch) cmax = c > cmax ? c : cmax;
        int rc;
        if ((rc = hip(hipMalloc((void **)&act, tot * N * sizeof(float)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&gb[0], (size_t)cmax * N * sizeof(float)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&gb[1], (size_t)cmax * N * sizeof(float)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&wt, (size_t)NET_MAXC * NET_MAXC * NET_K * sizeof(float)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&partials, ((N + 255) / 256 + 1) * sizeof(double)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&dloss, sizeof(double)), "hipMalloc(net)")) ||
            (rc = hip(hipMalloc((void **)&wpart, conv3_wgrad_workspace((uint32_t)N) * sizeof(float)), "hipMalloc(net)")))
            return rc;
        cap = N;
        return LBMIX_OK;
    }
    ConvArgs conv(int l, const float *x, float *y, uint32_t nx, uint32_t ny, uint32_t nz, int zwalls) const {
        ConvArgs a{};
        a.x = x;
        a.y = y;
        a.w = p + woff[l];
        a.b = p + boff[l];
        a.nx = nx; a.ny = ny; a.nz = nz; a.N = nx * ny * nz;
        a.cin = ch[l];
        a.cout = ch[l + 1];
        a.zwalls = zwalls;
        a.relu = l + 1 < layers() ? 1 : 0;
        return a;
    }
};

namespace {

// splitmix64 stream mapped to [-1, 1)
struct Rng {
    uint64_t s;
    double next() {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
};

int check_dims(lbmix_net *net, int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1 || (double)nx * ny * nz > 2147483647.0)
        return net->fail(LBMIX_EINVAL, "bad lattice extents");
    return LBMIX_OK;
}

}  // namespace

namespace lbmix {

int net_in_channels(const lbmix_net *net) { return net->ch[0]; }
int net_device(const lbmix_net *net) { return net->device; }

int net_forward(lbmix_net *net, const float *x, float *y, uint32_t nx, uint32_t ny, uint32_t nz, int zwalls,
                hipStream_t stream) {
    const size_t N = (size_t)nx * ny * nz;
    int rc = net->workspace(N);
    if (rc) return rc;
    const float *in = x;
    for (int l = 0; l < net->layers(); ++l) {
        float *out = (l + 1 == net->layers() && y) ? y : net->act + net->act_offset(l, N);
        if ((rc = net->hip(launch_conv3(net->conv(l, in, out, nx, ny, nz, zwalls), stream), "conv3"))) return rc;
        in = out;
    }
    return LBMIX_OK;
}

int net_gradient(lbmix_net *net, const float *x, const float *t, uint32_t nx, uint32_t ny, uint32_t nz, int zwalls,
                 double *loss, hipStream_t stream) {
    const size_t N = (size_t)nx * ny * nz;
    int rc = net_forward(net, x, nullptr, nx, ny, nz, zwalls, stream);
    if (rc) return rc;
    const int L = net->layers();
    const float *y = net->act + net->act_offset(L - 1, N);
    uint32_t nb = 0;
    float *g = net->gb[0], *g2 = net->gb[1];
    if ((rc = net->hip(launch_mse(y, t, g, (uint32_t)N, net->partials, &nb, stream), "mse"))) return rc;
    for (int l = L - 1; l >= 0; --l) {
        const float *in = l == 0 ? x : net->act + net->act_offset(l - 1, N);
        const float *out = net->act + net->act_offset(l, N);
        ConvArgs a = net->conv(l, in, nullptr, nx, ny, nz, zwalls);
        if (a.relu && (rc = net->hip(launch_relu_mask(g, out, (uint32_t)(a.cout * N), stream), "relu_mask"))) return rc;
        if ((rc = net->hip(launch_conv3_wgrad(a, g, net->g + net->woff[l], net->g + net->boff[l], net->wpart, stream),
                           "wgrad")))
            return rc;
        if (l == 0) break;
        // gradient of the layer's input: the transposed convolution of g
        if ((rc = net->hip(launch_flip_weights(a.w, net->wt, a.cout, a.cin, stream), "flip"))) return rc;
        ConvArgs b{};
        b.x = g; b.y = g2; b.w = net->wt; b.b = nullptr;
        b.nx = nx; b.ny = ny; b.nz = nz; b.N = (uint32_t)N;
        b.cin = a.cout; b.cout = a.cin; b.zwalls = zwalls; b.relu = 0;
        if ((rc = net->hip(launch_conv3(b, stream), "conv3(transposed)"))) return rc;
        std::swap(g, g2);
    }
    if (loss) {
        std::vector<double> h(nb);
        if ((rc = net->hip(hipMemcpyAsync(h.data(), net->partials, nb * sizeof(double), hipMemcpyDeviceToHost, stream),
                           "copy loss")) ||
            (rc = net->hip(hipStreamSynchronize(stream), "hipStreamSynchronize")))
            return rc;
        double s = 0.0;
        for (double d : h) s += d;
        *loss = s / (double)N;
    }
    return LBMIX_OK;
}

double net_output_scale(const lbmix_net *net) { return net->out_scale; }
void net_set_output_scale(lbmix_net *net, double alpha) { net->out_scale = alpha; }

int net_rms(lbmix_net *net, const float *t, uint32_t N, double *rms, hipStream_t stream) {
    int rc = net->workspace(N);
    if (rc) return rc;
    // mean square of t against a zero target, with the loss kernel (its gradient output is
    // written to scratch)
    float *zero = net->gb[1], *scratch = net->gb[0];
    if ((rc = net->hip(hipMemsetAsync(zero, 0, (size_t)N * sizeof(float), stream), "hipMemset"))) return rc;
    uint32_t nb = 0;
    if ((rc = net->hip(launch_mse(t, zero, scratch, N, net->partials, &nb, stream), "mse"))) return rc;
    std::vector<double> h(nb);
    if ((rc = net->hip(hipMemcpyAsync(h.data(), net->partials, nb * sizeof(double), hipMemcpyDeviceToHost, stream),
                       "copy")) ||
        (rc = net->hip(hipStreamSynchronize(stream), "hipStreamSynchronize")))
        return rc;
    double s = 0.0;
    for (double d : h) s += d;
    *rms = std::sqrt(s / (double)N);
    return LBMIX_OK;
}

int net_adam(lbmix_net *net, float lr, hipStream_t stream) {
    net->adam_steps++;
    return net->hip(launch_adam(net->p, net->g, net->m, net->v, (uint32_t)net->nparams, lr, 0.9f, 0.999f, 1e-8f,
                                net->adam_steps, stream),
                    "adam");
}

}  // namespace lbmix

extern "C" {

int lbmix_net_create(lbmix_net **out, int in_channels, int hidden, int layers, unsigned long long seed) {
    if (!out) return LBMIX_EINVAL;
    *out = nullptr;
    if (in_channels < 1 || in_channels > NET_MAXC || hidden < 1 || hidden > NET_MAXC || layers < 1 || layers > 16)
        return LBMIX_EINVAL;
    lbmix_net *n = new (std::nothrow) lbmix_net();
    if (!n) return LBMIX_ENOMEM;
    n->ch.push_back(in_channels);
    for (int l = 1; l < layers; ++l) n->ch.push_back(hidden);
    n->ch.push_back(1);
    for (int l = 0; l < layers; ++l) {
        n->woff.push_back(n->nparams);
        n->nparams += (size_t)n->ch[l + 1] * n->ch[l] * NET_K;
        n->boff.push_back(n->nparams);
        n->nparams += (size_t)n->ch[l + 1];
    }
    // uniform initialisation scaled by 1 / sqrt(fan-in) (x sqrt(6) for the ReLU layers), biases 0
    std::vector<float> h(n->nparams, 0.0f);
    Rng rng{seed};
    for (int l = 0; l < layers; ++l) {
        const double fan = (double)n->ch[l] * NET_K;
        const double lim = (l + 1 < layers ? std::sqrt(6.0) : 1.0) / std::sqrt(fan);
        for (size_t i = 0; i < (size_t)n->ch[l + 1] * n->ch[l] * NET_K; ++i) h[n->woff[l] + i] = (float)(lim * rng.next());
    }
    int rc = n->hip(hipGetDevice(&n->device), "hipGetDevice");
    const size_t bytes = n->nparams * sizeof(float);
    if (!rc) rc = n->hip(hipMalloc((void **)&n->p, bytes), "hipMalloc(net)");
    if (!rc) rc = n->hip(hipMalloc((void **)&n->g, bytes), "hipMalloc(net)");
    if (!rc) rc = n->hip(hipMalloc((void **)&n->m, bytes), "hipMalloc(net)");
    if (!rc) rc = n->hip(hipMalloc((void **)&n->v, bytes), "hipMalloc(net)");
    if (!rc) rc = n->hip(hipMemcpy(n->p, h.data(), bytes, hipMemcpyHostToDevice), "copy params");
    if (!rc) rc = n->hip(hipMemset(n->g, 0, bytes), "hipMemset");
    if (!rc) rc = n->hip(hipMemset(n->m, 0, bytes), "hipMemset");
    if (!rc) rc = n->hip(hipMemset(n->v, 0, bytes), "hipMemset");
    if (rc) {
        lbmix_net_destroy(n);
        return rc;
    }
    *out = n;
    return LBMIX_OK;
}

int lbmix_net_num_params(const lbmix_net *net) { return net ? (int)net->nparams : LBMIX_EINVAL; }

int lbmix_net_get_params(lbmix_net *net, float *host) {
    if (!net || !host) return LBMIX_EINVAL;
    return net->hip(hipMemcpy(host, net->p, net->nparams * sizeof(float), hipMemcpyDeviceToHost), "copy params");
}

int lbmix_net_set_params(lbmix_net *net, const float *host) {
    if (!net || !host) return LBMIX_EINVAL;
    for (size_t i = 0; i < net->nparams; ++i)
        if (!std::isfinite(host[i])) return net->fail(LBMIX_EINVAL, "non-finite parameter %zu", i);
    int rc = net->hip(hipMemcpy(net->p, host, net->nparams * sizeof(float), hipMemcpyHostToDevice), "copy params");
    if (rc) return rc;
    net->adam_steps = 0;
    const size_t bytes = net->nparams * sizeof(float);
    if ((rc = net->hip(hipMemset(net->m, 0, bytes), "hipMemset"))) return rc;
    return net->hip(hipMemset(net->v, 0, bytes), "hipMemset");
}

int lbmix_net_get_gradient(lbmix_net *net, float *host) {
    if (!net || !host) return LBMIX_EINVAL;
    return net->hip(hipMemcpy(host, net->g, net->nparams * sizeof(float), hipMemcpyDeviceToHost), "copy gradient");
}

int lbmix_net_forward(lbmix_net *net, const float *x_dev, float *y_dev, int nx, int ny, int nz, int z_walls,
                      void *stream) {
    if (!net || !x_dev || !y_dev) return LBMIX_EINVAL;
    int rc = check_dims(net, nx, ny, nz);
    if (rc) return rc;
    return net_forward(net, x_dev, y_dev, nx, ny, nz, z_walls ? 1 : 0, static_cast<hipStream_t>(stream));
}

int lbmix_net_forward_noalloc(lbmix_net *net, const float *x_dev, float *y_dev, int nx, int ny, int nz,
                              int z_walls, void *stream) {
    if (!net || !x_dev || !y_dev) return LBMIX_EINVAL;
    int rc = check_dims(net, nx, ny, nz);
    if (rc) return rc;
    const size_t N = (size_t)nx * ny * nz;
    const int L = net->layers();
    int cmax = 0;
    for (int k = 1; k < L; ++k) cmax = net->ch[k] > cmax ? net->ch[k] : cmax;
    const size_t nbuf = L > 2 ? 2 : (size_t)(L - 1);   // hidden outputs alive at once
    const size_t need = nbuf * (size_t)cmax * N * sizeof(float);
    if (need > NET_SCRATCH_BYTES)
        return net->fail(LBMIX_EINVAL, "%zu nodes need %zu bytes of activation scratch; the static scratch holds %zu",
                         N, need, NET_SCRATCH_BYTES);
    int dev = -1;
    if ((rc = net->hip(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    if (dev != net->device)
        return net->fail(LBMIX_EINVAL, "device %d is current; the network lives on device %d", dev, net->device);
    if (dev < 0 || dev >= MAX_DEVICES) return net->fail(LBMIX_EINVAL, "device ordinal %d out of range", dev);
    float *buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (!scratch_addr[dev]) {
            void *p = nullptr;
            if ((rc = net->hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")))
                return rc;
            scratch_addr[dev] = p;
        }
        buf = static_cast<float *>(scratch_addr[dev]);
    }
    // every output element of a layer is written, so nothing in the scratch needs clearing
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t ux = (uint32_t)nx, uy = (uint32_t)ny, uz = (uint32_t)nz;
    const float *in = x_dev;
    for (int l = 0; l < L; ++l) {
        float *out = (l + 1 == L) ? y_dev : buf + (size_t)(l & 1) * (size_t)cmax * N;
        if ((rc = net->hip(launch_conv3(net->conv(l, in, out, ux, uy, uz, z_walls ? 1 : 0), st), "conv3"))) return rc;
        in = out;
    }
    return LBMIX_OK;
}

int lbmix_net_gradient(lbmix_net *net, const float *x_dev, const float *t_dev, int nx, int ny, int nz, int z_walls,
                       double *loss, void *stream) {
    if (!net || !x_dev || !t_dev) return LBMIX_EINVAL;
    int rc = check_dims(net, nx, ny, nz);
    if (rc) return rc;
    return net_gradient(net, x_dev, t_dev, nx, ny, nz, z_walls ? 1 : 0, loss, static_cast<hipStream_t>(stream));
}

int lbmix_net_adam(lbmix_net *net, float lr, void *stream) {
    if (!net || !(lr > 0.0f)) return LBMIX_EINVAL;
    return net_adam(net, lr, static_cast<hipStream_t>(stream));
}

int lbmix_net_output_scale(lbmix_net *net, double scale, double *current) {
    if (!net || !std::isfinite(scale)) return LBMIX_EINVAL;
    if (scale > 0.0) net->out_scale = scale;
    if (current) *current = net->out_scale;
    return LBMIX_OK;
}

const char *lbmix_net_last_error(const lbmix_net *net) { return net ? net->err.c_str() : "null network"; }

void lbmix_net_destroy(lbmix_net *net) {
    if (!net) return;
    for (float *q : {net->p, net->g, net->m, net->v, net->act, net->gb[0], net->gb[1], net->wt})
        if (q) (void)hipFree(q);
    if (net->partials) (void)hipFree(net->partials);
    if (net->dloss) (void)hipFree(net->dloss);
    if (net->wpart) (void)hipFree(net->wpart);
    delete net;
}

}  // extern "C"
