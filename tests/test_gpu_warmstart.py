"""The learned warm start of the Poisson solve on the GPU against its FP64 reference.

Every convolution of the library rounds its weights and its inputs to BF16 (nearest-even,
unit roundoff u = 2^-9) and accumulates in FP32; the bars follow from that:

* one layer against the FP64 reference fed the same BF16-rounded weights and inputs: only the
  FP32 accumulation differs, K 2^-24 sum |w| |x| with K = 27 cin + 1 products and bias;
* the whole network against the exact FP64 reference (FP32 parameters and inputs): per layer
  the products carry (2 u + u^2) |w| |x| from rounding both operands plus the accumulation,
  and the error of the layer's input goes through |W| (ReLU does not increase it), so
  |y - y_ref| <= e_L elementwise with e_{l+1} = |W_l| * e_l + c |W_l| * (|a_l| + e_l),
  c = 2 u + u^2 + K 2^-24 (* the convolution, a_l the reference activations);
* back-propagated gradient against FP64 central finite differences of the loss, on a sample
  of parameters of every layer: both passes round every operand, about eight BF16 roundings
  along each path of the three-layer network, so 3e-2 of max|g| + 3e-2 |g|;
* the first Adam step: p - lr g / (|g| + eps);
* training through the lattice lowers the loss, and the multigrid solve started from the
  learned guess reaches the same potential as the direct solve.
"""
import numpy as np
import pytest

import workloads as WL
from oracle import warmstart_net as R

pytestmark = pytest.mark.gpu

U = 2.0 ** -9          # BF16 unit roundoff (nearest-even)
E32 = 2.0 ** -24       # FP32 unit roundoff


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    return P


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def bf16(a):
    """Round float32 values to BF16, nearest-even (finite values), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(w, a, zwalls):
    """sum_k w[:, :, k] x shifted by tap k (the reference's convolution, no bias)."""
    y = np.zeros((w.shape[0],) + a.shape[1:])
    for k, (dz, dy, dx) in enumerate(R.TAPS):
        y += np.einsum("oc,c...->o...", w[:, :, k], R.shifted(a, dz, dy, dx, zwalls))
    return y


def rounding_bound(params, ch, x, zwalls):
    """Elementwise bound e_L of |BF16-operand network - FP64 network| (module docstring)."""
    a = np.asarray(x, dtype=np.float64)
    e = np.zeros_like(a)
    L = R.layers(params, ch)
    for l, (w, b) in enumerate(L):
        K = 27 * w.shape[1] + 1
        c = 2 * U + U * U + K * E32
        aw = np.abs(w)
        e = conv(aw, e, zwalls) + c * (conv(aw, np.abs(a) + e, zwalls) + np.abs(b)[:, None, None, None])
        y = conv(w, a, zwalls) + b[:, None, None, None]
        a = np.maximum(y, 0.0) if l + 1 < len(L) else y
    return e


@pytest.mark.parametrize("cin,zwalls", [(16, True), (16, False), (5, True)])
def test_one_layer_is_bf16_products_with_fp32_sums(P, cin, zwalls):
    """A one-layer network cin -> 1: 16 channel pairs run on the BF16 matrix cores, 5 on the
    per-node kernel.  Against the FP64 reference fed the BF16-rounded weights and inputs, only
    the FP32 accumulation of the K = 27 cin products and the bias remains."""
    nx, ny, nz = 9, 6, 7
    net = P.Net(cin, 16, 1, seed=4)
    rng = np.random.default_rng(9)
    p = rng.uniform(-1, 1, net.num_params).astype(np.float32)
    net.set_params(p)
    x = rng.standard_normal((cin, nz, ny, nx)).astype(np.float32)
    y = net.forward(_cuda(x), z_walls=zwalls).cpu().numpy()[0]
    [(w, b)] = R.layers(p.astype(np.float64), [cin, 1])
    wr, xr = bf16(w), bf16(x)
    want = conv(wr, xr, zwalls)[0] + b[0]
    K = 27 * cin + 1
    bound = K * E32 * (conv(np.abs(wr), np.abs(xr), zwalls)[0] + abs(b[0]))
    assert np.all(np.abs(y - want) <= bound), (np.abs(y - want) / bound).max()
    # against the unrounded weights and inputs the difference is of the BF16 size, far above
    # FP32 rounding
    exact = conv(w, x.astype(np.float64), zwalls)[0] + b[0]
    assert np.abs(y - exact).max() > 1e-4 * np.abs(exact).max()


@pytest.mark.parametrize("zwalls,dims", [(True, (8, 6, 5)), (False, (7, 4, 6)), (True, (33, 3, 4))])
def test_forward_matches_fp64_reference_within_bf16_rounding(P, zwalls, dims):
    nx, ny, nz = dims
    net = P.Net(2, 16, 4, seed=3)
    rng = np.random.default_rng(1)
    p = net.params()
    p[-1] = 0.05   # a non-zero output bias
    net.set_params(p)
    x = rng.standard_normal((2, nz, ny, nx)).astype(np.float32)
    y = net.forward(_cuda(x), z_walls=zwalls).cpu().numpy()
    ch = [2, 16, 16, 16, 1]
    ref = R.forward(p, ch, x, zwalls)
    bound = rounding_bound(p.astype(np.float64), ch, x, zwalls)
    assert np.all(np.abs(y - ref) <= bound), (np.abs(y - ref) / (bound + 1e-300)).max()
    # the rounding is really BF16: the error is far above FP32 rounding
    assert np.abs(y - ref).max() > 1e-5 * np.abs(ref).max()


def test_gradient_matches_finite_differences(P):
    nx, ny, nz = 6, 5, 4
    ch = [2, 8, 8, 1]
    net = P.Net(2, 8, 3, seed=5)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, nz, ny, nx)).astype(np.float32)
    t = rng.standard_normal((1, nz, ny, nx)).astype(np.float32)
    loss = net.loss_and_gradient(_cuda(x), _cuda(t), z_walls=True)
    p = net.params().astype(np.float64)
    assert abs(loss - R.loss(p, ch, x, t, True)) <= 2e-2 * loss
    g = net.gradient()
    # every bias and a random sample of the weights of every layer
    offs, o = [], 0
    for l in range(3):
        n_w = ch[l + 1] * ch[l] * 27
        offs += list(rng.choice(np.arange(o, o + n_w), size=12, replace=False)) + list(range(o + n_w, o + n_w + ch[l + 1]))
        o += n_w + ch[l + 1]
    fd = R.fd_gradient(p, ch, x, t, True, offs)
    got = g[offs]
    assert np.all(np.abs(got - fd) <= 3e-2 * np.abs(g).max() + 3e-2 * np.abs(fd)), np.abs(got - fd).max()


def test_first_adam_step(P):
    net = P.Net(2, 4, 2, seed=7)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 4, 4)).astype(np.float32)
    t = rng.standard_normal((1, 4, 4, 4)).astype(np.float32)
    p0 = net.params()
    net.loss_and_gradient(_cuda(x), _cuda(t))
    g = net.gradient()
    net.adam(1e-2)
    p1 = net.params()
    want = p0 - 1e-2 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, want, rtol=0, atol=2e-6)


def test_training_and_learned_warm_start_on_a_charged_slit(P):
    w = WL.charged_slit(nx=16, ny=16, nz=34, n_ion=1e-3, debye_length=4.0, sigma=-3e-4, Ex=1e-4, sc=100.0)
    net = P.Net(5, 16, 4, seed=11)
    lat = P.from_workload(w, storage="f64", poisson=dict(method="direct"))
    losses = lat.train_warm_start(net, 150, lr=2e-3)[3:]   # samples start once three solutions exist
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.5 * losses[:20].mean(), (losses[:20].mean(), losses[-20:].mean())
    # multigrid from the learned guess, against the direct solve of the same states
    a = P.from_workload(w, storage="f64", poisson=dict(method="multigrid", rel_tol=1e-11, max_sweeps=100))
    a.set_warm_start_net(net)
    a.set_poisson(method="multigrid", rel_tol=1e-11, max_sweeps=100, warm_start="learned")
    b = P.from_workload(w, storage="f64", poisson=dict(method="direct"))
    a.step(30)
    b.step(30)
    pa, pb = a.potential(), b.potential()
    assert np.abs(pa - pb).max() <= 1e-8 * np.abs(pb).max()
    assert a.stats()["last_residual"] <= 1e-11


def test_learned_warm_start_gain_on_the_section4_slit(P):
    """What the trained network gains over the method without it, on the charged slit of
    Sec. IV (64 x 64 x 130, lambda_D = 8, sigma = -1e-4, E_x = 1e-4, Sc = 100, f32s): the
    network (5 -> 16 -> 16 -> 16 -> 1, BF16 operands) is trained for 300 steps on the exact
    corrections of the extrapolated guess after 200 steps of developed flow; then multigrid
    to a relative residual of 1e-8 is run for 200 + 50 steps from each warm start and its
    V-cycles per step over the last 50 are counted.  Measured on MI355X by the warm-start
    bench (600 training steps, 100 counted steps): previous potential 3.84, extrapolation
    1.15, learned 5.8 to 6.1 cycles per step (two runs).  The extrapolation beats the previous potential, and the learned correction, whose
    error is above that of the extrapolation it corrects, makes multigrid work harder: the
    network gains nothing over the extrapolation, and multigrid still reaches the tolerance
    from its guess."""
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    net = P.Net(5, 16, 4, seed=1)
    lat = P.from_workload(w, storage="f32s", poisson=dict(method="direct"))
    lat.step(200)
    losses = lat.train_warm_start(net, 300, lr=1e-3)[3:]
    assert np.all(np.isfinite(losses))
    cycles = {}
    for warm in ("previous", "extrapolated", "learned"):
        a = P.from_workload(w, storage="f32s", poisson=dict(method="multigrid", rel_tol=1e-8, max_sweeps=1000))
        if warm == "learned":
            a.set_warm_start_net(net)
        a.set_poisson(method="multigrid", rel_tol=1e-8, max_sweeps=1000, warm_start=warm)
        a.step(200)
        s0 = a.stats()
        a.step(50)
        s1 = a.stats()
        cycles[warm] = (s1["total_sweeps"] - s0["total_sweeps"]) / 50
        assert s1["last_residual"] <= 1e-8
    assert cycles["extrapolated"] < cycles["previous"], cycles
    assert cycles["learned"] > cycles["extrapolated"], cycles
