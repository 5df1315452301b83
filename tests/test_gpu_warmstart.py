"""The learned warm start of the Poisson solve on the GPU against its FP64 reference.

* forward pass of the network (FP32) against oracle/warmstart_net.py (FP64) on the same
  float32 parameters and inputs: 2e-5 of max|y| (about 4 x 27 x 16 FP32 accumulations);
* back-propagated gradient against FP64 central finite differences of the loss, on a
  sample of parameters of every layer: 2e-4 of max|g| + 1e-3 |g|;
* the first Adam step: p - lr g / (|g| + eps);
* training through the lattice lowers the loss, and the multigrid solve started from the
  learned guess reaches the same potential as the direct solve.
"""
import numpy as np
import pytest

import workloads as WL
from oracle import warmstart_net as R

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("zwalls,dims", [(True, (8, 6, 5)), (False, (7, 4, 6)), (True, (33, 3, 4))])
def test_forward_matches_fp64_reference(P, zwalls, dims):
    nx, ny, nz = dims
    net = P.Net(2, 16, 4, seed=3)
    rng = np.random.default_rng(1)
    p = net.params()
    p[-1] = 0.05   # a non-zero output bias
    net.set_params(p)
    x = rng.standard_normal((2, nz, ny, nx)).astype(np.float32)
    y = net.forward(_cuda(x), z_walls=zwalls).cpu().numpy()
    ref = R.forward(p, [2, 16, 16, 16, 1], x, zwalls)
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def test_gradient_matches_finite_differences(P):
    nx, ny, nz = 6, 5, 4
    ch = [2, 8, 8, 1]
    net = P.Net(2, 8, 3, seed=5)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, nz, ny, nx)).astype(np.float32)
    t = rng.standard_normal((1, nz, ny, nx)).astype(np.float32)
    loss = net.loss_and_gradient(_cuda(x), _cuda(t), z_walls=True)
    p = net.params().astype(np.float64)
    assert abs(loss - R.loss(p, ch, x, t, True)) <= 1e-5 * loss
    g = net.gradient()
    # every bias and a random sample of the weights of every layer
    offs, o = [], 0
    for l in range(3):
        n_w = ch[l + 1] * ch[l] * 27
        offs += list(rng.choice(np.arange(o, o + n_w), size=12, replace=False)) + list(range(o + n_w, o + n_w + ch[l + 1]))
        o += n_w + ch[l + 1]
    fd = R.fd_gradient(p, ch, x, t, True, offs)
    got = g[offs]
    assert np.all(np.abs(got - fd) <= 2e-4 * np.abs(g).max() + 1e-3 * np.abs(fd)), np.abs(got - fd).max()


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
    net = P.Net(4, 16, 4, seed=11)
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
