"""lbmix_net_forward_noalloc (activation scratch in the library's static device array, no
allocation) against lbmix_net_forward (workspace the library allocates), through the C ABI.

Both run the same convolution kernels on the same inputs, so the outputs must agree bitwise.
Two calls in a row, the second on a smaller lattice (the scratch keeps the first call's
contents), then a lattice beyond the scratch size, which must be refused before any launch.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    return P


def inputs(shape, seed):
    import torch
    g = np.random.default_rng(seed)
    return torch.tensor(g.standard_normal((4,) + shape).astype(np.float32), device="cuda")


@pytest.mark.parametrize("z_walls", [False, True])
def test_noalloc_forward_matches_allocating_forward(P, z_walls):
    import torch

    net = P.Net(4, 16, 4, seed=3)
    for shape, seed in (((20, 24, 32), 1), ((6, 10, 12), 2)):   # [nz][ny][nx], the second smaller
        x = inputs(shape, seed)
        ref = net.forward(x, z_walls=z_walls)
        y = torch.full((1,) + shape, float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, y, z_walls=z_walls)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), y.cpu().numpy()
        assert np.isfinite(b).all()
        np.testing.assert_array_equal(a, b)


def test_noalloc_forward_other_shapes_and_limit(P):
    import torch

    # two layers (one hidden buffer) and a one-layer network (no scratch at all)
    for layers in (2, 1):
        net = P.Net(4, 8, layers, seed=5)
        x = inputs((5, 7, 9), 4)
        y = torch.empty((1, 5, 7, 9), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, y)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(net.forward(x).cpu().numpy(), y.cpu().numpy())
    # 16 hidden channels: 2 x 16 x N x 4 bytes must fit in 64 MiB, so N = 64 x 64 x 129 is refused
    net = P.Net(4, 16, 4, seed=3)
    x = torch.zeros((4, 129, 64, 64), dtype=torch.float32, device="cuda")
    y = torch.zeros((1, 129, 64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(P.LbmixError) as e:
        net.forward_noalloc(x, y)
    assert e.value.code == P.EINVAL
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0     # nothing was launched
