"""Pins of the FP64 network reference used to check the library's learned warm start:
a one-layer linear network is a 27-point stencil (closed form on a delta input), the
zero-padded and periodic z ends, and the finite-difference gradient against the gradient of
a linear layer in closed form."""
import numpy as np

from oracle import warmstart_net as R


def test_single_tap_is_a_shift():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 5, 4, 6))
    for k, (dz, dy, dx) in enumerate(R.TAPS):
        p = np.zeros(28)
        p[k] = 1.0
        y = R.forward(p, [1, 1], x, zwalls=False)[0]
        for z in range(5):
            assert np.array_equal(y[z], np.roll(x[0, (z + dz) % 5], (-dy, -dx), axis=(0, 1)))
        yw = R.forward(p, [1, 1], x, zwalls=True)[0]
        for z in range(5):
            want = np.roll(x[0, z + dz], (-dy, -dx), axis=(0, 1)) if 0 <= z + dz < 5 else 0.0
            assert np.all(yw[z] == want)


def test_relu_hidden_layer_and_bias():
    x = np.zeros((2, 3, 3, 3))
    x[0, 1, 1, 1] = 2.0
    x[1] = 1.0
    # layer 1 (2 -> 1): centre tap of channel 0 weight -1, bias 0.5; layer 2 (1 -> 1): centre 3
    p = np.zeros(2 * 27 + 1 + 27 + 1)
    p[13] = -1.0
    p[54] = 0.5
    p[55 + 13] = 3.0
    y = R.forward(p, [2, 1, 1], x, zwalls=True)[0]
    want = np.full((3, 3, 3), 1.5)
    want[1, 1, 1] = 0.0        # relu(-2 + 0.5) = 0
    assert np.array_equal(y, want)


def test_fd_gradient_of_linear_layer_closed_form():
    """One linear layer: dL/dw[k] = 2 mean((y - t) shift_k(x)), dL/db = 2 mean(y - t)."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 5, 6))
    t = rng.standard_normal((1, 4, 5, 6))
    p = rng.standard_normal(28) * 0.2
    y = R.forward(p, [1, 1], x, zwalls=True)
    d = y - t
    exact = [2.0 * np.mean(d[0] * R.shifted(x, dz, dy, dx, True)[0]) for (dz, dy, dx) in R.TAPS] + [2.0 * np.mean(d)]
    fd = R.fd_gradient(p, [1, 1], x, t, True, range(28))
    np.testing.assert_allclose(fd, exact, rtol=1e-7, atol=1e-9)
