"""Pins of the drag with one frequency per pair of species (Sec. II: the friction of the
pair (alpha, beta); for equal masses F^alpha / m = -sum_beta omega^{alpha beta} (n^beta / n)
(u^alpha - u^beta), omega symmetric because gamma^{alpha beta} n / n^beta is).

* the paper's gamma form: -sum_b gamma^{ab} (u^a - u^b) with gamma^{ab} from the molecular
  diameters (equal masses) equals the oracle's pair drag with omega^{ab} = gamma^{ab} n / n^b;
* third law for a symmetric matrix, independence of the diagonal, reduction to one omega;
* uniform relaxation: the species velocities follow u(t) = (I - W)^t u(0) exactly;
* a binary with a pair matrix is the binary with omega = omega^{AB};
* a dilute tracer in a two-species background diffuses with D = v_T^2 (1/omega_eff - 1/2),
  omega_eff = sum_b omega^{Tb} n^b / n.
"""
import math

import numpy as np
import pytest

import workloads as WL

CS2 = 1.0 / 3.0


def sym(rng, ns, lo=0.3, hi=1.9):
    a = rng.uniform(lo, hi, (ns, ns))
    return 0.5 * (a + a.T)


@pytest.mark.parametrize("ns", [2, 3, 5])
def test_pair_drag_third_law_diagonal_and_reduction(oracle_mod, ns):
    rng = np.random.default_rng(10 + ns)
    n = rng.uniform(0.01, 1.0, ns)
    ua = rng.uniform(-0.05, 0.05, (ns, 3))
    om = sym(rng, ns)
    F = oracle_mod.drag_pair(n, ua, om)
    assert np.abs((n[:, None] * F).sum(axis=0)).max() < 1e-16
    om2 = om.copy()
    np.fill_diagonal(om2, 123.0)
    assert np.array_equal(oracle_mod.drag_pair(n, ua, om2), F)
    same = np.full((ns, ns), 1.37)
    np.testing.assert_allclose(oracle_mod.drag_pair(n, ua, same), oracle_mod.drag(n, ua, 1.37), rtol=0, atol=2e-17)


def test_pair_drag_is_the_papers_gamma_form(oracle_mod):
    """gamma^{ab} = (8 / 3m) sigma_ab^2 n^b sqrt(m_a m_b / (m_a + m_b) 2 kT / pi) g_ab with equal
    masses m and sigma_ab = (sigma_a + sigma_b) / 2 (Sec. II); the force per unit mass is
    -sum_b gamma^{ab} (u^a - u^b)."""
    rng = np.random.default_rng(3)
    m, kT = 1.0, CS2
    diam = np.array([1.0, 0.6, 1.4])
    gcon = np.array([[1.2, 1.1, 1.3], [1.1, 1.0, 1.05], [1.3, 1.05, 1.5]])
    n = np.array([0.7, 0.2, 0.1])
    ua = rng.uniform(-0.03, 0.03, (3, 3))
    sab = 0.5 * (diam[:, None] + diam[None, :])
    gamma = (8.0 / (3.0 * m)) * sab ** 2 * n[None, :] * math.sqrt(m * m / (2 * m) * 2 * kT / math.pi) * gcon
    F_paper = -np.einsum("ab,abd->ad", gamma, ua[:, None, :] - ua[None, :, :])
    omega = gamma * n.sum() / n[None, :]
    np.testing.assert_allclose(omega, omega.T, rtol=1e-15)
    np.testing.assert_allclose(oracle_mod.drag_pair(n, ua, omega), F_paper, rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("t", [1, 7, 30])
def test_pair_drag_uniform_relaxation_matrix_power(oracle_mod, t):
    """Uniform ternary, no field: the collision changes each species' momentum by n^a F^a and
    nothing else moves, so u(t + 1) = (I - W) u(t) with W_ab = delta_ab sum_c omega^{ac} n^c / n
    - omega^{ab} n^b / n."""
    shape = (2, 2, 2)
    n = np.array([0.5, 0.3, 0.2])
    om = np.array([[0.0, 0.4, 1.3], [0.4, 0.0, 1.9], [1.3, 1.9, 0.0]])
    u0 = np.array([[0.02, -0.01, 0.004], [-0.015, 0.02, 0.0], [0.01, 0.005, -0.02]])
    o = oracle_mod.Oracle(2, 2, 2, 3, 0.8, 1.0, drag_pair=om)
    for s in range(3):
        o.set_state(s, np.full(shape, n[s]), np.broadcast_to(u0[s][:, None, None, None], (3,) + shape))
    o.step(t)
    W = -om * n[None, :] / n.sum()
    W[np.diag_indices(3)] = (om * n[None, :] / n.sum()).sum(axis=1) - np.diag(om) * n / n.sum()
    want = np.linalg.matrix_power(np.eye(3) - W, t) @ u0
    for s in range(3):
        _, j = o.moments(s)
        np.testing.assert_allclose(j[:, 0, 0, 0] / n[s], want[s], rtol=1e-11, atol=1e-17)


def test_binary_pair_matrix_equals_scalar_drag(oracle_mod):
    w = WL.binary_multimode(n=12, amp=1e-2, nmodes=3, shear=1e-2, sc=30.0, seed=4)
    om = w.omega_drag
    a = oracle_mod.Oracle(12, 12, 12, 2, w.omega_visc, om)
    b = oracle_mod.Oracle(12, 12, 12, 2, w.omega_visc, 0.1, drag_pair=[[9.0, om], [om, 4.0]])
    for o in (a, b):
        for s in range(2):
            o.set_state(s, w.n[s], w.u[s])
        o.step(40)
    for s in range(2):
        fa, fb = a.populations(s), b.populations(s)
        assert np.abs(fa - fb).max() <= 1e-14 * np.abs(fa - fa.mean()).max()


def test_tracer_diffusion_with_pair_drag(oracle_mod):
    """Tracer T (1e-4 of the density) in a uniform A + B background: its concentration wave
    decays with D = v_T^2 (1/omega_eff - 1/2), omega_eff = (omega^{TA} n^A + omega^{TB} n^B) / n."""
    L = 128
    k = 2 * np.pi / L
    nA, nB, nT = 0.6, 0.4, 1e-4
    om = np.array([[0.0, 0.7, 1.2], [0.7, 0.0, 0.6], [1.2, 0.6, 0.0]])
    o = oracle_mod.Oracle(L, 1, 1, 3, 1.0, 1.0, drag_pair=om)
    x = np.arange(L)
    shape = (1, 1, L)
    o.set_state(0, np.full(shape, nA))
    o.set_state(1, np.full(shape, nB))
    o.set_state(2, (nT * (1.0 + 0.01 * np.sin(k * x)))[None, None, :])
    basis = np.sin(k * x)

    def amp():
        n, _ = o.moments(2)
        return float(((n[0, 0] - nT) * basis).sum())

    o.step(200)
    a1 = amp()
    o.step(3000)
    a2 = amp()
    D = -math.log(a2 / a1) / 3000 / k ** 2
    om_eff = (om[2, 0] * nA + om[2, 1] * nB) / (nA + nB + nT)
    assert abs(D / (CS2 * (1.0 / om_eff - 0.5)) - 1) < 2e-3
