"""Pins of the oracle's per-node pieces: lattice, equilibrium, forcing, drag.

Each check is a fact fixed by the paper or by the mathematics, not a retyping of the
oracle's formula: isotropy of the velocity set, the moments that the Hermite construction
of the Appendix guarantees, Newton's third law for the drag (Sec. III), and the identity
that reduces the paper's orthogonalised equilibrium to the equilibrium at the species
velocity.
"""
from fractions import Fraction

import numpy as np
import pytest


def test_d3q19_isotropy_exact(oracle_mod):
    c, w, opp = oracle_mod.d3q19()
    # weights are 1/3, 1/18, 1/36 exactly (as binary doubles of those fractions)
    fw = [Fraction(x).limit_denominator(100) for x in w]
    assert sum(fw) == 1
    assert sorted(set(fw)) == [Fraction(1, 36), Fraction(1, 18), Fraction(1, 3)]
    cs2 = Fraction(1, 3)
    for i in range(3):
        assert sum(fw[p] * c[p, i] for p in range(19)) == 0
        for j in range(3):
            assert sum(fw[p] * c[p, i] * c[p, j] for p in range(19)) == (cs2 if i == j else 0)
            for k in range(3):
                assert sum(fw[p] * c[p, i] * c[p, j] * c[p, k] for p in range(19)) == 0
                for l in range(3):
                    got = sum(fw[p] * c[p, i] * c[p, j] * c[p, k] * c[p, l] for p in range(19))
                    want = cs2 * cs2 * ((i == j) * (k == l) + (i == k) * (j == l) + (i == l) * (j == k))
                    assert got == want
    for p in range(19):
        assert (c[opp[p]] == -c[p]).all()
    # every lattice vector appears once, and they are the 19 of D3Q19
    vecs = {tuple(v) for v in c}
    assert len(vecs) == 19
    assert all(sum(abs(x) for x in v) <= 2 and max(abs(x) for x in v) <= 1 for v in vecs)


@pytest.mark.parametrize("seed", range(5))
def test_phi_perp_moments_and_reduction(oracle_mod, seed):
    """Moments of phi_perp (Appendix): density n, momentum n u^a and second moment
    n (cs2 I + u^a u^a); and phi_perp does not depend on the barycentric u at all (the
    paper's bracket simplifies to (u^a.c)^2 - cs2 |u^a|^2)."""
    rng = np.random.default_rng(seed)
    c, w, _ = oracle_mod.d3q19()
    n = rng.uniform(0.1, 2.0)
    ua = rng.uniform(-0.1, 0.1, 3)
    u = rng.uniform(-0.1, 0.1, 3)
    phi = oracle_mod.phi_perp(n, ua, u)
    assert abs(phi.sum() - n) < 1e-15 * 19
    np.testing.assert_allclose(phi @ c, n * ua, rtol=0, atol=1e-16 * 19)
    second = np.einsum("p,pi,pj->ij", phi, c, c)
    np.testing.assert_allclose(second, n * (np.eye(3) / 3.0 + np.outer(ua, ua)), rtol=0, atol=1e-15 * 19)
    for _ in range(3):
        u2 = rng.uniform(-0.2, 0.2, 3)
        np.testing.assert_allclose(oracle_mod.phi_perp(n, ua, u2), phi, rtol=0, atol=2e-16)


def test_phi_perp_null_projection_of_correction(oracle_mod):
    """phi_perp - phi (phi = equilibrium at the barycentric u) has zero density, and its
    momentum is n (u^a - u): the correction only moves momentum between species."""
    c, w, _ = oracle_mod.d3q19()
    n, ua, u = 0.7, np.array([0.03, -0.01, 0.02]), np.array([0.01, 0.0, -0.02])
    d = oracle_mod.phi_perp(n, ua, u) - oracle_mod.phi_perp(n, u, u)
    assert abs(d.sum()) < 1e-16 * 19
    np.testing.assert_allclose(d @ c, n * (ua - u), rtol=0, atol=1e-16 * 19)


@pytest.mark.parametrize("seed", range(5))
def test_forcing_moments(oracle_mod, seed):
    """g_p (Appendix, eq. ourforc): sum g = 0, sum g c = n F, sum g c c = n (F u + u F)."""
    rng = np.random.default_rng(100 + seed)
    c, w, _ = oracle_mod.d3q19()
    n = rng.uniform(0.1, 2.0)
    F = rng.uniform(-1e-2, 1e-2, 3)
    u = rng.uniform(-0.1, 0.1, 3)
    g = oracle_mod.forcing(n, F, u)
    assert abs(g.sum()) < 1e-17 * 19
    np.testing.assert_allclose(g @ c, n * F, rtol=0, atol=1e-17 * 19)
    second = np.einsum("p,pi,pj->ij", g, c, c)
    np.testing.assert_allclose(second, n * (np.outer(F, u) + np.outer(u, F)), rtol=0, atol=1e-17 * 19)


@pytest.mark.parametrize("ns", [1, 2, 3, 5])
def test_drag_newton_third_law(oracle_mod, ns):
    """sum_a n^a F^{a,drag} = 0 (Sec. III: the drag forces cancel in the total momentum),
    and with equal masses the pairwise sum equals -omega (u^a - u)."""
    rng = np.random.default_rng(ns)
    n = rng.uniform(0.01, 1.0, ns)
    ua = rng.uniform(-0.05, 0.05, (ns, 3))
    om = 1.7
    F = oracle_mod.drag(n, ua, om)
    assert np.abs((n[:, None] * F).sum(axis=0)).max() < 1e-16
    u = (n[:, None] * ua).sum(axis=0) / n.sum()
    np.testing.assert_allclose(F, -om * (ua - u), rtol=0, atol=1e-16)


def test_drag_zero_density_species(oracle_mod):
    F = oracle_mod.drag([0.0, 0.0], [[0.1, 0, 0], [0, 0, 0]], 1.0)
    assert (F == 0).all()
