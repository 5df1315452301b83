"""Pins of reading R3b (the drag of Sec. II acts on the mid-step species velocities) against
the literal reading (the drag acts on the plain first moments of the pre-collision
populations), both run by the oracle.

In a state with no particle flux, the literal reading leaves a pre-collision momentum
j = -n F / 2 per species (F the total force per particle), and the drag answers it:
F (1 - omega_drag / 2) = a for a dilute species under a field acceleration a.  Every field
force is then amplified by 1 / (1 - omega_drag / 2) = tau_drag / (tau_drag - 1/2), which is
101 at Sc = 100 with tau_visc = 1.  Measurable consequences, each with its closed form:

* the uniform steady current of the ternary electrolyte is (n+ + n-) E / omega_drag
  (Drude with the continuum D = v_T^2 / omega_drag), against (D / v_T^2)(n+ + n-) E with the
  discrete D = v_T^2 (1/omega_drag - 1/2) of Sec. IV under R3b;
* the zero-flux profile of a dilute charged tracer in a uniform field grows as
  exp(a z / (v_T^2 (1 - omega_drag / 2))) instead of the Boltzmann factor exp(a z / v_T^2);
* in the charged slit of Sec. IV at Sc = 100 the amplified force screens the wall charge
  within a fraction of a node, and the Boltzmann relation ln n^+- +- psi~ = const, which R3b
  keeps to the O(h^2) error of the field, fails outright.
"""
import numpy as np
import pytest

import workloads as WL

CS2 = 1.0 / 3.0


def bulk(oracle_mod, omega_drag, forcing):
    Ex = 1e-4
    w = WL.bulk_electrolyte(n=2, ratio=1e-2, Ex=Ex, tau_visc=1.0, tau_drag=1.0 / omega_drag)
    o = oracle_mod.Oracle(w.nx, w.ny, w.nz, 3, w.omega_visc, w.omega_drag, valence=w.valence,
                          E=w.E, forcing=forcing)
    for s in range(3):
        o.set_state(s, w.n[s], w.u[s])
    steps = int(np.ceil(np.log(1e-14) / np.log(max(abs(1 - omega_drag), 1e-3)))) + 5
    o.step(max(steps, 5))
    n = [o.moments(s)[0][0, 0, 0] for s in range(3)]
    j = [o.moments(s)[1][:, 0, 0, 0] for s in range(3)]
    return Ex, n, j


@pytest.mark.parametrize("omega_drag", [0.5, 1.0, 1.5, 1.9])
def test_literal_drag_bulk_current_is_continuum_drude(oracle_mod, omega_drag):
    Ex, n, j = bulk(oracle_mod, omega_drag, "literal")
    current = j[1][0] - j[2][0]
    np.testing.assert_allclose(current, (n[1] + n[2]) * Ex / omega_drag, rtol=1e-10)
    # each ion's pre-collision velocity is exactly z E / omega_drag; the mixture is at rest
    np.testing.assert_allclose(j[1][0] / n[1], Ex / omega_drag, rtol=1e-10)
    assert abs(sum(jj[0] for jj in j)) < 1e-18
    # the same lattice under R3b carries the current of the discrete D: their ratio is
    # exactly 1 / (1 - omega_drag / 2)
    Ex, n2, j2 = bulk(oracle_mod, omega_drag, "paper")
    ratio = current / (j2[1][0] - j2[2][0])
    np.testing.assert_allclose(ratio, 1.0 / (1.0 - 0.5 * omega_drag), rtol=1e-9)


def tracer_slope(oracle_mod, forcing, sc, E=1e-4, nz=10, steps=60000):
    """Dilute charged tracer (valence +1, 1e-6 of the solvent) in a slit 1 x 1 x nz with a
    uniform field E along z and no Poisson solve; returns the mean of ln(n(z+1) / n(z)) over
    the interior of the steady profile (two consecutive steps averaged)."""
    tau_d = WL.tau_drag_for_schmidt(1.0, sc)
    o = oracle_mod.Oracle(1, 1, nz, 2, 1.0, 1.0 / tau_d, geometry="slit", valence=[0, 1],
                          E=(0.0, 0.0, E), forcing=forcing)
    o.set_state(0, np.ones((nz, 1, 1)))
    o.set_state(1, np.full((nz, 1, 1), 1e-6))
    o.step(steps)
    a = o.moments(1)[0][1:-1, 0, 0]
    o.step(1)
    n = 0.5 * (a + o.moments(1)[0][1:-1, 0, 0])
    g = np.diff(np.log(n))
    return g[1:-1].mean(), np.ptp(g[1:-1]), 1.0 / tau_d


@pytest.mark.parametrize("sc", [10.0, 100.0])
def test_literal_drag_amplifies_the_barometric_law(oracle_mod, sc):
    E = 1e-4
    g_paper, spread_p, _ = tracer_slope(oracle_mod, "paper", sc, E)
    g_lit, spread_l, om = tracer_slope(oracle_mod, "literal", sc, E)
    # R3b: the Boltzmann factor, ln n grows by a / v_T^2 per node
    assert abs(g_paper / (E / CS2) - 1) < 1e-3
    # literal: amplified by 1 / (1 - omega_drag / 2) (11 at Sc = 10, 101 at Sc = 100)
    amp = 1.0 / (1.0 - 0.5 * om)
    assert abs(g_lit / (E / CS2) / amp - 1) < 0.02
    # both profiles are exponential in the interior
    assert spread_p < 1e-3 * abs(g_paper) and spread_l < 0.02 * abs(g_lit)


def charged_slit_boltzmann(oracle_mod, forcing, steps):
    nz = 34
    w = WL.charged_slit(nx=1, ny=1, nz=nz, n_solvent=1.0, n_ion=1e-3, debye_length=4.0,
                        sigma=-1e-4, Ex=0.0, tau_visc=1.0, sc=100.0)
    o = oracle_mod.Oracle(1, 1, nz, 3, w.omega_visc, w.omega_drag, geometry="slit",
                          valence=w.valence, bjerrum=w.bjerrum, sigma=w.sigma, E=w.E,
                          poisson="direct", forcing=forcing)
    for s in range(3):
        o.set_state(s, w.n[s])
    o.step(steps)
    n1 = [o.moments(s)[0][1:-1, 0, 0] for s in range(3)]
    p1 = o.potential()[1:-1, 0, 0]
    o.step(1)
    n = [0.5 * (a + o.moments(s)[0][1:-1, 0, 0]) for s, a in enumerate(n1)]
    p = 0.5 * (p1 + o.potential()[1:-1, 0, 0])
    return n, p, w.omega_drag


def test_literal_drag_breaks_the_boltzmann_relation_at_sc100(oracle_mod):
    """The charged slit of Sec. IV at Sc = 100 (lambda_D = 4, sigma = -1e-4, no field)."""
    n, p, om = charged_slit_boltzmann(oracle_mod, "paper", 20000)
    span_paper = np.ptp(p)
    assert np.ptp(np.log(n[1]) + p) < 0.03 * span_paper and np.ptp(np.log(n[2]) - p) < 0.03 * span_paper
    n, p, om = charged_slit_boltzmann(oracle_mod, "literal", 20000)
    span = np.ptp(p)
    # the amplified force screens as if the Debye length were lambda_D (1 - omega_drag / 2)^(1/2)
    # = 0.4 nodes: the double layer collapses into the first fluid planes and the potential
    # drop across the channel shrinks by more than the continuum factor 101^(1/2) = 10
    assert span < 0.1 * span_paper
    # ln n^+- +- psi~ is far from constant: it varies more than 100 times as much as psi~
    bp, bn = np.log(n[1]) + p, np.log(n[2]) - p
    assert np.ptp(bp) > 100 * span and np.ptp(bn) > 100 * span
