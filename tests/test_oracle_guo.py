"""Pins of the oracle's Guo-type forcing variant (the species move with v^a = u^a + F^a / 2
in the equilibrium and in the implicit drag; the forcing term carries 1 - omega_visc / 2).

* a uniform binary relaxes its relative velocity by exactly (1 - omega/2) / (1 + omega/2)
  per step, whatever the densities (closed form of the implicit drag);
* so the mutual diffusivity is D = v_T^2 / omega_drag, the continuum formula of the drag
  model (checked on a concentration wave, Richardson-extrapolated in k); this is why the
  variant cannot reach the large Schmidt numbers of the paper: D >= v_T^2 / 2;
* Drude: the uniform electrolyte's steady current uses the same D (Einstein relation);
* the shear viscosity is unchanged.
"""
import numpy as np
import pytest

import workloads as WL

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("omega", [0.3, 1.0, 1.7, 1.99])
def test_guo_uniform_relaxation_factor(oracle_mod, omega):
    shape = (2, 2, 2)
    nA, nB = 0.3, 0.7
    uA = np.array([0.02, -0.01, 0.005])
    uB = -uA * nA / nB + np.array([0.001, 0.0, -0.002])
    for t in (1, 6, 25):
        o = oracle_mod.Oracle(2, 2, 2, 2, 0.9, omega, forcing="guo")
        o.set_state(0, np.full(shape, nA), np.broadcast_to(uA[:, None, None, None], (3,) + shape))
        o.set_state(1, np.full(shape, nB), np.broadcast_to(uB[:, None, None, None], (3,) + shape))
        o.step(t)
        _, jA = o.moments(0)
        _, jB = o.moments(1)
        w = jA[:, 0, 0, 0] / nA - jB[:, 0, 0, 0] / nB
        r = (1 - omega / 2) / (1 + omega / 2)
        np.testing.assert_allclose(w, r ** t * (uA - uB), rtol=1e-12, atol=2e-16)
        # total momentum is conserved
        np.testing.assert_allclose(jA[:, 0, 0, 0] + jB[:, 0, 0, 0], nA * uA + nB * uB, rtol=0, atol=1e-16)


def make(oracle_mod, w, **kw):
    o = oracle_mod.Oracle(w.nx, w.ny, w.nz, w.nspecies, w.omega_visc, w.omega_drag, geometry=w.geometry,
                          valence=w.valence, E=w.E, **kw)
    for s in range(w.nspecies):
        o.set_state(s, w.n[s], w.u[s])
    return o


@pytest.mark.parametrize("tau_drag", [0.7, 1.5])
def test_guo_diffusivity_is_the_continuum_formula(oracle_mod, tau_drag):
    Ds = []
    for L in (128, 64):
        k = 2 * np.pi / L
        w = WL.binary_sine(L, 1, 1, amp=1e-6, tau_visc=1.0, sc=1.0)
        w.tau_drag = tau_drag
        o = make(oracle_mod, w, forcing="guo")
        basis = np.sin(k * np.arange(L))
        o.step(60)
        a1 = float(((o.moments(0)[0][0, 0] - 0.5) * basis).sum())
        o.step(2000)
        a2 = float(((o.moments(0)[0][0, 0] - 0.5) * basis).sum())
        Ds.append(-np.log(a2 / a1) / 2000 / k ** 2)
    D0 = (4 * Ds[0] - Ds[1]) / 3.0
    assert abs(D0 / (CS2 / w.omega_drag) - 1) < 1e-4, (D0, CS2 / w.omega_drag)
    # and not the literal scheme's v_T^2 (1/omega - 1/2)
    assert abs(D0 / (CS2 * (1 / w.omega_drag - 0.5)) - 1) > 0.1


def test_guo_drude_and_viscosity(oracle_mod):
    w = WL.bulk_electrolyte(n=2, Ex=1e-4, tau_visc=1.0, tau_drag=0.7)
    o = make(oracle_mod, w, forcing="guo")
    o.step(400)
    n = [o.moments(s)[0][0, 0, 0] for s in range(3)]
    j = [o.moments(s)[1][0, 0, 0, 0] for s in range(3)]
    ubar = sum(j) / sum(n)
    mob = (j[1] / n[1] - ubar) / 1e-4
    np.testing.assert_allclose(mob, 1.0 / w.omega_drag, rtol=1e-9)   # D / v_T^2 with D = v_T^2 / omega
    # shear wave: nu = v_T^2 (1/omega_visc - 1/2) whatever the forcing scheme
    L = 64
    k = 2 * np.pi / L
    u = np.zeros((3, 1, 1, L))
    u[1] = 1e-6 * np.sin(k * np.arange(L))
    ws = WL.Workload("shear", L, 1, 1, "periodic", [0.5, 0.5], [0, 0], 0.8, 0.6,
                     [np.full((1, 1, L), 0.5)] * 2, [u, u])
    amps = []
    for forcing in ("paper", "guo"):
        o = make(oracle_mod, ws, forcing=forcing)
        o.step(50)
        a1 = sum(float((o.moments(s)[1][1, 0, 0] * np.sin(k * np.arange(L))).sum()) for s in range(2))
        o.step(500)
        a2 = sum(float((o.moments(s)[1][1, 0, 0] * np.sin(k * np.arange(L))).sum()) for s in range(2))
        amps.append(-np.log(a2 / a1) / 500 / k ** 2)
    np.testing.assert_allclose(amps[1], amps[0], rtol=1e-6)
