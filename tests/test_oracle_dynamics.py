"""Pins of the oracle's time stepping against what the paper and the mathematics fix.

* uniform relaxation of the relative velocity: w(t) = (1 - omega_drag)^t w(0) exactly;
* species mass and total momentum conservation (Sec. III, eq. continuityb and the
  remark that the drag forces cancel in eq. globalmomentumcont);
* decay of a concentration wave against the exact discrete eigenvalue, and its
  continuum limit against D = v_T^2 (1/omega_drag - 1/2) of Sec. IV;
* decay of a shear wave against nu = v_T^2 (1/omega_visc - 1/2) of Sec. IV, independent of
  omega_drag (Sec. IV: the viscosity "remains unaltered");
* omega_drag = omega_visc reduces to the single-relaxation BGK mixture (Sec. V), with a
  closed-form remainder quadratic in the velocity differences;
* indifferentiability (Sec. II): identical species behave as one;
* bulk conductivity of the ternary electrolyte (Sec. III eq. Drude, Sec. IV);
* brute-force agreement with an independent NumPy implementation on tiny lattices.
"""
import numpy as np
import pytest

import workloads as WL
from brute_numpy import C as BC, W as BW, feq as b_feq
from linear_modes import diffusion_eigenvalue, shear_eigenvalue

CS2 = 1.0 / 3.0


def make(oracle_mod, w, **kw):
    o = oracle_mod.Oracle(w.nx, w.ny, w.nz, w.nspecies, w.omega_visc, w.omega_drag,
                          geometry=w.geometry, valence=w.valence, bjerrum=w.bjerrum,
                          sigma=w.sigma, E=w.E, **kw)
    for s in range(w.nspecies):
        o.set_state(s, w.n[s], w.u[s])
    return o


@pytest.mark.parametrize("omega_drag", [0.3, 1.0, 1.5, 1.818181818, 1.998002])
def test_uniform_relative_velocity_relaxation(oracle_mod, omega_drag):
    shape = (2, 2, 2)
    nA, nB = 0.3, 0.7
    uA = np.array([0.02, -0.01, 0.005])
    uB = -uA * nA / nB
    o = oracle_mod.Oracle(2, 2, 2, 2, 0.9, omega_drag)
    o.set_state(0, np.full(shape, nA), np.broadcast_to(uA[:, None, None, None], (3,) + shape))
    o.set_state(1, np.full(shape, nB), np.broadcast_to(uB[:, None, None, None], (3,) + shape))
    w0 = uA - uB
    for t in (1, 5, 40):
        o2 = oracle_mod.Oracle(2, 2, 2, 2, 0.9, omega_drag)
        o2.set_state(0, np.full(shape, nA), np.broadcast_to(uA[:, None, None, None], (3,) + shape))
        o2.set_state(1, np.full(shape, nB), np.broadcast_to(uB[:, None, None, None], (3,) + shape))
        o2.step(t)
        _, jA = o2.moments(0)
        _, jB = o2.moments(1)
        wt = jA[:, 0, 0, 0] / nA - jB[:, 0, 0, 0] / nB
        np.testing.assert_allclose(wt, (1.0 - omega_drag) ** t * w0, rtol=1e-12, atol=2e-16)
        # barycentric velocity stays zero
        assert np.abs(jA[:, 0, 0, 0] + jB[:, 0, 0, 0]).max() < 1e-15


@pytest.mark.parametrize("geometry", ["periodic", "slit"])
def test_mass_and_momentum_conservation(oracle_mod, geometry):
    w = WL.random_state(8, 6, 10, 3, geometry=geometry, seed=7, dn=0.05, du=0.02, tau_visc=0.7,
                        tau_drag=0.55)
    o = make(oracle_mod, w)
    m0 = o.mass_totals()
    p0 = sum(o.moments(s)[1].sum(axis=(1, 2, 3)) for s in range(3))
    o.step(500)
    m1 = o.mass_totals()
    np.testing.assert_allclose(m1, m0, rtol=1e-13)
    if geometry == "periodic":
        p1 = sum(o.moments(s)[1].sum(axis=(1, 2, 3)) for s in range(3))
        np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-13 * m0.sum())


def test_total_momentum_conserved_with_neutral_field(oracle_mod):
    """A uniform field on a neutral electrolyte exerts no net force (sum n z E = 0)."""
    w = WL.random_state(6, 4, 4, 3, seed=11, rho0=[1.0, 0.01, 0.01], valence=[0, 1, -1],
                        E=(1e-3, 0.0, 0.0), dn=0.0, du=0.01)
    o = make(oracle_mod, w)
    p0 = sum(o.moments(s)[1].sum(axis=(1, 2, 3)) for s in range(3))
    o.step(200)
    p1 = sum(o.moments(s)[1].sum(axis=(1, 2, 3)) for s in range(3))
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-14)


def _wave_amplitude(o, s, basis, rho0):
    n, _ = o.moments(s)
    return float(((n[0, 0, :] - rho0) * basis).sum())


@pytest.mark.parametrize("sc", [1.0, 10.0, 100.0, 1000.0])
def test_concentration_wave_vs_exact_eigenvalue(oracle_mod, sc):
    """Per-step decay factor of a small concentration wave = the diffusion eigenvalue of the
    linearised discrete scheme (complex-step Jacobian of the independent brute force)."""
    L = 64
    w = WL.binary_sine(L, 1, 1, amp=1e-6, tau_visc=1.0, sc=sc)
    lam = diffusion_eigenvalue([0.5, 0.5], w.omega_visc, w.omega_drag, [2 * np.pi / L, 0, 0]).real
    o = make(oracle_mod, w)
    basis = np.sin(2 * np.pi * np.arange(L) / L)
    # wait until the flux transient (factor |1 - omega_drag| per step) is below 1e-9
    t1 = int(np.ceil(np.log(1e-9) / np.log(max(abs(1.0 - w.omega_drag), 1e-3)))) + 10
    o.step(t1)
    a1 = _wave_amplitude(o, 0, basis, 0.5)
    o.step(1000)
    a2 = _wave_amplitude(o, 0, basis, 0.5)
    fit = (a2 / a1) ** (1.0 / 1000)
    assert abs(fit - lam) / (1.0 - lam) < 1e-5


@pytest.mark.parametrize("sc", [1.0, 10.0, 100.0])
def test_diffusion_coefficient_continuum_limit(oracle_mod, sc):
    """-ln(lambda)/k^2 -> D = v_T^2 (1/omega_drag - 1/2) (Sec. IV) as k -> 0: the O(k^2)
    remainder is removed by Richardson extrapolation over k and 2k."""
    Ds = []
    for L in (128, 64):
        k = 2 * np.pi / L
        w = WL.binary_sine(L, 1, 1, amp=1e-6, tau_visc=1.0, sc=sc)
        o = make(oracle_mod, w)
        basis = np.sin(k * np.arange(L))
        t1 = int(np.ceil(np.log(1e-9) / np.log(max(abs(1.0 - w.omega_drag), 1e-3)))) + 10
        o.step(t1)
        a1 = _wave_amplitude(o, 0, basis, 0.5)
        o.step(2000)
        a2 = _wave_amplitude(o, 0, basis, 0.5)
        Ds.append(-np.log(a2 / a1) / 2000 / k ** 2)
    D0 = (4 * Ds[0] - Ds[1]) / 3.0
    Dth = CS2 * (1.0 / w.omega_drag - 0.5)
    assert abs(D0 / Dth - 1) < 2e-5
    # and the continuum D = v_T^2 / omega_drag of eq. (mutualdiffusion) is not what the
    # lattice gives unless omega_drag is small: the -1/2 is a lattice term
    assert abs(Ds[0] / (CS2 / w.omega_drag) - 1) > 0.1


@pytest.mark.parametrize("sc", [1.0, 1000.0])
def test_shear_wave_viscosity_independent_of_drag(oracle_mod, sc):
    L = 64
    k = 2 * np.pi / L
    shape = (1, 1, L)
    u = np.zeros((3,) + shape)
    u[1] = 1e-6 * np.sin(k * np.arange(L))
    tv = 0.8
    w = WL.Workload("shear", L, 1, 1, "periodic", [0.5, 0.5], [0, 0], tv,
                    WL.tau_drag_for_schmidt(tv, sc), [np.full(shape, 0.5)] * 2, [u, u])
    lam = shear_eigenvalue([0.5, 0.5], w.omega_visc, w.omega_drag, [k, 0, 0]).real
    o = make(oracle_mod, w)
    basis = np.sin(k * np.arange(L))

    def amp():
        return sum(float((o.moments(s)[1][1, 0, 0, :] * basis).sum()) for s in range(2))

    o.step(50)
    a1 = amp()
    o.step(1000)
    a2 = amp()
    fit = (a2 / a1) ** (1.0 / 1000)
    assert abs(fit - lam) / (1.0 - lam) < 1e-6
    nu_fit = -np.log(fit) / k ** 2
    nu_th = CS2 * (1.0 / w.omega_visc - 0.5)
    assert abs(nu_fit / nu_th - 1) < 2e-3       # O(k^2) at L = 64


def test_bgk_limit_closed_form(oracle_mod):
    """omega_drag = omega_visc: the step equals the single-relaxation BGK mixture step
    f - omega (f - feq(n^a, u)) exactly up to omega w n^a [(c.d)^2/(2 cs2^2) - |d|^2/(2 cs2)],
    d = u^a - u, a remainder quadratic in the velocity differences (Sec. V)."""
    rng = np.random.default_rng(5)
    om = 1.3
    shape = (1, 1, 1)    # one periodic node: streaming is the identity
    o = oracle_mod.Oracle(1, 1, 1, 2, om, om)
    ns = [0.4, 0.6]
    us = [rng.uniform(-0.05, 0.05, 3), rng.uniform(-0.05, 0.05, 3)]
    fs = []
    for s in range(2):
        f = b_feq(np.array(ns[s]), us[s]) * (1.0 + 0.01 * rng.uniform(-1, 1, 19))
        fs.append(f)
        o.set_populations(s, f.reshape(19, 1, 1, 1))
    o.step(1)
    n = np.array([f.sum() for f in fs])
    j = np.array([f @ BC for f in fs])
    ua = j / n[:, None]
    u = j.sum(axis=0) / n.sum()
    for s in range(2):
        bgk = fs[s] - om * (fs[s] - b_feq(np.array(n[s]), u))
        d = ua[s] - u
        cd = BC @ d
        rem = om * BW * n[s] * (cd ** 2 / (2 * CS2 ** 2) - (d @ d) / (2 * CS2))
        np.testing.assert_allclose(o.populations(s).reshape(19), bgk + rem, rtol=0, atol=1e-16)


def test_indifferentiability(oracle_mod):
    """Identical species with a uniform composition ratio: f^A + f^B follows the
    single-species BGK exactly and the ratio f^A / f^B stays fixed (Sec. II)."""
    w1 = WL.random_state(6, 4, 8, 1, seed=21, rho0=[1.0], tau_visc=0.7, tau_drag=0.55)
    frac = 0.3
    o1 = make(oracle_mod, w1)
    o2 = oracle_mod.Oracle(6, 4, 8, 2, w1.omega_visc, 1.6)
    o2.set_state(0, frac * w1.n[0], w1.u[0])
    o2.set_state(1, (1 - frac) * w1.n[0], w1.u[0])
    o1.step(50)
    o2.step(50)
    fa, fb, f1 = o2.populations(0), o2.populations(1), o1.populations(0)
    np.testing.assert_allclose(fa + fb, f1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(fa, frac * f1, rtol=0, atol=1e-15)


@pytest.mark.parametrize("omega_drag", [0.5, 1.0, 1.5, 1.9])
def test_bulk_conductivity_drude(oracle_mod, omega_drag):
    """Uniform ternary electrolyte, n+/n0 = 1e-2 (Sec. IV), field E_x: the steady current
    is sigma E with sigma = e^2 (D / v_T^2)(n+ + n-), D = v_T^2 (1/omega_drag - 1/2)
    (Sec. III eq. Drude with the discrete D of Sec. IV), and u^0 = u = 0."""
    Ex = 1e-4
    w = WL.bulk_electrolyte(n=2, ratio=1e-2, Ex=Ex, tau_visc=1.0, tau_drag=1.0 / omega_drag)
    o = make(oracle_mod, w)
    steps = int(np.ceil(np.log(1e-14) / np.log(max(abs(1 - omega_drag), 1e-3)))) + 5
    o.step(max(steps, 5))
    n = [o.moments(s)[0][0, 0, 0] for s in range(3)]
    j = [o.moments(s)[1][:, 0, 0, 0] for s in range(3)]
    current = j[1][0] - j[2][0]
    D = CS2 * (1.0 / omega_drag - 0.5)
    sigma = (D / CS2) * (n[1] + n[2])
    np.testing.assert_allclose(current, sigma * Ex, rtol=1e-10)
    u = sum(j) / sum(n)
    assert np.abs(u).max() < 1e-18
    assert abs(j[0][0] / n[0]) < 1e-18


@pytest.mark.parametrize("geometry,charged", [("periodic", False), ("periodic", True),
                                               ("slit", False), ("slit", True)])
def test_brute_force_agreement(oracle_mod, geometry, charged):
    from brute_numpy import Brute
    ns = 3 if charged else 2
    val = [0, 1, -1] if charged else [0, 0]
    lb = 0.4 if charged else 0.0
    w = WL.random_state(6, 4, 8, ns, geometry=geometry, seed=3, valence=val, bjerrum=lb,
                        sigma=(-0.002, -0.001), E=(1e-3, 2e-4, -1e-4), dn=0.1, du=0.03)
    o = make(oracle_mod, w)
    b = Brute(w.nx, w.ny, w.nz, ns, w.omega_visc, w.omega_drag, slit=(geometry == "slit"),
              valence=val, bjerrum=lb, sigma=w.sigma, E=w.E)
    for s in range(ns):
        b.set_state(s, w.n[s], w.u[s])
    o.step(9)
    b.step(9)
    for s in range(ns):
        np.testing.assert_allclose(o.populations(s), b.f[s], rtol=0, atol=1e-15)
    if charged:
        np.testing.assert_allclose(o.potential(), b.psi, rtol=0, atol=1e-14)


def test_unlagged_and_lagged_reach_same_steady_state(oracle_mod):
    w = WL.charged_slit(nx=1, ny=1, nz=18, debye_length=3.0, sigma=-2e-4, Ex=0.0, sc=1.0)
    lagged = make(oracle_mod, w, lagged=True)
    direct = make(oracle_mod, w, lagged=False)
    lagged.step(3000)
    direct.step(3000)
    for s in range(3):
        np.testing.assert_allclose(lagged.moments(s)[0], direct.moments(s)[0], rtol=1e-9)
    np.testing.assert_allclose(lagged.potential(), direct.potential(), rtol=0, atol=1e-9)
