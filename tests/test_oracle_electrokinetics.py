"""Electrokinetic pins of the oracle in a charged slit (Sec. III-IV).

* Boltzmann (Gouy-Chapman) equilibrium: with no field, ln n^+- +- psi~ is constant across
  the channel, in the linear (Debye-Hueckel) and in the non-linear regime;
* Helmholtz-Smoluchowski: at low diffusivity the steady flow is
  u_x(z) = E_x (psi~(z) - psi~_wall) / (4 pi l_B eta), eta = rho nu, from eq.
  (globalmomentumcontc) with Poisson's equation;
* the paper's mass flow and electro-osmotic current formulas (eqs. theomassflow, theo),
  read as integrals over the half channel (the full-channel integral is twice them);
* at high diffusivity the solvent and barycentric velocities part (Sec. IV, Fig. 4).
"""
import math

import numpy as np
import pytest

import workloads as WL

CS2 = 1.0 / 3.0


def run_slit(oracle_mod, nz=34, lam=4.0, sigma=-1e-4, Ex=0.0, sc=100.0, steps=20000):
    w = WL.charged_slit(nx=1, ny=1, nz=nz, n_solvent=1.0, n_ion=1e-3, debye_length=lam,
                        sigma=sigma, Ex=Ex, tau_visc=1.0, sc=sc)
    o = oracle_mod.Oracle(1, 1, nz, 3, w.omega_visc, w.omega_drag, geometry="slit",
                          valence=w.valence, bjerrum=w.bjerrum, sigma=w.sigma, E=w.E,
                          poisson="direct")
    for s in range(3):
        o.set_state(s, w.n[s])
    o.step(steps)
    # average two consecutive steps: this removes the undamped period-2 (space and time)
    # checkerboard that the start-up transient leaves at the 1e-10 level
    n1 = [o.moments(s)[0][1:-1, 0, 0] for s in range(3)]
    j1 = [o.moments(s)[1][:, 1:-1, 0, 0] for s in range(3)]
    psi1 = o.potential()[:, 0, 0]
    o.step(1)
    n = [0.5 * (a + o.moments(s)[0][1:-1, 0, 0]) for s, a in enumerate(n1)]
    j = [0.5 * (a + o.moments(s)[1][:, 1:-1, 0, 0]) for s, a in enumerate(j1)]
    psi = 0.5 * (psi1 + o.potential()[:, 0, 0])
    return w, n, j, psi


@pytest.mark.parametrize("sigma,sc", [(-1e-4, 1.0), (-1e-4, 100.0), (-3e-3, 1.0)])
def test_boltzmann_equilibrium(oracle_mod, sigma, sc):
    w, n, j, psi = run_slit(oracle_mod, sigma=sigma, sc=sc, steps=20000 if sc > 1 else 4000)
    p = psi[1:-1]
    bp = np.log(n[1]) + p
    bn = np.log(n[2]) - p
    span = np.ptp(p)
    # the O(h^2) error of the central-difference field, relative to the potential drop
    assert np.ptp(bp) < 0.03 * span
    assert np.ptp(bn) < 0.03 * span
    # no particle flux: the solvent is at rest, and each ion's mid-step momentum
    # j + n a / 2 vanishes, a = -z cs2 d(psi)/dz (ghost values from the wall charge)
    k = 4 * math.pi * w.bjerrum
    ext = np.concatenate([[psi[1] + k * sigma], p, [psi[-2] + k * sigma]])
    dpsi = 0.5 * (ext[2:] - ext[:-2])
    assert np.abs(j[0]).max() < 1e-3 * np.abs(0.5 * n[1] * CS2 * dpsi).max()
    for s, zv in ((1, 1.0), (2, -1.0)):
        a = -zv * CS2 * dpsi
        mid = j[s][2] + 0.5 * n[s] * a
        assert np.abs(mid).max() < 1e-3 * np.abs(0.5 * n[s] * a).max()
    if sigma == -3e-3:
        assert span > 0.2     # non-linear regime: psi~ of order one


def test_debye_profile_matches_closed_form(oracle_mod):
    w, n, j, psi = run_slit(oracle_mod, sigma=-1e-4, sc=1.0, steps=4000)
    nz = 34
    dh = WL.debye_huckel_potential(np.arange(nz, dtype=float), nz, 4.0, w.bjerrum, -1e-4)
    ref = dh[1:-1] - dh[1:-1].mean()
    err = np.abs(psi[1:-1] - ref).max() / np.abs(dh).max()
    assert err < 2 * (1.0 / (12 * 4.0 ** 2)) + 0.01 * np.abs(dh).max()


def test_helmholtz_smoluchowski_flow_and_paper_currents(oracle_mod):
    Ex = 1e-5
    sigma = -1e-4
    lam = 4.0
    nz = 34
    H = nz - 2
    w, n, j, psi = run_slit(oracle_mod, nz=nz, lam=lam, sigma=sigma, Ex=Ex, sc=100.0, steps=30000)
    rho = n[0] + n[1] + n[2]
    ux = (j[0][0] + j[1][0] + j[2][0]) / rho
    nu = CS2 * (1.0 / w.omega_visc - 0.5)
    k = 4 * math.pi * w.bjerrum
    psi_wall = psi[1] + 0.5 * k * sigma          # extrapolated to the wall surface z = 1/2
    hs = Ex * (psi[1:-1] - psi_wall) / (k * nu * rho)
    c = H // 2
    assert abs(ux[c] / hs[c] - 1) < 2e-3
    assert np.abs(ux - hs).max() < 0.02 * np.abs(hs).max()
    # paper's mass flow (eq. theomassflow) and EO current (eq. theo): twice them over the
    # full channel
    kd = 1.0 / lam
    Im = (rho * ux).sum()
    Im_th = (Ex * sigma / nu) / kd ** 2 * (1 - (kd * H / 2) / math.tanh(kd * H / 2))
    assert abs(Im / (2 * Im_th) - 1) < 0.01
    eta = nu * rho.mean()
    Ieo = ((n[1] - n[2]) * ux).sum()
    Ieo_th = -(Ex * sigma ** 2 / (eta * kd * math.tanh(kd * H / 2) ** 2)) * (
        (math.sinh(kd * H) + kd * H) / (4 * math.cosh(kd * H / 2) ** 2)
        - math.sinh(kd * H / 2) / math.cosh(kd * H / 2))
    assert abs(Ieo / (2 * Ieo_th) - 1) < 0.02
    # the Ohmic current dominates the convective one (Sec. IV, Fig. 5)
    I = (j[1][0] - j[2][0]).sum()
    assert I / Ieo > 100


def test_solvent_velocity_departs_at_high_diffusivity(oracle_mod):
    """Sec. IV (Fig. 4): at large omega_drag the solvent moves with the barycentric velocity,
    at small omega_drag the two part."""
    out = {}
    for sc in (1.0, 100.0):
        w, n, j, psi = run_slit(oracle_mod, sigma=-1e-4, Ex=1e-5, sc=sc, steps=20000)
        rho = n[0] + n[1] + n[2]
        ux = (j[0][0] + j[1][0] + j[2][0]) / rho
        u0 = j[0][0] / n[0]
        out[sc] = np.abs(u0 - ux).max() / np.abs(ux).max()
    assert out[1.0] > 30 * out[100.0]
