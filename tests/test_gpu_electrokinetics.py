"""The paper's charged-slit experiment at full size on the GPU (Sec. IV): 64 x 64 x 130 lattice
(fluid 64 x 64 x 128), solvent + cation + anion, lambda_D = 8, surface charge -1e-4 per wall,
E_x = 1e-4, Sc = 100, shifted FP32 populations, direct Poisson solve, 80 000 steps from rest
(the slowest Stokes mode of the channel decays as exp(-t nu pi^2 / H^2): 3e-4 of it is left).

Closed forms, independent of the oracle:
* Helmholtz-Smoluchowski: u_x(z) = E_x (psi~(z) - psi~_wall) / (4 pi l_B eta), eta = rho nu;
* the paper's mass flow and electro-osmotic current (eqs. theomassflow, theo), read as
  integrals over half the channel, so the full-channel values are twice them;
* the Ohmic current dominates the convective one (Sec. IV).
The bars allow the O(h^2 / lambda_D^2) error of the lattice double layer.
"""
import math

import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def run():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    lat = P.from_workload(w, storage="f32s", poisson=dict(method="direct"))
    lat.step(80000)
    # average two consecutive steps: removes the period-2 checkerboard of the start-up
    pr = lat.zprofiles()
    psi = lat.potential().mean(axis=(1, 2))
    lat.step(1)
    pr = 0.5 * (pr + lat.zprofiles())
    psi = 0.5 * (psi + lat.potential().mean(axis=(1, 2)))
    return w, pr[:, :, 1:-1], psi[1:-1], lat.mass_totals()


def test_helmholtz_smoluchowski_profile(run):
    w, pr, psi, _ = run
    rho = pr[:, 0].sum(0)
    ux = pr[:, 1].sum(0) / rho
    nu = CS2 * (w.tau_visc - 0.5)
    k = 4 * math.pi * w.bjerrum
    psi_wall = psi[0] + 0.5 * k * w.sigma[0]      # extrapolated to the wall surface
    hs = w.E[0] * (psi - psi_wall) / (k * nu * rho)
    H = w.nz - 2
    centre = 0.5 * (ux[H // 2 - 1] + ux[H // 2])
    hs_centre = 0.5 * (hs[H // 2 - 1] + hs[H // 2])
    assert abs(centre / hs_centre - 1) < 5e-3, (centre, hs_centre)
    assert np.abs(ux - hs).max() < 0.02 * np.abs(hs).max()


def test_paper_mass_flow_and_electroosmotic_current(run):
    w, pr, psi, _ = run
    Ex, sigma, H = w.E[0], w.sigma[0], w.nz - 2
    n = pr[:, 0]
    rho = n.sum(0)
    ux = pr[:, 1].sum(0) / rho
    nu = CS2 * (w.tau_visc - 0.5)
    kd = 1.0 / 8.0
    Im = (rho * ux).sum()
    Im_th = (Ex * sigma / nu) / kd ** 2 * (1 - (kd * H / 2) / math.tanh(kd * H / 2))
    assert abs(Im / (2 * Im_th) - 1) < 0.01, (Im, 2 * Im_th)
    eta = nu * rho.mean()
    Ieo = ((n[1] - n[2]) * ux).sum()
    Ieo_th = -(Ex * sigma ** 2 / (eta * kd * math.tanh(kd * H / 2) ** 2)) * (
        (math.sinh(kd * H) + kd * H) / (4 * math.cosh(kd * H / 2) ** 2)
        - math.sinh(kd * H / 2) / math.cosh(kd * H / 2))
    assert abs(Ieo / (2 * Ieo_th) - 1) < 0.02, (Ieo, 2 * Ieo_th)
    I = (pr[1, 1] - pr[2, 1]).sum()
    assert I / Ieo > 100


def test_fp32_stochastic_rounding_mobility():
    """The same slit with FP32 storage rounded stochastically from FP64 arithmetic: the
    electro-osmotic mobility stays within 1e-3 of Helmholtz-Smoluchowski, where nearest
    rounding of the FP32 store is biased by 2e-3 at this flow speed (u ~ 5e-7)."""
    import paper_1507_04891_amd as P
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    lat = P.from_workload(w, storage="f32s", stochastic=True, seed=1, poisson=dict(method="direct"))
    lat.step(80000)
    pr = lat.zprofiles()
    psi = lat.potential().mean(axis=(1, 2))
    lat.step(1)
    pr = (0.5 * (pr + lat.zprofiles()))[:, :, 1:-1]
    psi = (0.5 * (psi + lat.potential().mean(axis=(1, 2))))[1:-1]
    rho = pr[:, 0].sum(0)
    ux = pr[:, 1].sum(0) / rho
    nu = CS2 * (w.tau_visc - 0.5)
    k = 4 * math.pi * w.bjerrum
    hs = w.E[0] * (psi - (psi[0] + 0.5 * k * w.sigma[0])) / (k * nu * rho)
    H = w.nz - 2
    c = lambda v: 0.5 * (v[H // 2 - 1] + v[H // 2])
    assert abs(c(ux) / c(hs) - 1) < 1e-3, c(ux) / c(hs) - 1


def test_mass_is_conserved(run):
    """The collision conserves mass exactly; FP32 storage rounds every stored deviation, so over
    80 000 steps the totals may move by the accumulated FP32 rounding (unit roundoff 6e-8 of
    deviations that are themselves far below the totals)."""
    w, _, _, tot = run
    want = np.array([float(a.sum()) for a in w.n])
    drift = np.abs(tot / want - 1)
    assert drift.max() < 1e-6, drift
