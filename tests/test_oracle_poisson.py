"""Pins of the oracle's Poisson solvers (eq. Poisson of Sec. II with the surface-charge
condition).  The operator is re-assembled here as a plain 7-point stencil with numpy, the
right-hand side is manufactured from a chosen potential, and the solvers must return it;
the Debye-Hueckel closed form pins the wall-charge treatment."""
import math

import numpy as np
import pytest

import workloads as WL


def stencil(psi, slit):
    """sum over neighbours (psi_nb - psi); slit: no neighbour across the planes z=0, nz-1."""
    nz = psi.shape[0]
    out = np.zeros_like(psi)
    for ax in (1, 2):
        out += np.roll(psi, 1, axis=ax) + np.roll(psi, -1, axis=ax) - 2 * psi
    if slit:
        for z in range(1, nz - 1):
            if z + 1 < nz - 1:
                out[z] += psi[z + 1] - psi[z]
            if z - 1 > 0:
                out[z] += psi[z - 1] - psi[z]
        out[0] = out[-1] = 0.0
    else:
        out += np.roll(psi, 1, axis=0) + np.roll(psi, -1, axis=0) - 2 * psi
    return out


def manufactured(nx, ny, nz, slit, lb, sig, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=(nz, ny, nx))
    fl = np.ones(psi.shape, bool)
    if slit:
        fl[0] = fl[-1] = False
        psi[~fl] = 0.0
    psi[fl] -= psi[fl].mean()
    b = stencil(psi, slit)
    k = 4 * math.pi * lb
    q = -b / k
    if slit:
        q[1] -= sig[0]
        q[nz - 2] -= sig[1]
        q[0] = q[-1] = 0.0
    return psi, q


@pytest.mark.parametrize("dims,slit", [((6, 4, 8), False), ((5, 3, 7), False), ((1, 1, 9), False),
                                       ((6, 4, 10), True), ((3, 1, 12), True), ((2, 2, 3), True),
                                       ((8, 8, 18), True)])
def test_direct_solver_inverts_operator(oracle_mod, dims, slit):
    nx, ny, nz = dims
    sig = (-3e-3, 1e-3)
    psi, q = manufactured(nx, ny, nz, slit, 0.7, sig, seed=nx * 100 + nz)
    o = oracle_mod.Oracle(nx, ny, nz, 1, 1.0, 1.0, geometry="slit" if slit else "periodic",
                          valence=[1], bjerrum=0.7, sigma=sig, poisson="direct")
    got, sweeps, resid, st = o.poisson(q)
    assert st == 0 and sweeps == 0
    np.testing.assert_allclose(got, psi, rtol=0, atol=1e-11 * np.abs(psi).max())
    assert resid < 1e-13


@pytest.mark.parametrize("dims,slit", [((6, 4, 8), False), ((6, 4, 10), True), ((8, 8, 18), True),
                                       ((2, 2, 34), True)])
def test_sor_converges_to_direct(oracle_mod, dims, slit):
    nx, ny, nz = dims
    sig = (-3e-3, 1e-3)
    psi, q = manufactured(nx, ny, nz, slit, 0.7, sig, seed=3)
    geo = "slit" if slit else "periodic"
    o = oracle_mod.Oracle(nx, ny, nz, 1, 1.0, 1.0, geometry=geo, valence=[1], bjerrum=0.7,
                          sigma=sig, poisson="sor", sor_tol=1e-12, sor_max=200000, sor_check=5)
    got, sweeps, resid, st = o.poisson(q)
    assert st == 0 and 0 < sweeps < 200000 and resid <= 1e-12
    np.testing.assert_allclose(got, psi, rtol=0, atol=1e-8 * np.abs(psi).max())
    # the residual is the one of the manufactured problem
    b = stencil(psi, slit)
    r = b - stencil(got, slit)
    fl = slice(1, nz - 1) if slit else slice(0, nz)
    assert np.sqrt((r[fl] ** 2).sum() / (b[fl] ** 2).sum()) <= 1.0001e-12


def test_sor_reports_non_convergence(oracle_mod):
    psi, q = manufactured(8, 8, 18, True, 0.7, (-1e-3, -1e-3), seed=4)
    o = oracle_mod.Oracle(8, 8, 18, 1, 1.0, 1.0, geometry="slit", valence=[1], bjerrum=0.7,
                          sigma=(-1e-3, -1e-3), poisson="sor", sor_tol=1e-10, sor_max=7,
                          sor_check=3)
    got, sweeps, resid, st = o.poisson(q)
    assert st == -5 and sweeps == 7 and resid > 1e-10


def test_sor_fixed_sweeps_and_warm_start(oracle_mod):
    psi, q = manufactured(6, 4, 10, True, 0.7, (-1e-3, 0.0), seed=5)
    mk = lambda m: oracle_mod.Oracle(6, 4, 10, 1, 1.0, 1.0, geometry="slit", valence=[1],  # noqa
                                     bjerrum=0.7, sigma=(-1e-3, 0.0), poisson="sor", sor_tol=0.0,
                                     sor_max=m)
    a, sa, _, st = mk(30).poisson(q)
    assert st == 0 and sa == 30
    b1, _, _, _ = mk(12).poisson(q)
    b2, _, _, _ = mk(18).poisson(q, psi0=b1)
    # 12 sweeps, gauge, then 18 more == 30 sweeps up to the gauge shift (mean removed twice)
    np.testing.assert_allclose(b2, a, rtol=0, atol=1e-12)
    # the exact solution is a fixed point
    c, _, r, _ = mk(5).poisson(q, psi0=psi)
    np.testing.assert_allclose(c, psi, rtol=0, atol=1e-13)


def test_debye_huckel_closed_form(oracle_mod):
    """With the charge of the linearised Boltzmann profile, q = -(k_D^2 / 4 pi l_B) psi_DH,
    the discrete solution matches psi_DH to the O(h^2 k_D^2 / 12) discretisation error;
    the wall potential of the paper's config (-6.25e-3 for lambda_D = 8, sigma = -1e-4) is
    reproduced."""
    nz = 130
    lam = 8.0
    lb = WL.bjerrum_for_debye(lam, 2e-3)
    sig = -1e-4
    z = np.arange(nz, dtype=float)
    dh = WL.debye_huckel_potential(z, nz, lam, lb, sig)
    q = np.zeros((nz, 2, 2))
    q[1:-1] = (-(1.0 / lam ** 2) / (4 * math.pi * lb) * dh[1:-1])[:, None, None]
    # the wall charge is carried by the walls; the fluid charge must cancel it
    q[1:-1] += (-(2 * sig) - q[1:-1, 0, 0].sum()) / (nz - 2)
    o = oracle_mod.Oracle(2, 2, nz, 1, 1.0, 1.0, geometry="slit", valence=[1], bjerrum=lb,
                          sigma=(sig, sig), poisson="direct")
    got, _, _, _ = o.poisson(q)
    ref = dh - dh[1:-1].mean()
    err = np.abs(got[1:-1, 0, 0] - ref[1:-1]).max() / np.abs(ref).max()
    assert err < 1.0 / (12 * lam ** 2) * 2
    # wall value in the paper's units: 4 pi l_B sigma lambda_D coth(H / 2 lambda_D)
    wall = 4 * math.pi * lb * sig * lam / math.tanh((nz - 2) / (2 * lam))
    assert abs(wall - (-6.25e-3)) < 1e-6
