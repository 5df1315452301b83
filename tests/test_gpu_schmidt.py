"""lbmix_set_schmidt under the paper's forcing, end to end against the oracle.

The GPU lattice gets its drag only from the Schmidt number (lbmix_set_schmidt, no
lbmix_set_tau_drag).  The oracle gets omega_drag computed here from the discrete transport
coefficients of Sec. IV, nu = v_T^2 (1/omega_visc - 1/2) and D = v_T^2 (1/omega_drag - 1/2),
with Sc = nu / D, so the library's own mapping is what is compared.  Bars as for every FP64
parity case: 1e-12 of the deviation from rest for densities and populations, 1e-11 of
max|j| for momenta, and a rounding floor of 1e-14 max|n|.
"""
import dataclasses

import numpy as np
import pytest

import workloads as WL
from parity_util import W as WQ, fluid, oracle_for, within

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    return P


def omega_drag_sec4(tau_visc, sc):
    """omega_drag with nu / D = sc, from the discrete nu and D of Sec. IV."""
    nu = CS2 * (tau_visc - 0.5)
    D = nu / sc
    return 1.0 / (D / CS2 + 0.5)


def compare(lat, o, w):
    m = fluid(w)
    for s in range(w.nspecies):
        ng, jg = lat.moments(s)
        no, jo = o.moments(s)
        F = 1e-14 * np.abs(no[m]).max()
        ok, err, bnd = within(ng, no, 1e-12, np.abs(no - w.rho0[s])[m].max(), F, m)
        assert ok, ("n", s, err, bnd)
        ok, err, bnd = within(jg, jo, 1e-11, np.abs(jo[:, m]).max(), F, m)
        assert ok, ("j", s, err, bnd)
        fg, fo = lat.populations(s), o.populations(s)
        rest = (WQ * w.rho0[s])[:, None, None, None]
        ok, err, bnd = within(fg, fo, 1e-12, np.abs(fo - rest)[:, m].max(), F, m)
        assert ok, ("f", s, err, bnd)


@pytest.mark.parametrize("sc", [10.0, 1000.0])
def test_schmidt_binary_fp64(P, oracle_mod, sc):
    """Binary concentration and shear modes, 24^3 periodic, tau_visc 0.9 (not 1, so that tau and
    omega cannot be confused unnoticed), 300 steps.  Mode amplitude 1e-2: the rounding floor of
    300 steps with 1 - omega_visc != 0 is about 70 units in the last place of n."""
    w = WL.binary_multimode(n=24, amp=1e-2, nmodes=4, shear=1e-3, tau_visc=0.9, sc=sc, seed=11)
    w = dataclasses.replace(w, tau_drag=1.0 / omega_drag_sec4(0.9, sc))
    lat = P.from_workload(w, storage="f64", schmidt=sc)
    o = oracle_for(oracle_mod, w)
    lat.step(300)
    o.step(300)
    compare(lat, o, w)


def test_schmidt_changes_the_dynamics(P):
    """The Schmidt number reaches the step: Sc 10 and 1000 give different states."""
    w = WL.binary_multimode(n=24, amp=1e-3, nmodes=4, shear=1e-3, tau_visc=0.9, sc=10.0, seed=11)
    a = P.from_workload(w, storage="f64", schmidt=10.0)
    b = P.from_workload(w, storage="f64", schmidt=1000.0)
    a.step(50)
    b.step(50)
    assert np.abs(a.moments(0)[0] - b.moments(0)[0]).max() > 1e-6


def test_schmidt_charged_slit_fp64(P, oracle_mod):
    """Charged ternary slit 8 x 6 x 18 under a field, Sc 100, direct Poisson solve."""
    sc = 100.0
    w = WL.charged_slit(nx=8, ny=6, nz=18, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4,
                        tau_visc=1.0, sc=sc)
    w = dataclasses.replace(w, tau_drag=1.0 / omega_drag_sec4(1.0, sc))
    lat = P.from_workload(w, storage="f64", schmidt=sc, poisson=dict(method="direct"))
    o = oracle_for(oracle_mod, w, poisson="direct")
    lat.step(120)
    o.step(120)
    compare(lat, o, w)
    # the potential: 1e-11 of max|psi| plus the rounding of q amplified by the inverse of the
    # 7-point operator (smallest eigenvalue about (pi / L)^2)
    m = fluid(w)
    L = max(w.nx, w.ny, w.nz - 2)
    qfloor = 2.2e-16 * sum(abs(z) * r for z, r in zip(w.valence, w.rho0))
    pg, po = lat.potential(), o.potential()
    ok, err, bnd = within(pg, po, 1e-11, np.abs(po[m]).max(), 4 * 4 * np.pi * w.bjerrum * qfloor * (L / np.pi) ** 2, m)
    assert ok, ("psi", err, bnd)
