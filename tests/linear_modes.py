"""Exact linear analysis of the binary LB step around a uniform rest state.

For a single Fourier mode exp(i k x) on a lattice that is uniform in y and z, one LB step
multiplies the population perturbation by L(k) = S(k) J, where J is the Jacobian of the
collision at the uniform state and S(k) = diag(exp(-i k c_px)) is the pull streaming.  J is
taken by complex-step differentiation of the brute-force collision (tests/brute_numpy.py),
which is exact to rounding, so the eigenvalues of L(k) are the exact per-step decay
factors of the discrete scheme: no continuum approximation enters.
"""
from __future__ import annotations

import numpy as np

from brute_numpy import C, CS2, feq, force_term


def _collide_node(f, ns, omega_visc, omega_drag):
    """Collision of one node; f is [ns*19] (may be complex); returns [ns*19]."""
    f = f.reshape(ns, 19)
    n = f.sum(axis=1)
    j = f @ C.astype(np.float64)              # [ns, 3]
    ua = j / n[:, None]
    u = j.sum(axis=0) / n.sum()
    out = np.empty_like(f)
    for s in range(ns):
        F = -omega_drag * (ua[s] - u)
        out[s] = f[s] - omega_visc * (f[s] - feq(n[s], ua[s])) + force_term(n[s], F, u)
    return out.reshape(-1)


def collision_jacobian(rho0, omega_visc, omega_drag, h=1e-30):
    ns = len(rho0)
    f0 = np.concatenate([feq(np.array(r), np.zeros(3)) for r in rho0]).astype(np.complex128)
    m = ns * 19
    J = np.zeros((m, m))
    for i in range(m):
        fp = f0.copy()
        fp[i] += 1j * h
        J[:, i] = _collide_node(fp, ns, omega_visc, omega_drag).imag / h
    return J


def step_operator(rho0, omega_visc, omega_drag, kvec):
    J = collision_jacobian(rho0, omega_visc, omega_drag)
    phase = np.exp(-1j * (C.astype(np.float64) @ np.asarray(kvec, dtype=np.float64)))
    S = np.diag(np.tile(phase, len(rho0)))
    return S @ J


def diffusion_eigenvalue(rho0, omega_visc, omega_drag, kvec):
    """Per-step factor of the concentration (interdiffusion) mode: the eigenvalue of L(k)
    closest to 1 - D k^2 with D = cs2 (1/omega_drag - 1/2)."""
    L = step_operator(rho0, omega_visc, omega_drag, kvec)
    ev = np.linalg.eigvals(L)
    k2 = float(np.dot(kvec, kvec))
    guess = 1.0 - CS2 * (1.0 / omega_drag - 0.5) * k2
    return ev[np.argmin(np.abs(ev - guess))]


def shear_eigenvalue(rho0, omega_visc, omega_drag, kvec):
    """Per-step factor of the transverse momentum (shear) mode: the eigenvalue closest to
    1 - nu k^2 with nu = cs2 (1/omega_visc - 1/2)."""
    L = step_operator(rho0, omega_visc, omega_drag, kvec)
    ev = np.linalg.eigvals(L)
    k2 = float(np.dot(kvec, kvec))
    guess = 1.0 - CS2 * (1.0 / omega_visc - 0.5) * k2
    return ev[np.argmin(np.abs(ev - guess))]
