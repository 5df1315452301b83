"""Helpers shared by the parity tests: running the oracle on a workload, comparing fields,
and light-cone patches for sampled checks of lattices too large for the oracle.

Light cone: D3Q19 moves information by at most one node per step in each axis, so after k
steps the state at a node depends only on the initial state within Chebyshev distance k.
On a periodic patch of width 2k + 3 centred on the node, the wrong values that enter at the
patch faces (distance k + 1) advance one node per step and stay at distance >= 2 after k
steps, so the centre is exact.  This holds for neutral runs only (the Poisson solve is
global).
"""
from __future__ import annotations

import numpy as np

import workloads as WL

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def oracle_for(oracle_mod, w, poisson="direct", lagged=True, sor_tol=1e-8, sor_max=100000,
               sor_check=10, sor_omega=None, drag_pairs=None, forcing="paper"):
    """The oracle for a workload; drag_pairs: [ns][ns] drag relaxation times per pair (the
    library's convention), passed on as frequencies 1 / tau; forcing: "paper" or "guo"."""
    pair = None
    if drag_pairs is not None:
        t = np.asarray(drag_pairs, dtype=np.float64)
        pair = np.where(np.eye(len(t), dtype=bool), 0.0, 1.0 / t)
    o = oracle_mod.Oracle(w.nx, w.ny, w.nz, w.nspecies, w.omega_visc, w.omega_drag,
                          geometry=w.geometry, valence=w.valence, bjerrum=w.bjerrum,
                          sigma=w.sigma, E=w.E, poisson=poisson, lagged=lagged, sor_omega=sor_omega,
                          sor_tol=sor_tol, sor_max=sor_max, sor_check=sor_check, drag_pair=pair,
                          forcing=forcing)
    for s in range(w.nspecies):
        o.set_state(s, w.n[s], w.u[s])
    return o


def fluid(w):
    m = np.ones((w.nz, w.ny, w.nx), bool)
    if w.geometry == "slit":
        m[0] = m[-1] = False
    return m


def rel_to_deviation(a, b, rest, mask=None):
    """max |a - b| / max |b - rest| over the mask."""
    rest = np.broadcast_to(rest, b.shape)
    if mask is not None:
        a, b, rest = a[..., mask], b[..., mask], rest[..., mask]
    den = np.abs(b - rest).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def within(a, b, rel, scale, floor, mask=None):
    """max |a - b| <= rel * scale + floor over the mask; returns (ok, max |a - b|, bound)."""
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    err = float(np.abs(a - b).max())
    bound = rel * scale + floor
    return err <= bound, err, bound


def rel_max(a, b, mask=None):
    """max |a - b| / max |b| over the mask."""
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def patch_workload(w, centre, k):
    """Periodic patch of width 2k + 3 around `centre` (z, y, x) of a periodic workload."""
    width = 2 * k + 3
    half = k + 1
    idx = [(np.arange(width) - half + c) % dim for c, dim in zip(centre, (w.nz, w.ny, w.nx))]
    sel = np.ix_(*idx)
    n = [a[sel] for a in w.n]
    u = [None if a is None else a[(slice(None),) + sel] for a in w.u]
    return WL.Workload(name=w.name + "_patch", nx=width, ny=width, nz=width, geometry="periodic",
                       rho0=w.rho0, valence=w.valence, tau_visc=w.tau_visc, tau_drag=w.tau_drag,
                       n=n, u=u, E=w.E), half
