"""Independent NumPy brute force of the multicomponent LB step, for tiny lattices.

Written separately from the C oracle and in a different form, so that an index, sign or
table mistake in either one shows up as a disagreement:
  * pull streaming with ``np.roll`` (the oracle pushes node by node);
  * the equilibrium in the textbook form w n (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u^2/(2 cs2))
    at the species velocity (the oracle evaluates the paper's orthogonalised expression);
  * the drag in the summed form -omega_drag (u^a - u) on mid-step velocities (the oracle
    evaluates the pairwise sum);
  * the Poisson problem by a dense least-squares solve of the assembled 7-point matrix
    (the oracle diagonalises the operator).
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0
# D3Q19 in the order documented by the C ABI: rest, +-x, +-y, +-z, then the face diagonals
# (xy, x-y, xz, x-z, yz, y-z), each followed by its opposite.
C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = np.array([int(np.nonzero((C == -C[p]).all(axis=1))[0][0]) for p in range(19)])


def feq(n, u):
    """n: [...], u: [3, ...] -> [19, ...]"""
    cu = np.tensordot(C.astype(np.float64), u, axes=(1, 0))
    uu = (u * u).sum(axis=0)
    return W.reshape((19,) + (1,) * n.ndim) * n * (1.0 + cu / CS2 + 0.5 * cu * cu / CS2 ** 2 - 0.5 * uu / CS2)


def force_term(n, F, u):
    cF = np.tensordot(C.astype(np.float64), F, axes=(1, 0))
    cu = np.tensordot(C.astype(np.float64), u, axes=(1, 0))
    Fu = (F * u).sum(axis=0)
    return W.reshape((19,) + (1,) * n.ndim) * n * (cF / CS2 + (cF * cu - CS2 * Fu) / CS2 ** 2)


class Brute:
    def __init__(self, nx, ny, nz, ns, omega_visc, omega_drag, slit=False, valence=None,
                 bjerrum=0.0, sigma=(0.0, 0.0), E=(0.0, 0.0, 0.0), lagged=True):
        self.nx, self.ny, self.nz, self.ns = nx, ny, nz, ns
        self.wv, self.wd = omega_visc, omega_drag
        self.slit = slit
        self.val = np.array(valence if valence is not None else [0] * ns, dtype=np.float64)
        self.lb = bjerrum
        self.sig = sigma
        self.E = np.array(E, dtype=np.float64)
        self.lagged = lagged
        self.fluid = np.ones((nz, ny, nx), dtype=bool)
        if slit:
            self.fluid[0] = self.fluid[-1] = False
        self.f = np.zeros((ns, 19, nz, ny, nx))
        self.psi = None
        self._A = None

    # -- state --------------------------------------------------------------------------
    def set_state(self, s, n, u=None):
        u = np.zeros((3,) + n.shape) if u is None else u
        self.f[s] = feq(n, u) * self.fluid
        self.psi = None

    def moments(self):
        n = self.f.sum(axis=1)
        j = np.tensordot(self.f, C.astype(np.float64), axes=(1, 0))   # [s, z, y, x, 3]
        j = np.moveaxis(j, -1, 1)                                     # [s, 3, z, y, x]
        return n, j

    # -- Poisson --------------------------------------------------------------------------
    def _assemble(self):
        idx = -np.ones((self.nz, self.ny, self.nx), dtype=np.int64)
        pts = np.argwhere(self.fluid)
        idx[tuple(pts.T)] = np.arange(len(pts))
        A = np.zeros((len(pts), len(pts)))
        for r, (z, y, x) in enumerate(pts):
            for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
                zz, yy, xx = z + dz, (y + dy) % self.ny, (x + dx) % self.nx
                if self.slit:
                    if not (0 < zz < self.nz - 1):
                        continue
                else:
                    zz %= self.nz
                A[r, idx[zz, yy, xx]] += 1.0
                A[r, r] -= 1.0
        self._A, self._pts = A, pts

    def solve_potential(self, q):
        if self._A is None:
            self._assemble()
        b = -4.0 * np.pi * self.lb * q.copy()
        if self.slit:
            b[1] += -4.0 * np.pi * self.lb * self.sig[0]
            b[self.nz - 2] += -4.0 * np.pi * self.lb * self.sig[1]
        bv = b[tuple(self._pts.T)]
        bv = bv - bv.mean()
        sol, *_ = np.linalg.lstsq(self._A, bv, rcond=None)
        sol -= sol.mean()
        psi = np.zeros((self.nz, self.ny, self.nx))
        psi[tuple(self._pts.T)] = sol
        return psi

    def _charged(self):
        return self.lb > 0 and np.any(self.val != 0)

    def _grad(self, psi):
        k = 4.0 * np.pi * self.lb
        gx = 0.5 * (np.roll(psi, -1, axis=2) - np.roll(psi, 1, axis=2))
        gy = 0.5 * (np.roll(psi, -1, axis=1) - np.roll(psi, 1, axis=1))
        up = np.roll(psi, -1, axis=0)
        dn = np.roll(psi, 1, axis=0)
        if self.slit:
            up[self.nz - 2] = psi[self.nz - 2] + k * self.sig[1]
            dn[1] = psi[1] + k * self.sig[0]
        gz = 0.5 * (up - dn)
        return np.stack([gx, gy, gz])

    # -- one step -----------------------------------------------------------------------
    def step(self, nsteps=1):
        for _ in range(nsteps):
            n, j = self.moments()
            q = (self.val[:, None, None, None] * n).sum(axis=0)
            if self._charged():
                if self.psi is None or not self.lagged:
                    self.psi = self.solve_potential(q)
                grad = self._grad(self.psi)
            else:
                grad = np.zeros((3, self.nz, self.ny, self.nx))
            with np.errstate(invalid="ignore", divide="ignore"):
                ua = np.where(n[:, None] != 0, j / n[:, None], 0.0)
            ntot = n.sum(axis=0)
            with np.errstate(invalid="ignore", divide="ignore"):
                u = np.where(ntot != 0, j.sum(axis=0) / ntot, 0.0)
            # field acceleration per species; the drag acts on the mid-step velocities
            acc = np.stack([self.val[s] * (self.E[:, None, None, None] - CS2 * grad)
                            for s in range(self.ns)])
            umid = ua + 0.5 * acc
            with np.errstate(invalid="ignore", divide="ignore"):
                ubar_mid = np.where(ntot != 0, (n[:, None] * umid).sum(axis=0) / ntot, 0.0)
            post = np.empty_like(self.f)
            for s in range(self.ns):
                F = -self.wd * (umid[s] - ubar_mid) + acc[s]
                eq = feq(n[s], ua[s])
                post[s] = self.f[s] - self.wv * (self.f[s] - eq) + force_term(n[s], F, u)
            post *= self.fluid
            new = np.zeros_like(self.f)
            for p in range(19):
                cx, cy, cz = C[p]
                moved = np.roll(post[:, p], shift=(cz, cy, cx), axis=(1, 2, 3))
                if self.slit:
                    # pull from a wall plane -> bounce back the opposite population in place
                    if cz == 1:
                        moved[:, 1] = post[:, OPP[p], 1]
                    elif cz == -1:
                        moved[:, self.nz - 2] = post[:, OPP[p], self.nz - 2]
                    moved[:, 0] = 0.0
                    moved[:, -1] = 0.0
                new[:, p] = moved
            self.f = new
            if self._charged() and self.lagged:
                self.psi = self.solve_potential(q)
