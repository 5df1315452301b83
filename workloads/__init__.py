"""Seeded synthetic inputs for the multicomponent lattice-Boltzmann runs.

This module only builds initial macroscopic fields (densities, velocities) and parameter
sets; it contains none of the method's arithmetic.  Both the GPU library's tests and the
oracle are fed from here.  All arrays are numpy float64 in ``[z][y][x]`` order (x fastest);
velocity fields are ``[3][z][y][x]``.

The shapes follow the paper's numerical experiments (Sec. IV): a sinusoidal concentration
profile in a periodic box for the diffusion coefficient, a sinusoidal shear wave for the
viscosity, a uniform ternary electrolyte under a field for the bulk conductivity, and a
charged slit channel (walls normal to z, field along x) for electro-osmosis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CS2 = 1.0 / 3.0


def omega_from_tau(tau: float) -> float:
    return 1.0 / tau


def tau_drag_for_schmidt(tau_visc: float, sc: float) -> float:
    """Drag relaxation time giving nu / D = sc with nu = cs2 (tau_visc - 1/2) and
    D = cs2 (tau_drag - 1/2) (Sec. IV, the discrete transport coefficients)."""
    return 0.5 + (tau_visc - 0.5) / sc


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    geometry: str                      # "periodic" or "slit"
    rho0: list                         # rest density per species (storage shift)
    valence: list
    tau_visc: float
    tau_drag: float
    n: list                            # per species [nz][ny][nx]
    u: list                            # per species [3][nz][ny][nx] or None
    bjerrum: float = 0.0
    sigma: tuple = (0.0, 0.0)
    E: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def nspecies(self) -> int:
        return len(self.rho0)

    @property
    def omega_visc(self) -> float:
        return 1.0 / self.tau_visc

    @property
    def omega_drag(self) -> float:
        return 1.0 / self.tau_drag

    @property
    def fluid_nodes(self) -> int:
        nzf = self.nz - 2 if self.geometry == "slit" else self.nz
        return self.nx * self.ny * nzf


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def binary_sine(nx=32, ny=32, nz=32, rho0=0.5, amp=0.01, mode=1, tau_visc=1.0, sc=10.0, steps=500):
    """Neutral binary mixture, concentration profile amp*sin(2 pi mode x / nx) in antiphase
    between the two species, zero velocity (the bulk diffusion experiment of Sec. IV)."""
    x, _, _ = _grid(nx, ny, nz)
    s = amp * np.sin(2.0 * np.pi * mode * x / nx)
    return Workload(name=f"binary_sine_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, geometry="periodic",
                    rho0=[rho0, rho0], valence=[0, 0], tau_visc=tau_visc,
                    tau_drag=tau_drag_for_schmidt(tau_visc, sc), n=[rho0 + s, rho0 - s],
                    u=[None, None], steps=steps, extra={"sc": sc, "amp": amp, "mode": mode})


def binary_multimode(n=256, rho0=0.5, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=100.0,
                     seed=2, steps=2000):
    """Neutral binary mixture on an n^3 periodic box: nmodes concentration modes (mode m along
    axis (m-1) mod 3, wavenumber 2 pi m / n, amplitude amp, phase uniform in [0, 2 pi) from
    `seed`), in antiphase between the species, plus a shear wave u_y = shear sin(2 pi x / n)
    shared by both species."""
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    ax = np.arange(n, dtype=np.float64)
    dn = np.zeros((n, n, n))
    for m in range(1, nmodes + 1):
        axis = (m - 1) % 3                       # 0 -> x, 1 -> y, 2 -> z
        prof = amp * np.sin(2.0 * np.pi * m * ax / n + phases[m - 1])
        shape = [1, 1, 1]
        shape[2 - axis] = n                      # array order is [z][y][x]
        dn += prof.reshape(shape)
    uy = shear * np.sin(2.0 * np.pi * ax / n)
    u = np.zeros((3, n, n, n))
    u[1] = uy.reshape(1, 1, n)
    return Workload(name=f"binary_multimode_{n}^3", nx=n, ny=n, nz=n, geometry="periodic",
                    rho0=[rho0, rho0], valence=[0, 0], tau_visc=tau_visc,
                    tau_drag=tau_drag_for_schmidt(tau_visc, sc), n=[rho0 + dn, rho0 - dn],
                    u=[u, u], steps=steps,
                    extra={"sc": sc, "seed": seed, "phases": phases.tolist(), "amp": amp,
                           "shear": shear})


def random_state(nx, ny, nz, nspecies, geometry="periodic", seed=0, rho0=None, dn=0.05, du=0.02,
                 valence=None, tau_visc=0.8, tau_drag=0.6, bjerrum=0.0, sigma=(0.0, 0.0),
                 E=(0.0, 0.0, 0.0)):
    """Uniformly random densities rho0*(1 + dn*U[-1,1]) and velocities du*U[-1,1] per node and
    species (wall planes of a slit are zero)."""
    rng = np.random.default_rng(seed)
    rho0 = list(rho0) if rho0 is not None else [1.0 / nspecies] * nspecies
    shape = (nz, ny, nx)
    ns, us = [], []
    for s in range(nspecies):
        n = rho0[s] * (1.0 + dn * rng.uniform(-1.0, 1.0, size=shape))
        u = du * rng.uniform(-1.0, 1.0, size=(3,) + shape)
        if geometry == "slit":
            n[0] = n[-1] = 0.0
            u[:, 0] = u[:, -1] = 0.0
        ns.append(n)
        us.append(u)
    return Workload(name=f"random_{nx}x{ny}x{nz}_s{nspecies}_{geometry}", nx=nx, ny=ny, nz=nz,
                    geometry=geometry, rho0=rho0,
                    valence=list(valence) if valence is not None else [0] * nspecies,
                    tau_visc=tau_visc, tau_drag=tau_drag, n=ns, u=us, bjerrum=bjerrum,
                    sigma=tuple(sigma), E=tuple(E), extra={"seed": seed})


def bjerrum_for_debye(debye_length: float, n_ion_total: float) -> float:
    """l_B such that lambda_D = 1 / sqrt(4 pi l_B (n+ + n-)) (Sec. IV)."""
    return 1.0 / (4.0 * math.pi * n_ion_total * debye_length ** 2)


def debye_huckel_potential(z, nz, debye_length, bjerrum, sigma):
    """Linearised (Debye-Hueckel) potential psi~ of a slit whose solid planes are z = 0 and
    z = nz-1 (wall surfaces at z = 0.5 and z = nz-1.5), both with surface charge sigma."""
    kd = 1.0 / debye_length
    H = nz - 2
    zc = 0.5 * (nz - 1)
    return (4.0 * math.pi * bjerrum * sigma / kd) * np.cosh(kd * (z - zc)) / math.sinh(kd * H / 2.0)


def charged_slit(nx=64, ny=64, nz=130, n_solvent=1.0, n_ion=1e-3, debye_length=8.0, sigma=-1e-4,
                 Ex=1e-4, tau_visc=1.0, sc=100.0, steps=20000):
    """Ternary electrolyte (solvent z=0, cation z=+1, anion z=-1) in a slit with solid planes
    z = 0 and z = nz-1, both carrying surface charge `sigma`, field Ex along x.  The ions
    start from the Debye-Hueckel Boltzmann profile n+- = n_ion exp(-+psi~_DH), rescaled so
    that the fluid carries exactly the opposite of the wall charge."""
    lb = bjerrum_for_debye(debye_length, 2.0 * n_ion)
    z = np.arange(nz, dtype=np.float64)
    psi = debye_huckel_potential(z, nz, debye_length, lb, sigma)
    P = np.exp(-psi)
    M = np.exp(psi)
    P[0] = P[-1] = M[0] = M[-1] = 0.0
    H = nz - 2
    # a*sum(P) - b*sum(M) = -2 sigma (per column), a*sum(P) + b*sum(M) = 2 n_ion H
    sP, sM = P.sum(), M.sum()
    target_q = -2.0 * sigma
    target_n = 2.0 * n_ion * H
    a = 0.5 * (target_n + target_q) / sP
    b = 0.5 * (target_n - target_q) / sM
    npos = (a * P)[:, None, None] * np.ones((nz, ny, nx))
    nneg = (b * M)[:, None, None] * np.ones((nz, ny, nx))
    nsol = np.full((nz, ny, nx), n_solvent)
    nsol[0] = nsol[-1] = 0.0
    return Workload(name=f"charged_slit_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, geometry="slit",
                    rho0=[n_solvent, n_ion, n_ion], valence=[0, 1, -1], tau_visc=tau_visc,
                    tau_drag=tau_drag_for_schmidt(tau_visc, sc), n=[nsol, npos, nneg],
                    u=[None, None, None], bjerrum=lb, sigma=(sigma, sigma), E=(Ex, 0.0, 0.0),
                    steps=steps, extra={"sc": sc, "debye_length": debye_length, "n_ion": n_ion})


def bulk_electrolyte(n=4, n_solvent=1.0, ratio=1e-2, Ex=1e-4, tau_visc=1.0, tau_drag=0.6):
    """Uniform ternary electrolyte, n+ = n- = ratio * n0, under a uniform field (the bulk
    conductivity experiment of Sec. IV)."""
    shape = (n, n, n)
    ni = ratio * n_solvent
    return Workload(name=f"bulk_electrolyte_{n}^3", nx=n, ny=n, nz=n, geometry="periodic",
                    rho0=[n_solvent, ni, ni], valence=[0, 1, -1], tau_visc=tau_visc,
                    tau_drag=tau_drag,
                    n=[np.full(shape, n_solvent), np.full(shape, ni), np.full(shape, ni)],
                    u=[None, None, None], E=(Ex, 0.0, 0.0))


@dataclass
class ChannelStack:
    """Independent charged slit channels of the same lateral extent, stacked along z (each
    with its own two wall planes): the batched form of the electro-osmosis experiment.
    Arrays cover all nz = sum (W_c + 2) planes."""
    name: str
    nx: int
    ny: int
    widths: list                       # fluid width of each channel
    rho0: list
    valence: list
    tau_visc: float
    tau_drags: list                    # per channel
    sigmas: list                       # per channel (sigma_lo, sigma_hi)
    n: list                            # per species [nz][ny][nx]
    u: list                            # per species [3][nz][ny][nx] or None
    bjerrum: float = 0.0
    E: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)
    geometry: str = "channels"

    @property
    def nz(self) -> int:
        return sum(w + 2 for w in self.widths)

    @property
    def nspecies(self) -> int:
        return len(self.rho0)

    def planes(self, c):
        """Slice of the full-lattice planes of channel c (walls included)."""
        z0 = sum(w + 2 for w in self.widths[:c])
        return slice(z0, z0 + self.widths[c] + 2)

    def channel(self, c) -> Workload:
        """Channel c alone, as a slit workload with the same initial fields."""
        sl = self.planes(c)
        return Workload(name=f"{self.name}_ch{c}", nx=self.nx, ny=self.ny, nz=self.widths[c] + 2,
                        geometry="slit", rho0=list(self.rho0), valence=list(self.valence),
                        tau_visc=self.tau_visc, tau_drag=self.tau_drags[c],
                        n=[a[sl].copy() for a in self.n],
                        u=[None if v is None else v[:, sl].copy() for v in self.u],
                        bjerrum=self.bjerrum, sigma=tuple(self.sigmas[c]), E=self.E)


def channel_stack(nx=32, ny=32, widths=(32, 48), sigmas=(-1e-4, -5e-4), scs=(10.0, 100.0), n_solvent=1.0,
                  n_ion=1e-3, debye_length=8.0, Ex=1e-4, tau_visc=1.0, lateral=0.0, seed=5):
    """Stack of charged slits (ternary electrolyte as charged_slit, one sigma on both walls of
    channel c, Schmidt number scs[c]).  lateral > 0 adds to the cation density of each
    channel lateral * n_ion * sin(2 pi (x / nx + y / ny) + phase_c) (zero sum over every
    plane: the channel stays neutral) with seeded random phases."""
    rng = np.random.default_rng(seed)
    parts = [charged_slit(nx=nx, ny=ny, nz=w + 2, n_solvent=n_solvent, n_ion=n_ion, debye_length=debye_length,
                          sigma=sg, Ex=Ex, tau_visc=tau_visc, sc=sc)
             for w, sg, sc in zip(widths, sigmas, scs)]
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    if lateral > 0.0:
        for p in parts:
            ph = rng.uniform(0.0, 2.0 * math.pi)
            bump = lateral * n_ion * np.sin(2.0 * math.pi * (x / nx + y / ny) + ph) * np.ones((p.nz, 1, 1))
            bump[0] = bump[-1] = 0.0
            p.n[1] = p.n[1] + bump
    n = [np.concatenate([p.n[s] for p in parts], axis=0) for s in range(3)]
    return ChannelStack(name=f"channel_stack_{len(widths)}x{nx}x{ny}", nx=nx, ny=ny, widths=list(widths),
                        rho0=[n_solvent, n_ion, n_ion], valence=[0, 1, -1], tau_visc=tau_visc,
                        tau_drags=[p.tau_drag for p in parts], sigmas=[tuple(p.sigma) for p in parts],
                        n=n, u=[None, None, None], bjerrum=parts[0].bjerrum, E=(Ex, 0.0, 0.0),
                        extra={"scs": list(scs), "debye_length": debye_length, "n_ion": n_ion})


def batched_channels(nch=64, nx=32, ny=32, wmin=32, wmax=256, seed=5, lateral=0.0):
    """The batched electro-osmosis workload: nch channels of fluid width W ~ U{wmin..wmax},
    lateral nx x ny, wall charge sigma ~ -U[1e-4, 1e-3], Schmidt number 10, 100, 1000 by
    channel index mod 3, lambda_D = 8, ions 1e-3, E_x = 1e-4, tau_visc = 1 (seeded)."""
    rng = np.random.default_rng(seed)
    widths = [int(w) for w in rng.integers(wmin, wmax + 1, size=nch)]
    sigmas = [-float(s) for s in rng.uniform(1e-4, 1e-3, size=nch)]
    scs = [(10.0, 100.0, 1000.0)[c % 3] for c in range(nch)]
    return channel_stack(nx=nx, ny=ny, widths=widths, sigmas=sigmas, scs=scs, lateral=lateral, seed=seed + 1)
