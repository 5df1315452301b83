"""FP64 CPU oracle of the multicomponent lattice-Boltzmann step (test infrastructure).

This package is the slow, plain reference that the GPU library is checked against.  It is
imported only by ``tests/``, by the smoke check and by the CPU-baseline leg of the
benchmark; the GPU path never imports it.  The arithmetic lives in ``lbmix_oracle.c``
(plain C, FP64), which cites the paper equation by equation:

* discrete update, eq. (latboeq) of Sec. IV, on the D3Q19 lattice;
* equilibrium ``phi_perp_p``: the last equation of the Appendix;
* forcing ``g_p``: eq. (ourforc) of the Appendix;
* drag force: Sec. II, the definition of ``F^{alpha,drag}/m`` for equal masses;
* electrostatic force and Poisson equation: eq. (evolution) and eq. (Poisson), Sec. II.

Arrays are numpy float64 in ``[z][y][x]`` order (x fastest), the same node order as the
GPU library's C ABI.  Vector fields are ``[3][z][y][x]``; populations ``[19][z][y][x]`` in
the D3Q19 order returned by :func:`d3q19`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbmix_oracle.c")
LIB_PATH = os.path.join(_HERE, "liblbmix_oracle.so")
MAXS = 8
Q = 19


BUILD_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC"]
# the same source built for the host it runs on, for timing it as the CPU baseline (no FMA
# contraction either, so the arithmetic is that of the default build)
NATIVE_FLAGS = ["-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC"]


def build(force: bool = True, native: bool = False, path: str | None = None) -> str:
    """Compile the oracle with gcc (plain ISO C, no FMA contraction, OpenMP over nodes).
    native: optimise for this host's CPU (-O3 -march=native) into `path`."""
    out = path or LIB_PATH
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", *(NATIVE_FLAGS if native else BUILD_FLAGS), "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("slit", ctypes.c_int), ("ns", ctypes.c_int),
        ("omega_visc", ctypes.c_double), ("omega_drag", ctypes.c_double),
        ("valence", ctypes.c_int * MAXS),
        ("bjerrum", ctypes.c_double), ("sigma_lo", ctypes.c_double), ("sigma_hi", ctypes.c_double),
        ("E", ctypes.c_double * 3),
        ("poisson", ctypes.c_int), ("lagged", ctypes.c_int),
        ("sor_omega", ctypes.c_double), ("sor_tol", ctypes.c_double),
        ("sor_max", ctypes.c_int), ("sor_check", ctypes.c_int),
        ("pair_drag", ctypes.c_int), ("drag_pair", ctypes.c_double * (MAXS * MAXS)),
        ("forcing", ctypes.c_int),
    ]


_libs = {}


def lib(path: str | None = None):
    """The loaded oracle library (the default build, or the one at `path`)."""
    path = path or LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            build(path=path)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.POINTER(_Params)]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_set_state.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
        L.ora_set_f.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.ora_get_f.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_moments.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
        L.ora_mass_totals.argtypes = [ctypes.c_void_p, dp]
        L.ora_get_psi.argtypes = [ctypes.c_void_p, dp]
        L.ora_get_q.argtypes = [ctypes.c_void_p, dp]
        L.ora_poisson.argtypes = [ctypes.c_void_p, dp, dp, ip, dp]
        L.ora_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_long), ip, dp]
        L.ora_d3q19.argtypes = [ip, dp, ip]
        L.ora_phi_perp.argtypes = [ctypes.c_double, dp, dp, dp]
        L.ora_forcing.argtypes = [ctypes.c_double, dp, dp, dp]
        L.ora_drag.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.ora_drag_pair.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, dp]
        _libs[path] = L
    return _libs[path]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def d3q19():
    """(c[19,3] int, w[19] float, opp[19] int) as the oracle defines them."""
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().ora_d3q19(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                    opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c.reshape(19, 3), w, opp


def phi_perp(n: float, ua, u) -> np.ndarray:
    out = np.zeros(19)
    lib().ora_phi_perp(float(n), _dp(_f64(ua)), _dp(_f64(u)), _dp(out))
    return out


def forcing(n: float, F, u) -> np.ndarray:
    out = np.zeros(19)
    lib().ora_forcing(float(n), _dp(_f64(F)), _dp(_f64(u)), _dp(out))
    return out


def drag(n, ua, omega_drag: float) -> np.ndarray:
    n = _f64(n)
    ua = _f64(ua).reshape(len(n), 3)
    F = np.zeros_like(ua)
    lib().ora_drag(len(n), _dp(n), _dp(ua), float(omega_drag), _dp(F))
    return F


def drag_pair(n, ua, omega) -> np.ndarray:
    """Drag with a frequency per pair: omega is [ns][ns] (symmetric)."""
    n = _f64(n)
    ua = _f64(ua).reshape(len(n), 3)
    om = _f64(omega).reshape(len(n), len(n))
    F = np.zeros_like(ua)
    lib().ora_drag_pair(len(n), _dp(n), _dp(ua), _dp(om), len(n), _dp(F))
    return F


def sor_omega_default(nx: int, ny: int, nzf: int) -> float:
    """Over-relaxation factor 2 / (1 + sin(pi / L)) with L the largest fluid extent."""
    L = max(nx, ny, nzf)
    return 2.0 / (1.0 + np.sin(np.pi / L))


class Oracle:
    """One lattice of the FP64 oracle.

    geometry: "periodic" (periodic in x, y, z) or "slit" (solid planes z = 0 and z = nz-1).
    poisson: "direct" (spectral solve of the 7-point operator) or "sor" (red-black SOR).
    forcing: "paper" (drag on mid-step velocities, reading R3b), "guo" (the Guo-type
    variant) or "literal" (drag on the plain first moments; only for the tests that pin R3b).
    lib_path: another build of the same source (e.g. the host-optimised one of build(native=True)).
    """

    def __init__(self, nx, ny, nz, nspecies, omega_visc, omega_drag, geometry="periodic",
                 valence=None, bjerrum=0.0, sigma=(0.0, 0.0), E=(0.0, 0.0, 0.0),
                 poisson="direct", lagged=True, sor_omega=None, sor_tol=1e-8,
                 sor_max=100000, sor_check=10, drag_pair=None, forcing="paper", lib_path=None):
        if nspecies > MAXS:
            raise ValueError("too many species")
        p = _Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.slit = 1 if geometry == "slit" else 0
        p.ns = nspecies
        p.omega_visc, p.omega_drag = omega_visc, omega_drag
        val = list(valence) if valence is not None else [0] * nspecies
        for i, v in enumerate(val):
            p.valence[i] = int(v)
        p.bjerrum = bjerrum
        p.sigma_lo, p.sigma_hi = sigma
        for d in range(3):
            p.E[d] = E[d]
        p.poisson = 0 if poisson == "direct" else 1
        p.lagged = 1 if lagged else 0
        nzf = nz - 2 if p.slit else nz
        p.sor_omega = sor_omega if sor_omega is not None else sor_omega_default(nx, ny, nzf)
        p.sor_tol = sor_tol
        p.sor_max = sor_max
        p.sor_check = sor_check
        p.forcing = {"paper": 0, "guo": 1, "literal": 2}[forcing]
        if drag_pair is not None:   # [ns][ns] drag frequencies omega^{ab}
            om = np.asarray(drag_pair, dtype=np.float64).reshape(nspecies, nspecies)
            p.pair_drag = 1
            for a in range(nspecies):
                for b in range(nspecies):
                    p.drag_pair[a * MAXS + b] = om[a, b]
        self.params = p
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.ns = nspecies
        self._L = lib(lib_path)
        self._h = self._L.ora_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the lattice parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.ora_destroy(h)
            self._h = None

    def set_state(self, s, n, u=None):
        n = _f64(n).reshape(self.shape)
        uu = None if u is None else _f64(u).reshape((3,) + self.shape)
        rc = self._L.ora_set_state(self._h, s, _dp(n), None if uu is None else _dp(uu))
        if rc:
            raise ValueError("bad species")

    def set_populations(self, s, f):
        f = _f64(f).reshape((19,) + self.shape)
        self._L.ora_set_f(self._h, s, _dp(f))

    def populations(self, s):
        f = np.zeros((19,) + self.shape)
        self._L.ora_get_f(self._h, s, _dp(f))
        return f

    def step(self, n=1):
        return self._L.ora_step(self._h, int(n))

    def moments(self, s):
        n = np.zeros(self.shape)
        j = np.zeros((3,) + self.shape)
        self._L.ora_moments(self._h, s, _dp(n), _dp(j))
        return n, j

    def mass_totals(self):
        out = np.zeros(self.ns)
        self._L.ora_mass_totals(self._h, _dp(out))
        return out

    def potential(self):
        out = np.zeros(self.shape)
        self._L.ora_get_psi(self._h, _dp(out))
        return out

    def charge(self):
        out = np.zeros(self.shape)
        self._L.ora_get_q(self._h, _dp(out))
        return out

    def poisson(self, q, psi0=None):
        """Solve the Poisson problem of this lattice for charge q; returns (psi, sweeps, resid, status)."""
        q = _f64(q).reshape(self.shape)
        psi = np.zeros(self.shape) if psi0 is None else _f64(psi0).reshape(self.shape).copy()
        sw = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = self._L.ora_poisson(self._h, _dp(q), _dp(psi), ctypes.byref(sw), ctypes.byref(rr))
        return psi, sw.value, rr.value, st

    def stats(self):
        step = ctypes.c_long(0)
        sw = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = self._L.ora_stats(self._h, ctypes.byref(step), ctypes.byref(sw), ctypes.byref(rr))
        return {"step": step.value, "sweeps": sw.value, "resid": rr.value, "status": st}
