"""Thin ctypes binding of liblbmix.so (the C ABI of include/lbmix.h).

Marshalling only: every step of the method runs in the library's gfx950 kernels.  There is
no CPU fallback; constructing a :class:`Lattice` raises if the library or a GPU is missing.
Host arrays are numpy float64 in [z][y][x] order (vector fields [3][z][y][x]); the device
read-back takes torch CUDA tensors (float64, contiguous).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbmix.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
PERIODIC, SLIT_Z, CHANNELS = 0, 1, 2
F64, F32, F32_SHIFTED, BF16_SHIFTED, F16_SHIFTED = 0, 1, 2, 3, 4
STORAGE = {"f64": F64, "f32": F32, "f32s": F32_SHIFTED, "bf16s": BF16_SHIFTED, "f16s": F16_SHIFTED}
GEOMETRY = {"periodic": PERIODIC, "slit": SLIT_Z, "channels": CHANNELS}
POISSON = {"sor": 0, "multigrid": 1, "direct": 2}
WARM_START = {"previous": 0, "extrapolated": 1, "learned": 2}
FORCING = {"paper": 0, "guo": 1}
ELEMENT_BYTES = {F64: 8, F32: 4, F32_SHIFTED: 4, BF16_SHIFTED: 2, F16_SHIFTED: 2}
Q = 19
MAX_SPECIES = 4
EXPORTS = (
    "lbmix_version", "lbmix_create", "lbmix_create_channels", "lbmix_set_channel", "lbmix_add_species",
    "lbmix_set_tau_visc", "lbmix_set_tau_drag", "lbmix_set_schmidt", "lbmix_set_drag_pairs", "lbmix_set_forcing",
    "lbmix_set_electrostatics",
    "lbmix_set_poisson", "lbmix_set_poisson_method", "lbmix_set_poisson_warm_start", "lbmix_set_rounding",
    "lbmix_set_storage_range", "lbmix_set_arithmetic", "lbmix_set_state", "lbmix_autotune", "lbmix_set_step_graph", "lbmix_step", "lbmix_get_moments", "lbmix_get_moments_device",
    "lbmix_get_populations", "lbmix_get_potential", "lbmix_get_mass_totals", "lbmix_get_step_mass",
    "lbmix_get_zprofiles", "lbmix_get_stats", "lbmix_sync", "lbmix_device_copy", "lbmix_save", "lbmix_load",
    "lbmix_last_error", "lbmix_destroy",
    "lbmix_net_create", "lbmix_net_num_params", "lbmix_net_get_params", "lbmix_net_set_params",
    "lbmix_net_get_gradient", "lbmix_net_forward", "lbmix_net_forward_noalloc", "lbmix_net_gradient", "lbmix_net_adam",
    "lbmix_net_output_scale", "lbmix_net_last_error", "lbmix_net_destroy", "lbmix_set_warm_start_net", "lbmix_train_warm_start",
)


class LbmixError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbmix error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_longlong), ("poisson_solves", ctypes.c_longlong),
                ("total_sweeps", ctypes.c_longlong), ("last_sweeps", ctypes.c_int),
                ("last_status", ctypes.c_int), ("last_residual", ctypes.c_double),
                ("fluid_nodes", ctypes.c_double), ("bytes_per_step", ctypes.c_double),
                ("block_x", ctypes.c_int), ("block_y", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load liblbmix.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1507_04891_amd.build; "
                           "there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "lbmix_version": ([], ctypes.c_int),
        "lbmix_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, vp], ctypes.c_int),
        "lbmix_create_channels": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
                                   vp], ctypes.c_int),
        "lbmix_set_channel": ([vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_int),
        "lbmix_add_species": ([vp, ctypes.c_double, ctypes.c_int, ip], ctypes.c_int),
        "lbmix_set_tau_visc": ([vp, ctypes.c_double], ctypes.c_int),
        "lbmix_set_tau_drag": ([vp, ctypes.c_double], ctypes.c_int),
        "lbmix_set_schmidt": ([vp, ctypes.c_double], ctypes.c_int),
        "lbmix_set_drag_pairs": ([vp, dp], ctypes.c_int),
        "lbmix_set_forcing": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_set_electrostatics": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp], ctypes.c_int),
        "lbmix_set_poisson": ([vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double], ctypes.c_int),
        "lbmix_set_poisson_method": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_set_poisson_warm_start": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_set_rounding": ([vp, ctypes.c_int, ctypes.c_ulonglong], ctypes.c_int),
        "lbmix_set_storage_range": ([vp, ctypes.c_int, ctypes.c_double], ctypes.c_int),
        "lbmix_set_arithmetic": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_set_state": ([vp, ctypes.c_int, dp, dp], ctypes.c_int),
        "lbmix_step": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_autotune": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_set_step_graph": ([vp, ctypes.c_int], ctypes.c_int),
        "lbmix_get_moments": ([vp, ctypes.c_int, dp, dp], ctypes.c_int),
        "lbmix_get_moments_device": ([vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "lbmix_get_populations": ([vp, ctypes.c_int, dp], ctypes.c_int),
        "lbmix_get_potential": ([vp, dp], ctypes.c_int),
        "lbmix_get_mass_totals": ([vp, dp], ctypes.c_int),
        "lbmix_get_step_mass": ([vp, dp], ctypes.c_int),
        "lbmix_get_zprofiles": ([vp, dp], ctypes.c_int),
        "lbmix_get_stats": ([vp, ctypes.POINTER(Stats)], ctypes.c_int),
        "lbmix_sync": ([vp], ctypes.c_int),
        "lbmix_device_copy": ([vp, vp, ctypes.c_ulonglong, vp], ctypes.c_int),
        "lbmix_save": ([vp, ctypes.c_char_p], ctypes.c_int),
        "lbmix_load": ([vp, ctypes.c_char_p], ctypes.c_int),
        "lbmix_last_error": ([vp], ctypes.c_char_p),
        "lbmix_destroy": ([vp], None),
        "lbmix_net_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong],
                             ctypes.c_int),
        "lbmix_net_num_params": ([vp], ctypes.c_int),
        "lbmix_net_get_params": ([vp, fp], ctypes.c_int),
        "lbmix_net_set_params": ([vp, fp], ctypes.c_int),
        "lbmix_net_get_gradient": ([vp, fp], ctypes.c_int),
        "lbmix_net_forward": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
        "lbmix_net_forward_noalloc": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp],
                                      ctypes.c_int),
        "lbmix_net_gradient": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, vp],
                               ctypes.c_int),
        "lbmix_net_adam": ([vp, ctypes.c_float, vp], ctypes.c_int),
        "lbmix_net_output_scale": ([vp, ctypes.c_double, dp], ctypes.c_int),
        "lbmix_net_last_error": ([vp], ctypes.c_char_p),
        "lbmix_net_destroy": ([vp], None),
        "lbmix_set_warm_start_net": ([vp, vp], ctypes.c_int),
        "lbmix_train_warm_start": ([vp, vp, ctypes.c_int, ctypes.c_float, dp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def device_copy(dst, src, stream=None):
    """Copy the torch CUDA tensor src into dst (same byte size, 16-byte aligned, a multiple of
    16 bytes) with the library's plain copy kernel (lbmix_device_copy), stream-ordered."""
    import torch
    L = load_library()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("dst and src must be CUDA tensors of the same byte size")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    rc = L.lbmix_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                             ctypes.c_void_p(s))
    if rc:
        raise LbmixError(rc, "lbmix_device_copy rejected the buffers")


class Lattice:
    """A lattice of the GPU library.

    geometry: "periodic", "slit" (solid planes z = 0 and z = nz-1) or "channels" (a stack of
    slit channels of fluid widths `widths`; nz is then sum(widths) + 2 len(widths)).
    storage: "f64", "f32", "f32s", "bf16s", "f16s" (see lbmix_storage).
    stream: a torch.cuda.Stream, a raw hipStream_t integer, or None for torch's current stream.
    """

    def __init__(self, nx, ny, nz=None, geometry="periodic", storage="f64", stream=None, widths=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbmix library has no CPU path")
        self._L = load_library()
        if stream is None:
            stream = torch.cuda.current_stream()
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.stream_handle = handle
        h = ctypes.c_void_p()
        if geometry == "channels":
            widths = [int(w) for w in widths]
            nz = sum(w + 2 for w in widths)
            wa = (ctypes.c_int * len(widths))(*widths)
            rc = self._L.lbmix_create_channels(ctypes.byref(h), nx, ny, len(widths), wa, STORAGE[storage],
                                               ctypes.c_void_p(handle))
        else:
            rc = self._L.lbmix_create(ctypes.byref(h), nx, ny, nz, GEOMETRY[geometry], STORAGE[storage],
                                      ctypes.c_void_p(handle))
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.geometry = geometry
        self.widths = widths
        self.storage = storage
        if rc:
            raise LbmixError(rc, "lbmix_create rejected the lattice")
        self._h = h
        self.nspecies = 0

    def _check(self, rc):
        if rc:
            msg = self._L.lbmix_last_error(self._h)
            raise LbmixError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._L.lbmix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up -------------------------------------------------------------------------
    def add_species(self, rho0, valence=0):
        i = ctypes.c_int(-1)
        self._check(self._L.lbmix_add_species(self._h, float(rho0), int(valence), ctypes.byref(i)))
        self.nspecies += 1
        return i.value

    def set_tau_visc(self, tau):
        self._check(self._L.lbmix_set_tau_visc(self._h, float(tau)))

    def set_tau_drag(self, tau):
        self._check(self._L.lbmix_set_tau_drag(self._h, float(tau)))

    def set_schmidt(self, sc):
        self._check(self._L.lbmix_set_schmidt(self._h, float(sc)))

    def set_drag_pairs(self, tau):
        """tau: [ns][ns] symmetric drag relaxation times per pair, or None for one drag frequency."""
        if tau is None:
            self._check(self._L.lbmix_set_drag_pairs(self._h, None))
            return
        t = _f64(tau, (self.nspecies, self.nspecies))
        self._check(self._L.lbmix_set_drag_pairs(self._h, _dp(t)))

    def set_forcing(self, scheme):
        """scheme: "paper" (the forcing of the Appendix, drag on mid-step velocities) or "guo"
        (the second-order Guo-type variant)."""
        if scheme not in FORCING:
            raise ValueError(f"forcing must be one of {sorted(FORCING)}")
        self._check(self._L.lbmix_set_forcing(self._h, FORCING[scheme]))

    def set_electrostatics(self, bjerrum, sigma_lo=0.0, sigma_hi=0.0, E=(0.0, 0.0, 0.0)):
        e = (ctypes.c_double * 3)(*[float(v) for v in E])
        self._check(self._L.lbmix_set_electrostatics(self._h, float(bjerrum), float(sigma_lo),
                                                     float(sigma_hi), e))

    def set_channel(self, c, tau_drag=0.0, sigma_lo=0.0, sigma_hi=0.0):
        self._check(self._L.lbmix_set_channel(self._h, int(c), float(tau_drag), float(sigma_lo), float(sigma_hi)))

    def set_poisson(self, rel_tol=1e-8, max_sweeps=200000, check_every=10, omega=-1.0, method="sor",
                    warm_start="previous"):
        self._check(self._L.lbmix_set_poisson(self._h, float(rel_tol), int(max_sweeps),
                                              int(check_every), float(omega)))
        self._check(self._L.lbmix_set_poisson_method(self._h, POISSON[method]))
        self._check(self._L.lbmix_set_poisson_warm_start(self._h, WARM_START[warm_start]))

    def set_rounding(self, stochastic=True, seed=0):
        self._check(self._L.lbmix_set_rounding(self._h, 1 if stochastic else 0, int(seed)))

    def set_arithmetic(self, wide=True):
        """wide: carry the density deviation beyond FP32 (default); False: FP32 collision
        arithmetic throughout (lbmix_set_arithmetic)."""
        self._check(self._L.lbmix_set_arithmetic(self._h, 1 if wide else 0))

    def set_storage_range(self, s, rel_range):
        self._check(self._L.lbmix_set_storage_range(self._h, int(s), float(rel_range)))

    def set_state(self, s, n, u=None):
        n = _f64(n, self.shape)
        uu = None if u is None else _f64(u, (3,) + self.shape)
        self._check(self._L.lbmix_set_state(self._h, int(s), _dp(n), _dp(uu)))

    # -- stepping -------------------------------------------------------------------------
    def step(self, n=1):
        return self._check(self._L.lbmix_step(self._h, int(n)))

    def set_step_graph(self, enable=True):
        """Replay steps as captured HIP graphs where no host decision is needed."""
        self._check(self._L.lbmix_set_step_graph(self._h, 1 if enable else 0))

    def autotune(self, reps=5):
        """Pick the fastest work-group shape of the step kernel; returns (block_x, block_y)."""
        self._check(self._L.lbmix_autotune(self._h, int(reps)))
        st = self.stats()
        return st["block_x"], st["block_y"]

    def set_warm_start_net(self, net):
        """Attach a Net for the learned warm start (kept alive by this lattice)."""
        self._ws_net = net
        self._check(self._L.lbmix_set_warm_start_net(self._h, net._h if net is not None else None))

    def train_warm_start(self, net, steps, lr=1e-3):
        """Advance `steps` steps with the direct solve, training `net` on exact corrections;
        returns the loss of every step."""
        losses = np.zeros(max(int(steps), 1))
        self._check(self._L.lbmix_train_warm_start(self._h, net._h, int(steps), float(lr), _dp(losses)))
        return losses[:int(steps)]

    def step_status(self, n=1):
        """Like step() but returns the status code instead of raising on ENOCONV."""
        rc = self._L.lbmix_step(self._h, int(n))
        if rc not in (OK, ENOCONV):
            self._check(rc)
        return rc

    def sync(self):
        self._check(self._L.lbmix_sync(self._h))

    # -- read-back ------------------------------------------------------------------------
    def moments(self, s):
        n = np.empty(self.shape)
        j = np.empty((3,) + self.shape)
        self._check(self._L.lbmix_get_moments(self._h, int(s), _dp(n), _dp(j)))
        return n, j

    def moments_device(self, s, n_dev, j_dev=None):
        """Write the moments of species s into torch float64 CUDA tensors (stream-ordered)."""
        for t in (n_dev, j_dev):
            if t is not None and (not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.float64"):
                raise ValueError("device outputs must be contiguous float64 CUDA tensors")
        if n_dev is not None and n_dev.numel() != self.nx * self.ny * self.nz:
            raise ValueError("n_dev has the wrong size")
        if j_dev is not None and j_dev.numel() != 3 * self.nx * self.ny * self.nz:
            raise ValueError("j_dev has the wrong size")
        self._check(self._L.lbmix_get_moments_device(
            self._h, int(s), ctypes.c_void_p(n_dev.data_ptr() if n_dev is not None else 0),
            ctypes.c_void_p(j_dev.data_ptr() if j_dev is not None else 0)))

    def populations(self, s):
        f = np.empty((19,) + self.shape)
        self._check(self._L.lbmix_get_populations(self._h, int(s), _dp(f)))
        return f

    def potential(self):
        p = np.empty(self.shape)
        self._check(self._L.lbmix_get_potential(self._h, _dp(p)))
        return p

    def mass_totals(self):
        out = np.empty(self.nspecies)
        self._check(self._L.lbmix_get_mass_totals(self._h, _dp(out)))
        return out

    def step_mass(self):
        """Per-species mass of the state the last step read, from the step's own FP64 partials."""
        out = np.empty(self.nspecies)
        self._check(self._L.lbmix_get_step_mass(self._h, _dp(out)))
        return out

    def metrics(self):
        """One record of the run's monitors: steps taken, the Poisson solver's work and last
        residual, and (after the first step) the per-species mass of the state the last step
        read, from the step's own partials (no extra pass over the populations)."""
        st = self.stats()
        rec = {"steps": st["steps"], "poisson_solves": st["poisson_solves"],
               "poisson_sweeps": st["total_sweeps"], "last_residual": st["last_residual"]}
        if st["steps"] > 0:
            rec["mass"] = [float(m) for m in self.step_mass()]
        return rec

    def zprofiles(self):
        out = np.empty((self.nspecies, 4, self.nz))
        self._check(self._L.lbmix_get_zprofiles(self._h, _dp(out)))
        return out

    def stats(self):
        st = Stats()
        self._check(self._L.lbmix_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def save(self, path):
        self._check(self._L.lbmix_save(self._h, str(path).encode()))

    def load(self, path):
        self._check(self._L.lbmix_load(self._h, str(path).encode()))


class MetricsLog:
    """Appends Lattice.metrics() records, one JSON object per line, with the wall time and
    species-site updates per second since the previous record."""

    def __init__(self, path):
        self._f = open(path, "a")
        self._last = None

    def write(self, lat, **extra):
        import json
        import time
        rec = lat.metrics()
        now = time.perf_counter()
        if self._last is not None and rec["steps"] > self._last[1]:
            sites = lat.nspecies * lat.stats()["fluid_nodes"]
            rec["glups"] = (rec["steps"] - self._last[1]) * sites / (now - self._last[0]) / 1e9
        self._last = (now, rec["steps"])
        rec.update(extra)
        self._f.write(json.dumps(rec) + "\n")
        self._f.flush()
        return rec

    def close(self):
        self._f.close()


class Net:
    """Network of the learned warm start (lbmix_net): 3 x 3 x 3 convolutions, in_channels ->
    hidden -> ... -> 1.  Device data are torch float32 CUDA tensors shaped [c][nz][ny][nx]."""

    def __init__(self, in_channels=2, hidden=16, layers=4, seed=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbmix library has no CPU path")
        self._L = load_library()
        h = ctypes.c_void_p()
        rc = self._L.lbmix_net_create(ctypes.byref(h), int(in_channels), int(hidden), int(layers), int(seed))
        if rc:
            raise LbmixError(rc, "lbmix_net_create failed")
        self._h = h
        self.in_channels = in_channels

    def _check(self, rc):
        if rc:
            msg = self._L.lbmix_net_last_error(self._h)
            raise LbmixError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._L.lbmix_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return self._L.lbmix_net_num_params(self._h)

    def params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(self._L.lbmix_net_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError("wrong parameter count")
        self._check(self._L.lbmix_net_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def output_scale(self, scale=0.0):
        """The warm start's output scale alpha (sets it when scale > 0)."""
        cur = ctypes.c_double(0.0)
        self._check(self._L.lbmix_net_output_scale(self._h, float(scale), ctypes.byref(cur)))
        return cur.value

    def gradient(self):
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(self._L.lbmix_net_get_gradient(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    @staticmethod
    def _dims(x):
        if x.dim() != 4 or not x.is_cuda or not x.is_contiguous() or str(x.dtype) != "torch.float32":
            raise ValueError("expected a contiguous float32 CUDA tensor [c][nz][ny][nx]")
        return x.shape[3], x.shape[2], x.shape[1]

    def forward(self, x, z_walls=False, stream=None):
        import torch
        nx, ny, nz = self._dims(x)
        y = torch.empty((1, nz, ny, nx), dtype=torch.float32, device=x.device)
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self._check(self._L.lbmix_net_forward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                              nx, ny, nz, 1 if z_walls else 0, ctypes.c_void_p(s)))
        return y

    def forward_noalloc(self, x, y, z_walls=False, stream=None):
        """y = net(x) into the caller's tensor y [1][nz][ny][nx], with the activation scratch in
        the library's static device array (lbmix_net_forward_noalloc: no allocation)."""
        import torch
        nx, ny, nz = self._dims(x)
        if tuple(self._dims(y)) != (nx, ny, nz) or y.shape[0] != 1:
            raise ValueError("y must be a float32 CUDA tensor [1][nz][ny][nx]")
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self._check(self._L.lbmix_net_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()),
                                                      ctypes.c_void_p(y.data_ptr()), nx, ny, nz,
                                                      1 if z_walls else 0, ctypes.c_void_p(s)))
        return y

    def loss_and_gradient(self, x, t, z_walls=False, stream=None):
        import torch
        nx, ny, nz = self._dims(x)
        self._dims(t)
        loss = ctypes.c_double(0.0)
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self._check(self._L.lbmix_net_gradient(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                               nx, ny, nz, 1 if z_walls else 0, ctypes.byref(loss), ctypes.c_void_p(s)))
        return loss.value

    def adam(self, lr, stream=None):
        import torch
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self._check(self._L.lbmix_net_adam(self._h, ctypes.c_float(lr), ctypes.c_void_p(s)))


def from_workload(w, storage="f64", stream=None, poisson=None, stochastic=None, seed=0, drag_pairs=None,
                  forcing="paper", schmidt=None, wide=True):
    """Build a Lattice from a workloads.Workload or workloads.ChannelStack description
    (parameters and initial fields).  stochastic: rounding of the stored populations (default:
    stochastic for the 16-bit forms, nearest for the FP32 ones); forcing: "paper" or "guo";
    schmidt: set the drag through lbmix_set_schmidt with this Schmidt number instead of the
    workload's tau_drag (single lattices only); wide: False for FP32 collision arithmetic
    throughout (lbmix_set_arithmetic)."""
    stack = w.geometry == "channels"
    lat = Lattice(w.nx, w.ny, w.nz, geometry=w.geometry, storage=storage, stream=stream,
                  widths=w.widths if stack else None)
    for s in range(w.nspecies):
        lat.add_species(w.rho0[s], w.valence[s])
    if storage in ("bf16s", "f16s"):
        lat.set_rounding(True if stochastic is None else stochastic, seed)
    elif storage in ("f32", "f32s") and stochastic:
        lat.set_rounding(True, seed)
    if not wide:
        lat.set_arithmetic(False)
    lat.set_tau_visc(w.tau_visc)
    if stack:
        for c in range(len(w.widths)):
            lat.set_channel(c, w.tau_drags[c], w.sigmas[c][0], w.sigmas[c][1])
        if w.bjerrum > 0 or any(w.E):
            lat.set_electrostatics(w.bjerrum, 0.0, 0.0, w.E)
    else:
        if schmidt is None:
            lat.set_tau_drag(w.tau_drag)
        else:
            lat.set_schmidt(schmidt)
        if w.bjerrum > 0 or any(w.E):
            lat.set_electrostatics(w.bjerrum, w.sigma[0], w.sigma[1], w.E)
    if drag_pairs is not None:
        lat.set_drag_pairs(drag_pairs)
    if forcing != "paper":
        lat.set_forcing(forcing)
    if poisson:
        lat.set_poisson(**poisson)
    for s in range(w.nspecies):
        lat.set_state(s, w.n[s], w.u[s])
    return lat
