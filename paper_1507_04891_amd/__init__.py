"""Multicomponent lattice Boltzmann at variable Schmidt number, native to MI355X (gfx950).

The library ``liblbmix.so`` (C ABI in ``include/lbmix.h``, kernels in ``csrc/``) implements
the fused per-species stream-and-collide step of Monteferrante, Melchionna and Marini
Bettolo Marconi (arXiv:1507.04891): modified BGK with separate momentum (omega_visc) and
mass-diffusion (omega_drag) time scales, interspecies drag, and the electrostatic force of
a lattice Poisson solve with charged walls.  :mod:`.lbmix` is its ctypes binding.
"""
from .lbmix import (  # noqa: F401
    Lattice, Net, MetricsLog, LbmixError, load_library, from_workload, device_copy, STORAGE, GEOMETRY, ELEMENT_BYTES, EXPORTS,
    OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOCONV, ENONFINITE,
)

__all__ = ["Lattice", "Net", "MetricsLog", "LbmixError", "load_library", "from_workload", "device_copy"]
