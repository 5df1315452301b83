"""The C-ABI library loads without a GPU, exports every symbol include/lbmix.h declares,
and its host-side validation answers without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    import paper_1507_04891_amd as P
    return P.load_library()


def declared():
    src = open(os.path.join(ROOT, "include", "lbmix.h")).read()
    return sorted(set(re.findall(r"\b(lbmix_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported(L):
    import paper_1507_04891_amd as P
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(P.EXPORTS) == names


def test_version_and_create_validation(L):
    assert L.lbmix_version() == 10000
    h = ctypes.c_void_p()
    assert L.lbmix_create(ctypes.byref(h), 0, 4, 4, 0, 0, None) == -1
    assert L.lbmix_create(ctypes.byref(h), 4, 4, 2, 1, 0, None) == -1     # slit needs nz >= 3
    assert L.lbmix_create(ctypes.byref(h), 4, 4, 4, 2, 0, None) == -1     # geometry
    assert L.lbmix_create(ctypes.byref(h), 4, 4, 4, 0, 9, None) == -1     # storage
    assert L.lbmix_create(ctypes.byref(h), 2048, 2048, 1024, 0, 0, None) == -1   # > 2^31 nodes
    # the 19 populations of a plane for 4 species must stay under 4 GiB: 7.06 M nodes in F64,
    # 28.3 M in the 16-bit forms
    assert L.lbmix_create(ctypes.byref(h), 4096, 2048, 1, 0, 0, None) == -1      # 8.4 M nodes, F64
    assert L.lbmix_create(ctypes.byref(h), 4096, 2048, 1, 0, 4, None) == 0       # the same plane in FP16
    L.lbmix_destroy(h)
    assert L.lbmix_create(ctypes.byref(h), 4096, 8192, 1, 0, 4, None) == -1      # 33.6 M nodes, FP16
    assert L.lbmix_create(ctypes.byref(h), 2048, 2048, 1, 0, 0, None) == 0       # 4.2 M nodes, F64
    L.lbmix_destroy(h)
    assert L.lbmix_create(ctypes.byref(h), 4, 4, 4, 0, 1, None) == 0
    L.lbmix_destroy(h)


def test_parameter_validation_without_device(L):
    h = ctypes.c_void_p()
    assert L.lbmix_create(ctypes.byref(h), 8, 8, 10, 1, 2, None) == 0
    i = ctypes.c_int(-1)
    assert L.lbmix_add_species(h, 1.0, 0, ctypes.byref(i)) == 0 and i.value == 0
    assert L.lbmix_add_species(h, -1.0, 0, ctypes.byref(i)) == -1
    for _ in range(3):
        L.lbmix_add_species(h, 0.01, 1, ctypes.byref(i))
    assert L.lbmix_add_species(h, 0.01, 1, ctypes.byref(i)) == -1       # max 4 species
    assert L.lbmix_set_tau_visc(h, 0.5) == -1
    assert L.lbmix_set_tau_visc(h, 0.8) == 0
    assert L.lbmix_set_tau_drag(h, 0.4) == -1
    assert L.lbmix_set_schmidt(h, 0.0) == -1
    assert L.lbmix_set_schmidt(h, 100.0) == 0
    E = (ctypes.c_double * 3)(1e-4, 0, 0)
    assert L.lbmix_set_electrostatics(h, -1.0, 0, 0, E) == -1
    assert L.lbmix_set_electrostatics(h, 0.6, -1e-4, -1e-4, E) == 0
    assert L.lbmix_set_poisson(h, -1.0, 10, 1, 1.5) == -1
    assert L.lbmix_set_poisson(h, 1e-8, 0, 1, 1.5) == -1
    assert L.lbmix_set_poisson(h, 1e-8, 10, 1, 2.0) == -1
    assert L.lbmix_set_poisson(h, 1e-8, 10, 1, -1.0) == 0
    # no state yet
    assert L.lbmix_step(h, 1) == -4
    assert L.lbmix_autotune(h, 3) == -4
    assert b"no state" in L.lbmix_last_error(h)
    # the first device call reports the missing GPU as EDEVICE (with a GPU present it allocates)
    st = L.lbmix_set_state(h, 0, (ctypes.c_double * (8 * 8 * 10))(), None)
    assert st in (0, -3)
    L.lbmix_destroy(h)
    L.lbmix_destroy(None)


def test_channel_stack_validation_without_device(L):
    h = ctypes.c_void_p()
    W = ctypes.c_int * 3
    assert L.lbmix_create_channels(ctypes.byref(h), 8, 8, 0, W(4, 5, 6), 2, None) == -1
    assert L.lbmix_create_channels(ctypes.byref(h), 8, 8, 3, None, 2, None) == -1
    assert L.lbmix_create_channels(ctypes.byref(h), 8, 8, 3, W(4, 0, 6), 2, None) == -1
    assert L.lbmix_create_channels(ctypes.byref(h), 8, 8, 3, W(4, 5, 6), 9, None) == -1
    assert L.lbmix_create_channels(ctypes.byref(h), 1024, 1024, 3, W(700, 700, 700), 2, None) == -1   # > 2^31
    assert L.lbmix_create_channels(ctypes.byref(h), 8, 8, 3, W(4, 5, 6), 2, None) == 0
    assert L.lbmix_set_channel(h, 3, 0.6, 0, 0) == -1              # index
    assert L.lbmix_set_channel(h, 0, 0.5, 0, 0) == -1              # tau_drag in (0, 1/2]
    assert L.lbmix_set_channel(h, 0, 0.6, -1e-4, -2e-4) == 0
    assert L.lbmix_set_channel(h, 1, 0.0, 0, 0) == 0               # the context's drag
    assert L.lbmix_set_poisson_method(h, 1) == 0                   # multigrid: z-line relaxation per channel
    assert L.lbmix_set_poisson_method(h, 2) == 0
    L.lbmix_destroy(h)
    assert L.lbmix_create(ctypes.byref(h), 8, 8, 10, 1, 2, None) == 0
    assert L.lbmix_set_channel(h, 0, 0.6, 0, 0) == -1              # not a stack
    L.lbmix_destroy(h)


def test_network_validation_without_device(L):
    h = ctypes.c_void_p()
    for args in [(0, 16, 4), (17, 16, 4), (2, 0, 4), (2, 17, 4), (2, 16, 0), (2, 16, 17)]:
        assert L.lbmix_net_create(ctypes.byref(h), *args, 0) == -1, args
    assert L.lbmix_net_num_params(None) == -1
    assert L.lbmix_net_adam(None, ctypes.c_float(1e-3), None) == -1
    assert L.lbmix_net_output_scale(None, ctypes.c_double(1.0), None) == -1
    assert L.lbmix_set_warm_start_net(None, None) == -1
    # a lattice without a network rejects the learned warm start
    assert L.lbmix_create(ctypes.byref(h), 8, 8, 10, 1, 2, None) == 0
    assert L.lbmix_set_poisson_warm_start(h, 2) == -1
    assert L.lbmix_set_poisson_warm_start(h, 3) == -1
    assert L.lbmix_set_step_graph(h, 1) == 0
    L.lbmix_destroy(h)
    L.lbmix_net_destroy(None)


def test_forcing_validation_without_device(L):
    h = ctypes.c_void_p()
    assert L.lbmix_set_forcing(None, 1) == -1
    assert L.lbmix_create(ctypes.byref(h), 8, 8, 8, 0, 0, None) == 0
    assert L.lbmix_set_forcing(h, 2) == -1
    assert b"forcing" in L.lbmix_last_error(h)
    assert L.lbmix_set_forcing(h, -1) == -1
    assert L.lbmix_set_forcing(h, 1) == 0
    assert L.lbmix_set_forcing(h, 0) == 0
    L.lbmix_destroy(h)
