"""The Guo-type forcing variant (every species moves with v = u + F/2, implicit drag solved in
closed form per node, forcing term scaled by 1 - omega_visc/2) on the GPU against the
oracle's variant, which solves the implicit drag as a dense linear system per node.

Bars as for the default forcing: FP64 1e-12 of the deviation from rest (1e-11 of max|j| for
momenta, the closed form and the elimination differ in rounding order only), FP32 1e-5 of
max|n| and 1e-3 of the deviation from rest.
"""
import os
import tempfile

import numpy as np
import pytest

import workloads as WL
from parity_util import oracle_for, rel_max, rel_to_deviation
from test_gpu_parity import P, check_potential, compare_fp64, pair_taus  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

CASES = ["binary_modes", "periodic_ternary_field", "slit_charged", "periodic_four_charged"]


def case(name):
    if name == "binary_modes":
        return WL.binary_multimode(n=16, amp=1e-2, nmodes=3, shear=1e-2, sc=1.0, tau_visc=1.2, seed=4), None
    if name == "periodic_ternary_field":
        return WL.random_state(20, 6, 8, 3, seed=21, rho0=[0.6, 0.25, 0.15], valence=[0, 1, -1], bjerrum=0.0,
                               E=(2e-3, -1e-3, 5e-4), dn=0.05, du=0.02, tau_drag=0.9), None
    if name == "slit_charged":
        w = WL.charged_slit(nx=8, ny=6, nz=18, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        return w, dict(method="direct")
    w = WL.random_state(10, 4, 6, 4, seed=22, rho0=[0.5, 0.2, 0.2, 0.1], valence=[0, 1, -1, 0], bjerrum=0.4,
                        E=(1e-3, 0, 0), dn=0.0, du=0.02, tau_drag=1.7)
    return w, dict(method="direct")


@pytest.mark.parametrize("name", CASES)
def test_guo_fp64_matches_oracle(P, oracle_mod, name):
    w, poisson = case(name)
    lat = P.from_workload(w, storage="f64", poisson=poisson, forcing="guo")
    o = oracle_for(oracle_mod, w, forcing="guo")
    lat.step(30)
    o.step(30)
    compare_fp64(lat, o, w)
    if w.bjerrum > 0:
        check_potential(lat.potential(), o.potential(), w)


@pytest.mark.parametrize("storage", ["f32", "f32s", "f32s:sr"])
def test_guo_fp32_matches_oracle(P, oracle_mod, storage):
    w, poisson = case("slit_charged")
    sr = storage.endswith(":sr")
    storage = storage.split(":")[0]
    lat = P.from_workload(w, storage=storage, poisson=poisson, forcing="guo", stochastic=True if sr else None, seed=2)
    o = oracle_for(oracle_mod, w, forcing="guo")
    lat.step(20)
    o.step(20)
    m = np.ones((w.nz, w.ny, w.nx), bool)
    m[0] = m[-1] = False
    for s in range(w.nspecies):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no, m) <= 1e-5, s
        if storage == "f32s":
            assert rel_to_deviation(ng, no, w.rho0[s], m) <= 1e-3, s
    assert rel_max(lat.potential(), o.potential(), m) <= 1e-5


def test_guo_differs_from_paper_forcing(P):
    """The variant changes the step (the drag relaxes differently)."""
    w, _ = case("binary_modes")
    a = P.from_workload(w, storage="f64", forcing="guo")
    b = P.from_workload(w, storage="f64")
    a.step(5)
    b.step(5)
    assert not np.array_equal(a.populations(0), b.populations(0))


def test_guo_schmidt_mapping(P):
    """Sc under the variant: tau_drag = (tau_visc - 1/2) / Sc, since D = v_T^2 tau_drag."""
    w, _ = case("binary_modes")
    a = P.from_workload(w, storage="f64", forcing="guo")
    a.set_schmidt(0.5)
    b = P.from_workload(w, storage="f64", forcing="guo")
    b.set_tau_drag((w.tau_visc - 0.5) / 0.5)
    a.step(4)
    b.step(4)
    np.testing.assert_array_equal(a.populations(1), b.populations(1))
    c = P.from_workload(w, storage="f64", forcing="guo")
    c.set_schmidt(2.0)                       # tau_drag = 0.35 < 1/2
    with pytest.raises(P.LbmixError) as e:
        c.step(1)
    assert "Guo" in str(e.value)


def test_guo_errors(P):
    w = WL.random_state(8, 4, 4, 3, seed=1, rho0=[0.6, 0.25, 0.15], valence=[0, 0, 0])
    with pytest.raises(ValueError):
        P.from_workload(w, storage="f64", forcing="implicit")
    lat = P.from_workload(w, storage="f64", forcing="guo", drag_pairs=pair_taus(3, 1))
    with pytest.raises(P.LbmixError) as e:
        lat.step(1)
    assert "pair" in str(e.value)
    ok = P.from_workload(w, storage="f64", forcing="guo")
    ok.step(1)
    with pytest.raises(P.LbmixError):
        ok.set_forcing("paper")


def test_guo_checkpoint_and_graph(P):
    """The scheme travels with a checkpoint; captured steps replay it bitwise."""
    w, poisson = case("slit_charged")
    a = P.from_workload(w, storage="f32s", poisson=poisson, forcing="guo")
    g = P.from_workload(w, storage="f32s", poisson=poisson, forcing="guo")
    g.set_step_graph(True)
    a.step(10)
    g.step(10)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(15)
        b = P.Lattice(w.nx, w.ny, w.nz, geometry="slit", storage="f32s")
        for s in range(w.nspecies):
            b.add_species(w.rho0[s], w.valence[s])
        b.load(path)
        b.step(15)
    g.step(15)
    for s in range(w.nspecies):
        np.testing.assert_array_equal(a.populations(s), b.populations(s))
        np.testing.assert_array_equal(a.populations(s), g.populations(s))


def test_guo_channel_stack_matches_each_channel(P, oracle_mod):
    """A stack of four slit channels (own drag and wall charge, lateral charge waves) under the
    Guo-type variant: every channel follows its own oracle slit at the FP64 bar."""
    from test_gpu_parity import SMALL_STACK, ChannelView, check_potential as chk
    st = WL.channel_stack(**SMALL_STACK)
    lat = P.from_workload(st, storage="f64", poisson=dict(method="direct"), forcing="guo")
    lat.step(25)
    for c in range(len(st.widths)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="direct", forcing="guo")
        o.step(25)
        view = ChannelView(lat, st.planes(c), 3)
        compare_fp64(view, o, wc)
        chk(view.potential(), o.potential(), wc)
