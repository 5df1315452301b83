"""GPU <-> oracle parity through the C ABI (liblbmix.so on gfx950).

Tolerances (derived from the arithmetic):
* FP64 storage: two independent FP64 implementations of the step (the C oracle and the NumPy
  brute force) differ after 500 steps of the 32^3 binary run by 3e-13 of the density
  perturbation and by 3e-16 absolute (1.2e-12 of max|j|) in the momentum, the rounding floor
  of sums of populations of size ~0.1.  The bar is 1e-12 relative to the deviation from rest
  for densities and populations, and 1e-11 of max|j| for momenta.
* FP32 storage: 1e-5 relative, populations and densities against max |f| and max |n|
  (unit roundoff 6e-8 per operation, ~10 operations per step, errors damped by the
  collision).  Momenta are checked against the population scale for plain FP32 (they are
  differences of populations that FP32 resolves to ~1e-8 absolute) and against max|j| for
  the shifted form, which stores deviations from rest.
"""
import math
import os
import tempfile

import numpy as np
import pytest

import workloads as WL
from parity_util import W as WQ, fluid, oracle_for, patch_workload, rel_max, rel_to_deviation, within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    return P


def gpu_for(P, w, storage="f64", poisson=None):
    return P.from_workload(w, storage=storage, poisson=poisson)


def compare_fp64(lat, o, w, pop_tol=1e-12, n_tol=1e-12, j_tol=1e-11, floor=1e-14):
    """FP64 bar: |dn| <= 1e-12 max|n - rho0| + F, |dj| <= 1e-11 max|j| + F and
    |df| <= 1e-12 max|f - w rho0| + F, with the rounding floor F = 1e-14 max|n| (about 45
    unit roundoffs of a sum of populations) for fields that barely leave rest."""
    m = fluid(w)
    for s in range(w.nspecies):
        ng, jg = lat.moments(s)
        no, jo = o.moments(s)
        F = floor * np.abs(no[m]).max()
        ok, err, bnd = within(ng, no, n_tol, np.abs(no - w.rho0[s])[m].max(), F, m)
        assert ok, ("n", s, err, bnd)
        ok, err, bnd = within(jg, jo, j_tol, np.abs(jo[:, m]).max(), F, m)
        assert ok, ("j", s, err, bnd)
        fg, fo = lat.populations(s), o.populations(s)
        rest = (WQ * w.rho0[s])[:, None, None, None]
        ok, err, bnd = within(fg, fo, pop_tol, np.abs(fo - rest)[:, m].max(), F, m)
        assert ok, ("f", s, err, bnd)
        assert np.all(ng[~m] == 0) and np.all(jg[:, ~m] == 0)


def test_config1_binary_32cubed_fp64_500_steps(P, oracle_mod):
    """Neutral binary 32^3 periodic FP64, 0.01 sin(2 pi x / 32) antiphase, tau 1, Sc 10."""
    w = WL.binary_sine(32, 32, 32, amp=0.01, tau_visc=1.0, sc=10.0)
    lat = gpu_for(P, w, "f64")
    o = oracle_for(oracle_mod, w)
    lat.step(500)
    o.step(500)
    compare_fp64(lat, o, w)
    st = lat.stats()
    assert st["steps"] == 500


CASES = [
    # nx, ny, nz, geometry, ns, charged, E
    (70, 6, 10, "periodic", 2, False, (0, 0, 0)),
    (130, 3, 5, "periodic", 3, False, (1e-3, 0, -2e-4)),
    (1, 1, 9, "periodic", 2, False, (0, 0, 0)),
    (300, 2, 3, "slit", 1, False, (2e-4, 0, 0)),
    (64, 4, 12, "slit", 3, True, (1e-3, 0, 0)),
    (66, 2, 6, "slit", 4, True, (0, 5e-4, 0)),
    (8, 8, 8, "periodic", 3, True, (0, 0, 1e-3)),
    (2, 2, 3, "slit", 3, True, (1e-4, 0, 0)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-{c[3]}-s{c[4]}{'-q' if c[5] else ''}")
def test_random_state_fp64(P, oracle_mod, case):
    nx, ny, nz, geo, ns, charged, E = case
    val = [0, 1, -1, 2][:ns] if charged else [0] * ns
    rho0 = [1.0, 0.02, 0.02, 0.01][:ns] if charged else [1.0 / ns] * ns
    if charged and ns == 4:
        rho0 = [1.0, 0.02, 0.04, 0.01]     # z = (0, 1, -1, 2): 0.02 - 0.04 + 0.02 = 0
    w = WL.random_state(nx, ny, nz, ns, geometry=geo, seed=nx * 7 + nz, rho0=rho0, valence=val,
                        bjerrum=0.5 if charged else 0.0, sigma=(0.0, 0.0), E=E, dn=0.0 if charged else 0.05,
                        du=0.02, tau_visc=0.8, tau_drag=0.6)
    sweeps = 30
    lat = gpu_for(P, w, "f64", poisson=dict(rel_tol=0.0, max_sweeps=sweeps))
    o = oracle_for(oracle_mod, w, poisson="sor", sor_tol=0.0, sor_max=sweeps)
    lat.step(25)
    o.step(25)
    compare_fp64(lat, o, w)
    if charged:
        check_potential(lat.potential(), o.potential(), w)


def check_potential(pg, po, w, rel=1e-11):
    """FP64 bar for the potential: 1e-11 of max|psi| plus the rounding of the charge density
    (a difference of ion densities, eps * sum |z| rho0) amplified by the inverse of the
    7-point operator, whose smallest eigenvalue is about (pi / L)^2."""
    m = fluid(w)
    L = max(w.nx, w.ny, w.nz - 2 if w.geometry == "slit" else w.nz)
    K = 4 * math.pi * w.bjerrum
    qfloor = 2.2e-16 * sum(abs(z) * r for z, r in zip(w.valence, w.rho0))
    ok, err, bnd = within(pg, po, rel, np.abs(po[m]).max(), 4 * K * qfloor * (L / math.pi) ** 2, m)
    assert ok, ("psi", err, bnd)


def test_charged_slit_converged_poisson_fp64(P, oracle_mod):
    """Residual-controlled SOR: both sides take the same number of sweeps."""
    w = WL.charged_slit(nx=8, ny=6, nz=18, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
    lat = gpu_for(P, w, "f64", poisson=dict(rel_tol=1e-10, max_sweeps=20000, check_every=5))
    o = oracle_for(oracle_mod, w, poisson="sor", sor_tol=1e-10, sor_max=20000, sor_check=5)
    lat.step(40)
    o.step(40)
    compare_fp64(lat, o, w)
    st, so = lat.stats(), o.stats()
    assert st["last_sweeps"] == so["sweeps"]
    assert st["last_residual"] <= 1e-10
    check_potential(lat.potential(), o.potential(), w)
    # against the direct solve, the iterative potential is good to the SOR tolerance
    od = oracle_for(oracle_mod, w, poisson="direct")
    od.step(40)
    assert rel_max(lat.potential(), od.potential(), fluid(w)) <= 1e-6


@pytest.mark.parametrize("storage", ["f32", "f32s"])
def test_fp32_binary(P, oracle_mod, storage):
    w = WL.binary_multimode(n=48, amp=1e-3, shear=1e-3, sc=100.0, seed=2)
    lat = gpu_for(P, w, storage)
    o = oracle_for(oracle_mod, w)
    lat.step(60)
    o.step(60)
    for s in range(2):
        ng, jg = lat.moments(s)
        no, jo = o.moments(s)
        assert rel_max(ng, no) <= 1e-5
        fg, fo = lat.populations(s), o.populations(s)
        assert rel_max(fg, fo) <= 1e-5
        if storage == "f32s":
            assert rel_max(jg, jo) <= 1e-5
            assert rel_to_deviation(ng, no, 0.5) <= 1e-4
        else:
            assert np.abs(jg - jo).max() <= 1e-5 * np.abs(no).max()


@pytest.mark.parametrize("storage", ["f32", "f32s"])
def test_fp32_charged_slit(P, oracle_mod, storage):
    w = WL.charged_slit(nx=16, ny=8, nz=34, n_ion=1e-3, debye_length=4.0, sigma=-1e-3, Ex=1e-4, sc=100.0)
    lat = gpu_for(P, w, storage, poisson=dict(rel_tol=0.0, max_sweeps=40))
    o = oracle_for(oracle_mod, w, poisson="sor", sor_tol=0.0, sor_max=40)
    lat.step(50)
    o.step(50)
    m = fluid(w)
    for s in range(3):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no, m) <= 1e-5
        assert rel_max(lat.populations(s), o.populations(s), m) <= 1e-5
    assert rel_max(lat.potential(), o.potential(), m) <= 1e-5


def test_determinism_and_mass_conservation(P):
    w = WL.random_state(40, 12, 10, 3, geometry="slit", seed=4, rho0=[1.0, 0.01, 0.01],
                        valence=[0, 1, -1], bjerrum=0.7, sigma=(0.0, 0.0), E=(1e-4, 0, 0), dn=0.0)
    runs = []
    for _ in range(2):
        lat = gpu_for(P, w, "f64", poisson=dict(rel_tol=1e-9, max_sweeps=5000))
        m0 = lat.mass_totals()
        lat.step(300)
        runs.append((lat.populations(1), lat.potential(), lat.mass_totals(), m0))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    np.testing.assert_array_equal(runs[0][2], runs[1][2])
    np.testing.assert_allclose(runs[0][2], runs[0][3], rtol=1e-13)


def test_checkpoint_restart_is_bitwise(P):
    w = WL.charged_slit(nx=8, ny=4, nz=14, debye_length=3.0, sigma=-2e-4, Ex=1e-4, sc=10.0)
    pp = dict(rel_tol=1e-9, max_sweeps=5000)
    a = gpu_for(P, w, "f32s", poisson=pp)
    a.step(20)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(30)
        b = P.Lattice(w.nx, w.ny, w.nz, geometry="slit", storage="f32s")
        for s in range(3):
            b.add_species(w.rho0[s], w.valence[s])
        b.load(path)
        b.step(30)
    for s in range(3):
        np.testing.assert_array_equal(a.populations(s), b.populations(s))
    np.testing.assert_array_equal(a.potential(), b.potential())
    assert b.stats()["steps"] == 50


def test_error_paths(P):
    w = WL.binary_sine(8, 4, 4, amp=0.01)
    # non-finite state latches ENONFINITE until set_state
    lat = gpu_for(P, w, "f64")
    bad = w.n[0].copy()
    bad[1, 2, 3] = np.nan
    lat.set_state(0, bad)
    lat.step(2)
    with pytest.raises(P.LbmixError) as e:
        lat.mass_totals()
    assert e.value.code == P.ENONFINITE
    with pytest.raises(P.LbmixError) as e:
        lat.step(1)
    assert e.value.code == P.ENONFINITE
    lat.set_state(0, w.n[0])
    lat.set_state(1, w.n[1])
    lat.step(1)
    assert np.isfinite(lat.mass_totals()).all()
    # sweep cap below need -> ENOCONV, steps still taken
    ws = WL.charged_slit(nx=4, ny=4, nz=18, debye_length=3.0, sigma=-3e-4, Ex=0.0, sc=1.0)
    lat = gpu_for(P, ws, "f64", poisson=dict(rel_tol=1e-12, max_sweeps=3, check_every=1))
    assert lat.step_status(2) == P.ENOCONV
    assert lat.stats()["steps"] == 2
    # non-neutral charged system -> EINVAL at the first step
    wn = WL.charged_slit(nx=4, ny=4, nz=10, sigma=-1e-3)
    lat = P.from_workload(wn, storage="f64")
    lat.set_electrostatics(wn.bjerrum, -2e-3, -2e-3, wn.E)
    with pytest.raises(P.LbmixError) as e:
        lat.step(1)
    assert e.value.code == P.EINVAL
    # odd periodic extent in a charged run -> EINVAL
    wo = WL.random_state(5, 4, 4, 3, seed=1, rho0=[1.0, 0.01, 0.01], valence=[0, 1, -1], bjerrum=0.5, dn=0.0)
    lat = P.from_workload(wo, storage="f64")
    with pytest.raises(P.LbmixError) as e:
        lat.step(1)
    assert e.value.code == P.EINVAL


def test_zprofiles_and_observables(P, oracle_mod):
    w = WL.charged_slit(nx=6, ny=4, nz=20, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
    lat = gpu_for(P, w, "f64", poisson=dict(rel_tol=0.0, max_sweeps=20))
    o = oracle_for(oracle_mod, w, poisson="sor", sor_tol=0.0, sor_max=20)
    lat.step(30)
    o.step(30)
    prof = lat.zprofiles()
    for s in range(3):
        n, j = o.moments(s)
        np.testing.assert_allclose(prof[s, 0], n.mean(axis=(1, 2)), rtol=1e-12, atol=1e-300)
        for d in range(3):
            np.testing.assert_allclose(prof[s, 1 + d], j[d].mean(axis=(1, 2)), rtol=0,
                                       atol=1e-11 * np.abs(j[d]).max() + 1e-14 * np.abs(n).max())


def test_moments_device_matches_host(P):
    import torch
    w = WL.binary_multimode(n=16, sc=10.0, seed=3)
    lat = gpu_for(P, w, "f32")
    lat.step(3)
    n_dev = torch.empty(w.nx * w.ny * w.nz, dtype=torch.float64, device="cuda")
    j_dev = torch.empty(3 * w.nx * w.ny * w.nz, dtype=torch.float64, device="cuda")
    lat.moments_device(1, n_dev, j_dev)
    torch.cuda.synchronize()
    n, j = lat.moments(1)
    np.testing.assert_array_equal(n_dev.cpu().numpy().reshape(n.shape), n)
    np.testing.assert_array_equal(j_dev.cpu().numpy().reshape(j.shape), j)


# --------------------------------------------------------------------------------------
# Full sizes, in the launch configuration the benchmark times.

@pytest.mark.parametrize("amp,k", [(1e-3, 6), (5e-2, 8)])
def test_full_size_binary_256cubed_fp32_sampled(P, oracle_mod, amp, k):
    """256^3 periodic binary FP32, the benchmark's kernel and launch shape (Sc = 100): after k
    steps the GPU populations at sampled nodes equal the oracle's on light-cone patches.  With
    the benchmark's amplitude (1e-3) a few steps move the populations by little more than the
    FP32 bar, so a second case with 50 times the amplitude also checks the change itself."""
    w = WL.binary_multimode(n=256, amp=amp, shear=amp, sc=100.0, seed=2)
    lat = gpu_for(P, w, "f32")
    f0 = [lat.populations(s) if amp > 1e-3 else None for s in range(2)]
    lat.step(k)
    rng = np.random.default_rng(0)
    centres = [(0, 0, 0), (255, 255, 255), (128, 0, 255)] + [tuple(rng.integers(0, 256, 3)) for _ in range(5)]
    fg = [lat.populations(s) for s in range(2)]
    for c in centres:
        pw, h = patch_workload(w, c, k)
        o = oracle_for(oracle_mod, pw)
        o.step(k)
        for s in range(2):
            got = fg[s][:, c[0], c[1], c[2]]
            want = o.populations(s)[:, h, h, h]
            assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max(), (c, s)
            if f0[s] is not None:
                start = f0[s][:, c[0], c[1], c[2]]
                change = np.abs(want - start).max()
                assert change > 20 * 1e-5 * np.abs(want).max(), (c, s, change)
                assert np.abs((got - start) - (want - start)).max() <= 2e-2 * change, (c, s)
    m = lat.mass_totals()
    np.testing.assert_allclose(m, [0.5 * 256 ** 3] * 2, rtol=1e-6)


def test_full_size_charged_slit_64x64x130_fp32(P, oracle_mod):
    """The charged-slit configuration at full size (64 x 64 x 130, FP32, Sc 100, lambda_D 8):
    a few steps against the oracle run on the whole lattice with the same SOR sweeps."""
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    sweeps = 12
    lat = gpu_for(P, w, "f32s", poisson=dict(rel_tol=0.0, max_sweeps=sweeps))
    o = oracle_for(oracle_mod, w, poisson="sor", sor_tol=0.0, sor_max=sweeps)
    lat.step(3)
    o.step(3)
    m = fluid(w)
    for s in range(3):
        ng, jg = lat.moments(s)
        no, jo = o.moments(s)
        assert rel_max(ng, no, m) <= 1e-5
        assert rel_to_deviation(ng, no, w.rho0[s], m) <= 1e-3
    assert rel_max(lat.potential(), o.potential(), m) <= 1e-5


@pytest.mark.parametrize("geometry,dims", [("slit", (16, 8, 34)), ("periodic", (16, 8, 12)), ("slit", (6, 4, 20))])
def test_multigrid_poisson_matches_direct_solve(P, oracle_mod, geometry, dims):
    """Multigrid V-cycles to a tight residual reproduce the oracle's exact (spectral) solve;
    the populations then follow the oracle to the precision the residual allows."""
    nx, ny, nz = dims
    if geometry == "slit":
        w = WL.charged_slit(nx=nx, ny=ny, nz=nz, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
    else:
        w = WL.random_state(nx, ny, nz, 3, seed=13, rho0=[1.0, 0.02, 0.02], valence=[0, 1, -1],
                            bjerrum=0.5, E=(1e-3, 0, 0), dn=0.0, du=0.02)
    lat = gpu_for(P, w, "f64", poisson=dict(rel_tol=1e-13, max_sweeps=200, method="multigrid"))
    o = oracle_for(oracle_mod, w, poisson="direct")
    lat.step(30)
    o.step(30)
    st = lat.stats()
    assert st["last_residual"] <= 1e-13 and st["last_sweeps"] <= 20
    assert rel_max(lat.potential(), o.potential(), fluid(w)) <= 1e-9
    compare_fp64(lat, o, w, pop_tol=1e-9, n_tol=1e-9, j_tol=1e-8)


def test_multigrid_cycles_on_the_charged_slit(P):
    """Full-size charged slit (64 x 64 x 130): from a cold start the solve reaches 1e-8 in a
    few V-cycles; later steps need a few, and fewer with the extrapolated warm start."""
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    per_step = {}
    for warm in ("previous", "extrapolated"):
        lat = gpu_for(P, w, "f32s", poisson=dict(rel_tol=1e-8, max_sweeps=100, method="multigrid",
                                                   warm_start=warm))
        lat.step(1)
        first = lat.stats()
        assert first["poisson_solves"] == 2 and first["last_residual"] <= 1e-8
        assert first["total_sweeps"] <= 30
        lat.step(40)
        st = lat.stats()
        assert st["last_residual"] <= 1e-8
        per_step[warm] = (st["total_sweeps"] - first["total_sweeps"]) / 40
    assert per_step["previous"] <= 6
    assert per_step["extrapolated"] <= per_step["previous"]


DIRECT_CASES = [("slit", (16, 8, 34)), ("periodic", (16, 8, 12)), ("slit", (7, 5, 13)), ("periodic", (9, 6, 7)),
                ("slit", (1, 1, 12)), ("periodic", (70, 3, 5)), ("slit", (130, 66, 8)),
                # more planes than transform work-groups (256 of 64 x 64, 1024 of 32 x 32); LDS
                # eliminations of 8 modes (segments of 257-1024 planes) and 4 modes (1025-2048),
                # and a segment longer than the LDS eliminations take
                ("slit", (40, 36, 300)), ("periodic", (12, 10, 1100)), ("slit", (6, 4, 1100)),
                ("slit", (2, 2, 2100)),
                # planes between 32 and 64 wide, fewer than 256: split in halves
                ("slit", (40, 36, 34)), ("periodic", (48, 33, 10)),
                # power-of-two planes wider than 64: FFT passes along x and y (8 to 1024 points,
                # work-groups that span planes, a partial last work-group), and along z in a box
                # of more than 64 planes
                ("slit", (128, 128, 10)), ("slit", (256, 8, 6)), ("periodic", (8, 1024, 3)),
                ("periodic", (128, 8, 128)), ("slit", (16, 512, 5))]


def charged_case(geometry, dims):
    nx, ny, nz = dims
    if geometry == "slit":
        return WL.charged_slit(nx=nx, ny=ny, nz=nz, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
    return WL.random_state(nx, ny, nz, 3, seed=13, rho0=[1.0, 0.02, 0.02], valence=[0, 1, -1],
                           bjerrum=0.5, E=(1e-3, 0, 0), dn=0.0, du=0.02)


@pytest.mark.parametrize("geometry,dims", DIRECT_CASES)
def test_direct_poisson_fp64_matches_oracle(P, oracle_mod, geometry, dims):
    """The direct solve (Fourier bases in x, y; tridiagonal or Fourier in z) against the
    oracle's eigenbasis solve: odd and one-node extents, ragged 64-wide transform tiles
    (70, 130, 66), planes looped within a transform work-group, 30 coupled steps at the
    full FP64 bar."""
    w = charged_case(geometry, dims)
    lat = gpu_for(P, w, "f64", poisson=dict(method="direct"))
    o = oracle_for(oracle_mod, w, poisson="direct")
    lat.step(30)
    o.step(30)
    compare_fp64(lat, o, w)
    check_potential(lat.potential(), o.potential(), w)
    st = lat.stats()
    assert st["last_sweeps"] == 1 and st["poisson_solves"] == 31
    assert st["last_residual"] <= 1e-13


def test_direct_poisson_full_size_charged_slit_fp32(P, oracle_mod):
    """64 x 64 x 130 charged slit, shifted FP32 populations, direct solve on both sides."""
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    lat = gpu_for(P, w, "f32s", poisson=dict(method="direct"))
    o = oracle_for(oracle_mod, w, poisson="direct")
    lat.step(3)
    o.step(3)
    m = fluid(w)
    for s in range(3):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no, m) <= 1e-5
        assert rel_to_deviation(ng, no, w.rho0[s], m) <= 1e-3
    assert rel_max(lat.potential(), o.potential(), m) <= 1e-5
    assert lat.stats()["last_residual"] <= 1e-12


def test_odd_extents_need_the_direct_solve(P):
    w = charged_case("slit", (7, 5, 13))
    lat = gpu_for(P, w, "f64")
    with pytest.raises(P.LbmixError):
        lat.step(1)
    lat = gpu_for(P, w, "f64", poisson=dict(method="direct"))
    lat.step(2)
    with pytest.raises(P.LbmixError):
        lat.set_poisson(method="sor")
    lat.step(1)


class ChannelView:
    """The planes of one channel of a stacked lattice, read back once."""

    def __init__(self, lat, sl, ns, populations=True):
        self.m = [lat.moments(s) for s in range(ns)]
        self.f = [lat.populations(s)[:, sl] for s in range(ns)] if populations else None
        self.psi = lat.potential()[sl]
        self.sl = sl

    def moments(self, s):
        n, j = self.m[s]
        return n[self.sl], j[:, self.sl]

    def populations(self, s):
        return self.f[s]

    def potential(self):
        return self.psi


SMALL_STACK = dict(nx=8, ny=6, widths=(5, 9, 1, 12), sigmas=(-1e-3, -4e-4, -2e-4, -7e-4),
                   scs=(10.0, 100.0, 1000.0, 1.0), n_ion=2e-3, debye_length=3.0, lateral=0.3)


@pytest.mark.parametrize("lateral", [(8, 6), (128, 8)], ids=["8x6", "128x8_fft"])
def test_channel_stack_direct_fp64_matches_each_channel(P, oracle_mod, lateral):
    """Four channels of widths 5, 9, 1, 12 (own drag and wall charge, lateral charge waves)
    in one stacked lattice: every channel follows its own oracle slit at the FP64 bar.  The
    128 x 8 planes take the FFT passes of the direct solve, the 8 x 6 planes the register
    transforms."""
    st = WL.channel_stack(**dict(SMALL_STACK, nx=lateral[0], ny=lateral[1]))
    lat = P.from_workload(st, storage="f64", poisson=dict(method="direct"))
    lat.step(25)
    for c in range(len(st.widths)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="direct")
        o.step(25)
        view = ChannelView(lat, st.planes(c), 3)
        compare_fp64(view, o, wc)
        check_potential(view.potential(), o.potential(), wc)
    m = lat.mass_totals()
    assert np.all(np.isfinite(m))


def test_channel_stack_sor_fixed_sweeps_fp64(P, oracle_mod):
    """The same stack with a fixed number of red-black SOR sweeps: each channel is coloured by
    its own lattice, so it takes exactly the oracle's iterates."""
    st = WL.channel_stack(**SMALL_STACK)
    omega, sweeps = 1.6, 30
    lat = P.from_workload(st, storage="f64", poisson=dict(rel_tol=0.0, max_sweeps=sweeps, omega=omega))
    lat.step(10)
    for c in range(len(st.widths)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="sor", sor_tol=0.0, sor_max=sweeps, sor_omega=omega)
        o.step(10)
        view = ChannelView(lat, st.planes(c), 3)
        compare_fp64(view, o, wc)
        check_potential(view.potential(), o.potential(), wc)


@pytest.mark.parametrize("lateral", [(8, 6), (8, 8)], ids=["8x6", "8x8"])
def test_channel_stack_multigrid_fp64_matches_each_channel(P, oracle_mod, lateral):
    """Multigrid in its channel form (x and y halved, whole z lines of each channel relaxed
    exactly) to a relative residual of 1e-13 on the same stack: every channel follows its own
    oracle slit with the direct solve at the FP64 bar, the potential to the tolerance times the
    condition number of the operator (about (L / pi)^2), below the FP64 bar.  8 x 8 coarsens
    down to one column per channel, where the line solve is the exact coarse solve; 8 x 6 stops
    at 1 x 6 and relaxes that level repeatedly."""
    st = WL.channel_stack(**dict(SMALL_STACK, nx=lateral[0], ny=lateral[1]))
    lat = P.from_workload(st, storage="f64", poisson=dict(method="multigrid", rel_tol=1e-13, max_sweeps=200))
    lat.step(25)
    stats = lat.stats()
    assert stats["last_residual"] <= 1e-13
    assert stats["total_sweeps"] / stats["poisson_solves"] < 40      # V-cycles per solve
    for c in range(len(st.widths)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="direct")
        o.step(25)
        view = ChannelView(lat, st.planes(c), 3)
        compare_fp64(view, o, wc)
        check_potential(view.potential(), o.potential(), wc)


def test_channel_stack_rejects_charged_channels(P):
    bad = WL.channel_stack(**SMALL_STACK)
    bad.sigmas[1] = (-4e-4, -3e-4)   # the fluid no longer balances the walls of channel 1
    lat = P.from_workload(bad, storage="f64", poisson=dict(method="direct"))
    with pytest.raises(P.LbmixError) as e:
        lat.step(1)
    assert "channel 1" in str(e.value)


def test_batched_channels_full_size_sampled(P, oracle_mod):
    """The batched workload at full size (64 channels of 32 x 32 x W, W in 32..256, 9.2 M fluid
    nodes, shifted FP32, direct solve): four sampled channels against their own oracle slits
    after 3 steps, to the FP32 bar; all channels keep their mass."""
    st = WL.batched_channels(lateral=0.2)
    lat = P.from_workload(st, storage="f32s", poisson=dict(method="direct"))
    lat.step(3)
    n_all = [lat.moments(s)[0] for s in range(3)]
    psi = lat.potential()
    rng = np.random.default_rng(11)
    for c in sorted(rng.choice(len(st.widths), size=4, replace=False)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="direct")
        o.step(3)
        sl = st.planes(c)
        m = fluid(wc)
        for s in range(3):
            no, _ = o.moments(s)
            assert rel_max(n_all[s][sl], no, m) <= 1e-5, (c, s)
            assert rel_to_deviation(n_all[s][sl], no, wc.rho0[s], m) <= 1e-3, (c, s)
        assert rel_max(psi[sl], o.potential(), m) <= 1e-5, c
    tot = lat.mass_totals()
    want = [sum(float(a[st.planes(c)].sum()) for c in range(len(st.widths))) for a in st.n]
    np.testing.assert_allclose(tot, want, rtol=1e-9)


def pair_taus(ns, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.52, 3.0, (ns, ns))
    t = 0.5 * (t + t.T)
    np.fill_diagonal(t, 1.0)
    return t


@pytest.mark.parametrize("case", ["periodic_ternary_field", "slit_charged", "periodic_four"])
def test_pair_drag_fp64_matches_oracle(P, oracle_mod, case):
    """Drag with one relaxation time per species pair against the oracle at the FP64 bar."""
    if case == "periodic_ternary_field":
        w = WL.random_state(20, 6, 8, 3, seed=21, rho0=[0.6, 0.25, 0.15], valence=[0, 1, -1], bjerrum=0.0,
                            E=(2e-3, -1e-3, 5e-4), dn=0.05, du=0.02)
        poisson = None
    elif case == "slit_charged":
        w = WL.charged_slit(nx=8, ny=6, nz=18, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        poisson = dict(method="direct")
    else:
        w = WL.random_state(10, 4, 6, 4, seed=22, rho0=[0.5, 0.2, 0.2, 0.1], valence=[0, 1, -1, 0], bjerrum=0.4,
                            E=(1e-3, 0, 0), dn=0.0, du=0.02)
        poisson = dict(method="direct")
    taus = pair_taus(w.nspecies, 5)
    lat = P.from_workload(w, storage="f64", poisson=poisson, drag_pairs=taus)
    o = oracle_for(oracle_mod, w, drag_pairs=taus)
    lat.step(30)
    o.step(30)
    compare_fp64(lat, o, w)
    if w.bjerrum > 0:
        check_potential(lat.potential(), o.potential(), w)


def test_pair_drag_fp32_and_binary_reduction(P, oracle_mod):
    w = WL.random_state(40, 4, 6, 3, seed=23, rho0=[0.6, 0.25, 0.15], valence=[0, 1, -1], bjerrum=0.0,
                        E=(2e-3, 0, 0), dn=0.05, du=0.02)
    taus = pair_taus(3, 6)
    lat = P.from_workload(w, storage="f32s", drag_pairs=taus)
    o = oracle_for(oracle_mod, w, drag_pairs=taus)
    lat.step(20)
    o.step(20)
    for s in range(3):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no) <= 1e-5
        assert rel_to_deviation(ng, no, w.rho0[s]) <= 1e-3
    # a binary's pair matrix is its single drag frequency
    wb = WL.binary_multimode(n=16, amp=1e-2, nmodes=3, shear=1e-2, sc=30.0, seed=4)
    t01 = wb.tau_drag
    a = P.from_workload(wb, storage="f64", drag_pairs=[[3.0, t01], [t01, 0.9]])
    b = P.from_workload(wb, storage="f64")
    a.step(20)
    b.step(20)
    for s in range(2):
        assert np.array_equal(a.populations(s), b.populations(s))


def test_pair_drag_errors(P):
    w = WL.random_state(8, 4, 4, 3, seed=1, rho0=[0.6, 0.25, 0.15], valence=[0, 0, 0])
    lat = P.Lattice(8, 4, 4, storage="f64")
    for s in range(3):
        lat.add_species(w.rho0[s])
    t = pair_taus(3, 1)
    bad = t.copy()
    bad[0, 1] += 0.1
    with pytest.raises(P.LbmixError):
        lat.set_drag_pairs(bad)
    low = t.copy()
    low[1, 2] = low[2, 1] = 0.5
    with pytest.raises(P.LbmixError):
        lat.set_drag_pairs(low)
    lat.set_drag_pairs(t)
    st = WL.channel_stack(**SMALL_STACK)
    lat2 = P.from_workload(st, storage="f64", poisson=dict(method="direct"), drag_pairs=pair_taus(3, 2))
    with pytest.raises(P.LbmixError) as e:
        lat2.step(1)
    assert "own drag" in str(e.value)


@pytest.mark.parametrize("dims,geometry", [((256, 8, 4), "periodic"), ((32, 32, 12), "slit"), ((7, 5, 6), "periodic")])
def test_autotuned_launch_gives_identical_results(P, dims, geometry):
    """The tuned work-group shape changes nothing but speed: populations bitwise equal."""
    nx, ny, nz = dims
    w = WL.random_state(nx, ny, nz, 2, geometry=geometry, seed=31, dn=0.05, du=0.02)
    a = P.from_workload(w, storage="f32s")
    b = P.from_workload(w, storage="f32s")
    bx, by = a.autotune(reps=3)
    assert 1 <= bx * by <= 512 and (bx >= 64 or bx == nx)
    a.step(6)
    b.step(6)
    for s in range(2):
        assert np.array_equal(a.populations(s), b.populations(s))


EPS16 = {"f16s": 2.0 ** -11, "bf16s": 2.0 ** -8, "f32s": 2.0 ** -24}


@pytest.mark.parametrize("storage", ["f16s", "bf16s", "f32s"])
def test_full_size_binary_512cubed_sampled(P, oracle_mod, storage):
    """The precision configuration at full size: 512^3 periodic binary, shifted storage
    (stochastic rounding for 16 bits), Sc 100, multimode noise and shear (seed 4).  After k
    steps the GPU moments at sampled nodes equal the oracle's on light-cone patches within
    k units in the last place per population and step bound: |dn| <= 19 * 2 k eps * dev, dev
    the largest deviation of a population from rest on the patch."""
    k = 4
    w = WL.binary_multimode(n=512, amp=1e-3, nmodes=8, shear=1e-3, sc=100.0, seed=4)
    lat = gpu_for(P, w, storage)
    lat.step(k)
    n_all = [lat.moments(s)[0] for s in range(2)]
    del lat
    rng = np.random.default_rng(4)
    centres = [(0, 0, 0), (511, 511, 511)] + [tuple(rng.integers(0, 512, 3)) for _ in range(4)]
    for c in centres:
        pw, h = patch_workload(w, c, k)
        o = oracle_for(oracle_mod, pw)
        o.step(k)
        for s in range(2):
            fo = o.populations(s)
            dev = np.abs(fo - (WQ * 0.5)[:, None, None, None]).max()
            no, _ = o.moments(s)
            err = abs(n_all[s][c] - no[h, h, h])
            assert err <= max(19 * 2 * k * EPS16[storage] * dev, 1e-5 * 0.5 if storage == "f32s" else 0.0), (c, s, err)


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_full_size_ternary_slit_128x128x258_sixteen_bit(P, oracle_mod, storage):
    """The precision slit at full size (128 x 128 x 258, ternary, lambda_D 8, sigma -1e-4,
    Sc 100), direct Poisson solve on both sides: densities on the whole lattice after k steps
    within the stochastic-rounding bound.  The rounding of every species' stored deviations
    reaches the others within a step through the drag and the barycentric velocity, so the
    bound uses the largest deviation of any species (the solvent itself barely leaves rest)."""
    k = 3
    w = WL.charged_slit(nx=128, ny=128, nz=258, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    lat = gpu_for(P, w, storage, poisson=dict(method="direct"))
    lat.step(k)
    o = oracle_for(oracle_mod, w, poisson="direct")
    o.step(k)
    m = fluid(w)
    dev = max(np.abs(o.populations(s) - (WQ * w.rho0[s])[:, None, None, None])[:, m].max() for s in range(3))
    for s in range(3):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        err = np.abs(ng - no)[m].max()
        assert err <= 19 * 2 * k * EPS16[storage] * dev, (s, err, dev)
        assert err > 0.0


@pytest.mark.parametrize("case", ["binary_f32s", "slit_direct_f32s", "slit_batched_f32s", "slit_fft_f32s",
                                  "channels_bf16s"])
def test_step_graph_is_bitwise_the_uncaptured_step(P, case):
    """Captured steps (fused step + direct solve + step count) replay exactly the uncaptured
    sequence, including the stochastic-rounding stream of the 16-bit forms."""
    if case == "binary_f32s":
        w, storage, poisson = WL.binary_multimode(n=24, amp=1e-2, nmodes=4, shear=1e-2, sc=30.0, seed=3), "f32s", None
    elif case == "slit_direct_f32s":
        w = WL.charged_slit(nx=16, ny=8, nz=34, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        storage, poisson = "f32s", dict(method="direct")
    elif case == "slit_batched_f32s":   # planes wider than 64: the batched products
        w = WL.charged_slit(nx=70, ny=66, nz=12, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        storage, poisson = "f32s", dict(method="direct")
    elif case == "slit_fft_f32s":   # power-of-two planes wider than 64: the FFT passes
        w = WL.charged_slit(nx=128, ny=16, nz=12, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        storage, poisson = "f32s", dict(method="direct")
    else:
        w, storage, poisson = WL.channel_stack(**SMALL_STACK), "bf16s", dict(method="direct")
    a = P.from_workload(w, storage=storage, poisson=poisson)
    b = P.from_workload(w, storage=storage, poisson=poisson)
    a.set_step_graph(True)
    a.step(3)
    a.step(9)
    b.step(12)
    for s in range(w.nspecies):
        assert np.array_equal(a.populations(s), b.populations(s)), s
    assert np.array_equal(a.potential(), b.potential())
    sa, sb = a.stats(), b.stats()
    assert sa["steps"] == sb["steps"] == 12 and sa["poisson_solves"] == sb["poisson_solves"]


def test_degenerate_cases(P, oracle_mod):
    """A species absent everywhere stays absent and leaves the others exactly as without it;
    step(0) changes nothing; a single-node lattice and the stiffest drag (Sc = 1000, omega_drag
    = 1.998) follow the oracle at the FP64 bar."""
    # absent species (R12: its velocity is 0 where its density is 0)
    w3 = WL.random_state(10, 6, 4, 3, seed=41, rho0=[0.6, 0.4, 0.3], dn=0.05, du=0.02)
    w3.n[2] = np.zeros_like(w3.n[2])
    w2 = WL.Workload("two", 10, 6, 4, "periodic", w3.rho0[:2], w3.valence[:2], w3.tau_visc, w3.tau_drag,
                     w3.n[:2], w3.u[:2])
    a = gpu_for(P, w3, "f64")
    b = gpu_for(P, w2, "f64")
    a.step(0)
    assert a.stats()["steps"] == 0
    a.step(15)
    b.step(15)
    n2, j2 = a.moments(2)
    assert np.all(n2 == 0.0) and np.all(j2 == 0.0)
    o = oracle_for(oracle_mod, w3)
    o.step(15)
    compare_fp64(a, o, w3)
    for s in range(2):
        np.testing.assert_allclose(a.moments(s)[0], b.moments(s)[0], rtol=0, atol=1e-15)
    # one node
    w1 = WL.random_state(1, 1, 1, 2, seed=42, dn=0.05, du=0.02)
    a = gpu_for(P, w1, "f64")
    o = oracle_for(oracle_mod, w1)
    a.step(25)
    o.step(25)
    compare_fp64(a, o, w1)
    # stiffest drag of the benchmark range
    ws = WL.binary_sine(16, 4, 4, amp=0.01, tau_visc=1.0, sc=1000.0)
    a = gpu_for(P, ws, "f64")
    o = oracle_for(oracle_mod, ws)
    a.step(60)
    o.step(60)
    compare_fp64(a, o, ws)


@pytest.mark.parametrize("case", ["slit_charged", "binary_modes"])
def test_fp32_stochastic_rounding_matches_oracle(P, oracle_mod, case):
    """Shifted FP32 storage with FP64 collision arithmetic and stochastically rounded stores
    against the oracle, to the FP32 bar (every store errs by less than one FP32 unit in the
    last place, with zero mean)."""
    if case == "slit_charged":
        w = WL.charged_slit(nx=8, ny=6, nz=18, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
        poisson = dict(method="direct")
    else:
        w = WL.binary_multimode(n=16, amp=1e-2, nmodes=3, shear=1e-2, sc=30.0, seed=4)
        poisson = None
    lat = P.from_workload(w, storage="f32s", stochastic=True, seed=3, poisson=poisson)
    o = oracle_for(oracle_mod, w)
    lat.step(20)
    o.step(20)
    m = fluid(w)
    for s in range(w.nspecies):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no, m) <= 1e-5, s
        assert rel_to_deviation(ng, no, w.rho0[s], m) <= 1e-3, s
    if w.bjerrum > 0:
        assert rel_max(lat.potential(), o.potential(), m) <= 1e-5


def test_fp32_stochastic_rounding_is_reproducible(P):
    """The rounding stream is a function of (seed, step, node): captured steps and a restored
    checkpoint continue it bitwise; another seed rounds differently."""
    w = WL.charged_slit(nx=16, ny=8, nz=20, n_ion=2e-3, debye_length=3.0, sigma=-3e-4, Ex=1e-4, sc=10.0)
    pp = dict(method="direct")
    a = P.from_workload(w, storage="f32s", stochastic=True, seed=5, poisson=pp)
    g = P.from_workload(w, storage="f32s", stochastic=True, seed=5, poisson=pp)
    c = P.from_workload(w, storage="f32s", stochastic=True, seed=6, poisson=pp)
    g.set_step_graph(True)
    for lat in (a, g, c):
        lat.step(10)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(10)
        b = P.Lattice(w.nx, w.ny, w.nz, geometry="slit", storage="f32s")
        for s in range(w.nspecies):
            b.add_species(w.rho0[s], w.valence[s])
        b.load(path)
        b.step(10)
    g.step(10)
    c.step(10)
    for s in range(w.nspecies):
        np.testing.assert_array_equal(a.populations(s), b.populations(s))
        np.testing.assert_array_equal(a.populations(s), g.populations(s))
    assert not np.array_equal(a.populations(0), c.populations(0))
    with pytest.raises(P.LbmixError):
        a.set_rounding(False)


def test_fp32_stochastic_rounding_channels_and_pair_drag(P, oracle_mod):
    """Stochastically rounded FP32 on a channel stack (each channel against its own oracle
    slit) and with a pair drag matrix on a ternary under a field, to the FP32 bar."""
    st = WL.channel_stack(**SMALL_STACK)
    lat = P.from_workload(st, storage="f32s", stochastic=True, seed=9, poisson=dict(method="direct"))
    lat.step(20)
    for c in range(len(st.widths)):
        wc = st.channel(c)
        o = oracle_for(oracle_mod, wc, poisson="direct")
        o.step(20)
        view = ChannelView(lat, st.planes(c), 3)
        m = fluid(wc)
        for s in range(3):
            ng, _ = view.moments(s)
            no, _ = o.moments(s)
            assert rel_max(ng, no, m) <= 1e-5, (c, s)
            assert rel_to_deviation(ng, no, wc.rho0[s], m) <= 1e-3, (c, s)
    w = WL.random_state(20, 6, 8, 3, seed=21, rho0=[0.6, 0.25, 0.15], valence=[0, 1, -1], bjerrum=0.0,
                        E=(2e-3, -1e-3, 5e-4), dn=0.05, du=0.02)
    taus = pair_taus(3, 5)
    lat = P.from_workload(w, storage="f32s", stochastic=True, seed=9, drag_pairs=taus)
    o = oracle_for(oracle_mod, w, drag_pairs=taus)
    lat.step(20)
    o.step(20)
    for s in range(3):
        ng, _ = lat.moments(s)
        no, _ = o.moments(s)
        assert rel_max(ng, no) <= 1e-5, s
        assert rel_to_deviation(ng, no, w.rho0[s]) <= 1e-3, s


def test_channel_stack_checkpoint_restart_is_bitwise(P):
    """A channel stack (per-channel drag and wall charges) saved mid-run and restored into a
    fresh context continues bitwise, potential included."""
    st = WL.channel_stack(**SMALL_STACK)
    a = P.from_workload(st, storage="f32s", poisson=dict(method="direct"))
    a.step(12)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(9)
        b = P.Lattice(st.nx, st.ny, geometry="channels", storage="f32s", widths=st.widths)
        for s in range(3):
            b.add_species(st.rho0[s], st.valence[s])
        b.load(path)
        b.step(9)
    for s in range(3):
        np.testing.assert_array_equal(a.populations(s), b.populations(s))
    np.testing.assert_array_equal(a.potential(), b.potential())


@pytest.mark.parametrize("nx", [320, 480])
def test_wide_rows_default_launch(P, oracle_mod, nx):
    """Planes wider than 256 nodes: rows of 320 nodes run as one 320-thread work-group, rows
    of 480 as one of 512 with 32 idle lanes; the FP64-arithmetic FP32 form takes rows of 64
    (320) or 256 (480), the 16-bit forms one row per work-group.  FP64 at the FP64 bar, the
    FP64-arithmetic FP32 form at the FP32 bar, FP16 within 2 k units in the last place."""
    w = WL.random_state(nx, 3, 4, 2, seed=17, dn=0.05, du=0.02)
    k = 5
    o = oracle_for(oracle_mod, w)
    o.step(k)
    lat = gpu_for(P, w, "f64")
    lat.step(k)
    compare_fp64(lat, o, w)
    m = fluid(w)
    sr = P.from_workload(w, storage="f32s", stochastic=True, seed=3)
    sr.step(k)
    for s in range(2):
        assert rel_max(sr.moments(s)[0], o.moments(s)[0], m) <= 1e-5, s
    h = P.from_workload(w, storage="f16s", seed=3)
    h.step(k)
    for s in range(2):
        fo = o.populations(s)
        dev = np.abs(fo - (WQ * w.rho0[s])[:, None, None, None]).max()
        assert np.abs(h.populations(s) - fo).max() <= 2 * k * 2.0 ** -11 * dev, s
    for lat_ in (lat, sr, h):
        assert lat_.stats()["block_x"] in (64, 256, 320, 512)
