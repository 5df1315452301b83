"""The FP64 mass partials of the fused step (continuity, eq. `continuityb`).

Every work-group of the stream-collide writes, per species, the FP64 sum of n - rho_bar over
its nodes; lbmix_get_step_mass adds them up.  Streaming moves or reflects every population, so
the sum is the mass of the state before the step, which lbmix_get_mass_totals computes by a
separate pass.  The shapes cover work-groups of whole waves (rows of 256 and 128 threads,
inactive lanes past the edge of a row) and work-groups that end in a partial wave (narrow
planes), which sum in LDS instead of by wave reductions.
"""
import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1507_04891_amd as P
    P.load_library()
    return P


# (nx, ny, nz): work-group of the default shape (threads), whole waves or not
SHAPES = [
    (96, 6, 5),    # 128 x 2 = 256 threads, lanes 96..127 of each row inactive
    (256, 4, 3),   # 256 x 2
    (16, 12, 10),  # 16 x 12 = 192 threads: three whole waves
    (24, 12, 6),   # 24 x 12 = 288 threads: the fifth wave is partial
    (8, 6, 10),    # 8 x 6 = 48 threads: one partial wave
]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("storage,kw,rtol", [
    ("f64", {}, 1e-13),
    ("f32s", {}, 1e-13),                      # FP64 sum of every stored value
    ("f32s", {"stochastic": True}, 1e-13),    # FP64 arithmetic
    ("f16s", {}, 1e-10),                      # FP64 combination of FP32 class sums
    ("bf16s", {}, 1e-10),
    ("f32s", {"wide": False}, 1e-8),          # FP32 sum per node
])
def test_step_mass_is_the_mass_of_the_state_the_step_read(P, dims, storage, kw, rtol):
    nx, ny, nz = dims
    w = WL.random_state(nx, ny, nz, 2, seed=11, rho0=[0.6, 0.4], dn=0.05, du=0.02)
    lat = P.from_workload(w, storage=storage, seed=5, **kw)
    with pytest.raises(P.LbmixError):
        lat.step_mass()          # no step yet
    lat.step(3)
    before = lat.mass_totals()
    lat.step(1)
    got = lat.step_mass()
    np.testing.assert_allclose(got, before, rtol=rtol, atol=0)


def test_step_mass_charged_slit_and_autotuned_shape(P):
    """A charged ternary slit (walls hold no populations), then the same after the autotuner
    has picked a shape: the partials follow the last launch's work-group count."""
    w = WL.random_state(40, 12, 10, 3, geometry="slit", seed=4, rho0=[1.0, 0.01, 0.01],
                        valence=[0, 1, -1], bjerrum=0.7, sigma=(0.0, 0.0), E=(1e-4, 0, 0), dn=0.0)
    lat = P.from_workload(w, storage="f64", poisson=dict(method="direct"))
    lat.step(2)
    before = lat.mass_totals()
    lat.step(1)
    np.testing.assert_allclose(lat.step_mass(), before, rtol=1e-13, atol=0)
    lat.autotune(reps=2)
    before = lat.mass_totals()
    lat.step(1)
    np.testing.assert_allclose(lat.step_mass(), before, rtol=1e-13, atol=0)


def test_metrics_log_records_mass_and_solver_work(P, tmp_path):
    """The JSONL monitor: one record per call, the mass from the step's own partials."""
    import json
    w = WL.random_state(32, 16, 12, 2, seed=2, rho0=[0.5, 0.5], dn=0.05, du=0.02)
    lat = P.from_workload(w, storage="f32s")
    log = P.MetricsLog(tmp_path / "run.jsonl")
    first = log.write(lat, note="start")
    assert first["steps"] == 0 and "mass" not in first
    masses = []
    for _ in range(3):
        lat.step(4)
        masses.append(lat.mass_totals())   # the state the fifth step reads
        lat.step(1)
        log.write(lat)
    log.close()
    recs = [json.loads(line) for line in open(tmp_path / "run.jsonl")]
    assert [r["steps"] for r in recs] == [0, 5, 10, 15]
    assert recs[0]["note"] == "start"
    for r, m in zip(recs[1:], masses):
        assert r["glups"] > 0
        np.testing.assert_allclose(r["mass"], m, rtol=1e-13, atol=0)
