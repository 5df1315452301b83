"""The charged step's XCD tile order on the host: the multiply-high division it uses is exact
for every dividend the launch can produce, and the map from a work-group's linear id to its tile
is a bijection onto the launch's tiles (tests/host_tile_order/check.cpp).  No GPU is needed."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tile_order_is_a_bijection_and_division_is_exact():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1507_04891_amd", "csrc"),
                        "-o", exe, os.path.join(ROOT, "tests", "host_tile_order", "check.cpp")],
                       check=True, capture_output=True, timeout=300)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout[-2000:]
        assert "tile order checks passed" in r.stdout
