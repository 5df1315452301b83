"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer: the two
host-heavy sources (the lattice context with the C ABI, and the network object) are rebuilt
with both sanitizers on their host code only and linked, with the other objects of the
in-tree build, into a driver that exercises the C ABI's host-side validation
(tests/host_sanitizers/driver.cpp).  No GPU is needed; on a machine without one the first
device call reports EDEVICE."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1507_04891_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1507_04891_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]
INSTRUMENTED = ("lbmix_runtime.hip", "lbmix_net_runtime.hip")


def test_c_abi_host_paths_under_sanitizers():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    others = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))
              if f.endswith(".o") and f[:-2] not in INSTRUMENTED] if os.path.isdir(BUILD) else []
    if len(others) < 7:
        pytest.skip("the in-tree build (paper_1507_04891_amd/build.py) has not run")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in INSTRUMENTED:
            obj = os.path.join(d, src + ".o")
            subprocess.run([HIPCC, *flags, *SANITIZE, "-c", "-o", obj, os.path.join(CSRC, src)],
                           check=True, capture_output=True, timeout=300)
            objs.append(obj)
        drv = os.path.join(d, "driver.o")
        subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", *SANITIZE, "-I", os.path.join(ROOT, "include"),
                        "-c", "-o", drv, os.path.join(ROOT, "tests", "host_sanitizers", "driver.cpp")],
                       check=True, capture_output=True, timeout=300)
        exe = os.path.join(d, "driver")
        subprocess.run([HIPCC, "--offload-arch=gfx950", *SANITIZE[:4], "-o", exe, drv, *objs, *others],
                       check=True, capture_output=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe, os.path.join(d, "scratch.bin")], capture_output=True, text=True, timeout=120,
                           env=env)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "host ABI checks passed" in r.stdout
