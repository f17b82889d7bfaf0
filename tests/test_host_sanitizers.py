"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The C-ABI library's host side: pimd_api.cpp is compiled with both
  sanitizers on its host pass (the device code is not instrumented) and
  linked with the library's kernel objects into a driver
  (sanitize/abi_driver.cpp) that runs the argument checks, the workspace
  layout and pimd_init's table building for every potential, precision,
  integrator, thermostat and bias option; without a GPU pimd_init then fails
  at its first device call, after all host work.
* The oracle's C core (oracle/bpnn_core.c) with a driver of its own
  (sanitize/oracle_driver.c): descriptors and their vector-Jacobian product,
  periodic and open, G4 and G5.
Any sanitizer report aborts the driver (no recovery), failing the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_core_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "bpnn_core.c"), "-o", exe, "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"), timeout=300)
    assert "ALL OK" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_abi_host_code_under_sanitizers(tmp_path):
    from paper_2503_23728_amd import build
    objs = [os.path.join(build.BUILD, s + ".o") for s in build.SOURCES if s != "pimd_api.cpp"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    inc = os.path.join(ROOT, "include")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "pimd_api.o")
    _run(["hipcc", "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={build.ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", inc, *san, "-c",
          os.path.join(build.CSRC, "pimd_api.cpp"), "-o", api], timeout=600)
    drv = str(tmp_path / "abi_driver.o")
    _run(["hipcc", "-O1", "-g", "-std=c++17", "-I", inc, *san, "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv],
         timeout=600)
    exe = str(tmp_path / "abi_driver")
    _run(["hipcc", f"--offload-arch={build.ARCH}", *san, drv, api, *objs, "-o", exe], timeout=600)
    r = _run([exe], env=ENV, timeout=300)
    assert "ALL OK" in r.stdout, r.stdout
