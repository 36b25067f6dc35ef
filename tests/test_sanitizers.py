"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle and the host side of the C ABI are compiled with the
sanitizers (the device code of the library's kernels is not: the sanitizer
flags are given to the host compilation only), linked with a driver
(tests/native/asan_driver.cpp) and run; the driver exercises the oracle's
evaluation, derivatives, VMC and DMC and the ABI's host-only entry points and
argument errors.  Any sanitizer report fails the run."""

import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2207_14715_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = "-fsanitize=address,undefined"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    objs = sorted(glob.glob(os.path.join(PKG, "_build", "*.hip.o")))
    if len(objs) < 7:
        from paper_2207_14715_amd import build as b
        b.build()
        objs = sorted(glob.glob(os.path.join(PKG, "_build", "*.hip.o")))
    d = tmp_path_factory.mktemp("asan")
    orc = str(d / "oracle.o")
    host = str(d / "host.o")
    drv = str(d / "driver.o")
    exe = str(d / "asan_driver")
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer"]
    # the oracle and the driver: plain host C++ with g++
    _run(["g++", SAN, "-fopenmp", "-ffp-contract=off"] + common +
         ["-c", os.path.join(ROOT, "oracle", "vbqmc_oracle.cpp"), "-o", orc])
    _run(["g++", SAN] + common + ["-c", os.path.join(ROOT, "tests", "native", "asan_driver.cpp"), "-o", drv])
    # the host side of the ABI through hipcc, sanitizers on the host pass only
    _run([HIPCC, "--offload-arch=gfx950", "-x", "hip", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + common +
         ["-c", os.path.join(PKG, "csrc", "vbqmc_host.cpp"), "-o", host])
    _run(["g++", SAN, "-fopenmp", drv, orc, host] + objs +
         ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe])
    return exe


def test_host_code_is_clean_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "sanitized host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
