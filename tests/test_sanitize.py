"""Sanitizer builds (CPU): the oracle and the C-ABI front end's host code under
AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (oracle/orbgrand_oracle.c) is compiled with gcc and the driver
  tests/sanitize/oracle_driver.c, which calls every entry point on small
  seeded codes with special LLR values (zeros of both signs, NaN, infinities,
  ties) and checks the decoders' invariants.
* capi.hip is compiled with hipcc, the sanitizers applied to its host code
  only, and linked with stand-ins for the device launchers
  (tests/sanitize/capi_stubs.cpp) and the driver tests/sanitize/capi_driver.cpp,
  which feeds every entry point arguments its checks must reject and checks
  status and message.  Leak detection is off for this binary: the HIP runtime
  keeps its allocations until the process ends.
Any sanitizer report aborts the binary (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", os.path.join(ROOT, "oracle", "orbgrand_oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "all checks passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_capi_host_checks_under_address_and_undefined_sanitizers(tmp_path):
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROOT, "paper_2202_13951_amd", "csrc"),
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src, host_only in ((os.path.join(ROOT, "paper_2202_13951_amd", "csrc", "capi.hip"), False),
                           (os.path.join(SAN, "capi_stubs.cpp"), True), (os.path.join(SAN, "capi_driver.cpp"), True)):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        mode = ["--cuda-host-only", "-x", "hip"] if host_only else ["--offload-arch=gfx950"]
        _run([HIPCC, *mode, *flags, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "capi_asan")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", *objs, "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"), timeout=120)
    assert "all checks passed" in r.stdout
