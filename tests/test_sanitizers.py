"""The oracle (plain C) and the library's host-side C++ built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU
(tests/sanitize/): every oracle routine on small generated problems, the host
aggregation on generated and malformed strength graphs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver ok" in r.stdout


@pytest.mark.skipif(shutil.which("/opt/rocm/bin/hipcc") is None, reason="hipcc not found")
def test_host_aggregation_under_sanitizers(tmp_path):
    obj = str(tmp_path / "agg.o")
    exe = str(tmp_path / "aggregate_driver")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", *san,
          "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "paper_1610_03154_amd", "csrc", "rn_aggregate_host.hip"), "-o", obj])
    drv = str(tmp_path / "drv.o")
    _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", *san,
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "aggregate_driver.cpp"), "-o", drv])
    _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", *san, drv, obj, "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "aggregate driver ok" in r.stdout
