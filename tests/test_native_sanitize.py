"""The host builds of the FFT building blocks (fft.h, fft2.h) under
AddressSanitizer and UndefinedBehaviorSanitizer: the same checks as
test_native_fft.py, host code only, halting on the first report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# sanitizers on the host pass only (the device code is never launched)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
       "-fno-omit-frame-pointer"]


@pytest.mark.parametrize("src", ["fft_host_check.cpp", "rdft_host_check.cpp"])
def test_host_checks_under_sanitizers(src, tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "check")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++20", "--offload-arch=gfx950", *SAN, os.path.join(HERE, "native", src),
                    "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-2000:]
    rows = [line.split() for line in res.stdout.strip().splitlines()]
    assert rows and all(float(r[-1]) < 1e-6 for r in rows)
