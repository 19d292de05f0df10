"""Host builds of the library's FFT building blocks against naive FP64 DFTs:
the Stockham line FFT (fft.h) and the compile-time register DFTs with the
two-pass split (fft2.h).  Runs on the CPU: the device code is never launched."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def run_check(src, tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "check")
    subprocess.run([HIPCC, "-O2", "-std=c++20", "--offload-arch=gfx950", os.path.join(HERE, "native", src), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return [line.split() for line in out.strip().splitlines()]


def test_stockham_lines(tmp_path):
    rows = run_check("fft_host_check.cpp", tmp_path)
    assert len(rows) >= 16
    for r in rows:
        assert float(r[-1]) < 1e-6, r


def test_register_dfts_and_two_pass_split(tmp_path):
    rows = run_check("rdft_host_check.cpp", tmp_path)
    kinds = {r[0] for r in rows}
    assert kinds == {"rdft", "split"}
    for r in rows:
        assert float(r[-1]) < 1e-6, r
