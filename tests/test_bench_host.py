"""bench.py's host logic on the CPU: the work model it divides by (the
algorithmic flops and bytes per launch stated for the high-field slice and
the volume), the source-hash gate on the stored byte counters, and the
one-GPU refusal of --gpus N."""
import dataclasses
import os
import subprocess
import sys

import bench
from paper_2601_05418_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_work_model_of_the_high_field_slice():
    g = synth.highfield_slice(0).geom
    # 8 K Nc Nt Ny flops per contraction: 8 x 64 x 32 x 1344 x 224
    assert bench.stage_work(g, "group_expand", "fp32") == ("mfma", 8.0 * 64 * 32 * 1344 * 224, "flop")
    assert bench.stage_work(g, "group_compress", "fp32")[1] == 4932501504.0
    # readout: image, coils, PSF and W, 8 bytes per complex value
    b = 8.0 * (224 * 224 + 32 * 224 * 224 + 224 * 1344 + 32 * 224 * 1344)
    assert bench.stage_work(g, "readout_fwd", "fp32") == ("hbm", b, "byte")
    # phase-encode normal: Z in and Z^T out once, 16 B per element of Np K Ny
    assert bench.stage_work(g, "pe_normal", "fp32")[1] == 16.0 * 42 * 64 * 224


def test_work_model_of_the_volume():
    v = synth.volume(0, n=192, nz=64, nc=32, os_=8, patch_len=32, k=56, ry=4, rz=3, shift=1, acs=16, cycles=8,
                     phase=6.0, periodic=True)
    gv = dataclasses.replace(v.geom, ny=v.geom.ny * v.nz)
    assert bench.stage_work(gv, "group_expand", "fp32")[1] == 8.0 * 56 * 32 * 1536 * 192 * 64


def test_traffic_gate_follows_the_sources(monkeypatch):
    """A stored counter line is used only while its source hash is the
    current one."""
    stored = {}
    for line in open(bench.TRAFFIC_FILE):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic-bytes":
            stored[f[1]] = (float(f[2]), f[4])
    assert set(stored) == set(bench.STAGE_SOURCES)
    value, h = stored["group_expand"]
    monkeypatch.setattr(bench, "source_hash", lambda files: h)
    assert bench.measured_traffic("group_expand") == value
    monkeypatch.setattr(bench, "source_hash", lambda files: "0" * 16)
    assert bench.measured_traffic("group_expand") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
