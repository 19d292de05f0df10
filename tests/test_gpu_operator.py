"""Parity of the HIP operator (through the C ABI) with the FP64 oracle.

Bound: relative L2 <= 1e-5 per FP32 application, and every element within
1e-5 of the largest reference magnitude.  Inputs are rounded to complex64
once and the oracle receives the same rounded values.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import compression as oc
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

ELEM = 1e-5


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def make(case, batch=1, compressed=True, bank="oracle"):
    sl = H.rounded_slice(H.CASES[case]())
    a = None
    if compressed:
        a = H.oracle_bank(sl)[0] if bank == "oracle" else H.random_bank(sl.geom)
    plan = gpjc.Plan.from_slice(sl, batch=batch, compressed=compressed)
    if compressed:
        plan.set_compression(torch.as_tensor(a).cuda())
    return sl, a, plan


def check(out, ref, bound=H.REL_L2_FP32):
    rl, mr = H.rel_l2(out, ref), H.max_rel(out, ref)
    print(f"rel_l2={rl:.3e} max_rel={mr:.3e}", flush=True)
    assert rl <= bound
    assert mr <= ELEM


@pytest.mark.parametrize("case", list(H.CASES))
def test_forward(gpu_lib, case):
    sl, a, plan = make(case)
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(1), (1, sl.geom.ny, sl.geom.nx)))
    out = host(plan.forward(dev(x)))
    check(out[0], ops["fwd"](x[0]))


@pytest.mark.parametrize("case", list(H.CASES))
def test_adjoint(gpu_lib, case):
    sl, a, plan = make(case)
    ops = H.oracle_ops(sl, a)
    y = H.round64(H.crandn(np.random.default_rng(2), plan.data_shape()))
    out = host(plan.adjoint(dev(y)))
    check(out[0], ops["adj"](y[0]))


@pytest.mark.parametrize("case", list(H.CASES))
def test_normal(gpu_lib, case):
    sl, a, plan = make(case)
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(3), (1, sl.geom.ny, sl.geom.nx)))
    out = host(plan.normal(dev(x)))
    check(out[0], ops["nrm"](x[0]))


def test_batched_images_are_independent(gpu_lib):
    sl, a, plan = make("rect", batch=3)
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(4), (3, sl.geom.ny, sl.geom.nx)))
    f = host(plan.forward(dev(x)))
    n = host(plan.normal(dev(x)))
    for b in range(3):
        check(f[b], ops["fwd"](x[b]))
        check(n[b], ops["nrm"](x[b]))


@pytest.mark.parametrize("case", ["small", "rect"])
def test_uncompressed(gpu_lib, case):
    sl, _, plan = make(case, compressed=False)
    ops = H.oracle_ops(sl, None)
    rng = np.random.default_rng(5)
    x = H.round64(H.crandn(rng, (1, sl.geom.ny, sl.geom.nx)))
    check(host(plan.forward(dev(x)))[0], ops["fwd_full"](x[0]))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj_full"](y[0]))
    check(host(plan.normal(dev(x)))[0], ops["nrm_full"](x[0]))


def test_uncompressed_normal_ragged_column_block(gpu_lib):
    """Ny = 16 splits as 8 x 2, so the column-FFT kernel takes 32 readout
    samples per work-group; Nt = 3 x 16 = 48 leaves a half-filled last block."""
    sl = H.rounded_slice(synth.tiny_slice(0, nx=16, ny=16, nc=3, os_=3, patch_len=4, k=6))
    plan = gpjc.Plan.from_slice(sl, compressed=False)
    ops = H.oracle_ops(sl, None)
    x = H.round64(H.crandn(np.random.default_rng(8), (1, 16, 16)))
    check(host(plan.normal(dev(x)))[0], ops["nrm_full"](x[0]))


@pytest.mark.parametrize("nx,ny,nc,os_,p", [(160, 16, 2, 16, 32), (512, 16, 4, 2, 16)])
def test_long_readout_and_wide_rows(gpu_lib, nx, ny, nc, os_, p):
    """Geometries that reach the readout kernels' remainder loops (their
    work-groups have 256 threads): 160 x 16 = 2560 readout samples, more than
    the 8 per thread held in registers, and four 512-pixel coil rows, more
    than one round of 2 set-up loads per thread.  Forward, adjoint and normal
    operator against the oracle (random orthonormal bank)."""
    sl = H.rounded_slice(synth.tiny_slice(0, nx=nx, ny=ny, nc=nc, os_=os_, patch_len=p, k=8))
    g = sl.geom
    a = H.random_bank(g, seed=3)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(4), (1, g.ny, g.nx)))
    check(host(plan.forward(dev(x)))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(np.random.default_rng(5), plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj"](y[0]))
    check(host(plan.normal(dev(x)))[0], ops["nrm"](x[0]))


@pytest.mark.parametrize("case", ["small", "rect"])
def test_adjoint_identity(gpu_lib, case):
    sl, a, plan = make(case)
    rng = np.random.default_rng(6)
    x = H.round64(H.crandn(rng, (1, sl.geom.ny, sl.geom.nx)))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    fx = host(plan.forward(dev(x)))
    ahy = host(plan.adjoint(dev(y)))
    lhs, rhs = np.vdot(fx, y), np.vdot(x, ahy)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("case", ["small", "rect"])
def test_compress_matches_oracle(gpu_lib, case):
    sl, a, plan = make(case)
    g = sl.geom
    ops = H.oracle_ops(sl, a)
    s = H.round64(ops["fwd_full"](sl.image))  # acquired k-space [Nc][Ms][Nt]
    out = host(plan.compress(dev(s[None])))
    check(out[0], oc.compress(s, a, g.patch_group, g.patch_len))


def test_highfield_full_size(gpu_lib):
    """224 x 224, 32 coils, 1344 samples, 42 groups, K = 64: forward and
    adjoint at full size in the launch configuration the benchmark uses,
    every element against the oracle (random orthonormal bank)."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    g = sl.geom
    a = H.random_bank(g, seed=7)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    x = H.round64(sl.image)[None]
    check(host(plan.forward(dev(x)))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(np.random.default_rng(8), plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj"](y[0]))


def test_highfield_uncompressed_normal_full_size(gpu_lib):
    """The plain operator's normal form at full size (column FFTs of
    224 = 16 x 14 over 32 x 1344 columns), every element against the oracle."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    plan = gpjc.Plan.from_slice(sl, compressed=False)
    ops = H.oracle_ops(sl, None)
    x = H.round64(sl.image)[None]
    check(host(plan.normal(dev(x)))[0], ops["nrm_full"](x[0]))


def test_highfield_adjoint_identity_full_size(gpu_lib):
    """<E' x, y> = <x, E'^H y> for the compressed FP32 operator at full size
    (224 x 224, 32 coils, 42 groups, K = 64) in the benchmark's launch
    configuration: a property of the pair that holds at any size."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    a = H.random_bank(sl.geom, seed=11)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    rng = np.random.default_rng(12)
    x = H.round64(H.crandn(rng, (1, sl.geom.ny, sl.geom.nx)))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    lhs = np.vdot(host(plan.forward(dev(x))), y)
    rhs = np.vdot(x, host(plan.adjoint(dev(y))))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_highfield_compress_full_size(gpu_lib):
    """Compression of acquired data (Eq. 13) at full size: 68 sampled lines
    give the contraction a ragged last column tile and no k-split.  Every
    element against the oracle."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    g = sl.geom
    a = H.random_bank(g, seed=13)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    s_acq = H.round64(H.crandn(np.random.default_rng(14), (g.nc, g.ms, g.nt)))
    out = host(plan.compress(dev(s_acq[None])))
    check(out[0], oc.compress(s_acq, a, g.patch_group, g.patch_len))


def test_state_and_argument_errors(gpu_lib):
    sl = H.rounded_slice(synth.small_slice(0))
    plan = gpjc.Plan.from_slice(sl)
    x = torch.zeros((1, 64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpjc.GpjcError) as e:
        plan.forward(x)
    assert e.value.status == gpjc.GPJC_E_STATE
    out = torch.full(plan.data_shape(), 7.0 + 0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(gpjc.GpjcError):
        plan.forward(x, prec=9, out=out)
    assert torch.all(out == 7.0)  # untouched on error


def test_runtime_is_torchs(gpu_lib):
    """libgpjc must share torch's HIP runtime, or device pointers would not
    be valid across the two."""
    import os
    path = gpjc.runtime_path()
    assert os.path.dirname(os.path.realpath(path)) == os.path.dirname(os.path.realpath(torch.__file__)) + "/lib", path


# Odd patch lengths: a contraction chunk of two complex samples may span two
# coils (P odd), and with Ns = Nc P odd the contraction ends mid-chunk.
ODD_CASES = {
    # P = 9, Nc = 3: Ns = 27 odd; 16 patches, ragged 2K = 14
    "odd9": lambda: synth._make_rect(0, nx=48, ny=32, nc=3, os_=3, patch_len=9, k=7, accel=3, acs=6, cycles=3,
                                     phase_max=2.0),
    # P = 3: a 16-sample k-tile crosses five coils; Ns = 15 odd
    "odd3": lambda: synth._make_rect(1, nx=32, ny=48, nc=5, os_=3, patch_len=3, k=4, accel=2, acs=4, cycles=2,
                                     phase_max=1.5),
    # P = 21, Nc = 4: Ns = 84 even, but chunks still straddle coils
    "odd21": lambda: synth._make_rect(2, nx=112, ny=64, nc=4, os_=3, patch_len=21, k=9, accel=3, acs=6,
                                      cycles=3, phase_max=2.0),
}


@pytest.mark.parametrize("bank", ["oracle", "random"])
@pytest.mark.parametrize("case", list(ODD_CASES))
def test_odd_patch_length(gpu_lib, case, bank):
    """Forward, adjoint, normal and data compression with an odd patch
    length (any divisor of Nt forms a partition, Section 2.3), every element
    against the oracle."""
    sl = H.rounded_slice(ODD_CASES[case]())
    g = sl.geom
    assert g.patch_len % 2 == 1 and g.nt % g.patch_len == 0
    a = H.oracle_bank(sl)[0] if bank == "oracle" else H.random_bank(g, seed=5)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    rng = np.random.default_rng(21)
    x = H.round64(H.crandn(rng, (1, g.ny, g.nx)))
    check(host(plan.forward(dev(x)))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj"](y[0]))
    check(host(plan.normal(dev(x)))[0], ops["nrm"](x[0]))
    s_acq = H.round64(H.crandn(rng, (g.nc, g.ms, g.nt)))
    check(host(plan.compress(dev(s_acq[None])))[0], oc.compress(s_acq, a, g.patch_group, g.patch_len))


def test_odd_patch_length_batched_images(gpu_lib):
    sl = H.rounded_slice(ODD_CASES["odd9"]())
    g = sl.geom
    a = H.random_bank(g, seed=6)
    plan = gpjc.Plan.from_slice(sl, batch=3)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(22), (3, g.ny, g.nx)))
    n = host(plan.normal(dev(x)))
    for b in range(3):
        check(n[b], ops["nrm"](x[b]))


def test_odd_patch_length_highfield_full_size(gpu_lib):
    """224 x 224, 32 coils, os 6 (1344 samples) cut into 64 patches of
    P = 21 (Ns = 672, K = 42: 16x), the odd divisor of 1344 that the uneven
    batch's patch-length draw admits: forward, adjoint and normal operator in
    the default launch configuration, every element against the oracle
    (random orthonormal bank)."""
    base = synth.highfield_slice(0)
    g0 = base.geom
    np_ = g0.nt // 21
    geom = dataclasses.replace(g0, patch_len=21, patch_group=synth.sequential_groups(np_), n_groups=np_, k=42)
    sl = H.rounded_slice(dataclasses.replace(base, geom=geom))
    g = sl.geom
    a = H.random_bank(g, seed=17)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    x = H.round64(sl.image)[None]
    check(host(plan.forward(dev(x)))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(np.random.default_rng(18), plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj"](y[0]))
    check(host(plan.normal(dev(x)))[0], ops["nrm"](x[0]))


def test_highfield_normal_full_size(gpu_lib):
    """E'^H E' in FP32 on the benchmark's slice and launch configuration
    (224 x 224, 32 coils, 42 groups of 32, K = 64; the compressing
    contraction's default k-split and the fused phase-encode stage for
    Ny = 224), every element against the oracle (random orthonormal bank)."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    a = H.random_bank(sl.geom, seed=19)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    cfg = plan.gemm_config("fp32")
    print(f"gemm config {cfg}", flush=True)
    ops = H.oracle_ops(sl, a)
    x = H.round64(sl.image)[None]
    check(host(plan.normal(dev(x)))[0], ops["nrm"](x[0]))


# The matrix sizes of the paper's scans: lengths of the form 2^a 3^b 5^c
# (180 = 15 x 12 and 280 = 14 x 20 in the two-pass readout and phase-encode
# kernels) and one with the prime factor 23 (230 = 10 x 23).
PAPER_SIZES = {
    # 180 x 180, 4 coils, os 8 (1440 samples), 45 patches of 32, K = 16
    "n180": lambda: synth._make_rect(3, nx=180, ny=180, nc=4, os_=8, patch_len=32, k=16, accel=4, acs=16, cycles=7,
                                     phase_max=4.0),
    # 230 x 230, 4 coils, os 4 (920 samples), 23 patches of 40, K = 20
    "n230": lambda: synth._make_rect(4, nx=230, ny=230, nc=4, os_=4, patch_len=40, k=20, accel=4, acs=16, cycles=5,
                                     phase_max=4.0),
    # 280 x 280, 4 coils, os 6 (1680 samples), 35 patches of 48, K = 24
    "n280": lambda: synth._make_rect(5, nx=280, ny=280, nc=4, os_=6, patch_len=48, k=24, accel=4, acs=16, cycles=7,
                                     phase_max=4.0),
}


@pytest.mark.parametrize("case", list(PAPER_SIZES))
def test_paper_matrix_sizes(gpu_lib, case):
    """Compressed forward, adjoint and normal operator, the uncompressed
    normal operator, and the BF16 / FP16 normal operator (2e-3 / 5e-4) at the
    paper's matrix sizes, against the oracle."""
    sl = H.rounded_slice(PAPER_SIZES[case]())
    g = sl.geom
    a = H.random_bank(g, seed=23)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    rng = np.random.default_rng(29)
    x = H.round64(H.crandn(rng, (1, g.ny, g.nx)))
    check(host(plan.forward(dev(x)))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    check(host(plan.adjoint(dev(y)))[0], ops["adj"](y[0]))
    ref = ops["nrm"](x[0])
    check(host(plan.normal(dev(x)))[0], ref)
    # 16-bit operands on the phantom (random complex images with a random
    # bank put more weight in the small samples that 16-bit storage loses)
    ph = sl.image[None]
    ref_ph = ops["nrm"](ph[0])
    assert H.rel_l2(host(plan.normal(dev(ph), prec="bf16"))[0], ref_ph) <= 2e-3
    assert H.rel_l2(host(plan.normal(dev(ph), prec="fp16"))[0], ref_ph) <= 5e-4
    unc = gpjc.Plan.from_slice(sl, compressed=False)
    check(host(unc.normal(dev(x)))[0], ops["nrm_full"](x[0]))
