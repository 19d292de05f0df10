"""3D volumes (gpjc_plan_create_3d): two phase-encode dimensions with a 2D
CAIPI mask, the readout model and group contraction on (z, y) rows, and
calibration over all voxels, against the oracle (oracle/volume.py).  Bounds
as for slices: FP32 rel-L2 <= 1e-5 and every element within 1e-5 of the
largest; BF16 <= 2e-3 per application; reconstructions NRMSE <= 1e-4 on the
oracle's same schedule."""
import numpy as np
import pytest
import torch

from oracle import compression as oc
from oracle import solvers as osv
from oracle import volume as ov
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

ELEM = 1e-5


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def check(out, ref, bound=H.REL_L2_FP32, elem=ELEM):
    rl, mr = H.rel_l2(out, ref), H.max_rel(out, ref)
    print(f"rel_l2={rl:.3e} max_rel={mr:.3e}", flush=True)
    assert rl <= bound
    assert mr <= elem


def rounded(v):
    import dataclasses
    return dataclasses.replace(v, image=H.round64(v.image), coils=H.round64(v.coils), psf=H.round64(v.psf))


CASES = {
    # 32 x 32 x 16, 4 coils, os 4 (128 samples), 8 patches of 16, K = 12, CAIPI 2 x 2 shift 1
    "small": lambda: rounded(synth.volume(0)),
    # ragged: 48 x 48 x 32, 3 coils, os 2 (96), 6 patches of 16, K = 10, CAIPI 3 x 2 shift 1, 4 x 4 centre
    "rect": lambda: rounded(synth.volume(1, n=48, nz=32, nc=3, os_=2, patch_len=16, k=10, ry=3, rz=2, shift=1,
                                         acs=4, cycles=2)),
    # K = 20: the inverse y pass takes its k in two blocks, the second partial
    "k20": lambda: rounded(synth.volume(2, n=32, nz=16, nc=4, os_=4, patch_len=16, k=20, ry=2, rz=2, shift=1,
                                        cycles=4)),
    # Nz = 48 and Ny = 80: both phase-encode FFTs take three radix passes (8 x 2 x 3, 8 x 2 x 5)
    "nz48": lambda: rounded(synth.volume(4, n=80, nz=48, nc=2, os_=2, patch_len=16, k=8, ry=2, rz=3, shift=1,
                                         cycles=2)),
}


def ops_for(v, a):
    g = v.geom
    args = (v.coils, v.psf, v.mask2, g.os, a, g.patch_group, g.patch_len)
    return (lambda x: ov.forward(x, *args), lambda y: ov.adjoint(y, *args), lambda x: ov.normal(x, *args))


def plan_with(v, a, batch=1):
    p = gpjc.Plan.from_volume(v, batch=batch)
    p.set_compression(torch.as_tensor(a).cuda())
    return p


@pytest.mark.parametrize("case", list(CASES))
def test_volume_operator_matches_oracle(gpu_lib, case):
    v = CASES[case]()
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    rng = np.random.default_rng(1)
    x = H.round64(H.crandn(rng, v.image.shape))
    check(host(plan.forward(dev(x[None])))[0], fwd(x))
    y = H.round64(H.crandn(rng, plan.data_shape()[1:]))
    check(host(plan.adjoint(dev(y[None])))[0], adj(y))
    check(host(plan.normal(dev(x[None])))[0], nrm(x))
    s = H.round64(ov.forward_full(v.image, v.coils, v.psf, v.mask2, g.os))
    check(host(plan.compress(dev(s[None])))[0], oc.compress(s, a, g.patch_group, g.patch_len))


def test_volume_batch(gpu_lib):
    v = CASES["small"]()
    g = v.geom
    a = H.random_bank(g, seed=4)
    plan = plan_with(v, a, batch=2)
    fwd, adj, nrm = ops_for(v, a)
    x = H.round64(H.crandn(np.random.default_rng(2), (2,) + v.image.shape))
    out = host(plan.normal(dev(x)))
    for b in range(2):
        check(out[b], nrm(x[b]))


@pytest.mark.parametrize("prec,bound", [("bf16", 2e-3), ("fp16", 5e-4)])
def test_volume_reduced_precision(gpu_lib, prec, bound):
    """The 16-bit contractions through the 2D phase-encode stage (Z^T as a
    hi + lo pair written by the inverse y pass): per-application bounds of
    the precision configuration, on the phantom with the calibrated bank."""
    v = CASES["small"]()
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    x = H.round64(v.image)
    y = H.round64(fwd(x))
    ef = H.rel_l2(host(plan.forward(dev(x[None]), prec=prec))[0], fwd(x))
    ea = H.rel_l2(host(plan.adjoint(dev(y[None]), prec=prec))[0], adj(y))
    en = H.rel_l2(host(plan.normal(dev(x[None]), prec=prec))[0], nrm(x))
    print(f"{prec}: forward {ef:.2e}, adjoint {ea:.2e}, normal {en:.2e}", flush=True)
    assert max(ef, ea, en) <= bound


def test_volume_phase_encode_sums_its_precisions_split(gpu_lib):
    """The 2D phase-encode stage sums as many partials of Z as the
    compressing contraction of the call's precision wrote: BF16 with a split
    other than FP32's, then FP32 again, each within its bound."""
    v = CASES["small"]()
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    f32 = plan.gemm_config("fp32")["ksplit"]
    c16 = plan.gemm_config("bf16")
    plan.set_gemm_config(c16["compress"], c16["expand"], 3 if f32 != 3 else 2, prec="bf16")
    x = H.round64(v.image)
    e16 = H.rel_l2(host(plan.normal(dev(x[None]), prec="bf16"))[0], nrm(x))
    ef16 = H.rel_l2(host(plan.forward(dev(x[None]), prec="bf16"))[0], fwd(x))
    print(f"bf16 normal {e16:.2e}, forward {ef16:.2e}", flush=True)
    assert max(e16, ef16) <= 2e-3
    check(host(plan.normal(dev(x[None])))[0], nrm(x))


@pytest.mark.parametrize("case", list(CASES))
def test_volume_calibration(gpu_lib, case):
    v = CASES[case]()
    g = v.geom
    a_ref, lam_ref = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    plan = gpjc.Plan.from_volume(v)
    eig, bank = plan.calibrate(want_eigvals=True, want_bank=True)
    assert np.max(np.abs(eig - lam_ref)) <= 1e-10 * lam_ref.max()
    gap = np.min((lam_ref[:, g.k - 1] - lam_ref[:, g.k]) / lam_ref[:, 0])
    assert np.max(np.abs(oc.projectors(bank.cpu().numpy()) - oc.projectors(a_ref))) <= 1e-9 / max(gap, 1e-3)


def test_volume_cg_and_fista(gpu_lib):
    v = CASES["small"]()
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    y = H.round64(fwd(v.image))
    b = adj(y)
    xg, hist = plan.recon_cg(dev(y[None]), 15, want_resid=True)
    xo, ho = osv.cg(nrm, b, 15)
    e = osv.nrmse(host(xg)[0], xo)
    print(f"CG-15 NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hist, ho, rtol=1e-3)
    # FISTA with the Haar term of every z partition: the 2D Haar of the
    # (z, y)-row image has the same coefficients (ny divisible by 2^levels)
    shp = v.image.shape
    flat = (shp[0] * shp[1], shp[2])
    nrm2 = lambda u: nrm(u.reshape(shp)).reshape(flat)
    lip = osv.power_iteration(nrm2, flat, iters=40, seed=0) * 1.01
    lam = 1e-3 * np.abs(osv.haar_fwd(b.reshape(flat), 2)).max()
    xf = host(plan.recon_fista(dev(y[None]), 20, lam, lip, levels=2))[0]
    xfo, _ = osv.fista(nrm2, b.reshape(flat), 20, lam, lip, 2)
    e = osv.nrmse(xf, xfo.reshape(shp))
    print(f"FISTA-20 NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_volume_refusals(gpu_lib):
    v = CASES["small"]()
    plan = plan_with(v, H.random_bank(v.geom))
    y = torch.zeros(plan.data_shape(), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpjc.GpjcError) as e:
        plan.recon_lsqr(y, 3)
    assert e.value.status == gpjc.GPJC_E_UNSUPPORTED
    with pytest.raises(gpjc.GpjcError) as e:
        plan.recon_fista_tv(y, 3, 1e-3, 1e-3, 1e-2, 4.0)
    assert e.value.status == gpjc.GPJC_E_UNSUPPORTED


def test_volume_moderate_size_forward(gpu_lib):
    """96 x 96 x 32, 16 coils, os 4 (384 samples), 24 patches of 16, K = 16,
    CAIPI 2 x 2 with an 8 x 8 centre (3072 rows, 24 x 16 planes of 32 x 96):
    forward and normal operator, every element against the oracle."""
    v = rounded(synth.volume(3, n=96, nz=32, nc=16, os_=4, patch_len=16, k=16, ry=2, rz=2, shift=1, acs=8,
                             cycles=4))
    a = H.random_bank(v.geom, seed=5)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    x = v.image
    check(host(plan.forward(dev(x[None])))[0], fwd(x))
    check(host(plan.normal(dev(x[None])))[0], nrm(x))


def full_ops(v):
    args = (v.coils, v.psf, v.mask2, v.geom.os)
    return (lambda x: ov.forward_full(x, *args), lambda y: ov.adjoint_full(y, *args),
            lambda x: ov.normal_full(x, *args))


@pytest.mark.parametrize("case", list(CASES))
def test_volume_uncompressed_operator_matches_oracle(gpu_lib, case):
    """The uncompressed E, E^H and E^H E of a volume: the 2D DFT of every
    (coil, readout sample) plane of W in place (y pass, z pass with the 2D
    mask, inverse passes), acquired rows gathered and scattered whole."""
    v = CASES[case]()
    plan = gpjc.Plan.from_volume(v, compressed=False)
    assert plan.data_shape() == (1, v.geom.nc, v.ms, v.geom.nt)
    fwd, adj, nrm = full_ops(v)
    rng = np.random.default_rng(6)
    x = H.round64(H.crandn(rng, v.image.shape))
    check(host(plan.forward(dev(x[None])))[0], fwd(x))
    y = H.round64(H.crandn(rng, plan.data_shape()[1:]))
    check(host(plan.adjoint(dev(y[None])))[0], adj(y))
    check(host(plan.normal(dev(x[None])))[0], nrm(x))
    # a second normal after the adjoint: every pass rewrites W whole
    check(host(plan.normal(dev(v.image[None])))[0], nrm(v.image))


def test_volume_uncompressed_batch_and_cg(gpu_lib):
    v = CASES["rect"]()
    plan = gpjc.Plan.from_volume(v, batch=2, compressed=False)
    fwd, adj, nrm = full_ops(v)
    x = H.round64(H.crandn(np.random.default_rng(7), (2,) + v.image.shape))
    out = host(plan.normal(dev(x)))
    for b in range(2):
        check(out[b], nrm(x[b]))
    one = gpjc.Plan.from_volume(v, compressed=False)
    y = H.round64(fwd(v.image))
    xg, hist = one.recon_cg(dev(y[None]), 12, want_resid=True)
    b = adj(y)
    xo, ho = osv.cg(nrm, b, 12)
    e = osv.nrmse(host(xg)[0], xo)
    print(f"uncompressed CG-12 NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hist, ho, rtol=1e-3)
    # FISTA with the Haar term of every z partition on the same schedule
    shp = v.image.shape
    flat = (shp[0] * shp[1], shp[2])
    nrm2 = lambda u: nrm(u.reshape(shp)).reshape(flat)
    lip = osv.power_iteration(nrm2, flat, iters=40, seed=0) * 1.01
    lam = 1e-3 * np.abs(osv.haar_fwd(b.reshape(flat), 2)).max()
    xf = host(one.recon_fista(dev(y[None]), 15, lam, lip, levels=2))[0]
    xfo, _ = osv.fista(nrm2, b.reshape(flat), 15, lam, lip, 2)
    e = osv.nrmse(xf, xfo.reshape(shp))
    print(f"uncompressed FISTA-15 NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_volume_uncompressed_moderate_size(gpu_lib):
    """96 x 96 x 32, 16 coils, os 4 (384 samples), CAIPI 2 x 2 with an 8 x 8
    centre: the uncompressed forward and normal operator, every element."""
    v = rounded(synth.volume(3, n=96, nz=32, nc=16, os_=4, patch_len=16, k=16, ry=2, rz=2, shift=1, acs=8,
                             cycles=4))
    plan = gpjc.Plan.from_volume(v, compressed=False)
    fwd, adj, nrm = full_ops(v)
    check(host(plan.forward(dev(v.image[None])))[0], fwd(v.image))
    check(host(plan.normal(dev(v.image[None])))[0], nrm(v.image))


def test_volume_full_size_properties(gpu_lib):
    """The 192 x 192 x 64 volume the benchmark times (32 coils, os 8, 48
    patches of 32 on 6 groups, K = 56, CAIPI 4 x 3 + 16 x 16 centre; W 4.8 GB),
    too large for the oracle: properties that hold at any size.  Compressing
    the uncompressed operator's data gives the compressed operator's (Eq. 13),
    and both operators satisfy the adjoint identity, every sum in FP64."""
    v = synth.volume(0, n=192, nz=64, nc=32, os_=8, patch_len=32, k=56, ry=4, rz=3, shift=1, acs=16, cycles=8,
                     phase=6.0, periodic=True)
    comp = plan_with(v, H.random_bank(v.geom, seed=7))
    full = gpjc.Plan.from_volume(v, compressed=False)
    rng = np.random.default_rng(9)
    x = H.crandn(rng, (1,) + v.image.shape)
    xd = dev(x)
    s_full = full.forward(xd)
    s_c = host(comp.forward(xd))
    check(host(comp.compress(s_full)), s_c)
    for plan, s in ((comp, s_c), (full, host(s_full))):
        y = H.crandn(rng, s.shape)
        ahy = host(plan.adjoint(dev(y)))
        lhs, rhs = np.vdot(s, y), np.vdot(x, ahy)
        rel = abs(lhs - rhs) / (np.linalg.norm(s) * np.linalg.norm(y))
        print(f"adjoint identity {rel:.2e}", flush=True)
        assert rel <= 1e-6
    # the autotuned tiles: the 4.8 GB operand needs a split the staged forms can address
    choice = comp.autotune("fp32")
    print(f"autotuned {choice}", flush=True)
    assert choice["ksplit"] >= 3
    check(host(comp.forward(xd)), s_c)
    comp.close()
    full.close()
