"""Reconstruction algorithm #1 (gpjc_recon_lsqr): hybrid-space LSQR over the
aliased sets of a regular mask (Section 3.4, Eq. 16), against the oracle's
same-schedule run (oracle/hybrid.py), NRMSE <= 1e-4; the residual history
against the oracle's; at full high-field size on sampled sets the oracle
solves one by one."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import compression as oc
from oracle import encoding as oe
from oracle import explicit as ox
from oracle import hybrid as oh
from oracle import solvers as osv
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def regular(sl, accel):
    return dataclasses.replace(sl, geom=dataclasses.replace(sl.geom, mask=oh.regular_mask(sl.geom.ny, accel)))


def wave_case(case, accel, seed=0):
    sl = regular(H.rounded_slice(H.CASES[case]()), accel)
    g = sl.geom
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    bmod = np.repeat(sl.psf.T[:, :, None], g.nx, axis=2)
    e_c = ox.compressed_matrices(sl.coils, bmod, a, g.patch_group, g.patch_len)
    rng = np.random.default_rng(seed)
    s = oe.forward(sl.image, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    s = H.round64(s + 0.02 * np.abs(s).max() * H.crandn(rng, s.shape))
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    return sl, g, a, e_c, s, plan


@pytest.mark.parametrize("case,accel", [("small", 4), ("rect", 4), ("periodic", 2), ("wide", 5)])
def test_lsqr_same_schedule(gpu_lib, case, accel):
    sl, g, a, e_c, s, plan = wave_case(case, accel)
    xg, hg = plan.recon_lsqr(dev(s[None]), 15, want_resid=True)
    xo, ho = oh.recon(s, e_c, g.mask, accel, 15)
    e = osv.nrmse(host(xg)[0], xo)
    print(f"{case} R={accel}: {g.ny // accel} sets, NRMSE vs oracle LSQR-15 {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hg, ho, rtol=1e-4)


def test_lsqr_batched_images_are_separate_sets(gpu_lib):
    sl, g, a, e_c, s, _ = wave_case("rect", 4)
    plan = gpjc.Plan.from_slice(sl, batch=2)
    plan.set_compression(torch.as_tensor(a).cuda())
    s2 = np.stack([s, H.round64(0.5 * s[:, :, ::-1])])
    x = host(plan.recon_lsqr(dev(s2), 10))
    for b in range(2):
        xo, _ = oh.recon(s2[b], e_c, g.mask, 4, 10)
        assert osv.nrmse(x[b], xo) <= H.NRMSE_RECON


def test_lsqr_converges_to_the_least_squares_solution(gpu_lib):
    """Run long on a well-conditioned case (R = 2), LSQR over the sets reaches
    the minimiser of Eq. 16: the oracle's FP64 LSQR run to convergence, which
    the oracle pins confirm is the global least-squares solution.  (On the
    R = 4 small case FP32 iterations stall near 1e-4 of it, as FP32 CG does.)"""
    sl, g, a, e_c, s, plan = wave_case("small", 2)
    xs, hs = oh.recon(s, e_c, g.mask, 2, 200)
    assert hs[-1] <= hs[0] and abs(hs[-1] - hs[-2]) <= 1e-10 * hs[0]  # converged reference
    x1 = host(plan.recon_lsqr(dev(s[None]), 60))[0]
    e = osv.nrmse(x1, xs)
    print(f"LSQR-60 vs converged FP64 LSQR: NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_lsqr_on_a_modulation_map(gpu_lib):
    sl = synth.local_b0_slice(0, n=64, nc=8, os_=4, patch_len=16, k=11, cycles=4)
    sl = dataclasses.replace(sl, image=H.round64(sl.image), coils=H.round64(sl.coils), bmod=H.round64(sl.bmod))
    sl = dataclasses.replace(sl, geom=dataclasses.replace(sl.geom, mask=oh.regular_mask(64, 4)))
    g = sl.geom
    a = H.random_bank(g, seed=2)
    e_c = ox.compressed_matrices(sl.coils, sl.bmod, a, g.patch_group, g.patch_len)
    s = H.round64(ox.forward(sl.image, e_c, g.mask))
    plan = gpjc.Plan.from_map_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    xg = host(plan.recon_lsqr(dev(s[None]), 15))[0]
    xo, _ = oh.recon(s, e_c, g.mask, 4, 15)
    e = osv.nrmse(xg, xo)
    print(f"map plan: NRMSE vs oracle LSQR-15 {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_lsqr_needs_a_regular_mask(gpu_lib):
    sl = H.rounded_slice(synth.small_slice(0))  # R = 3 with 8 calibration lines
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(H.random_bank(sl.geom)).cuda())
    with pytest.raises(gpjc.GpjcError) as e:
        plan.recon_lsqr(torch.zeros(plan.data_shape(), dtype=torch.complex64, device="cuda"), 5)
    assert e.value.status == gpjc.GPJC_E_UNSUPPORTED


def test_lsqr_highfield_full_size_sampled_sets(gpu_lib):
    """224 x 224, 32 coils, 1344 samples, 42 groups of 32, K = 64, R = 4
    regular (56 aliased sets of 4 x 224 unknowns and 2688 samples): the GPU
    solves every set; the oracle solves three of them on its own (their
    readout models built from those image rows only), LSQR-20."""
    base = regular(H.rounded_slice(synth.highfield_slice(0)), 4)
    g = base.geom
    a = H.random_bank(g, seed=31)
    s = oe.forward(base.image, base.coils, base.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    s = H.round64(s + 0.02 * np.abs(s).max() * H.crandn(np.random.default_rng(32), s.shape))
    plan = gpjc.Plan.from_slice(base)
    plan.set_compression(torch.as_tensor(a).cuda())
    xg = host(plan.recon_lsqr(dev(s[None]), 20))[0]
    h = oh.set_data(s, g.mask, 4)
    sets = oh.aliased_sets(g.ny, 4)
    for yr in (0, 23, 55):
        rows = sets[yr]
        bmod = np.repeat(base.psf[rows].T[:, :, None], g.nx, axis=2)
        e_c = ox.compressed_matrices(base.coils[:, rows], bmod, a, g.patch_group, g.patch_len)  # [R][Np][K][Nx]
        m = np.concatenate([e_c[q].reshape(-1, g.nx) for q in range(4)], axis=1) / 2.0
        xo, _ = oh.lsqr(lambda v: m @ v, lambda u: m.conj().T @ u, h[yr], 20)
        ref = xo.reshape(4, g.nx)
        e = osv.nrmse(xg[rows], ref)
        print(f"set {yr}: NRMSE vs oracle LSQR-20 {e:.2e}", flush=True)
        assert e <= H.NRMSE_RECON
