"""FISTA on the full Eq. 17 (gpjc_recon_fista_tv): smoothed total variation
plus Haar wavelet l1, with project-generated variable-density Poisson-disc
masks, against the oracle's same-schedule run (NRMSE <= 1e-4; objective
history 1e-5 relative)."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import solvers as osv
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def pd_case(case, accel, seed=5):
    sl = H.rounded_slice(H.CASES[case]())
    mask = synth.poisson_disc_mask(sl.geom.ny, accel, np.random.default_rng(seed), center=6)
    sl = dataclasses.replace(sl, geom=dataclasses.replace(sl.geom, mask=mask))
    a = H.oracle_bank(sl)[0]
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    rng = np.random.default_rng(seed + 1)
    y = ops["fwd"](sl.image)
    y = H.round64(y + 0.01 * np.abs(y).max() * H.crandn(rng, y.shape))
    return sl, plan, ops, y


@pytest.mark.parametrize("case,accel", [("small", 3), ("rect", 4)])
def test_fista_tv_same_schedule(gpu_lib, case, accel):
    sl, plan, ops, y = pd_case(case, accel)
    b = ops["adj"](y)
    lam = 1e-3 * np.abs(osv.haar_fwd(b, 2)).max()
    lam_tv, eps = 2e-3 * np.abs(b).max(), 1e-2 * np.abs(b).max()
    lip = osv.power_iteration(ops["nrm"], b.shape, iters=50, seed=0) * 1.01 + 8 * lam_tv / eps
    dm = osv.detail_mask(b.shape, 2)

    def objective(x):
        r = ops["fwd"](x) - y
        return (0.5 * np.vdot(r, r).real + lam * np.sum(np.abs(osv.haar_fwd(x, 2)[dm]))
                + lam_tv * osv.tv_smooth(x, eps))

    xg, obj = plan.recon_fista_tv(dev(y[None]), 25, lam, lam_tv, eps, lip, levels=2, want_obj=True)
    xo, objo = osv.fista_tv(ops["nrm"], b, 25, lam, lam_tv, eps, lip, 2, objective=objective)
    e = osv.nrmse(host(xg)[0], xo)
    rel = np.max(np.abs(obj - objo) / objo)
    print(f"{case} PD R~{accel} ({int(sl.geom.mask.sum())} lines): NRMSE {e:.2e}, objective rel {rel:.2e}",
          flush=True)
    assert e <= H.NRMSE_RECON
    assert rel <= 1e-5
    # the TV term changes the result (it is not a no-op)
    x0 = host(plan.recon_fista(dev(y[None]), 25, lam, lip, levels=2))[0]
    assert osv.nrmse(x0, xo) > 10 * H.NRMSE_RECON


def test_fista_tv_zero_weight_is_fista(gpu_lib):
    sl, plan, ops, y = pd_case("small", 3)
    x1 = plan.recon_fista(dev(y[None]), 10, 1e-3, 3.0, levels=3)
    x2 = plan.recon_fista_tv(dev(y[None]), 10, 1e-3, 0.0, 0.5, 3.0, levels=3)
    assert torch.equal(x1, x2)
    with pytest.raises(gpjc.GpjcError):
        plan.recon_fista_tv(dev(y[None]), 1, 1e-3, 1.0, 0.0, 3.0)  # tv_eps must be positive


def test_cg_with_a_poisson_disc_mask(gpu_lib):
    sl, plan, ops, y = pd_case("rect", 4)
    xg = host(plan.recon_cg(dev(y[None]), 20))[0]
    xo, _ = osv.cg(ops["nrm"], ops["adj"](y), 20)
    assert osv.nrmse(xg, xo) <= H.NRMSE_RECON


def test_fista_tv_highfield_full_size(gpu_lib):
    """224 x 224, 32 coils, 42 groups, K = 64 with a variable-density
    Poisson-disc mask (~4x), three FISTA-TV iterations (the TV gradient enters
    from the second) against the oracle's same schedule."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    g = sl.geom
    mask = synth.poisson_disc_mask(g.ny, 4, np.random.default_rng(9), center=16)
    sl = dataclasses.replace(sl, geom=dataclasses.replace(g, mask=mask))
    a = H.random_bank(g, seed=41)
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    y = H.round64(ops["fwd"](sl.image))
    b = ops["adj"](y)
    lam = 1e-3 * np.abs(osv.haar_fwd(b, 3)).max()
    lam_tv, eps = 2e-3 * np.abs(b).max(), 1e-2 * np.abs(b).max()
    lip = 8.0 + 8 * lam_tv / eps  # above ||E'^H E'|| for an orthonormal bank and unit-norm coil sums
    xg = host(plan.recon_fista_tv(dev(y[None]), 3, lam, lam_tv, eps, lip, levels=3))[0]
    xo, _ = osv.fista_tv(ops["nrm"], b, 3, lam, lam_tv, eps, lip, 3)
    e = osv.nrmse(xg, xo)
    print(f"full size FISTA-TV-3: NRMSE {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON
