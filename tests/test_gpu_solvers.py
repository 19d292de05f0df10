"""CG and FISTA on the GPU against the oracle's same-schedule FP64 runs
(NRMSE <= 1e-4, Section 3.4's metric)."""
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


def setup(case):
    sl = H.rounded_slice(H.CASES[case]())
    a = H.oracle_bank(sl)[0]
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    y = H.round64(ops["fwd"](sl.image))
    return sl, plan, ops, y


@pytest.mark.parametrize("case", ["small", "rect"])
def test_cg_same_schedule(gpu_lib, case):
    sl, plan, ops, y = setup(case)
    x, hist = plan.recon_cg(dev(y[None]), 20, want_resid=True)
    xg = host(x)[0]
    xo, ho = osv.cg(ops["nrm"], ops["adj"](y), 20, x0=np.zeros_like(sl.image))
    e = osv.nrmse(xg, xo)
    print(f"{case}: nrmse vs oracle CG-20 = {e:.3e}; truth nrmse = {osv.nrmse(xg, sl.image):.3e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hist, ho, rtol=1e-3, atol=1e-6 * ho[0])


def test_cg_warm_start_and_zero_iterations(gpu_lib):
    sl, plan, ops, y = setup("small")
    x0 = dev(H.round64(sl.image)[None] * 0.5)
    x = host(plan.recon_cg(dev(y[None]), 0, x0=x0))
    assert np.array_equal(x, host(x0))
    xg = host(plan.recon_cg(dev(y[None]), 10, x0=x0))[0]
    xo, _ = osv.cg(ops["nrm"], ops["adj"](y), 10, x0=H.round64(sl.image) * 0.5)
    assert osv.nrmse(xg, xo) <= H.NRMSE_RECON


@pytest.mark.parametrize("case", ["small", "rect"])
def test_fista_same_schedule(gpu_lib, case):
    sl, plan, ops, y = setup(case)
    b = ops["adj"](y)
    lip = osv.power_iteration(ops["nrm"], b.shape, iters=50, seed=0) * 1.01
    lam = 1e-3 * np.abs(osv.haar_fwd(b, 3)).max()
    xg = host(plan.recon_fista(dev(y[None]), 30, lam, lip, levels=3))[0]
    xo, _ = osv.fista(ops["nrm"], b, 30, lam, lip, 3)
    e = osv.nrmse(xg, xo)
    print(f"{case}: fista nrmse vs oracle = {e:.3e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_fista_strong_penalty_matches(gpu_lib):
    """A large lambda makes many coefficients exactly zero: checks the
    threshold path, not only the gradient path."""
    sl, plan, ops, y = setup("small")
    b = ops["adj"](y)
    lip = osv.power_iteration(ops["nrm"], b.shape, iters=50, seed=0) * 1.01
    lam = 0.05 * np.abs(osv.haar_fwd(b, 3)).max()
    xg = host(plan.recon_fista(dev(y[None]), 15, lam, lip, levels=2))[0]
    xo, _ = osv.fista(ops["nrm"], b, 15, lam, lip, 2)
    assert osv.nrmse(xg, xo) <= H.NRMSE_RECON


def test_power_iteration_matches_oracle(gpu_lib):
    sl, plan, ops, y = setup("small")
    rng = np.random.default_rng(4)
    x0 = H.round64(H.crandn(rng, (sl.geom.ny, sl.geom.nx)))
    lam = plan.power_iteration(dev(x0[None]), 30)
    # oracle power iteration from the same start
    v = x0 / np.linalg.norm(x0)
    ref = 0.0
    for _ in range(30):
        w = ops["nrm"](v)
        ref = np.vdot(v, w).real
        v = w / np.linalg.norm(w)
    assert abs(lam - ref) <= 1e-5 * ref


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_wavelet_absmax(gpu_lib, levels):
    sl, plan, ops, y = setup("rect")
    x = H.round64(H.crandn(np.random.default_rng(5), (sl.geom.ny, sl.geom.nx)))
    got = plan.wavelet_absmax(dev(x[None]), levels)
    ref = np.abs(osv.haar_fwd(x, levels)).max()
    assert abs(got - ref) <= 1e-6 * ref


def test_stage_timing_counts(gpu_lib):
    sl, plan, ops, y = setup("small")
    plan.stage_timing(True)
    plan.recon_fista(dev(y[None]), 4, 1e-3, 2.0, levels=3)
    t = plan.stage_times()
    plan.stage_timing(False)
    assert t["readout_fwd"][1] == 4 and t["group_compress"][1] == 4 and t["readout_adj"][1] == 5
    assert t["solver"][1] == 4 and all(v[0] >= 0 for v in t.values())


def test_stage_timing_select_times_only_named_stages(gpu_lib):
    sl, plan, ops, y = setup("small")
    plan.stage_timing(True, stages=["group_expand"])
    plan.recon_fista(dev(y[None]), 4, 1e-3, 2.0, levels=3)
    t = plan.stage_times()
    plan.stage_timing(False)
    assert t["group_expand"][1] == 5 and t["group_expand"][0] > 0
    assert all(v[1] == 0 for k, v in t.items() if k != "group_expand")
    assert plan.lib.gpjc_stage_timing_select(plan.handle, 1 << len(gpjc.STAGES)) == gpjc.GPJC_E_INVAL


def test_highfield_fista50_against_stored_oracle(gpu_lib):
    """The benchmark's reconstruction end to end: 224 x 224, 32 coils, 42
    groups of 32, K = 64, R = 4 + 16 ACS, SNR 30.  The GPU calibrates its own
    bank, compresses the acquired k-space (Eq. 13) and runs FISTA-50 with
    3-level Haar and the oracle's lambda and L (Section 3.4, Eq. 17).  FISTA
    depends on the bank only through the projectors A_g^H A_g, so the result
    must match the oracle's stored same-schedule run (its own calibration) to
    NRMSE <= 1e-4, and the objective history to 1e-5 relative.  The GPU's own
    lambda = 1e-3 max|W E'^H S'| and power-iteration L from the same start
    agree with the oracle's."""
    from tests.golden.make_golden import FISTA_FILE, FISTA_ITERS, LEVELS, POWER_ITERS, highfield_inputs
    gold = np.load(FISTA_FILE)
    lam, lip = float(gold["lam"]), float(gold["lip"])
    sl, s = highfield_inputs()
    g = sl.geom
    plan = gpjc.Plan.from_slice(sl)
    plan.calibrate()
    y = plan.compress(dev(s[None]))
    x, obj = plan.recon_fista(y, FISTA_ITERS, lam, lip, levels=LEVELS, want_obj=True)
    e = osv.nrmse(host(x)[0], gold["x"].astype(np.complex128))
    rel = np.abs(obj - gold["obj"]) / gold["obj"]
    print(f"FISTA-{FISTA_ITERS}: NRMSE vs stored oracle {e:.2e}; objective rel err max {rel.max():.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert rel.max() <= 1e-5
    lam_gpu = 1e-3 * plan.wavelet_absmax(plan.adjoint(y), LEVELS)
    rng = np.random.default_rng(0)  # the oracle's power-iteration start
    v0 = rng.standard_normal((g.ny, g.nx)) + 1j * rng.standard_normal((g.ny, g.nx))
    lip_gpu = 1.01 * plan.power_iteration(dev(v0[None]), POWER_ITERS)
    print(f"lambda {lam_gpu:.6e} vs {lam:.6e}; L {lip_gpu:.6e} vs {lip:.6e}", flush=True)
    assert abs(lam_gpu - lam) <= 1e-5 * lam
    assert abs(lip_gpu - lip) <= 1e-5 * lip
