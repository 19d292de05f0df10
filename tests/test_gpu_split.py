"""BF16X6: FP32 storage with both group contractions on the BF16 MFMA, every
FP32 operand split into three BF16 pieces and the six leading piece products
accumulated in FP32.  The products it drops are below 2^-26 of each product,
so it is held to the FP32 bars against the FP64 oracle: relative L2 <= 1e-5
per application and every element within 1e-5 of the largest reference
magnitude; reconstructions NRMSE <= 1e-4 on the oracle's same schedule.
Covers every built tile shape, odd patch lengths, the high-field slice in the
benchmark's launch configuration, CG / FISTA, the batch and a 3D volume.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import solvers as osv
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H
from tests.test_gpu_operator import ODD_CASES

pytestmark = pytest.mark.gpu

ELEM = 1e-5
X6 = "bf16x6"


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def check(out, ref, bound=H.REL_L2_FP32):
    rl, mr = H.rel_l2(out, ref), H.max_rel(out, ref)
    print(f"rel_l2={rl:.3e} max_rel={mr:.3e}", flush=True)
    assert rl <= bound
    assert mr <= ELEM


def make(sl, bank="oracle", seed=0, batch=1):
    a = H.oracle_bank(sl)[0] if bank == "oracle" else H.random_bank(sl.geom, seed=seed)
    plan = gpjc.Plan.from_slice(sl, batch=batch)
    plan.set_compression(torch.as_tensor(a).cuda())
    return a, plan


def all_three(plan, ops, g, seed):
    rng = np.random.default_rng(seed)
    x = H.round64(H.crandn(rng, (1, g.ny, g.nx)))
    check(host(plan.forward(dev(x), prec=X6))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(rng, plan.data_shape()))
    check(host(plan.adjoint(dev(y), prec=X6))[0], ops["adj"](y[0]))
    check(host(plan.normal(dev(x), prec=X6))[0], ops["nrm"](x[0]))


@pytest.mark.parametrize("case", list(H.CASES))
def test_operator(gpu_lib, case):
    sl = H.rounded_slice(H.CASES[case]())
    a, plan = make(sl)
    all_three(plan, H.oracle_ops(sl, a), sl.geom, 31)


@pytest.mark.parametrize("case", list(ODD_CASES))
def test_odd_patch_length(gpu_lib, case):
    """Odd P: the data operand is fetched in 8-byte halves that may lie in two
    coils, as in the FP32 form."""
    sl = H.rounded_slice(ODD_CASES[case]())
    assert sl.geom.patch_len % 2 == 1
    a, plan = make(sl, bank="random", seed=5)
    all_three(plan, H.oracle_ops(sl, a), sl.geom, 32)


@pytest.mark.parametrize("case", ["rect", "odd9"])
def test_every_tile_shape_and_split(gpu_lib, case):
    """Every built shape of both contractions (ragged row and column tiles on
    these sizes), each with a split of 1 and of 3, against the oracle."""
    sl = H.rounded_slice(H.CASES[case]() if case in H.CASES else ODD_CASES[case]())
    g = sl.geom
    a, plan = make(sl, bank="random", seed=9)
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(33), (1, g.ny, g.nx)))
    ref = ops["nrm"](x[0])
    cfg = plan.gemm_config(X6)
    nvc, nve = cfg["n_compress"], cfg["n_expand"]
    assert nvc == nve == 8
    for v in range(nvc):
        for ks in (1, 3):
            plan.set_gemm_config(v, v, ks, prec=X6)
            print(f"variant {v} split {ks}: ", end="", flush=True)
            check(host(plan.normal(dev(x), prec=X6))[0], ref)


def test_configuration_is_its_own(gpu_lib):
    """BF16X6 keeps a configuration of its own: changing it leaves FP32's
    alone, and the phase-encode stage sums the partials BF16X6 wrote."""
    sl = H.rounded_slice(H.CASES["rect"]())
    a, plan = make(sl, bank="random", seed=10)
    ops = H.oracle_ops(sl, a)
    f32 = plan.gemm_config("fp32")
    plan.set_gemm_config(3, 2, 5, prec=X6)
    assert plan.gemm_config("fp32") == f32
    c = plan.gemm_config(X6)
    assert (c["compress"], c["expand"], c["ksplit"]) == (3, 2, 5)
    assert f32["ksplit"] != 5
    x = H.round64(H.crandn(np.random.default_rng(34), (1, sl.geom.ny, sl.geom.nx)))
    check(host(plan.normal(dev(x), prec=X6))[0], ops["nrm"](x[0]))
    check(host(plan.normal(dev(x)))[0], ops["nrm"](x[0]))


def test_highfield_full_size(gpu_lib):
    """224 x 224, 32 coils, 1344 samples, 42 groups of 32, K = 64 in the
    default BF16X6 launch configuration: forward, adjoint and E'^H E', every
    element against the oracle (random orthonormal bank)."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    a, plan = make(sl, bank="random", seed=19)
    print(f"gemm config {plan.gemm_config(X6)}", flush=True)
    ops = H.oracle_ops(sl, a)
    x = H.round64(sl.image)[None]
    check(host(plan.forward(dev(x), prec=X6))[0], ops["fwd"](x[0]))
    y = H.round64(H.crandn(np.random.default_rng(8), plan.data_shape()))
    check(host(plan.adjoint(dev(y), prec=X6))[0], ops["adj"](y[0]))
    check(host(plan.normal(dev(x), prec=X6))[0], ops["nrm"](x[0]))


def test_highfield_odd_patch_full_size(gpu_lib):
    """The high-field slice cut into 64 patches of P = 21 (K = 42)."""
    base = synth.highfield_slice(0)
    np_ = base.geom.nt // 21
    geom = dataclasses.replace(base.geom, patch_len=21, patch_group=synth.sequential_groups(np_), n_groups=np_, k=42)
    sl = H.rounded_slice(dataclasses.replace(base, geom=geom))
    a, plan = make(sl, bank="random", seed=17)
    ops = H.oracle_ops(sl, a)
    x = H.round64(sl.image)[None]
    check(host(plan.normal(dev(x), prec=X6))[0], ops["nrm"](x[0]))


@pytest.mark.parametrize("case", ["small", "rect"])
def test_cg_and_fista_same_schedule(gpu_lib, case):
    sl = H.rounded_slice(H.CASES[case]())
    a, plan = make(sl)
    ops = H.oracle_ops(sl, a)
    y = H.round64(ops["fwd"](sl.image))
    x, hist = plan.recon_cg(dev(y[None]), 20, prec=X6, want_resid=True)
    xo, ho = osv.cg(ops["nrm"], ops["adj"](y), 20, x0=np.zeros_like(sl.image))
    e = osv.nrmse(host(x)[0], xo)
    print(f"{case}: CG-20 nrmse vs oracle {e:.3e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hist, ho, rtol=1e-3, atol=1e-6 * ho[0])
    b = ops["adj"](y)
    lip = osv.power_iteration(ops["nrm"], b.shape, iters=50, seed=0) * 1.01
    lam = 1e-3 * np.abs(osv.haar_fwd(b, 3)).max()
    xf = host(plan.recon_fista(dev(y[None]), 30, lam, lip, levels=3, prec=X6))[0]
    xo, _ = osv.fista(ops["nrm"], b, 30, lam, lip, 3)
    e = osv.nrmse(xf, xo)
    print(f"{case}: FISTA-30 nrmse vs oracle {e:.3e}", flush=True)
    assert e <= H.NRMSE_RECON


def test_highfield_fista50_against_stored_oracle(gpu_lib):
    """The benchmark's reconstruction with BF16X6 contractions: own
    calibration, compression of the acquired k-space, FISTA-50 with the
    oracle's lambda and L, against the oracle's stored run (NRMSE <= 1e-4,
    objective history within 1e-5 relative)."""
    from tests.golden.make_golden import FISTA_FILE, FISTA_ITERS, LEVELS, highfield_inputs
    gold = np.load(FISTA_FILE)
    lam, lip = float(gold["lam"]), float(gold["lip"])
    sl, s = highfield_inputs()
    plan = gpjc.Plan.from_slice(sl)
    plan.calibrate()
    y = plan.compress(dev(s[None]))
    x, obj = plan.recon_fista(y, FISTA_ITERS, lam, lip, levels=LEVELS, prec=X6, want_obj=True)
    e = osv.nrmse(host(x)[0], gold["x"].astype(np.complex128))
    rel = np.abs(obj - gold["obj"]) / gold["obj"]
    print(f"FISTA-{FISTA_ITERS}: NRMSE vs stored oracle {e:.2e}; objective rel err max {rel.max():.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert rel.max() <= 1e-5


def test_batch_equals_separate(gpu_lib):
    """The batch's captured iteration runs the same BF16X6 kernels with the
    same shapes as separate solves: equal bit for bit, on two replays."""
    from tests.test_gpu_batch import plans_for, separate, uneven_slices
    plans, _, ys = plans_for(uneven_slices(), seed=4)
    ref = separate(plans, ys, 10, prec=X6)
    batch = gpjc.Batch(plans, lanes=2)
    for rep in range(2):
        xs, hs = batch.recon_cg([dev(y) for y in ys], 10, prec=X6, want_resid=True)
        for i, (xr, hr) in enumerate(ref):
            assert np.array_equal(host(xs[i]), xr), (rep, i)
            assert np.array_equal(hs[i], hr), (rep, i)
    batch.close()


def test_volume(gpu_lib):
    """3D volume (32 x 32 x 16, CAIPI 2 x 2): forward, adjoint and normal."""
    from tests.test_gpu_volume import CASES, ops_for, plan_with
    v = CASES["small"]()
    g = v.geom
    a = H.random_bank(g, seed=3)
    plan = plan_with(v, a)
    fwd, adj, nrm = ops_for(v, a)
    rng = np.random.default_rng(35)
    x = H.round64(H.crandn(rng, v.image.shape))
    check(host(plan.forward(dev(x[None]), prec=X6))[0], fwd(x))
    y = H.round64(H.crandn(rng, plan.data_shape()[1:]))
    check(host(plan.adjoint(dev(y[None]), prec=X6))[0], adj(y))
    check(host(plan.normal(dev(x[None]), prec=X6))[0], nrm(x))


def test_autotune(gpu_lib, tmp_path):
    """The autotuner times the BF16X6 shapes under a key of their own; the
    installed choice still meets the FP32 bar."""
    sl = H.rounded_slice(H.CASES["rect"]())
    a, plan = make(sl, bank="random", seed=12)
    path = str(tmp_path / "tune.txt")
    c = plan.autotune(prec=X6, cache_path=path)
    with open(path) as fh:
        assert "bf16x6/" in fh.read()
    got = plan.gemm_config(X6)
    assert all(got[k] == c[k] for k in ("compress", "expand", "ksplit"))
    ops = H.oracle_ops(sl, a)
    x = H.round64(H.crandn(np.random.default_rng(36), (1, sl.geom.ny, sl.geom.nx)))
    check(host(plan.normal(dev(x), prec=X6))[0], ops["nrm"](x[0]))


def test_plans_without_contractions_run_their_fp32_path(gpu_lib):
    """The uncompressed operator and the explicit model of a modulation map
    have no group contraction: BF16X6 runs their FP32 kernels, bit for bit."""
    from tests.test_gpu_explicit import CASES as MAP_CASES
    from tests.test_gpu_explicit import plan_with as map_plan
    sl = H.rounded_slice(H.CASES["rect"]())
    unc = gpjc.Plan.from_slice(sl, compressed=False)
    msl = MAP_CASES["small"]()
    mp = map_plan(msl, H.random_bank(msl.geom, seed=2))
    for plan, g in ((unc, sl.geom), (mp, msl.geom)):
        x = dev(H.round64(H.crandn(np.random.default_rng(37), (1, g.ny, g.nx))))
        assert np.array_equal(host(plan.normal(x, prec=X6)), host(plan.normal(x)))
        assert np.array_equal(host(plan.forward(x, prec=X6)), host(plan.forward(x)))


def test_lsqr_sums_its_own_split(gpu_lib):
    """Algorithm #1 with BF16X6 column stages, the split set apart from
    FP32's: same-schedule LSQR against the oracle."""
    from oracle import hybrid as oh
    from tests.test_gpu_hybrid import wave_case
    sl, g, a, e_c, s, plan = wave_case("rect", 4)
    c = plan.gemm_config(X6)
    ks = 3 if plan.gemm_config("fp32")["ksplit"] != 3 else 2
    plan.set_gemm_config(c["compress"], c["expand"], ks, prec=X6)
    xg, hg = plan.recon_lsqr(dev(s[None]), 15, prec=X6, want_resid=True)
    xo, ho = oh.recon(s, e_c, g.mask, 4, 15)
    e = osv.nrmse(host(xg)[0], xo)
    print(f"LSQR-15 BF16X6 (split {ks}): NRMSE vs oracle {e:.2e}", flush=True)
    assert e <= H.NRMSE_RECON
    assert np.allclose(hg, ho, rtol=1e-4)


def test_unrolled_network_matches_fp32(gpu_lib):
    """The unrolled network (10 checkpointed GD steps, 2 images) with BF16X6
    contractions: loss and gradients agree with the FP32 network to the FP32
    bars (the two differ only by rounding inside the contractions)."""
    from paper_2601_05418_amd import autograd as ga
    from tests.test_gpu_autograd import setup
    sl, plan, ops, y, x0, t, lip = setup(seed=6)
    res = {}
    for prec in ("fp32", X6):
        torch.manual_seed(0)
        net = ga.UnrolledGD(plan, steps=10, alpha0=0.8 / lip, checkpoint_every=2, prec=prec)
        x = dev(x0).requires_grad_(True)
        loss = 0.5 * (net(dev(y), x) - dev(t)).abs().pow(2).sum()
        loss.backward()
        res[prec] = (float(loss.detach()), x.grad.detach().cpu().numpy().astype(np.complex128),
                     net.alpha.grad.detach().cpu().numpy().astype(np.float64))
    (l0, gx0, ga0), (l1, gx1, ga1) = res["fp32"], res[X6]
    print(f"loss {l0:.6e} / {l1:.6e}; x-grad rel {H.rel_l2(gx1, gx0):.2e}; "
          f"alpha-grad rel {np.linalg.norm(ga1 - ga0) / np.linalg.norm(ga0):.2e}", flush=True)
    assert abs(l1 - l0) <= 1e-5 * abs(l0)
    assert H.rel_l2(gx1, gx0) <= 1e-5
    assert np.linalg.norm(ga1 - ga0) <= 1e-5 * np.linalg.norm(ga0)


@pytest.mark.parametrize("case", ["n180", "n230", "n280"])
def test_paper_matrix_sizes(gpu_lib, case):
    """The matrix sizes of the paper's scans (180, 230 = 10 x 23, 280): forward,
    adjoint and E'^H E' at the FP32 bars (random orthonormal bank)."""
    from tests.test_gpu_operator import PAPER_SIZES
    sl = H.rounded_slice(PAPER_SIZES[case]())
    a, plan = make(sl, bank="random", seed=23)
    all_three(plan, H.oracle_ops(sl, a), sl.geom, 38)
