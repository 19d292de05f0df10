"""Differentiable operator and unrolled gradient descent.

Pins (the loss is quadratic in x0 and in each step size, so every check is
exact up to rounding):
- autograd of Encode / Adjoint gives E'^H v / E' v (oracle adjoint);
- one GDStep equals the oracle's x - alpha (E'^H E' x - b);
- the x0-gradient of 1/2 ||x_K - t||^2 equals the closed form
  M (M x0 + c - t), M = prod_k (I - alpha_k E'^H E') (Hermitian), with the
  oracle's FP64 operator;
- step-size gradients equal PyTorch FP64 autograd through the oracle
  operator, and central differences of the GPU loss;
- checkpointing changes nothing, bit for bit;
- at the full unrolled-network size (8 x 256^2, 32 coils, os 8, 64 groups,
  K = 80) the gradients match central differences along a random direction
  and in one step size.
"""
import numpy as np
import pytest
import torch

from oracle import encoding as oe
from oracle import solvers as osv
from paper_2601_05418_amd import autograd as ga
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

STEPS = 10


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def setup(case="rect", batch=2, seed=0):
    sl = H.rounded_slice(H.CASES[case]())
    g = sl.geom
    a = H.random_bank(g, seed)
    plan = gpjc.Plan.from_slice(sl, batch=batch)
    plan.set_compression(torch.as_tensor(a).cuda())
    rng = np.random.default_rng(seed + 20)
    y = H.round64(H.crandn(rng, plan.data_shape()))
    x0 = H.round64(0.3 * H.crandn(rng, plan.image_shape()))
    t = H.round64(H.crandn(rng, plan.image_shape()))
    ops = H.oracle_ops(sl, a)
    lip = 1.01 * osv.power_iteration(ops["nrm"], (g.ny, g.nx), iters=40, seed=seed)
    return sl, plan, ops, y, x0, t, lip


def per_image(fn, x):
    return np.stack([fn(x[b]) for b in range(x.shape[0])])


def test_encode_and_adjoint_gradients(gpu_lib):
    sl, plan, ops, y, x0, t, _ = setup()
    x = dev(x0).requires_grad_(True)
    v = dev(y)
    out = ga.Encode.apply(x, plan)
    (out.conj() * v).real.sum().backward()
    assert H.rel_l2(host(x.grad), per_image(ops["adj"], y)) <= H.REL_L2_FP32
    yy = dev(y).requires_grad_(True)
    w = dev(t)
    out = ga.Adjoint.apply(yy, plan)
    (out.conj() * w).real.sum().backward()
    assert H.rel_l2(host(yy.grad), per_image(ops["fwd"], t)) <= H.REL_L2_FP32


def test_gd_step_forward_and_residual(gpu_lib):
    sl, plan, ops, y, x0, t, lip = setup()
    b = per_image(ops["adj"], y)
    alpha = torch.tensor([0.7 / lip], dtype=torch.float32, device="cuda")
    xo, r = plan.gd_step(dev(x0), dev(b), alpha)
    r_ref = per_image(ops["nrm"], x0) - b
    a = float(alpha.item())
    assert H.rel_l2(host(r), r_ref) <= H.REL_L2_FP32
    assert H.rel_l2(host(xo), x0 - a * r_ref) <= H.REL_L2_FP32


def oracle_unrolled(ops, y, x0, alphas):
    b = per_image(ops["adj"], y)
    x = x0.copy()
    for a in alphas:
        x = x - a * (per_image(ops["nrm"], x) - b)
    return x


def test_x0_gradient_closed_form(gpu_lib):
    sl, plan, ops, y, x0, t, lip = setup()
    alphas = np.linspace(0.5, 1.2, STEPS) / lip
    net = ga.UnrolledGD(plan, steps=STEPS, checkpoint_every=2)
    with torch.no_grad():
        net.alpha.copy_(torch.as_tensor(alphas, dtype=torch.float32))
    al = net.alpha.detach().cpu().numpy().astype(np.float64)
    x = dev(x0).requires_grad_(True)
    xk = net(dev(y), x)
    loss = 0.5 * (xk - dev(t)).abs().pow(2).sum()
    loss.backward()
    xk_ref = oracle_unrolled(ops, y, x0, al)
    assert H.rel_l2(host(xk), xk_ref) <= 1e-5
    e = xk_ref - t
    for a in al:  # M e, factors in any order (they commute)
        e = e - a * per_image(ops["nrm"], e)
    err = H.rel_l2(host(x.grad), e)
    print(f"x0-gradient vs closed form: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_step_size_gradients_vs_fp64_autograd_and_differences(gpu_lib):
    sl, plan, ops, y, x0, t, lip = setup(seed=3)
    g = sl.geom
    alphas = np.linspace(1.1, 0.6, STEPS) / lip
    net = ga.UnrolledGD(plan, steps=STEPS, checkpoint_every=2)
    with torch.no_grad():
        net.alpha.copy_(torch.as_tensor(alphas, dtype=torch.float32))
    al = net.alpha.detach().cpu().numpy().astype(np.float64)
    xk = net(dev(y), dev(x0))
    loss = 0.5 * (xk - dev(t)).abs().pow(2).sum()
    loss.backward()
    grad_gpu = net.alpha.grad.detach().cpu().numpy().astype(np.float64)

    # PyTorch FP64 autograd through the oracle operator (CPU)
    class Normal(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v):
            return torch.as_tensor(per_image(ops["nrm"], v.detach().numpy()))

        @staticmethod
        def backward(ctx, gv):  # Hermitian
            return torch.as_tensor(per_image(ops["nrm"], gv.detach().numpy()))

    a64 = torch.tensor(al, dtype=torch.float64, requires_grad=True)
    b = torch.as_tensor(per_image(ops["adj"], y))
    x = torch.as_tensor(x0)
    for k in range(STEPS):
        x = x - a64[k] * (Normal.apply(x) - b)
    l64 = 0.5 * (x - torch.as_tensor(t)).abs().pow(2).sum()
    l64.backward()
    grad_ref = a64.grad.numpy()
    err = np.linalg.norm(grad_gpu - grad_ref) / np.linalg.norm(grad_ref)
    print(f"step-size gradient vs FP64 autograd: {err:.2e}", flush=True)
    assert err <= 1e-4

    # central differences at eps = 1e-3 (relative to alpha_k) of the FP64
    # network: the GPU gradient within 1e-3
    def loss64(a):
        xx = x0.copy()
        for k in range(STEPS):
            xx = xx - a[k] * (per_image(ops["nrm"], xx) - b.numpy())
        return 0.5 * np.sum(np.abs(xx - t) ** 2)

    for k in (0, STEPS // 2, STEPS - 1):
        h = 1e-3 * al[k]
        ap, am = al.copy(), al.copy()
        ap[k] += h
        am[k] -= h
        fd64 = (loss64(ap) - loss64(am)) / (2 * h)
        print(f"alpha_{k}: GPU {grad_gpu[k]:.6e}, FP64 differences {fd64:.6e}", flush=True)
        assert abs(grad_gpu[k] - fd64) <= 1e-3 * abs(fd64)
    assert abs(float(loss.detach()) - float(l64.detach())) <= 1e-5 * float(l64.detach())

    # central differences of the GPU loss (quadratic in each step size)
    eps = 1e-2 / lip
    for k in (0, STEPS - 1):
        vals = []
        for s in (1, -1):
            with torch.no_grad():
                net.alpha.copy_(torch.as_tensor(al, dtype=torch.float32))
                net.alpha[k] += s * eps
                ak = float(net.alpha[k]) - float(al[k])
                xk = net(dev(y), dev(x0))
            vals.append((0.5 * np.sum(np.abs(host(xk) - t) ** 2), ak))
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        print(f"alpha_{k}: autograd {grad_gpu[k]:.6e}, differences {fd:.6e}", flush=True)
        assert abs(fd - grad_gpu[k]) <= 2e-3 * abs(grad_gpu[k]) + 1e-6 * float(l64.detach())


def test_checkpointing_is_exact(gpu_lib):
    sl, plan, ops, y, x0, t, lip = setup(seed=5)
    grads = []
    for every in (0, 2, 3):
        torch.manual_seed(0)
        net = ga.UnrolledGD(plan, steps=STEPS, alpha0=0.8 / lip, checkpoint_every=every)
        x = dev(x0).requires_grad_(True)
        loss = 0.5 * (net(dev(y), x) - dev(t)).abs().pow(2).sum()
        loss.backward()
        grads.append((float(loss.detach()), host(x.grad), net.alpha.grad.detach().cpu().numpy()))
    for other in grads[1:]:
        assert other[0] == grads[0][0]
        assert np.array_equal(other[1], grads[0][1])
        assert np.array_equal(other[2], grads[0][2])


def test_unrolled_full_size_directional_differences(gpu_lib):
    slices = synth.unrolled_slices(8, 0)
    sl = H.rounded_slice(slices[0])
    g = sl.geom
    rng = np.random.default_rng(41)
    plan = gpjc.Plan.from_slice(sl, batch=8)
    plan.set_compression(torch.as_tensor(synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng)).cuda())
    truth = dev(np.stack([s.image for s in slices]))
    y = plan.forward(truth)
    lip = plan.power_iteration(dev(synth.unit_noise(plan.image_shape(), rng)), 30) * 1.01
    net = ga.UnrolledGD(plan, steps=STEPS, alpha0=1.0 / lip, checkpoint_every=2)
    x0 = dev(0.1 * synth.unit_noise(plan.image_shape(), rng)).requires_grad_(True)
    loss = 0.5 * (net(y, x0) - truth).abs().pow(2).sum()
    loss.backward()
    # along the gradient itself the directional derivative is ||grad|| (a
    # random direction is nearly orthogonal to it and tests little)
    v = x0.grad.detach().clone()
    v = v / torch.linalg.vector_norm(v)
    eps = 1.0

    def loss_at(x, alpha=None):
        with torch.no_grad():
            if alpha is not None:
                net.alpha.copy_(alpha)
            out = net(y, x)
            return 0.5 * np.sum(np.abs(host(out) - host(truth)) ** 2)

    a_keep = net.alpha.detach().clone()
    fd = (loss_at(x0.detach() + eps * v) - loss_at(x0.detach() - eps * v)) / (2 * eps)
    ad = float(torch.sum((x0.grad.conj() * v).real))
    print(f"full size: loss {float(loss.detach()):.6e}, directional autograd {ad:.6e}, differences {fd:.6e}", flush=True)
    assert abs(fd - ad) <= 2e-3 * abs(ad)
    h = 1e-2 / lip
    ap, am = a_keep.clone(), a_keep.clone()
    ap[3] += h
    am[3] -= h
    fa = (loss_at(x0.detach(), ap) - loss_at(x0.detach(), am)) / float(ap[3] - am[3])
    ga3 = float(net.alpha.grad[3])
    print(f"full size alpha_3: autograd {ga3:.6e}, differences {fa:.6e}", flush=True)
    assert abs(fa - ga3) <= 5e-3 * abs(ga3) + 1e-6 * float(loss.detach())


def _adjoint_gap(plan, x, v):
    """|<E'x, v> - <x, E'^H v>| / (||E'x|| ||v||) with E'^H v from autograd
    through Encode (its backward is the library's adjoint)."""
    xt = dev(x).requires_grad_(True)
    out = ga.Encode.apply(xt, plan)
    (out.conj() * dev(v)).real.sum().backward()
    ex = host(out)
    lhs = np.vdot(ex, v)
    rhs = np.vdot(x, host(xt.grad))
    return abs(lhs - rhs) / (np.linalg.norm(ex) * np.linalg.norm(v))


def test_adjoint_dot_product_test(gpu_lib):
    """The dot-product test at 1e-6, normalised by the Cauchy-Schwarz bound
    ||E'x|| ||v|| (a plain ratio of the two inner products would divide by an
    inner product of random vectors, itself ~||E'x|| ||v|| / sqrt(n)): on the
    rect case (B = 2) and at the unrolled network's full size (8 x 256^2, 32
    coils, os 8, 64 groups, K = 80)."""
    sl, plan, ops, y, x0, t, lip = setup()
    gap = _adjoint_gap(plan, x0, y)
    print(f"rect: adjoint gap {gap:.2e}", flush=True)
    assert gap <= 1e-6
    slices = synth.unrolled_slices(8, 0)
    sl = H.rounded_slice(slices[0])
    g = sl.geom
    rng = np.random.default_rng(44)
    big = gpjc.Plan.from_slice(sl, batch=8)
    big.set_compression(torch.as_tensor(synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng)).cuda())
    x = H.round64(synth.unit_noise(big.image_shape(), rng))
    v = H.round64(synth.unit_noise(big.data_shape(), rng))
    gap = _adjoint_gap(big, x, v)
    print(f"full size: adjoint gap {gap:.2e}", flush=True)
    assert gap <= 1e-6


def test_unrolled_full_size_gradient_vs_fp64_differences(gpu_lib):
    """Full size (8 x 256^2, 32 coils, os 8, 64 groups, K = 80), zero data:
    the GPU autograd directional derivative of 1/2 ||x_10 - truth||^2 along a
    unit direction v on image 0 against central differences at eps = 1e-3 of
    the same network evaluated in FP64 by the oracle (stored by
    tests/golden/make_golden.py); relative error <= 1e-3.  (FP32 evaluations
    of the loss carry ~1e-5 relative rounding, too much for differences at
    this eps; the quadratic loss has no truncation error.)"""
    from tests.golden.make_golden import UNROLLED_FILE, unrolled_inputs
    sl, bank, x0, v, truth, alphas = unrolled_inputs()
    gold = np.load(UNROLLED_FILE)
    assert np.array_equal(gold["alphas"], alphas) and float(gold["eps"]) == 1e-3
    plan = gpjc.Plan.from_slice(sl, batch=8)
    plan.set_compression(torch.as_tensor(bank).cuda())
    net = ga.UnrolledGD(plan, steps=STEPS, checkpoint_every=2)
    with torch.no_grad():
        net.alpha.copy_(torch.as_tensor(alphas, dtype=torch.float32))
    y = torch.zeros(plan.data_shape(), dtype=torch.complex64, device="cuda")
    x = dev(x0).requires_grad_(True)
    loss = 0.5 * (net(y, x) - dev(truth)).abs().pow(2).sum()
    loss.backward()
    ad = float(np.vdot(host(x.grad)[0], v).real)  # dL = Re <g, dx>
    fd = float(gold["fd"])
    print(f"full size: autograd {ad:.9e}, FP64 differences {fd:.9e}, rel {abs(ad - fd) / abs(fd):.2e}", flush=True)
    assert abs(ad - fd) <= 1e-3 * abs(fd)
