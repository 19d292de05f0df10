"""Pins for the oracle's reconstruction (CPU only): CG against a dense
least-squares solve, the Haar transform against hand-computed and
closed-form values, soft-thresholding, FISTA against the closed-form
proximal solution and the least-squares limit, the Beck-Teboulle rate, and
NRMSE on a hand example (Section 3.4)."""
import numpy as np
import pytest

from oracle import compression as oc
from oracle import encoding as oe
from oracle import solvers as osv
from paper_2601_05418_amd import synth

RNG = np.random.default_rng(3)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def small_problem(nx=16, k=12, accel=2, acs=4, nc=3):
    sl = synth.tiny_slice(nx=nx, ny=nx, os_=2, nc=nc, patch_len=4, k=k, accel=accel, acs=acs)
    g = sl.geom
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)

    def op(x):
        return oe.normal(x, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)

    y = oe.forward(sl.image, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    b = oe.adjoint(y, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    return sl, op, b


def dense_matrix(op, shape):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n, complex)
        e[i] = 1
        cols.append(op(e.reshape(shape)).reshape(-1))
    return np.stack(cols, 1)


def test_cg_reaches_dense_solution():
    sl, op, b = small_problem()
    m = dense_matrix(op, b.shape)
    xstar = np.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    x, hist = osv.cg(op, b, 200)
    assert osv.rel_l2(x, xstar) < 1e-8
    # energy-norm error decreases monotonically
    errs = []
    for it in (1, 2, 4, 8, 16, 32):
        xi, _ = osv.cg(op, b, it)
        d = (xi - xstar).reshape(-1)
        errs.append(np.vdot(d, m @ d).real)
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))
    assert hist[0] == pytest.approx(np.linalg.norm(b))


def test_cg_refinement_same_limit():
    sl, op, b = small_problem()
    x1, _ = osv.cg(op, b, 150)
    x2, _ = osv.cg(op, b, 150, refine_every=10)
    assert osv.rel_l2(x2, x1) < 1e-8


def test_haar_hand_example():
    c = osv.haar_fwd(np.array([[1.0, 2.0], [3.0, 4.0]]), 1)
    assert np.allclose(c, [[5.0, -1.0], [-2.0, 0.0]], atol=1e-15)


def test_haar_constant_and_parseval():
    x = np.full((16, 24), 2.5 - 1j)
    c = osv.haar_fwd(x, 3)
    assert np.allclose(c[:2, :3], (2.5 - 1j) * 8)
    c2 = c.copy()
    c2[:2, :3] = 0
    assert np.allclose(c2, 0, atol=1e-13)
    z = crandn(32, 16)
    cz = osv.haar_fwd(z, 3)
    assert np.linalg.norm(cz) == pytest.approx(np.linalg.norm(z), rel=1e-14)
    assert np.allclose(osv.haar_inv(cz, 3), z, atol=1e-13)
    # separability: one level on a rank-one image is the outer product of 1D transforms
    u, v = RNG.standard_normal(8), RNG.standard_normal(8)
    h1 = lambda s: np.concatenate([s[0::2] + s[1::2], s[0::2] - s[1::2]]) / np.sqrt(2)
    assert np.allclose(osv.haar_fwd(np.outer(u, v), 1), np.outer(h1(u), h1(v)), atol=1e-14)


def test_soft_threshold():
    z = crandn(200)
    out = osv.soft(z, 0.7)
    assert np.allclose(np.abs(out), np.maximum(np.abs(z) - 0.7, 0), atol=1e-14)
    nz = np.abs(out) > 0
    assert np.allclose(np.angle(out[nz]), np.angle(z[nz]))
    assert np.array_equal(osv.soft(z, 0.0), z)
    assert osv.soft(np.array([0j]), 0.1)[0] == 0


def _prox_by_hand(b, lam, levels):
    """W^H soft(W b, lam) with the final low-pass block (top-left
    Ny/2^levels x Nx/2^levels) sliced out by hand."""
    c = osv.haar_fwd(b, levels)
    h, w = b.shape[0] >> levels, b.shape[1] >> levels
    keep = c[:h, :w].copy()
    mag = np.abs(c)
    c = np.where(mag > lam, c * (1 - lam / np.maximum(mag, 1e-300)), 0)
    c[:h, :w] = keep
    return osv.haar_inv(c, levels)


def test_detail_mask_counts():
    m = osv.detail_mask((16, 24), 3)
    assert m.sum() == 16 * 24 - 2 * 3 and not m[:2, :3].any() and m[2:, :].all() and m[:, 3:].all()


@pytest.mark.parametrize("scale", [1.0, 0.5, 3.0])
def test_fista_scaled_identity_gives_closed_form(scale):
    """With E'^H E' = c I the problem c/2||x||^2 - Re<x, b> + lam ||W x||_1
    has the closed-form solution W^H soft(W b, lam) / c (W orthonormal);
    FISTA with L = c reaches it at the first iterate and stays there."""
    b = crandn(16, 16)
    lam = 0.8
    ref = _prox_by_hand(b, lam, 3) / scale
    x, _ = osv.fista(lambda v: scale * v, b, 5, lam, scale, 3)
    assert np.allclose(x, ref, atol=1e-13)


def test_fista_overestimated_lipschitz_same_minimiser():
    """A step 1/L with L above the true constant converges to the same
    minimiser (the threshold scales with the step)."""
    b = crandn(16, 16)
    x, _ = osv.fista(lambda v: v, b, 300, 0.8, 2.0, 3)
    assert np.allclose(x, _prox_by_hand(b, 0.8, 3), atol=1e-10)


def test_fista_first_momentum_is_zero():
    """t_1 = 1 makes the first extrapolation weight (t_1 - 1)/t_2 vanish, so
    two FISTA iterations equal two proximal-gradient steps."""
    sl, op, b = small_problem()
    lip = osv.power_iteration(op, b.shape, iters=100) * 1.01
    lam = 1e-2 * np.abs(osv.haar_fwd(b, 3)).max()
    x = np.zeros_like(b)
    for _ in range(2):
        x = _prox_by_hand(x - (op(x) - b) / lip, lam / lip, 3)
    xf, _ = osv.fista(op, b, 2, lam, lip, 3)
    assert np.allclose(xf, x, atol=1e-13)
    # and the third differs from a third plain step (momentum is active)
    x3 = _prox_by_hand(x - (op(x) - b) / lip, lam / lip, 3)
    xf3, _ = osv.fista(op, b, 3, lam, lip, 3)
    assert not np.allclose(xf3, x3, atol=1e-6)


def test_fista_momentum_weights_follow_t_recursion():
    """On a 1-pixel-per-band quadratic (E'^H E' = d I, lam = 0) the error
    of FISTA obeys e_{k+1} = (1 - d/L)(y_k - x*) with
    y_{k+1} = x_k + w_k (x_k - x_{k-1}); the published t-sequence
    1, 1.618.., 2.194.., 2.750.. gives weights 0, 0.2818, 0.4340, 0.5311."""
    d, lip = 0.3, 1.0
    b = np.full((8, 8), 1.0 + 0j)
    xs = b / d
    xk, _ = osv.fista(lambda v: d * v, b, 5, 0.0, lip, 3)
    weights = [0.0, 0.28176, 0.43400, 0.53105]
    r = 1 - d / lip
    e_prev, y = -xs, -xs  # x_0 - x*, y_1 - x*
    for w in weights + [0.60]:
        e = r * y
        y = e + w * (e - e_prev)
        e_prev = e
    # five iterations use the first four tabulated weights (the fifth is unused)
    assert np.allclose(xk - xs, e_prev, rtol=2e-4)


def test_fista_without_penalty_is_least_squares():
    sl, op, b = small_problem(k=16, accel=1, acs=0, nc=4)
    m = dense_matrix(op, b.shape)
    xstar = np.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    lip = np.linalg.eigvalsh(m).max()
    x, _ = osv.fista(op, b, 3000, 0.0, lip, 3)
    assert osv.rel_l2(x, xstar) < 1e-6


def test_fista_rate_bound():
    """Beck-Teboulle: F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k + 1)^2."""
    sl, op, b = small_problem()
    m = dense_matrix(op, b.shape)
    lip = np.linalg.eigvalsh(m).max()
    lam = 1e-2 * np.abs(osv.haar_fwd(b, 3)).max()
    y = oe.forward(sl.image, sl.coils, sl.psf, sl.geom.mask, sl.geom.os,
                   *oc.calibrate(sl.coils, sl.psf, sl.geom.os, sl.geom.patch_len,
                                 sl.geom.patch_group, sl.geom.n_groups, sl.geom.k)[:1],
                   sl.geom.patch_group, sl.geom.patch_len)
    yy = np.vdot(y, y).real

    def f(x):
        # 1/2||E'x - S'||^2 = 1/2 <x, M x> - Re<x, b> + 1/2 ||S'||^2
        v = x.reshape(-1)
        quad = 0.5 * np.vdot(v, m @ v).real - np.vdot(v, b.reshape(-1)).real + 0.5 * yy
        return quad + lam * np.abs(osv.haar_fwd(x, 3)[osv.detail_mask(x.shape, 3)]).sum()

    xs, _ = osv.fista(op, b, 2000, lam, lip, 3)
    fstar = f(xs)
    _, objs = osv.fista(op, b, 60, lam, lip, 3, objective=f)
    for k, fk in enumerate(objs, start=1):
        assert fk - fstar <= 2 * lip * np.linalg.norm(xs) ** 2 / (k + 1) ** 2 + 1e-9


def test_power_iteration():
    q, _ = np.linalg.qr(crandn(20, 20))
    lam = np.linspace(0.1, 3.0, 20)
    m = (q * lam) @ q.conj().T
    est = osv.power_iteration(lambda v: (m @ v.reshape(-1)).reshape(v.shape), (4, 5), iters=300)
    assert est == pytest.approx(3.0, rel=1e-6)


def test_nrmse_hand_example():
    ref = np.array([1.0, 3.0, 2.0, 5.0])
    x = ref + np.array([0.4, 0, 0, 0])
    assert osv.nrmse(x, ref) == pytest.approx(0.2 / 4.0)


# ---------------------------------------------------------------------------
# Total variation (smoothed) and FISTA with it (Eq. 17)
# ---------------------------------------------------------------------------
def _crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_tv_difference_adjoint_and_norm_bound():
    rng = np.random.default_rng(0)
    x = _crandn(rng, (12, 10))
    qx, qy = _crandn(rng, (12, 10)), _crandn(rng, (12, 10))
    dx, dy = osv.tv_diff(x)
    lhs = np.vdot(dx, qx) + np.vdot(dy, qy)
    assert abs(lhs - np.vdot(x, osv.tv_diff_adj(qx, qy))) <= 1e-12 * abs(lhs)
    v = _crandn(rng, (12, 10))
    for _ in range(200):  # power iteration on D^H D
        v = osv.tv_diff_adj(*osv.tv_diff(v))
        lam = np.linalg.norm(v)
        v /= lam
    assert lam <= 8.0


def test_tv_hand_example_and_constant_image():
    x = np.array([[0.0, 3.0], [4.0, 0.0]], complex)
    # pixel (0,0): dx = 3, dy = 4 -> 5; (0,1): dx = 0, dy = -3 -> 3; (1,0): dx = -4 -> 4; (1,1): 0
    assert abs(osv.tv_smooth(x, 0.0) - 12.0) <= 1e-12
    c = np.full((6, 5), 2.0 - 1.0j)
    assert abs(osv.tv_smooth(c, 0.1) - 30 * 0.1) <= 1e-12
    assert np.all(osv.tv_grad(c, 0.1) == 0)


def test_tv_gradient_against_differences():
    """Re <grad, v> = d/dt TV_eps(x + t v) at t = 0 (central differences, FP64)."""
    rng = np.random.default_rng(1)
    x, v = _crandn(rng, (9, 11)), _crandn(rng, (9, 11))
    h = 1e-6
    fd = (osv.tv_smooth(x + h * v, 0.05) - osv.tv_smooth(x - h * v, 0.05)) / (2 * h)
    ad = np.vdot(osv.tv_grad(x, 0.05), v).real
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_fista_tv_reduces_to_fista_and_reaches_a_stationary_point():
    rng = np.random.default_rng(2)
    n = 16
    q = _crandn(rng, (n * n, n * n)) / n
    a = q.conj().T @ q + 0.5 * np.eye(n * n)
    op = lambda v: (a @ v.reshape(-1)).reshape(n, n)
    b = _crandn(rng, (n, n))
    lip = np.linalg.eigvalsh(a).max()
    x1, _ = osv.fista(op, b, 30, 0.1, lip * 1.01, 2)
    x2, _ = osv.fista_tv(op, b, 30, 0.1, 0.0, 0.05, lip * 1.01, 2)
    assert np.array_equal(x1, x2)
    # lam = 0: the minimiser of the smooth objective, where its gradient vanishes
    lam_tv, eps = 0.3, 0.1
    x, _ = osv.fista_tv(op, b, 3000, 0.0, lam_tv, eps, lip + 8 * lam_tv / eps, 2)
    g = op(x) - b + lam_tv * osv.tv_grad(x, eps)
    assert np.linalg.norm(g) <= 1e-6 * np.linalg.norm(b)
