"""FP64 oracle: reconstruction on top of the compressed operator.

TEST INFRASTRUCTURE (see the package docstring of ``oracle.encoding``).

* Least squares (Eq. 16) is solved by conjugate gradients on the normal
  equations E'^H E' x = E'^H S', which has the same minimiser.
* The regularised problem (Eq. 17) is solved by FISTA (Beck and Teboulle) on
  1/2 ||E' x - S'||^2 + lam_tv TV_eps(x) + lam ||W x||_1, W an orthonormal
  separable Haar transform; the wavelet term is applied by soft-thresholding
  and the total variation through a smooth approximation (Section 3.4).
* Quality: NRMSE normalised by the range of the reference (Section 3.4).
"""
from __future__ import annotations

import numpy as np


def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a, b))


def cg(normal_op, b, iters, x0=None, refine_every=0, refine_op=None):
    """Conjugate gradients for normal_op(x) = b with a fixed iteration count.

    Every ``refine_every`` iterations (if > 0) the residual is recomputed as
    b - refine_op(x) and the search direction restarted from it.
    Returns (x, residual norms ||r_k|| for k = 0..iters)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - normal_op(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = vdot(r, r).real
    hist = [np.sqrt(rr)]
    for it in range(iters):
        q = normal_op(p)
        alpha = rr / vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rr_new = vdot(r, r).real
        if refine_every and (it + 1) % refine_every == 0 and it + 1 < iters:
            r = b - (refine_op or normal_op)(x)
            p = r.copy()
            rr = vdot(r, r).real
        else:
            p = r + (rr_new / rr) * p
            rr = rr_new
        hist.append(np.sqrt(rr))
    return x, np.array(hist)


def haar_fwd(x, levels):
    """Orthonormal separable 2D Haar: per level, along x then along y on the
    current low-pass block, a = (u + v)/sqrt2, d = (u - v)/sqrt2, low-pass
    first (Mallat layout)."""
    c = np.array(x, dtype=np.complex128)
    h, w = c.shape
    s = np.sqrt(0.5)
    for _ in range(levels):
        blk = c[:h, :w]
        ev, od = blk[:, 0::2], blk[:, 1::2]
        blk = np.concatenate([(ev + od) * s, (ev - od) * s], axis=1)
        ev, od = blk[0::2, :], blk[1::2, :]
        c[:h, :w] = np.concatenate([(ev + od) * s, (ev - od) * s], axis=0)
        h //= 2
        w //= 2
    return c


def haar_inv(c, levels):
    """Inverse of :func:`haar_fwd`."""
    x = np.array(c, dtype=np.complex128)
    ny, nx = x.shape
    s = np.sqrt(0.5)
    for lev in reversed(range(levels)):
        h, w = ny >> lev, nx >> lev
        blk = x[:h, :w]
        lo, hi = blk[:h // 2, :], blk[h // 2:, :]
        tmp = np.empty_like(blk)
        tmp[0::2, :] = (lo + hi) * s
        tmp[1::2, :] = (lo - hi) * s
        lo, hi = tmp[:, :w // 2], tmp[:, w // 2:]
        out = np.empty_like(blk)
        out[:, 0::2] = (lo + hi) * s
        out[:, 1::2] = (lo - hi) * s
        x[:h, :w] = out
    return x


def detail_mask(shape, levels):
    """True for every Haar coefficient except the final low-pass block."""
    m = np.ones(shape, bool)
    m[:shape[0] >> levels, :shape[1] >> levels] = False
    return m


def soft(z, tau):
    """Complex soft-threshold: z max(0, 1 - tau/|z|), 0 at z = 0."""
    mag = np.abs(z)
    scale = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    return z * scale if tau > 0 else np.array(z, dtype=np.complex128)


def wavelet_prox(v, tau, levels):
    """W^H soft(W v, tau) with the final low-pass band left untouched."""
    c = haar_fwd(v, levels)
    m = detail_mask(c.shape, levels)
    c[m] = soft(c[m], tau)
    return haar_inv(c, levels)


def fista(normal_op, b, iters, lam, lipschitz, levels, objective=None):
    """FISTA for 1/2 ||E'x - S'||^2 + lam ||W x||_1 with gradient
    E'^H E' y - b and step 1/L; x_0 = y_1 = 0, t_1 = 1.
    Returns (x, objective values per iteration if ``objective`` is given)."""
    x_prev = np.zeros_like(b)
    y = np.zeros_like(b)
    t = 1.0
    objs = []
    for _ in range(iters):
        grad = normal_op(y) - b
        x = wavelet_prox(y - grad / lipschitz, lam / lipschitz, levels)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
        if objective is not None:
            objs.append(objective(x))
    return x_prev, np.array(objs)


# ----------------------------------------------------------------------------
# Total variation (Eq. 17's TV term), smoothed as the paper does in practice:
#   TV_eps(x) = sum over pixels of sqrt(|Dx x|^2 + |Dy x|^2 + eps^2),
# Dx, Dy forward differences along x and y with a zero difference at the last
# column / row.  Its gradient (the conjugate-Wirtinger gradient, as used for
# 1/2 ||E'x - S'||^2) is D^H (D x / m), m = sqrt(|Dx x|^2 + |Dy x|^2 + eps^2);
# it is Lipschitz with constant ||D||^2 / eps <= 8 / eps.
# ----------------------------------------------------------------------------
def tv_diff(x):
    dx = np.zeros_like(x)
    dy = np.zeros_like(x)
    dx[:, :-1] = x[:, 1:] - x[:, :-1]
    dy[:-1, :] = x[1:, :] - x[:-1, :]
    return dx, dy


def tv_diff_adj(qx, qy):
    """D^H (qx, qy): the adjoint of tv_diff."""
    out = np.zeros_like(qx)
    out[:, :-1] -= qx[:, :-1]
    out[:, 1:] += qx[:, :-1]
    out[:-1, :] -= qy[:-1, :]
    out[1:, :] += qy[:-1, :]
    return out


def tv_smooth(x, eps):
    dx, dy = tv_diff(x)
    return float(np.sum(np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2 + eps * eps)))


def tv_grad(x, eps):
    dx, dy = tv_diff(x)
    m = np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2 + eps * eps)
    return tv_diff_adj(dx / m, dy / m)


def fista_tv(normal_op, b, iters, lam, lam_tv, eps, lipschitz, levels, objective=None):
    """FISTA on 1/2 ||E'x - S'||^2 + lam_tv TV_eps(x) + lam ||W x||_1 (Eq. 17):
    the smoothed TV term joins the gradient step, the wavelet term stays the
    proximal step; step 1/L with L >= ||E'^H E'|| + 8 lam_tv / eps.
    lam_tv = 0 is :func:`fista`."""
    x_prev = np.zeros_like(b)
    y = np.zeros_like(b)
    t = 1.0
    objs = []
    for _ in range(iters):
        grad = normal_op(y) - b + lam_tv * tv_grad(y, eps)
        x = wavelet_prox(y - grad / lipschitz, lam / lipschitz, levels)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
        if objective is not None:
            objs.append(objective(x))
    return x_prev, np.array(objs)


def power_iteration(normal_op, shape, iters=50, seed=0):
    """Largest eigenvalue of the (Hermitian PSD) normal operator, from a
    seeded complex-normal start."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = normal_op(v)
        lam = vdot(v, w).real
        v = w / np.linalg.norm(w)
    return lam


def nrmse(x, ref):
    """sqrt(mean |x - ref|^2) / (max |ref| - min |ref|)."""
    mag = np.abs(ref)
    return float(np.sqrt(np.mean(np.abs(np.asarray(x) - ref) ** 2)) / (mag.max() - mag.min()))


def rel_l2(a, ref):
    return float(np.linalg.norm(np.asarray(a) - ref) / np.linalg.norm(ref))
