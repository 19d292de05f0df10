"""FP64 oracle: reconstruction algorithm #1 of Section 3.4 (hybrid-space
least squares over aliased sets, Eq. 16, solved per set by LSQR).

TEST INFRASTRUCTURE (see the package docstring of ``oracle.encoding``).

With a regular R-fold phase-encode mask without calibration lines (lines
with (ky - Ny/2) divisible by R; Ms = Ny / R of them), the inverse DFT of the
acquired lines folds the image rows y = yr + q Ms (q < R) onto one another.
The least-squares problem therefore splits into Ms independent problems, one
per aliased set yr (Section 3.4, Fig. 6A): unknowns rho[yr + q Ms][x]
(R Nx of them), data the Np K compressed samples of one readout line, and the
dense readout model per set

    M_yr = R^(-1/2) [ E'_yr | E'_(yr + Ms) | ... | E'_(yr + (R-1) Ms) ],
    h_yr = R^(1/2) zf[:, :, yr],   zf = zero-filled inverse DFT of S',

with E'_y the compressed readout matrix of column y (oracle.explicit; for
the Wave operator the map is the PSF repeated over x).  Each set is solved by
LSQR (Paige and Saunders), as the paper does, for a fixed number of
iterations, and the solutions are assembled.
"""
from __future__ import annotations

import numpy as np

from . import encoding as oe


def lsqr(matvec, rmatvec, b, iters):
    """LSQR (Paige and Saunders' bidiagonalisation with Givens updates) for
    min ||A x - b|| from x = 0, complex A, a fixed number of iterations.
    Returns (x, [||r_k|| estimates for k = 0..iters])."""
    beta = np.linalg.norm(b)
    u = b / beta if beta > 0 else np.zeros_like(b)
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    v = v / alpha if alpha > 0 else v
    w = v.copy()
    x = np.zeros_like(v)
    phibar, rhobar = beta, alpha
    hist = [phibar]
    for _ in range(iters):
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        v = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        rho = np.hypot(rhobar, beta)
        if rho > 0:
            c, s = rhobar / rho, beta / rho
            theta = s * alpha
            rhobar = -c * alpha
            phi = c * phibar
            phibar = s * phibar
            x = x + (phi / rho) * w
            w = v - (theta / rho) * w
        hist.append(phibar)
    return x, np.array(hist)


def regular_mask(ny, accel):
    """The R-fold regular mask without calibration lines."""
    ky = np.arange(ny) - ny // 2
    return (ky % accel == 0).astype(np.uint8)


def aliased_sets(ny, accel):
    """Row indices of every aliased set: [yr + q Ms for q < R], yr < Ms."""
    ms = ny // accel
    return [np.array([yr + q * ms for q in range(accel)]) for yr in range(ms)]


def set_model(e_c, rows, accel):
    """M_yr [(p, k)][(q, x)] from the compressed readout matrices e_c [Ny][Np][K][Nx]."""
    blocks = [e_c[y].reshape(-1, e_c.shape[3]) for y in rows]
    return np.concatenate(blocks, axis=1) / np.sqrt(accel)


def set_data(s_prime, mask, accel):
    """h [Ms][Np K] = sqrt(R) times the zero-filled inverse DFT at rows yr < Ms."""
    zf = oe.pe_encode_adj(s_prime, mask)  # [Np][K][Ny]
    ms = len(mask) // accel
    return np.sqrt(accel) * np.moveaxis(zf[:, :, :ms], 2, 0).reshape(ms, -1)


def recon(s_prime, e_c, mask, accel, iters):
    """Algorithm #1: inverse DFT along the phase encodes, LSQR per aliased set,
    assembly.  Returns (image [Ny][Nx], residual estimate per iteration summed
    over the sets, sqrt(sum_sets ||r||^2))."""
    ny, nx = e_c.shape[0], e_c.shape[3]
    h = set_data(s_prime, mask, accel)
    img = np.zeros((ny, nx), dtype=np.complex128)
    r2 = np.zeros(iters + 1)
    for yr, rows in enumerate(aliased_sets(ny, accel)):
        m = set_model(e_c, rows, accel)
        x, hist = lsqr(lambda v: m @ v, lambda u: m.conj().T @ u, h[yr], iters)
        img[rows] = x.reshape(accel, nx)
        r2 += hist ** 2
    return img, np.sqrt(r2)
