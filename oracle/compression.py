"""FP64 oracle: group-patch joint compression (Section 2.4, Eqs. 6-14).

TEST INFRASTRUCTURE (see the package docstring of ``oracle.encoding``).

For a group g whose first member patch starts at readout sample t0, the
composite encoding vector of pixel r (Eq. 6) stacks, over coils n and patch
samples j (index n * P + j, coil-major):

    E_g[r][(n, j)] = c_n(r) * exp(-i k_m(t0 + j, r)) * DFT(t0 + j, ix)

i.e. coil map (E_RF) x modulation phase (E_NG; the Wave PSF) x the readout
DFT row (E_LG, the "synthesized DFT matrix" of Section 3.3).  P_g sums the
outer products of these vectors with their pseudo-inverses over the ROI
(Eq. 7); Eqs. 9-11 give the same matrix as one weighted matrix product.
"""
from __future__ import annotations

import numpy as np


def virtual_channels(coils, psf, os_, patch_len, t0):
    """Composite encoding maps E_g of Eq. 6 as an [Ns][L] matrix, Ns = Nc P,
    L = Ny Nx (pixel index iy * Nx + ix)."""
    nc, ny, nx = coils.shape
    nt = os_ * nx
    t = t0 + np.arange(patch_len)
    ix = np.arange(nx)
    dft = np.exp(-2j * np.pi * np.outer(t - nt / 2, ix - nx / 2) / nt) / np.sqrt(nt)  # [P][Nx]
    mod = psf[:, t].T  # [P][Ny]
    e = coils[:, None, :, :] * mod[None, :, :, None] * dft[None, :, None, :]  # [Nc][P][Ny][Nx]
    return e.reshape(nc * patch_len, ny * nx)


def gram_pinv(e, roi=None):
    """Eq. 7 literally: sum over ROI pixels of e e^+ with the pseudo-inverse of
    each column vector.  Pixels whose vector is zero are excluded."""
    ns, npix = e.shape
    sel = np.ones(npix, bool) if roi is None else np.asarray(roi, bool).reshape(-1)
    p = np.zeros((ns, ns), dtype=np.complex128)
    for r in range(npix):
        col = e[:, r:r + 1]
        if not sel[r] or not np.any(col):
            continue
        p += col @ np.linalg.pinv(col)
    return p


def gram(e, roi=None):
    """Eqs. 9-11: P_g = (E_g N) E_g^H with N = diag(1 / sum_Ns |E_g|^2).
    Pixels outside the ROI or with a zero vector get weight 0."""
    npix = e.shape[1]
    sel = np.ones(npix, bool) if roi is None else np.asarray(roi, bool).reshape(-1)
    energy = np.sum(np.abs(e) ** 2, axis=0)
    keep = sel & (energy > 0)
    w = np.zeros(npix)
    w[keep] = 1.0 / energy[keep]
    return (e * w[None, :]) @ e.conj().T


def whitening(noise_cov):
    """T = Q^{-1} with Psi = Q Q^H (Cholesky), the noise-decorrelation matrix
    of Eq. 12."""
    q = np.linalg.cholesky(np.asarray(noise_cov, dtype=np.complex128))
    return np.linalg.inv(q)


def compression_matrix(p_g, k, patch_len, t=None):
    """Eqs. 8 and 12: eigen-decompose P_g = U F U^H, order the eigenpairs by
    decreasing eigenvalue, and keep the first K rows of U^H, then apply the
    whitening T (x) I_P on the coil-major joint index.

    Each kept eigenvector is scaled by a unit phase so that its entry of
    largest magnitude (lowest index on ties) is real and positive.
    Returns (A [K][Ns], eigenvalues in decreasing order [Ns])."""
    lam, u = np.linalg.eigh(p_g)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    u = u[:, order]
    for c in range(u.shape[1]):
        i = int(np.argmax(np.abs(u[:, c])))
        u[:, c] *= np.conj(u[i, c]) / np.abs(u[i, c])
    a = u[:, :k].conj().T
    if t is not None:
        a = a @ np.kron(t, np.eye(patch_len))
    return a, lam


def first_members(patch_group, n_groups):
    """First patch of every group (the patch whose maps define P_g)."""
    firsts = []
    for g in range(n_groups):
        members = np.nonzero(np.asarray(patch_group) == g)[0]
        if len(members) == 0:
            raise ValueError(f"group {g} has no patch")
        firsts.append(int(members[0]))
    return firsts


def groups_legal(psf, patch_len, patch_group, tol=1e-6):
    """A group may only reuse one matrix across patches that see the same
    modulation (Section 2.3: the B0 encoding functions are shift-invariant
    across modulation cycles).  True if every member patch's PSF block equals
    the first member's within ``tol``."""
    pg = np.asarray(patch_group)
    for g in range(int(pg.max()) + 1):
        members = np.nonzero(pg == g)[0]
        ref = psf[:, members[0] * patch_len:(members[0] + 1) * patch_len]
        for p in members[1:]:
            blk = psf[:, p * patch_len:(p + 1) * patch_len]
            if np.max(np.abs(blk - ref)) > tol:
                return False
    return True


def calibrate(coils, psf, os_, patch_len, patch_group, n_groups, k, roi=None, noise_cov=None):
    """The calibration steps of Section 2.4 for every group: composite maps
    (Eq. 6, whitened coil maps when a noise covariance is given), P_g
    (Eqs. 9-11), eigen-decomposition and selection (Eqs. 8, 12).

    Returns (A bank [G][K][Nc][P], eigenvalues [G][Ns])."""
    nc = coils.shape[0]
    t = None
    maps = coils
    if noise_cov is not None:
        t = whitening(noise_cov)
        maps = np.einsum("ab,byx->ayx", t, coils)
    banks, eigs = [], []
    for g, p in enumerate(first_members(patch_group, n_groups)):
        e = virtual_channels(maps, psf, os_, patch_len, p * patch_len)
        a, lam = compression_matrix(gram(e, roi), k, patch_len, t)
        banks.append(a.reshape(k, nc, patch_len))
        eigs.append(lam)
    return np.stack(banks), np.stack(eigs)


def compress(s, a_bank, patch_group, patch_len):
    """Eq. 13 on acquired k-space S [Nc][Ms][Nt]:
    S'[p][k][m] = sum_{n,j} A_{g(p)}[k][n][j] S[n][m][p P + j]."""
    nc, ms, nt = s.shape
    n_p = nt // patch_len
    out = np.empty((n_p, a_bank.shape[1], ms), dtype=np.complex128)
    for p in range(n_p):
        out[p] = np.einsum("knj,nmj->km", a_bank[patch_group[p]],
                           s[:, :, p * patch_len:(p + 1) * patch_len])
    return out


def projectors(a_bank):
    """Pi_g = A_g^H A_g [G][Ns][Ns]: the basis-free object the reconstructions
    depend on."""
    g, k = a_bank.shape[:2]
    a = a_bank.reshape(g, k, -1)
    return np.einsum("gki,gkj->gij", a.conj(), a)
