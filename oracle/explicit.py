"""FP64 oracle: the readout model for a general modulation map k_m(t, x, y)
and its compressed form stored explicitly per phase-encode column.

TEST INFRASTRUCTURE (see the package docstring of ``oracle.encoding``).

Nonlinear B0 fields (a local B0 coil array, Section 3.1; Eqs. 1-3) make the
modulation phase depend on x as well as y, so it no longer factors into a
point-spread function along the readout.  The modulation is the same on
every phase-encode step, so the phase-encode dimension is still Fourier
(Section 2.3): the inverse DFT along the acquired lines leaves, per image
column y, a dense readout model

    E_y[(n, t)][x] = c_n(x, y) exp(-i k_m(t, x, y)) F_Nt[t][x + (Nt - Nx)/2]

and compression stores E'_y = blockdiag_p(A_g(p)) E_y explicitly (Eq. 14,
the compressed readout matrices of Section 5 and Table S2), one
(Np K) x Nx matrix per column.  With k_m independent of x this is the Wave
operator of ``oracle.encoding`` (psf[y][t] = exp(-i k_m(t, y))).

Shapes: bmod [Nt][Ny][Nx] = exp(-i k_m(t, x, y)); E_y [Nc][Nt][Nx];
E' [Ny][Np][K][Nx]; Z [Np][K][Ny]; S' [Np][K][Ms].
"""
from __future__ import annotations

import numpy as np

from . import compression as oc
from . import encoding as oe


def readout_dft(nt: int, nx: int) -> np.ndarray:
    """F[t][ix] = exp(-2 pi i (t - Nt/2)(ix - Nx/2) / Nt) / sqrt(Nt): the
    centred Nt-point DFT restricted to the Nx zero-padded input positions."""
    t = np.arange(nt)
    ix = np.arange(nx)
    return np.exp(-2j * np.pi * np.outer(t - nt / 2, ix - nx / 2) / nt) / np.sqrt(nt)


def readout_matrix(coils, bmod, y):
    """E_y [Nc][Nt][Nx] of image column y."""
    nt = bmod.shape[0]
    nx = coils.shape[2]
    return coils[:, y, :][:, None, :] * (bmod[:, y, :] * readout_dft(nt, nx))[None, :, :]


def readout_encode(image, coils, bmod):
    """W [Nc][Ny][Nt] with W[n][y] = E_y[n] image[y]."""
    nc, ny, nx = coils.shape
    nt = bmod.shape[0]
    w = np.empty((nc, ny, nt), dtype=np.complex128)
    for y in range(ny):
        w[:, y, :] = readout_matrix(coils, bmod, y) @ image[y]
    return w


def forward_full(image, coils, bmod, mask):
    """Uncompressed E: S [Nc][Ms][Nt] (readout model per column, then the
    phase-encode DFT at the acquired lines)."""
    w = readout_encode(image, coils, bmod)
    return oe.cdft(w, axis=1)[:, oe.sampled_lines(mask), :]


def compressed_matrices(coils, bmod, a_bank, patch_group, patch_len):
    """E' [Ny][Np][K][Nx]: E'_y[(p, k)][x] = sum_{n,j} A_g(p)[k][n][j] E_y[n][pP + j][x]."""
    nc, ny, nx = coils.shape
    nt = bmod.shape[0]
    n_p = nt // patch_len
    k = a_bank.shape[1]
    out = np.empty((ny, n_p, k, nx), dtype=np.complex128)
    for y in range(ny):
        e = readout_matrix(coils, bmod, y)
        for p in range(n_p):
            blk = e[:, p * patch_len:(p + 1) * patch_len, :]  # [Nc][P][Nx]
            out[y, p] = np.einsum("knj,njx->kx", a_bank[patch_group[p]], blk)
    return out


def forward(image, e_c, mask):
    """Compressed E' from the stored matrices: Z[p][k][y] = sum_x E'_y[(p,k)][x]
    image[y][x], then the phase-encode DFT (``oracle.encoding.pe_encode``)."""
    z = np.einsum("ypkx,yx->pky", e_c, image)
    return oe.pe_encode(z, mask)


def adjoint(s, e_c, mask):
    z = oe.pe_encode_adj(s, mask)
    return np.einsum("ypkx,pky->yx", np.conj(e_c), z)


def normal(image, e_c, mask):
    return adjoint(forward(image, e_c, mask), e_c, mask)


def virtual_channels(coils, bmod, patch_len, t0):
    """Composite maps of Eq. 6 for the general modulation, [Ns][L]:
    E_g[(n, j)][r] = c_n(r) exp(-i k_m(t0 + j, r)) F[t0 + j][ix]."""
    nc, ny, nx = coils.shape
    nt = bmod.shape[0]
    t = t0 + np.arange(patch_len)
    dft = readout_dft(nt, nx)[t]  # [P][Nx]
    e = coils[:, None, :, :] * bmod[t][None, :, :, :] * dft[None, :, None, :]  # [Nc][P][Ny][Nx]
    return e.reshape(nc * patch_len, ny * nx)


def groups_legal(bmod, patch_len, patch_group, tol=1e-6):
    """One matrix may serve a group if its member patches are encoded alike
    (Section 2.3): their modulation blocks agree within tol.  With P = 1 a
    patch's channels differ from another's only by one unit phase per pixel,
    which cancels in Eq. 7, so every grouping is legal."""
    if patch_len == 1:
        return True
    pg = np.asarray(patch_group)
    for g in range(int(pg.max()) + 1):
        members = np.nonzero(pg == g)[0]
        ref = bmod[members[0] * patch_len:(members[0] + 1) * patch_len]
        for p in members[1:]:
            if np.max(np.abs(bmod[p * patch_len:(p + 1) * patch_len] - ref)) > tol:
                return False
    return True


def calibrate(coils, bmod, patch_len, patch_group, n_groups, k, roi=None, noise_cov=None):
    """Section 2.4 for the general modulation: composite maps (Eq. 6), P_g
    (Eqs. 9-11), eigen-decomposition and selection (Eqs. 8, 12); the Gram,
    eigen and selection steps are ``oracle.compression``'s.
    Returns (A bank [G][K][Nc][P], eigenvalues [G][Ns])."""
    nc = coils.shape[0]
    t = None
    maps = coils
    if noise_cov is not None:
        t = oc.whitening(noise_cov)
        maps = np.einsum("ab,byx->ayx", t, coils)
    banks, eigs = [], []
    for g, p in enumerate(oc.first_members(patch_group, n_groups)):
        e = virtual_channels(maps, bmod, patch_len, p * patch_len)
        a, lam = oc.compression_matrix(oc.gram(e, roi), k, patch_len, t)
        banks.append(a.reshape(k, nc, patch_len))
        eigs.append(lam)
    return np.stack(banks), np.stack(eigs)


def dense_encoding(coils, bmod, mask):
    """E entry by entry from the discretised signal equation (Eqs. 1-4) for
    tiny inputs: row (n, m, t), column (iy, ix),
        c_n(r) exp(-i [k(t) . r + k_m(t, r)]) / sqrt(Nt Ny)
    with k(t) . r = 2 pi [(t - Nt/2)(ix - Nx/2)/Nt + (l_m - Ny/2)(iy - Ny/2)/Ny]
    and exp(-i k_m(t, r)) = bmod[t][iy][ix]."""
    nc, ny, nx = coils.shape
    nt = bmod.shape[0]
    lines = oe.sampled_lines(mask)
    e = np.zeros((nc, len(lines), nt, ny, nx), dtype=np.complex128)
    for n in range(nc):
        for m, lm in enumerate(lines):
            for t in range(nt):
                for iy in range(ny):
                    for ix in range(nx):
                        ph = 2 * np.pi * ((t - nt / 2) * (ix - nx / 2) / nt + (lm - ny / 2) * (iy - ny / 2) / ny)
                        e[n, m, t, iy, ix] = coils[n, iy, ix] * np.exp(-1j * ph) * bmod[t, iy, ix]
    return e.reshape(nc * len(lines) * nt, ny * nx) / np.sqrt(nt * ny)
