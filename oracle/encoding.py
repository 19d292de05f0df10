"""FP64 oracle: the Wave encoding operator E and its group-compressed form E'.

TEST INFRASTRUCTURE.  This package is a plain, slow CPU reference written from
the paper.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the library never does, and it shares no code with the HIP
path.

Conventions (the paper does not state FFT centring or scaling; the reading
taken here is a centred, unitary DFT):

* readout sample t has k coordinate t - Nt/2, phase-encode line i has
  k coordinate i - Ny/2, pixel (iy, ix) sits at (iy - Ny/2, ix - Nx/2);
* F_N[k, i] = exp(-2 pi i (k - N/2)(i - N/2) / N) / sqrt(N);
* the oversampled readout zero-pads pixel ix to index ix + (Nt - Nx)/2;
* the modulation enters as exp(-i k_m(t, r)) (Eq. 1); for Wave it depends on
  (y, t) only and is stored as psf[iy][t].

Shapes: image [Ny][Nx], coils [Nc][Ny][Nx], psf [Ny][Nt],
W (hybrid readout data) [Nc][Ny][Nt], A bank [G][K][Nc][P],
Z (compressed hybrid data) [Np][K][Ny], S' (compressed k-space) [Np][K][Ms],
S (k-space) [Nc][Ms][Nt].
"""
from __future__ import annotations

import numpy as np


def cdft(x: np.ndarray, axis: int) -> np.ndarray:
    """Centred unitary DFT along ``axis`` (even lengths)."""
    n = x.shape[axis]
    y = np.fft.fft(np.fft.ifftshift(x, axes=axis), axis=axis)
    return np.fft.fftshift(y, axes=axis) / np.sqrt(n)


def cidft(x: np.ndarray, axis: int) -> np.ndarray:
    """Inverse (= conjugate transpose) of :func:`cdft`."""
    n = x.shape[axis]
    y = np.fft.ifft(np.fft.ifftshift(x, axes=axis), axis=axis)
    return np.fft.fftshift(y, axes=axis) * np.sqrt(n)


def sampled_lines(mask: np.ndarray) -> np.ndarray:
    """Indices of the acquired phase-encode lines, ascending."""
    return np.nonzero(np.asarray(mask))[0]


# ----------------------------------------------------------------------------
# The three stages of the hybrid-space Wave model (Section 2.3: the
# phase-encode dimension is handled by FFT, only the readout is non-Fourier;
# Section 3.4 reconstructs the phase-encode dimension by FFT).
# ----------------------------------------------------------------------------

def readout_encode(image, coils, psf, os_):
    """F1: coil weighting, zero-padded oversampled readout DFT, then the
    modulation PSF.  Returns W [Nc][Ny][Nt]."""
    nc, ny, nx = coils.shape
    nt = os_ * nx
    off = (nt - nx) // 2
    padded = np.zeros((nc, ny, nt), dtype=np.complex128)
    padded[:, :, off:off + nx] = coils * image[None]
    return cdft(padded, axis=2) * psf[None]


def readout_encode_adj(w, coils, psf, os_):
    """Adjoint of :func:`readout_encode`: conj PSF, inverse DFT, crop, coil
    combine with conj maps.  Returns image [Ny][Nx]."""
    nc, ny, nx = coils.shape
    nt = os_ * nx
    off = (nt - nx) // 2
    u = cidft(w * np.conj(psf)[None], axis=2)[:, :, off:off + nx]
    return np.sum(np.conj(coils) * u, axis=0)


def group_compress(w, a_bank, patch_group, patch_len):
    """F2: apply each patch's group matrix to the Nc x P virtual channels of
    that patch (Eq. 13 / Eq. 14 applied to hybrid data).
    Z[p][k][y] = sum_{n,j} A_{g(p)}[k][n][j] W[n][y][p P + j]."""
    nc, ny, nt = w.shape
    n_p = nt // patch_len
    k = a_bank.shape[1]
    z = np.empty((n_p, k, ny), dtype=np.complex128)
    for p in range(n_p):
        wp = w[:, :, p * patch_len:(p + 1) * patch_len]
        z[p] = np.einsum("knj,nyj->ky", a_bank[patch_group[p]], wp)
    return z


def group_expand(z, a_bank, patch_group, patch_len, nc, nt):
    """Adjoint of :func:`group_compress`:
    W[n][y][p P + j] = sum_k conj(A_{g(p)}[k][n][j]) Z[p][k][y]."""
    n_p, k, ny = z.shape
    w = np.empty((nc, ny, nt), dtype=np.complex128)
    for p in range(n_p):
        w[:, :, p * patch_len:(p + 1) * patch_len] = np.einsum(
            "knj,ky->nyj", np.conj(a_bank[patch_group[p]]), z[p])
    return w


def pe_encode(z, mask):
    """F3: centred DFT along the phase-encode axis (last axis of ``z``), keep
    the acquired lines."""
    return cdft(z, axis=-1)[..., sampled_lines(mask)]


def pe_encode_adj(s, mask):
    """Adjoint of :func:`pe_encode`: zero-fill the missing lines, inverse DFT."""
    ny = len(mask)
    full = np.zeros(s.shape[:-1] + (ny,), dtype=np.complex128)
    full[..., sampled_lines(mask)] = s
    return cidft(full, axis=-1)


# ----------------------------------------------------------------------------
# Whole operators.  Uncompressed: S = E rho (Eq. 4).  Compressed: S' = E' rho
# (Eq. 15) with E'_g = A_g E_g (Eq. 14).
# ----------------------------------------------------------------------------

def forward_full(image, coils, psf, mask, os_):
    """Uncompressed E: returns S [Nc][Ms][Nt]."""
    w = readout_encode(image, coils, psf, os_)
    return cdft(w, axis=1)[:, sampled_lines(mask), :]


def adjoint_full(s, coils, psf, mask, os_):
    nc, ny, nx = coils.shape
    full = np.zeros((nc, ny, s.shape[2]), dtype=np.complex128)
    full[:, sampled_lines(mask), :] = s
    return readout_encode_adj(cidft(full, axis=1), coils, psf, os_)


def normal_full(image, coils, psf, mask, os_):
    return adjoint_full(forward_full(image, coils, psf, mask, os_), coils, psf, mask, os_)


def forward(image, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    """Compressed E': returns S' [Np][K][Ms]."""
    w = readout_encode(image, coils, psf, os_)
    return pe_encode(group_compress(w, a_bank, patch_group, patch_len), mask)


def adjoint(s, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    nc, ny, nx = coils.shape
    z = pe_encode_adj(s, mask)
    w = group_expand(z, a_bank, patch_group, patch_len, nc, os_ * nx)
    return readout_encode_adj(w, coils, psf, os_)


def normal(image, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    """E'^H E' (the operator inside CG and FISTA)."""
    s = forward(image, coils, psf, mask, os_, a_bank, patch_group, patch_len)
    return adjoint(s, coils, psf, mask, os_, a_bank, patch_group, patch_len)


def dense_encoding(coils, psf, mask, os_):
    """E written out entry by entry from the discretised signal equation
    (Eqs. 1 and 4) for tiny inputs: row (n, m, t), column (iy, ix),

        E = c_n(r) exp(-i [k(t) . r + k_m(t, r)]) / sqrt(Nt Ny)

    with k(t) . r = 2 pi [(t - Nt/2)(ix - Nx/2)/Nt + (l_m - Ny/2)(iy - Ny/2)/Ny]
    for the m-th acquired line l_m and exp(-i k_m) = psf[iy][t]."""
    nc, ny, nx = coils.shape
    nt = os_ * nx
    lines = sampled_lines(mask)
    e = np.zeros((nc, len(lines), nt, ny, nx), dtype=np.complex128)
    for n in range(nc):
        for m, lm in enumerate(lines):
            for t in range(nt):
                for iy in range(ny):
                    for ix in range(nx):
                        ph = 2 * np.pi * ((t - nt / 2) * (ix - nx / 2) / nt
                                          + (lm - ny / 2) * (iy - ny / 2) / ny)
                        e[n, m, t, iy, ix] = coils[n, iy, ix] * np.exp(-1j * ph) * psf[iy, t]
    return e.reshape(nc * len(lines) * nt, ny * nx) / np.sqrt(nt * ny)
