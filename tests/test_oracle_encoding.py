"""Pins for the oracle's encoding operator (CPU only).

Each check compares the oracle with something other than itself: the signal
equation written out entry by entry (Eqs. 1, 4), closed forms of special
cases, and the adjoint identity.
"""
import numpy as np
import pytest

from oracle import compression as oc
from oracle import encoding as oe
from paper_2601_05418_amd import synth

RNG = np.random.default_rng(11)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


@pytest.mark.parametrize("nx,ny,os_", [(8, 8, 2), (8, 6, 2), (6, 8, 3)])
def test_fft_form_equals_signal_equation(nx, ny, os_):
    """Hybrid FFT factorisation (Section 2.3) == E built entry by entry from
    the discretised signal model (Eqs. 1, 4)."""
    sl = synth.tiny_slice(nx=nx, ny=ny, os_=os_, patch_len=2, k=2)
    g = sl.geom
    e = oe.dense_encoding(sl.coils, sl.psf, g.mask, g.os)
    x = crandn(ny, nx)
    s = oe.forward_full(x, sl.coils, sl.psf, g.mask, g.os)
    assert np.max(np.abs(s.reshape(-1) - e @ x.reshape(-1))) <= 1e-13 * np.max(np.abs(s))
    y = crandn(*s.shape)
    xa = oe.adjoint_full(y, sl.coils, sl.psf, g.mask, g.os)
    assert np.max(np.abs(xa.reshape(-1) - e.conj().T @ y.reshape(-1))) <= 1e-12 * np.max(np.abs(xa))


def test_cartesian_sense_reduction():
    """PSF = 1, os = 1, all lines: E is coil weighting followed by a centred
    2D FFT (textbook Cartesian SENSE)."""
    nx, ny, nc = 12, 10, 3
    coils = crandn(nc, ny, nx)
    x = crandn(ny, nx)
    psf = np.ones((ny, nx))
    mask = np.ones(ny, np.uint8)
    s = oe.forward_full(x, coils, psf, mask, 1)  # [Nc][Ny][Nx]
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(coils * x, axes=(1, 2))), axes=(1, 2))
    ref /= np.sqrt(nx * ny)
    assert np.allclose(s, ref, rtol=0, atol=1e-12)


def test_oversampling_without_modulation_adds_nothing():
    """Section 2.2: without modulation an oversampled readout only widens the
    readout FOV; every os-th sample around the centre is the unoversampled
    spectrum scaled by 1/sqrt(os)."""
    nx, ny, nc, os_ = 8, 6, 2, 4
    coils = crandn(nc, ny, nx)
    x = crandn(ny, nx)
    mask = np.ones(ny, np.uint8)
    s1 = oe.forward_full(x, coils, np.ones((ny, nx)), mask, 1)
    s4 = oe.forward_full(x, coils, np.ones((ny, os_ * nx)), mask, os_)
    nt = os_ * nx
    t = nt // 2 + os_ * (np.arange(nx) - nx // 2)
    assert np.allclose(s4[:, :, t], s1 / np.sqrt(os_), atol=1e-12)


def test_normal_closed_form_full_sampling():
    """All lines and a unit-modulus PSF: E^H E = diag(sum_n |c_n|^2)."""
    nx, ny, nc, os_ = 8, 8, 3, 3
    coils = crandn(nc, ny, nx)
    psf = np.exp(1j * RNG.uniform(-np.pi, np.pi, (ny, os_ * nx)))
    x = crandn(ny, nx)
    out = oe.normal_full(x, coils, psf, np.ones(ny, np.uint8), os_)
    assert np.allclose(out, np.sum(np.abs(coils) ** 2, 0) * x, atol=1e-12)


def test_single_unit_coil_is_unitary():
    nx, ny, os_ = 8, 6, 2
    coils = np.ones((1, ny, nx))
    psf = np.exp(1j * RNG.uniform(-np.pi, np.pi, (ny, os_ * nx)))
    x = crandn(ny, nx)
    out = oe.normal_full(x, coils, psf, np.ones(ny, np.uint8), os_)
    assert np.allclose(out, x, atol=1e-13)


@pytest.mark.parametrize("compressed", [False, True])
def test_adjoint_identity(compressed):
    sl = synth.tiny_slice(nx=16, ny=8, os_=2, nc=3, patch_len=4, k=5)
    g = sl.geom
    x = crandn(g.ny, g.nx)
    if compressed:
        a = crandn(g.n_groups, g.k, g.nc, g.patch_len)
        fwd = oe.forward(x, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
        y = crandn(*fwd.shape)
        adj = oe.adjoint(y, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    else:
        fwd = oe.forward_full(x, sl.coils, sl.psf, g.mask, g.os)
        y = crandn(*fwd.shape)
        adj = oe.adjoint_full(y, sl.coils, sl.psf, g.mask, g.os)
    lhs = np.vdot(fwd, y)
    rhs = np.vdot(x, adj)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_compressed_dense_matches_group_sum():
    """E' rows are A_g times the rows of E of the patch (Eq. 14), with E from
    the entry-by-entry signal equation."""
    sl = synth.tiny_slice(nx=8, ny=8, os_=2, nc=2, patch_len=4, k=3)
    g = sl.geom
    a = crandn(g.n_groups, g.k, g.nc, g.patch_len)
    e = oe.dense_encoding(sl.coils, sl.psf, g.mask, g.os).reshape(g.nc, g.ms, g.nt, -1)
    x = crandn(g.ny, g.nx)
    ex = e @ x.reshape(-1)  # [Nc][Ms][Nt]
    ref = np.empty((g.n_patches, g.k, g.ms), complex)
    for p in range(g.n_patches):
        blk = ex[:, :, p * g.patch_len:(p + 1) * g.patch_len]  # [Nc][Ms][P]
        ref[p] = np.einsum("knj,nmj->km", a[g.patch_group[p]], blk)
    out = oe.forward(x, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    assert np.allclose(out, ref, atol=1e-12)


def test_full_rank_compression_is_lossless():
    """K = Ns with the calibrated (unitary) A_g: E'^H E' = E^H E."""
    sl = synth.tiny_slice(nx=8, ny=8, os_=2, nc=2, patch_len=4, k=8)
    g = sl.geom
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.ns)
    x = crandn(g.ny, g.nx)
    lhs = oe.normal(x, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    rhs = oe.normal_full(x, sl.coils, sl.psf, g.mask, g.os)
    assert np.allclose(lhs, rhs, atol=1e-12)
