"""Pins of the 3D oracle (oracle/volume.py): the dense signal equation with
two phase encodes (Eqs. 1-4) and its conjugate transpose for the
uncompressed adjoint and normal operators, reduction to the 2D operator at Nz = 1, the
adjoint identity, Eq. 13 on acquired data, losslessness at full rank, and
the R-fold point spread of a CAIPI mask."""
import numpy as np

from oracle import compression as oc
from oracle import encoding as oe
from oracle import volume as ov
from paper_2601_05418_amd import synth


def tiny_volume(k=3, ry=2, rz=2, shift=1):
    return synth.volume(0, n=4, nz=4, nc=2, os_=2, patch_len=2, k=k, ry=ry, rz=rz, shift=shift, cycles=1, phase=1.5)


def test_dense_signal_equation_two_phase_encodes():
    v = tiny_volume()
    e = ov.dense_encoding(v.coils, v.psf, v.mask2, v.geom.os)
    s = ov.forward_full(v.image, v.coils, v.psf, v.mask2, v.geom.os)
    assert np.allclose(s.reshape(-1), e @ v.image.reshape(-1), atol=1e-12)


def test_uncompressed_adjoint_and_normal_are_the_dense_ones():
    """E^H and E^H E of the uncompressed volume operator against the
    conjugate transpose of the dense signal equation, entry by entry."""
    v = tiny_volume()
    args = (v.coils, v.psf, v.mask2, v.geom.os)
    e = ov.dense_encoding(*args)
    rng = np.random.default_rng(3)
    s = ov.forward_full(v.image, *args)
    y = rng.standard_normal(s.shape) + 1j * rng.standard_normal(s.shape)
    assert np.allclose(ov.adjoint_full(y, *args).reshape(-1), e.conj().T @ y.reshape(-1), atol=1e-12)
    x = rng.standard_normal(v.image.shape) + 1j * rng.standard_normal(v.image.shape)
    assert np.allclose(ov.normal_full(x, *args).reshape(-1), e.conj().T @ (e @ x.reshape(-1)), atol=1e-11)


def test_single_partition_is_the_2d_operator():
    sl = synth.tiny_slice(0, nx=8, ny=8, nc=2, os_=2, patch_len=4, k=3)
    g = sl.geom
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    mask2 = g.mask[None, :]
    s3 = ov.forward(sl.image[None], sl.coils[:, None], sl.psf[None], mask2, g.os, a, g.patch_group, g.patch_len)
    s2 = oe.forward(sl.image, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    assert np.allclose(s3, s2, atol=1e-12)
    f3 = ov.forward_full(sl.image[None], sl.coils[:, None], sl.psf[None], mask2, g.os)
    assert np.allclose(f3, oe.forward_full(sl.image, sl.coils, sl.psf, g.mask, g.os), atol=1e-12)
    a3h = ov.adjoint_full(f3, sl.coils[:, None], sl.psf[None], mask2, g.os)
    assert np.allclose(a3h[0], oe.adjoint_full(f3, sl.coils, sl.psf, g.mask, g.os), atol=1e-12)
    a3, _ = ov.calibrate(sl.coils[:, None], sl.psf[None], g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    assert np.allclose(oc.projectors(a3), oc.projectors(a), atol=1e-10)


def test_adjoint_identity_and_compression_of_acquired_data():
    v = synth.volume(0, n=8, nz=4, nc=2, os_=2, patch_len=4, k=5, cycles=2)
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(v.image.shape) + 1j * rng.standard_normal(v.image.shape)
    fx = ov.forward(x, v.coils, v.psf, v.mask2, g.os, a, g.patch_group, g.patch_len)
    y = rng.standard_normal(fx.shape) + 1j * rng.standard_normal(fx.shape)
    ahy = ov.adjoint(y, v.coils, v.psf, v.mask2, g.os, a, g.patch_group, g.patch_len)
    assert abs(np.vdot(fx, y) - np.vdot(x, ahy)) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(y)
    s = ov.forward_full(v.image, v.coils, v.psf, v.mask2, g.os)
    assert np.allclose(oc.compress(s, a, g.patch_group, g.patch_len),
                       ov.forward(v.image, v.coils, v.psf, v.mask2, g.os, a, g.patch_group, g.patch_len), atol=1e-12)


def test_full_rank_is_lossless():
    v = synth.volume(0, n=8, nz=4, nc=2, os_=2, patch_len=4, k=8, cycles=2)
    g = v.geom
    a, _ = ov.calibrate(v.coils, v.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.ns)
    args = (v.coils, v.psf, v.mask2, g.os)
    n1 = ov.normal(v.image, *args, a, g.patch_group, g.patch_len)
    s = ov.forward_full(v.image, *args)
    e = ov.dense_encoding(*args)
    n2 = (e.conj().T @ s.reshape(-1)).reshape(v.image.shape)
    assert np.allclose(n1, n2, atol=1e-10 * np.abs(n2).max())


def test_caipi_point_spread_is_r_fold():
    """The zero-filled inverse 2D DFT of a CAIPI mask (no calibration block)
    has exactly R = ry rz nonzero points, each of magnitude Ms / sqrt(N) =
    sqrt(N) / R (unitary DFTs, N = 144): the aliasing that fold-over
    reconstruction separates."""
    for ry, rz, shift in ((2, 2, 1), (3, 2, 1), (2, 3, 1), (2, 2, 0)):
        m = synth.caipi_mask(12, 12, ry, rz, shift)
        r = ry * rz
        assert m.sum() == 144 // r
        psf = ov.pe_encode_adj(np.ones(int(m.sum())), m)
        mag = np.abs(psf)
        nz_pts = mag > 1e-9 * mag.max()
        assert np.sum(nz_pts) == r
        assert np.allclose(mag[nz_pts], 12.0 / r, rtol=1e-12)
