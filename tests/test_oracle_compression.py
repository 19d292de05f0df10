"""Pins for the oracle's calibration and compression (CPU only).

Eq. 7 (per-pixel pseudo-inverse) against Eqs. 9-11, the trace and
positivity of P_g, the Dirichlet-kernel closed form for a single coil
without modulation, the RF-only reduction of Eq. 6 for P = 1, reuse of one
matrix across modulation cycles, the Ky Fan optimality of the kept
subspace, unitarity and whitening of A_g, and Eq. 13 against Eq. 15.
"""
import numpy as np
import pytest

from oracle import compression as oc
from oracle import encoding as oe
from paper_2601_05418_amd import synth

RNG = np.random.default_rng(7)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def tiny():
    return synth.tiny_slice(nx=8, ny=8, os_=2, nc=2, patch_len=4, k=3)


def test_eq7_equals_eq10():
    sl = tiny()
    g = sl.geom
    e = oc.virtual_channels(sl.coils, sl.psf, g.os, g.patch_len, 4)
    roi = RNG.uniform(size=(g.ny, g.nx)) > 0.3
    assert np.allclose(oc.gram_pinv(e, roi), oc.gram(e, roi), atol=1e-12)


def test_virtual_channels_are_rows_of_E():
    """Eq. 6: the composite vectors are the readout block of E (Eq. 4) for one
    acquired line, up to that line's per-pixel unit phase."""
    sl = tiny()
    g = sl.geom
    p0 = 1
    t0 = p0 * g.patch_len
    e = oc.virtual_channels(sl.coils, sl.psf, g.os, g.patch_len, t0)
    mask = np.zeros(g.ny, np.uint8)
    mask[g.ny // 2] = 1  # ky = 0: the phase-encode factor is 1/sqrt(Ny) everywhere
    dense = oe.dense_encoding(sl.coils, sl.psf, mask, g.os).reshape(g.nc, g.nt, -1)
    ref = dense[:, t0:t0 + g.patch_len, :].reshape(g.ns, -1) * np.sqrt(g.ny)
    assert np.allclose(e, ref, atol=1e-13)


def test_gram_trace_hermitian_psd():
    sl = tiny()
    g = sl.geom
    e = oc.virtual_channels(sl.coils, sl.psf, g.os, g.patch_len, 0)
    roi = RNG.uniform(size=(g.ny, g.nx)) > 0.5
    p = oc.gram(e, roi)
    assert abs(np.trace(p) - roi.sum()) < 1e-12
    assert np.allclose(p, p.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(p).min() > -1e-12


def test_dirichlet_closed_form():
    """One coil, no modulation: P[j, j'] = (Ny/P) sum_{x=-Nx/2}^{Nx/2-1}
    exp(-2 pi i (j - j') x / Nt), a Dirichlet kernel, summed here as a
    geometric series."""
    nx, ny, os_, plen = 16, 6, 4, 12
    nt = os_ * nx
    coils = crandn(1, ny, nx)
    e = oc.virtual_channels(coils, np.ones((ny, nt)), os_, plen, 20)
    p = oc.gram(e)
    d = np.subtract.outer(np.arange(plen), np.arange(plen))
    z = np.exp(-2j * np.pi * d / nt)
    with np.errstate(invalid="ignore", divide="ignore"):
        geo = z ** (-nx / 2) * (1 - z ** nx) / (1 - z)
    geo[d == 0] = nx
    assert np.allclose(p, ny / plen * geo, atol=1e-11)
    # Section 2.2: oversampling without modulation adds no information -- the
    # spectrum concentrates in about P/os eigenvalues.
    lam = np.linalg.eigvalsh(p)
    big = int(np.sum(lam > 0.5 * lam.max()))
    assert abs(big - plen // os_) <= 1


def test_p1_reduces_to_rf_only():
    """P = 1: Eq. 6 reduces to the coil maps, so every group's P_g is
    sum_r c c^H / ||c||^2 whatever the modulation."""
    sl = synth.tiny_slice(nx=8, ny=8, os_=2, nc=3, patch_len=1, k=2)
    g = sl.geom
    c = sl.coils.reshape(g.nc, -1)
    ref = (c / np.sum(np.abs(c) ** 2, 0)) @ c.conj().T
    for t0 in (0, 3, 11):
        e = oc.virtual_channels(sl.coils, sl.psf, g.os, 1, t0)
        assert np.allclose(oc.gram(e), ref, atol=1e-12)


def test_periodic_reuse_of_projectors():
    """Sections 2.3-2.4: patches one modulation period apart share P_g."""
    sl = synth.tiny_slice(nx=8, ny=8, os_=2, nc=2, patch_len=4, k=3, cycles=2)
    g = sl.geom  # nt = 16, period 8 = 2 patches
    a, lam = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    pis = oc.projectors(a)
    assert np.allclose(pis[0], pis[2], atol=1e-10)
    assert np.allclose(pis[1], pis[3], atol=1e-10)
    assert not np.allclose(pis[0], pis[1], atol=1e-3)
    assert oc.groups_legal(sl.psf, g.patch_len, synth.periodic_groups(4, 2))
    assert not oc.groups_legal(sl.psf, g.patch_len, np.array([0, 0, 1, 1], np.int32))


def test_eigen_selection_is_optimal():
    """Eqs. 8, 12: rows of A_g are orthonormal, eigenpairs satisfy
    P U = U F in decreasing order, and the kept subspace retains
    sum_{k<K} lambda_k of the normalised pixel energy -- no other K-dim
    subspace retains more (Ky Fan)."""
    sl = tiny()
    g = sl.geom
    e = oc.virtual_channels(sl.coils, sl.psf, g.os, g.patch_len, 0)
    p = oc.gram(e)
    a, lam = oc.compression_matrix(p, g.k, g.patch_len)
    assert np.all(np.diff(lam) <= 1e-12)
    assert np.allclose(a @ a.conj().T, np.eye(g.k), atol=1e-13)
    assert np.allclose(p @ a.conj().T, a.conj().T * lam[:g.k], atol=1e-12 * np.abs(p).max())
    en = e / np.linalg.norm(e, axis=0)
    kept = np.sum(np.abs(a @ en) ** 2)
    assert abs(kept - lam[:g.k].sum()) < 1e-10
    for _ in range(20):
        q, _ = np.linalg.qr(crandn(g.ns, g.k))
        assert np.sum(np.abs(q.conj().T @ en) ** 2) <= kept + 1e-10
    # each kept vector has its largest-magnitude entry real and positive
    for row in a.conj():
        i = np.argmax(np.abs(row))
        assert abs(row[i].imag) < 1e-14 and row[i].real > 0


def test_whitened_channels_have_unit_noise():
    """Eq. 12 with T = Q^{-1}, Psi = Q Q^H: compressed channels carry white
    noise, A_g (Psi x I_P) A_g^H = I."""
    sl = tiny()
    g = sl.geom
    m = crandn(g.nc, g.nc)
    psi = m @ m.conj().T + g.nc * np.eye(g.nc)
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k,
                        noise_cov=psi)
    cov = np.kron(psi, np.eye(g.patch_len))
    for ag in a.reshape(g.n_groups, g.k, -1):
        assert np.allclose(ag @ cov @ ag.conj().T, np.eye(g.k), atol=1e-12)


def test_compress_matches_compressed_forward():
    """Eq. 13 on noise-free data equals Eq. 15: A S = E' rho."""
    sl = synth.tiny_slice(nx=8, ny=8, os_=2, nc=2, patch_len=4, k=3)
    g = sl.geom
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    s = oe.forward_full(sl.image, sl.coils, sl.psf, g.mask, g.os)
    lhs = oc.compress(s, a, g.patch_group, g.patch_len)
    rhs = oe.forward(sl.image, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("kfrac", [0.25, 0.5])
def test_joint_beats_rf_only_at_equal_factor(kfrac):
    """Section 4 (Figs. 7, 10): at one compression factor the joint subspace
    keeps more encoding energy than coil-only compression of the same
    patch."""
    sl = synth.tiny_slice(nx=16, ny=16, os_=4, nc=4, patch_len=8, k=4, cycles=3, phase_max=3.0)
    g = sl.geom
    e = oc.virtual_channels(sl.coils, sl.psf, g.os, g.patch_len, 8)
    en = e / np.linalg.norm(e, axis=0)
    kk = int(g.ns * kfrac)
    lam_joint = np.linalg.eigvalsh(oc.gram(e))[::-1]
    c = sl.coils.reshape(g.nc, -1)
    lam_rf = np.linalg.eigvalsh((c / np.sum(np.abs(c) ** 2, 0)) @ c.conj().T)[::-1]
    kc = kk // g.patch_len
    joint = lam_joint[:kk].sum() / np.sum(np.abs(en) ** 2)
    rf = lam_rf[:kc].sum() / (g.ny * g.nx)
    assert joint > rf
