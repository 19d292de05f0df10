"""Pins of the general-modulation oracle (oracle/explicit.py) against things
other than itself: the Wave special case against the FFT-based operator and
calibration of oracle/encoding.py and oracle/compression.py, the dense signal
equation (Eqs. 1-4), compression of acquired data (Eq. 13), the Gram forms
of Eqs. 7 and 10, RF-only reduction at P = 1, reuse across modulation
periods, and losslessness at full rank."""
import dataclasses

import numpy as np
import pytest

from oracle import compression as oc
from oracle import encoding as oe
from oracle import explicit as ox
from paper_2601_05418_amd import synth


def small_map_slice(seed=0, n=16, nc=3, os_=2, patch_len=4, k=5, cycles=2, periodic=False):
    return synth.local_b0_slice(seed, n=n, nc=nc, os_=os_, patch_len=patch_len, k=k, accel=2, acs=4,
                                cycles=cycles, phase_max=2.5, periodic=periodic)


def wave_as_map(sl):
    """bmod[t][y][x] = psf[y][t] for every x: the Wave modulation as a map."""
    return np.repeat(sl.psf.T[:, :, None], sl.geom.nx, axis=2)


def test_wave_special_case_matches_fft_operator():
    sl = synth.tiny_slice(0, nx=16, ny=16, nc=3, os_=2, patch_len=4, k=5)
    g = sl.geom
    bmod = wave_as_map(sl)
    x = sl.image
    assert np.allclose(ox.readout_encode(x, sl.coils, bmod), oe.readout_encode(x, sl.coils, sl.psf, g.os),
                       atol=1e-12)
    a, lam = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    a2, lam2 = ox.calibrate(sl.coils, bmod, g.patch_len, g.patch_group, g.n_groups, g.k)
    assert np.allclose(lam, lam2, atol=1e-12)
    assert np.allclose(oc.projectors(a), oc.projectors(a2), atol=1e-10)
    e_c = ox.compressed_matrices(sl.coils, bmod, a, g.patch_group, g.patch_len)
    ref = oe.forward(x, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len)
    assert np.allclose(ox.forward(x, e_c, g.mask), ref, atol=1e-12)
    y = np.random.default_rng(1).standard_normal(ref.shape) + 0j
    assert np.allclose(ox.adjoint(y, e_c, g.mask),
                       oe.adjoint(y, sl.coils, sl.psf, g.mask, g.os, a, g.patch_group, g.patch_len), atol=1e-12)


def test_dense_signal_equation_with_nonlinear_map():
    sl = small_map_slice(n=8, nc=2, os_=2, patch_len=4, k=3)
    g = sl.geom
    # the map really depends on x
    assert np.max(np.abs(np.diff(np.angle(sl.bmod), axis=2))) > 1e-3
    e = ox.dense_encoding(sl.coils, sl.bmod, g.mask)
    s = ox.forward_full(sl.image, sl.coils, sl.bmod, g.mask)
    assert np.allclose(s.reshape(-1), e @ sl.image.reshape(-1), atol=1e-12)


def test_compressed_matrices_compress_the_acquired_data():
    """Eq. 13 on S = E rho equals the stored compressed model E' rho."""
    sl = small_map_slice()
    g = sl.geom
    a, _ = ox.calibrate(sl.coils, sl.bmod, g.patch_len, g.patch_group, g.n_groups, g.k)
    e_c = ox.compressed_matrices(sl.coils, sl.bmod, a, g.patch_group, g.patch_len)
    s = ox.forward_full(sl.image, sl.coils, sl.bmod, g.mask)
    assert np.allclose(ox.forward(sl.image, e_c, g.mask), oc.compress(s, a, g.patch_group, g.patch_len),
                       atol=1e-12)


def test_adjoint_identity():
    sl = small_map_slice()
    g = sl.geom
    rng = np.random.default_rng(3)
    a = rng.standard_normal((g.n_groups, g.k, g.nc, g.patch_len)) + 1j * rng.standard_normal(
        (g.n_groups, g.k, g.nc, g.patch_len))
    e_c = ox.compressed_matrices(sl.coils, sl.bmod, a, g.patch_group, g.patch_len)
    x = rng.standard_normal((g.ny, g.nx)) + 1j * rng.standard_normal((g.ny, g.nx))
    fx = ox.forward(x, e_c, g.mask)
    y = rng.standard_normal(fx.shape) + 1j * rng.standard_normal(fx.shape)
    assert abs(np.vdot(fx, y) - np.vdot(x, ox.adjoint(y, e_c, g.mask))) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(y)


def test_full_rank_compression_is_lossless():
    sl = small_map_slice(k=12)  # Ns = 3 * 4 = 12
    g = sl.geom
    a, _ = ox.calibrate(sl.coils, sl.bmod, g.patch_len, g.patch_group, g.n_groups, g.ns)
    e_c = ox.compressed_matrices(sl.coils, sl.bmod, a, g.patch_group, g.patch_len)
    x = sl.image
    full = ox.forward_full(x, sl.coils, sl.bmod, g.mask)
    nc, ny, nx = sl.coils.shape
    # E^H E x through the dense matrix
    e = ox.dense_encoding(sl.coils, sl.bmod, g.mask) if g.nx <= 8 else None
    ehe = None
    if e is not None:
        ehe = (e.conj().T @ (e @ x.reshape(-1))).reshape(ny, nx)
    else:
        # adjoint of the uncompressed model: E_y^H per column after the inverse phase-encode DFT
        w = np.zeros((nc, ny, full.shape[2]), complex)
        w[:, oe.sampled_lines(g.mask), :] = full
        w = oe.cidft(w, axis=1)
        ehe = np.stack([np.einsum("ntx,nt->x", np.conj(ox.readout_matrix(sl.coils, sl.bmod, yy)), w[:, yy, :])
                        for yy in range(ny)])
    assert np.allclose(ox.normal(x, e_c, g.mask), ehe, atol=1e-10 * np.abs(ehe).max())


def test_gram_eq7_equals_eq10_and_trace():
    sl = small_map_slice(n=8, nc=2, os_=2, patch_len=4, k=3)
    e = ox.virtual_channels(sl.coils, sl.bmod, 4, 4)
    p7, p10 = oc.gram_pinv(e), oc.gram(e)
    assert np.allclose(p7, p10, atol=1e-12)
    assert abs(np.trace(p10).real - 64) <= 1e-10  # one unit-trace term per pixel


def test_p1_makes_every_group_the_rf_only_gram():
    """With P = 1 the modulation and DFT factors of a patch are one unit
    scalar per pixel and cancel: every P_g is sum c c^H / |c|^2 (Eq. 6 with
    E_RF only), whatever the map."""
    sl = small_map_slice(patch_len=1, k=2)
    rf = oc.gram(sl.coils.reshape(sl.geom.nc, -1))
    for t0 in (0, 5, 17):
        assert np.allclose(oc.gram(ox.virtual_channels(sl.coils, sl.bmod, 1, t0)), rf, atol=1e-12)
    assert ox.groups_legal(sl.bmod, 1, np.zeros(sl.geom.nt, np.int32))


def test_periodic_map_reuses_projectors_and_legality():
    """cycles = 2 over 32 samples: period 16 = 4 patches of 4; patches p and
    p + 4 see the same modulation (Section 2.3), their projectors agree and
    the periodic grouping is legal, the same grouping of a non-periodic map
    is not."""
    sl = small_map_slice(cycles=2)
    g = sl.geom
    proj = []
    for p in (1, 5):
        e = ox.virtual_channels(sl.coils, sl.bmod, g.patch_len, p * g.patch_len)
        a, _ = oc.compression_matrix(oc.gram(e), g.k, g.patch_len)
        proj.append(a.conj().T @ a)
    assert np.allclose(proj[0], proj[1], atol=1e-10)
    pg = synth.periodic_groups(g.n_patches, 4)
    assert ox.groups_legal(sl.bmod, g.patch_len, pg)
    bad = small_map_slice(cycles=3)
    assert not ox.groups_legal(bad.bmod, g.patch_len, pg)
