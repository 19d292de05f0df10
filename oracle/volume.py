"""FP64 oracle: 3D volumes with two phase-encode dimensions (Section 3.4: the
phase-encoding dimensions are reconstructed by 2D FFT; Table S2, Figs. 8-9).

TEST INFRASTRUCTURE (see the package docstring of ``oracle.encoding``).

The modulation repeats on every (ky, kz) phase-encode step, so both
phase-encode dimensions stay Fourier and the readout model of each image
column (z, y) is that of the 2D operator: the readout stage, the group
contraction and the calibration act on rows (z, y) exactly as on the rows y
of a 2D slice.  The phase-encode stage is the centred unitary 2D DFT over
(z, y), sampled at the acquired (kz, ky) points of a 2D mask (e.g. CAIPI),
listed in raster order (kz major, ky fastest).

Shapes: image [Nz][Ny][Nx]; coils [Nc][Nz][Ny][Nx]; psf [Nz][Ny][Nt];
mask [Nz][Ny]; Z [Np][K][Nz][Ny]; S' [Np][K][Ms]; S [Nc][Ms][Nt].
"""
from __future__ import annotations

import numpy as np

from . import compression as oc
from . import encoding as oe


def flat(a, lead):
    """Merge the (Nz, Ny) axes that follow `lead` leading axes into one row axis."""
    s = a.shape
    return a.reshape(s[:lead] + (s[lead] * s[lead + 1],) + s[lead + 2:])


def sampled_points(mask):
    """Raster indices (kz * Ny + ky) of the acquired points, ascending."""
    return np.nonzero(np.asarray(mask).reshape(-1))[0]


def pe_encode(z, mask):
    """Centred 2D DFT over the last two axes (z, y), then the acquired points."""
    f = oe.cdft(oe.cdft(z, axis=-1), axis=-2)
    return f.reshape(f.shape[:-2] + (-1,))[..., sampled_points(mask)]


def pe_encode_adj(s, mask):
    nz, ny = mask.shape
    full = np.zeros(s.shape[:-1] + (nz * ny,), dtype=np.complex128)
    full[..., sampled_points(mask)] = s
    full = full.reshape(s.shape[:-1] + (nz, ny))
    return oe.cidft(oe.cidft(full, axis=-1), axis=-2)


def readout_encode(image, coils, psf, os_):
    nz, ny = image.shape[:2]
    w = oe.readout_encode(flat(image, 0), flat(coils, 1), flat(psf, 0), os_)  # [Nc][Nz Ny][Nt]
    return w.reshape(w.shape[0], nz, ny, w.shape[2])


def readout_encode_adj(w, coils, psf, os_):
    nz, ny = coils.shape[1:3]
    img = oe.readout_encode_adj(flat(w, 1), flat(coils, 1), flat(psf, 0), os_)
    return img.reshape(nz, ny, -1)


def forward(image, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    """Compressed E': S' [Np][K][Ms]."""
    w = readout_encode(image, coils, psf, os_)
    nc, nz, ny, nt = w.shape
    z = oe.group_compress(w.reshape(nc, nz * ny, nt), a_bank, patch_group, patch_len)  # [Np][K][Nz Ny]
    return pe_encode(z.reshape(z.shape[0], z.shape[1], nz, ny), mask)


def adjoint(s, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    nc, nz, ny, nx = coils.shape
    z = pe_encode_adj(s, mask)  # [Np][K][Nz][Ny]
    w = oe.group_expand(z.reshape(z.shape[0], z.shape[1], nz * ny), a_bank, patch_group, patch_len, nc,
                        os_ * nx)
    return readout_encode_adj(w.reshape(nc, nz, ny, -1), coils, psf, os_)


def normal(image, coils, psf, mask, os_, a_bank, patch_group, patch_len):
    return adjoint(forward(image, coils, psf, mask, os_, a_bank, patch_group, patch_len), coils, psf, mask, os_,
                   a_bank, patch_group, patch_len)


def forward_full(image, coils, psf, mask, os_):
    """Uncompressed E: S [Nc][Ms][Nt]."""
    w = readout_encode(image, coils, psf, os_)  # [Nc][Nz][Ny][Nt]
    f = oe.cdft(oe.cdft(w, axis=2), axis=1)
    nc, nz, ny, nt = f.shape
    return f.reshape(nc, nz * ny, nt)[:, sampled_points(mask), :]


def adjoint_full(s, coils, psf, mask, os_):
    """Uncompressed E^H: S [Nc][Ms][Nt] -> image [Nz][Ny][Nx].  The acquired
    points are zero-filled into every (coil, sample) plane, each plane goes
    through the inverse centred 2D DFT, then the readout adjoint."""
    nc, ms, nt = s.shape
    nz, ny = mask.shape
    full = np.zeros((nc, nz * ny, nt), dtype=np.complex128)
    full[:, sampled_points(mask), :] = s
    w = oe.cidft(oe.cidft(full.reshape(nc, nz, ny, nt), axis=2), axis=1)
    return readout_encode_adj(w, coils, psf, os_)


def normal_full(image, coils, psf, mask, os_):
    """Uncompressed E^H E."""
    return adjoint_full(forward_full(image, coils, psf, mask, os_), coils, psf, mask, os_)


def calibrate(coils, psf, os_, patch_len, patch_group, n_groups, k, roi=None, noise_cov=None):
    """Section 2.4 over all voxels of the volume: the 2D calibration on the
    (z, y) rows."""
    r = None if roi is None else flat(np.asarray(roi), 0)
    return oc.calibrate(flat(coils, 1), flat(psf, 0), os_, patch_len, patch_group, n_groups, k, roi=r,
                        noise_cov=noise_cov)


def dense_encoding(coils, psf, mask, os_):
    """E entry by entry from the discretised signal equation (Eqs. 1-4) with two
    phase encodes, for tiny inputs: row (n, m, t), column (iz, iy, ix),
        c_n(r) exp(-i [k(t) . r + k_m(t, r)]) / sqrt(Nt Ny Nz)
    with k(t) . r = 2 pi [(t - Nt/2)(ix - Nx/2)/Nt + (ky_m - Ny/2)(iy - Ny/2)/Ny
    + (kz_m - Nz/2)(iz - Nz/2)/Nz] and exp(-i k_m) = psf[iz][iy][t]."""
    nc, nz, ny, nx = coils.shape
    nt = os_ * nx
    pts = sampled_points(mask)
    e = np.zeros((nc, len(pts), nt, nz, ny, nx), dtype=np.complex128)
    for n in range(nc):
        for m, pt in enumerate(pts):
            kz, ky = divmod(int(pt), ny)
            for t in range(nt):
                for iz in range(nz):
                    for iy in range(ny):
                        for ix in range(nx):
                            ph = 2 * np.pi * ((t - nt / 2) * (ix - nx / 2) / nt + (ky - ny / 2) * (iy - ny / 2) / ny
                                              + (kz - nz / 2) * (iz - nz / 2) / nz)
                            e[n, m, t, iz, iy, ix] = coils[n, iz, iy, ix] * np.exp(-1j * ph) * psf[iz, iy, t]
    return e.reshape(nc * len(pts) * nt, nz * ny * nx) / np.sqrt(nt * ny * nz)
