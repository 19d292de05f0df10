"""Seeded synthetic inputs for the Wave / joint-compression workloads.

This module only draws inputs: phantoms, coil maps, Wave point-spread
functions, phase-encode masks, patch-to-group maps and unit noise.  It holds
none of the method's arithmetic (no encoding, no Gram, no eigen-solve), so the
CPU oracle and the HIP path can both be fed from it without sharing code.

The in-vivo and ex-vivo scans of the paper (Section 3.2, Data Availability)
are not available; these draws stand in for their shapes: 2D matrices
64-256, 8-32 coils, readout oversampling 4-8 (paper: 8, Section 3.2),
patches of 16-48 samples (paper: 5-16, Section 3.3) and joint compression
factors 11-20 (paper: 11-24, Abstract).

Coordinates (shared convention): pixel (iy, ix) sits at x = (ix - Nx/2)/Nx,
y = (iy - Ny/2)/Ny in field-of-view units; phase-encode line i has k-space
coordinate i - Ny/2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Child-stream indices of every configuration's SeedSequence.
_PHANTOM, _COILS, _B1, _NOISE, _DRAWS, _PROBE = range(6)


def _streams(config_id: int, seed: int = 0):
    ss = np.random.SeedSequence([5418, int(config_id), int(seed)])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(6)]


@dataclasses.dataclass
class Geometry:
    """Sizes of one 2D slice and its compression partition.

    nt = os * nx readout samples per line; the readout is cut into
    np_ = nt // patch_len patches, patch p belongs to group patch_group[p].
    """

    nx: int
    ny: int
    nc: int
    os: int
    patch_len: int
    patch_group: np.ndarray  # int32 [nt // patch_len]
    n_groups: int
    k: int
    mask: np.ndarray  # uint8 [ny]

    @property
    def nt(self) -> int:
        return self.os * self.nx

    @property
    def n_patches(self) -> int:
        return self.nt // self.patch_len

    @property
    def ns(self) -> int:
        return self.nc * self.patch_len

    @property
    def lines(self) -> np.ndarray:
        return np.nonzero(self.mask)[0].astype(np.int32)

    @property
    def ms(self) -> int:
        return int(self.mask.sum())


@dataclasses.dataclass
class Slice:
    geom: Geometry
    image: np.ndarray  # complex128 [ny][nx]
    coils: np.ndarray  # complex128 [nc][ny][nx]
    psf: np.ndarray  # complex128 [ny][nt]
    noise: Optional[np.ndarray]  # complex128 [nc][ms][nt] unit-variance, or None
    snr: Optional[float]
    wave_cycles: int
    wave_phase: float


def grid(nx: int, ny: int):
    """Pixel centres in field-of-view units, arrays of shape [ny][nx]."""
    x = (np.arange(nx) - nx / 2) / nx
    y = (np.arange(ny) - ny / 2) / ny
    return np.meshgrid(x, y)  # X[iy][ix], Y[iy][ix]


def ellipse_phantom(nx: int, ny: int, rng: np.random.Generator, n_ellipses: int = 6) -> np.ndarray:
    """Painter's-order sum of filled ellipses with random complex values.

    Centres U(-0.35, 0.35), semi-axes U(0.05, 0.3) (FOV units), rotation
    U(0, pi), magnitude U(0.2, 1), phase U(-pi, pi).  Later ellipses
    overwrite earlier ones.
    """
    X, Y = grid(nx, ny)
    img = np.zeros((ny, nx), dtype=np.complex128)
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.35, 0.35, size=2)
        a, b = rng.uniform(0.05, 0.3, size=2)
        th = rng.uniform(0.0, np.pi)
        mag = rng.uniform(0.2, 1.0)
        ph = rng.uniform(-np.pi, np.pi)
        xr = (X - cx) * np.cos(th) + (Y - cy) * np.sin(th)
        yr = -(X - cx) * np.sin(th) + (Y - cy) * np.cos(th)
        inside = (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
        img[inside] = mag * np.exp(1j * ph)
    return img


def gaussian_coils(nx: int, ny: int, nc: int, rng: np.random.Generator,
                   b1_rng: Optional[np.random.Generator] = None,
                   sigma: float = 0.4, radius: float = 0.6) -> np.ndarray:
    """Receive maps: Gaussian bumps on a circle, each with a random linear phase.

    c_n(r) = exp(-|r - r_n|^2 / (2 sigma^2)) exp(i (a_n x + b_n y + phi_n)),
    r_n at angle 2 pi n / nc on a circle of the given radius, a_n, b_n,
    phi_n ~ U(-pi, pi).  With b1_rng, each coil also gets a smooth B1 phase:
    a second-order polynomial in (x, y) with N(0, 1) coefficients.
    """
    X, Y = grid(nx, ny)
    coils = np.empty((nc, ny, nx), dtype=np.complex128)
    for n in range(nc):
        ang = 2.0 * np.pi * n / nc
        cx, cy = radius * np.cos(ang), radius * np.sin(ang)
        a, b, phi = rng.uniform(-np.pi, np.pi, size=3)
        mag = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma ** 2))
        phase = a * X + b * Y + phi
        if b1_rng is not None:
            q = b1_rng.standard_normal(5)
            phase = phase + q[0] * X + q[1] * Y + q[2] * X * X + q[3] * X * Y + q[4] * Y * Y
        coils[n] = mag * np.exp(1j * phase)
    return coils


def wave_psf(ny: int, nt: int, cycles: int, phase_max: float) -> np.ndarray:
    """Sinusoidal-G_y Wave point-spread function, [ny][nt].

    PSF(iy, t) = exp(-i phase_max ((iy - ny/2)/(ny/2)) sin(2 pi cycles t / nt)),
    i.e. a phase excursion of +-phase_max at the field-of-view edge, following
    the exp(-i k_m) form of the modulation term in Eq. 1.
    """
    yy = (np.arange(ny) - ny / 2) / (ny / 2)
    t = np.arange(nt)
    return np.exp(-1j * phase_max * yy[:, None] * np.sin(2.0 * np.pi * cycles * t / nt)[None, :])


def local_b0_modulation(nx: int, ny: int, nt: int, rng: np.random.Generator, n_b0: int = 8,
                        cycles: int = 4, phase_max: float = 6.0, sigma: float = 0.35,
                        radius: float = 0.75) -> np.ndarray:
    """exp(-i k_m(t, x, y)), [nt][ny][nx], for an array of n_b0 local B0 coils
    driven with sinusoidal currents (Eqs. 2-3: k_m = sum_l B_l(r) int I_l):

        k_m(t, r) = sum_l a_l B_l(r) sin(2 pi cycles t / nt + phi_l),

    B_l a Gaussian bump (sigma in FOV units) centred on a circle of the given
    radius (the coils sit around the object), a_l ~ U(0.5, 1) * phase_max,
    phi_l ~ U(0, 2 pi).  The field is nonlinear in x and y, so the phase does
    not factor into a readout point-spread function.  Periodic in t with
    period nt / cycles."""
    X, Y = grid(nx, ny)
    t = np.arange(nt)
    km = np.zeros((nt, ny, nx))
    for lam in range(n_b0):
        ang = 2.0 * np.pi * lam / n_b0
        cx, cy = radius * np.cos(ang), radius * np.sin(ang)
        amp = rng.uniform(0.5, 1.0) * phase_max
        phi = rng.uniform(0.0, 2.0 * np.pi)
        field = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma ** 2))
        km += amp * field[None] * np.sin(2.0 * np.pi * cycles * t / nt + phi)[:, None, None]
    return np.exp(-1j * km)


def pe_mask(ny: int, accel: int, acs: int) -> np.ndarray:
    """Regular phase-encode undersampling plus a centred calibration block.

    Line i (k coordinate ky = i - ny/2) is kept if ky % accel == 0 or
    -acs/2 <= ky < acs/2.
    """
    ky = np.arange(ny) - ny // 2
    m = (ky % accel == 0) | ((ky >= -(acs // 2)) & (ky < acs // 2))
    return m.astype(np.uint8)


def poisson_disc_mask(ny: int, accel: float, rng: np.random.Generator, center: int = 8,
                      density_power: float = 2.0, max_tries: int = 2000) -> np.ndarray:
    """Variable-density Poisson-disc phase-encode mask [ny] (the PD-VD
    undersampling of Section 3.4, here drawn by the project rather than by an
    external tool): the `center` lines around ky = 0 are always acquired;
    further lines are accepted in random order (dart throwing) if no acquired
    line lies within r(ky) = r0 (1 + |ky| / (ny/2))^density_power, and r0 is
    set by bisection so that about ny / accel lines are acquired."""
    ky = np.arange(ny) - ny // 2
    target = max(center, int(round(ny / accel)))

    def draw(r0, seed_rng):
        m = np.zeros(ny, bool)
        m[np.abs(ky + 0.5) < center / 2] = True
        order = seed_rng.permutation(ny)
        radius = r0 * (1.0 + np.abs(ky) / (ny / 2)) ** density_power
        for i in order:
            if m[i]:
                continue
            lo, hi = int(np.floor(i - radius[i])), int(np.ceil(i + radius[i]))
            near = np.nonzero(m[max(0, lo):min(ny, hi + 1)])[0] + max(0, lo)
            if np.all(np.abs(near - i) >= radius[i]):
                m[i] = True
        return m

    state = rng.bit_generator.state
    lo, hi = 0.0, float(ny)
    best = None
    for _ in range(40):
        r0 = 0.5 * (lo + hi)
        rng.bit_generator.state = state
        m = draw(r0, rng)
        if best is None or abs(int(m.sum()) - target) < abs(int(best.sum()) - target):
            best = m
        if m.sum() > target:
            lo = r0
        else:
            hi = r0
    return best.astype(np.uint8)


def wave_caipi_psf(ny: int, nz: int, nt: int, cycles: int, phase_y: float, phase_z: float) -> np.ndarray:
    """3D Wave-CAIPI point-spread function [nz][ny][nt]: sinusoidal G_y and
    cosinusoidal G_z (a corkscrew k-space trajectory),
        exp(-i [phase_y yn sin(2 pi c t / nt) + phase_z zn cos(2 pi c t / nt)]),
    yn = (iy - ny/2)/(ny/2), zn = (iz - nz/2)/(nz/2)."""
    yn = (np.arange(ny) - ny / 2) / (ny / 2)
    zn = (np.arange(nz) - nz / 2) / (nz / 2)
    t = 2.0 * np.pi * cycles * np.arange(nt) / nt
    ph = phase_y * yn[None, :, None] * np.sin(t)[None, None, :] + phase_z * zn[:, None, None] * np.cos(t)[None, None, :]
    return np.exp(-1j * ph)


def caipi_mask(ny: int, nz: int, ry: int, rz: int, shift: int, acs: int = 0) -> np.ndarray:
    """2D CAIPIRINHA phase-encode mask [nz][ny]: point (kz, ky), with
    centred coordinates ky - ny/2 = ry a, acquired when
    (kz - nz/2 - shift a) is divisible by rz; plus an acs x acs centre block."""
    ky = np.arange(ny) - ny // 2
    kz = np.arange(nz) - nz // 2
    m = np.zeros((nz, ny), bool)
    for iy, y in enumerate(ky):
        if y % ry:
            continue
        a = y // ry
        m[:, iy] = (kz - shift * a) % rz == 0
    if acs:
        cz = np.abs(kz + 0.5) < acs / 2
        cy = np.abs(ky + 0.5) < acs / 2
        m[np.ix_(cz, cy)] = True
    return m.astype(np.uint8)


@dataclasses.dataclass
class Volume:
    """A 3D volume: geom.ny is the in-plane phase-encode size, nz the second
    phase-encode size; geom.mask is unused (mask2 [nz][ny] holds the points)."""
    geom: Geometry
    nz: int
    mask2: np.ndarray  # uint8 [nz][ny]
    image: np.ndarray  # complex128 [nz][ny][nx]
    coils: np.ndarray  # complex128 [nc][nz][ny][nx]
    psf: np.ndarray  # complex128 [nz][ny][nt]

    @property
    def ms(self) -> int:
        return int(self.mask2.sum())


def volume(seed: int = 0, n: int = 32, nz: int = 16, nc: int = 4, os_: int = 4, patch_len: int = 16, k: int = 12,
           ry: int = 2, rz: int = 2, shift: int = 1, acs: int = 0, cycles: int = 4, phase: float = 3.0,
           periodic: bool = False) -> Volume:
    """A seeded 3D Wave-CAIPI volume: n x n x nz, nc coils (3D Gaussian bumps:
    the 2D maps of each slice scaled by a bump along z), os-fold readout, a
    corkscrew PSF, an ry x rz CAIPI mask with the given shift.  The phantom is
    ellipsoidal: the 2D ellipses scaled by a z-profile per ellipse."""
    rs = _streams(7, seed)
    nt = os_ * n
    np_ = nt // patch_len
    pg = periodic_groups(np_, (nt // cycles) // patch_len) if periodic else sequential_groups(np_)
    geom = Geometry(nx=n, ny=n, nc=nc, os=os_, patch_len=patch_len, patch_group=pg.astype(np.int32),
                    n_groups=int(pg.max()) + 1, k=k, mask=np.ones(n, np.uint8))
    zc = (np.arange(nz) - nz / 2) / nz
    img = np.zeros((nz, n, n), complex)
    for e in range(4):
        sl = ellipse_phantom(n, n, rs[_PHANTOM], n_ellipses=2)
        z0, zr = rs[_PHANTOM].uniform(-0.2, 0.2), rs[_PHANTOM].uniform(0.15, 0.4)
        prof = (np.abs(zc - z0) <= zr).astype(float)
        img = np.where(np.abs(sl)[None] > 0, sl[None] * prof[:, None, None], img)
    c2 = gaussian_coils(n, n, nc, rs[_COILS])
    zoff = rs[_B1].uniform(-0.3, 0.3, size=nc)
    coils = c2[:, None] * np.exp(-((zc[None, :] - zoff[:, None]) ** 2) / (2 * 0.5 ** 2))[:, :, None, None]
    psf = wave_caipi_psf(n, nz, nt, cycles, phase, phase)
    return Volume(geom, nz, caipi_mask(n, nz, ry, rz, shift, acs), img, coils, psf)


def sequential_groups(n_patches: int) -> np.ndarray:
    return np.arange(n_patches, dtype=np.int32)


def periodic_groups(n_patches: int, patches_per_period: int) -> np.ndarray:
    return (np.arange(n_patches) % patches_per_period).astype(np.int32)


def unit_noise(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex normal draws with unit total variance (1/2 per component)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def scaled_noise(signal: np.ndarray, unit: np.ndarray, snr: float) -> np.ndarray:
    """unit * sigma with sigma = rms(signal) / snr (linear SNR)."""
    sigma = math.sqrt(float(np.mean(np.abs(signal) ** 2))) / snr
    return unit * sigma


# ----------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------

def _make(config_id, seed, n, nc, os_, cycles, phase_max, patch_len, k, accel, acs,
          b1=False, snr=None, groups=None):
    rs = _streams(config_id, seed)
    nt = os_ * n
    np_ = nt // patch_len
    pg = sequential_groups(np_) if groups is None else groups
    geom = Geometry(nx=n, ny=n, nc=nc, os=os_, patch_len=patch_len,
                    patch_group=pg.astype(np.int32), n_groups=int(pg.max()) + 1, k=k,
                    mask=pe_mask(n, accel, acs))
    image = ellipse_phantom(n, n, rs[_PHANTOM])
    coils = gaussian_coils(n, n, nc, rs[_COILS], rs[_B1] if b1 else None)
    psf = wave_psf(n, nt, cycles, phase_max)
    noise = unit_noise((nc, geom.ms, nt), rs[_NOISE]) if snr is not None else None
    return Slice(geom, image, coils, psf, noise, snr, cycles, phase_max)


def small_slice(seed: int = 0) -> Slice:
    """64x64, 8 coils, os 4, wave 5 cycles / +-3 rad, 16 patches of 16, K = 11,
    R = 3 with 8 calibration lines, noise-free."""
    return _make(1, seed, 64, 8, 4, 5, 3.0, 16, 11, 3, 8)


def highfield_slice(seed: int = 0, periodic: bool = False) -> Slice:
    """224x224, 32 coils with B1 phase, os 6 (1344 samples), wave 7 cycles /
    +-6 rad, 42 patches of 32 samples (1024 virtual channels each), K = 64,
    R = 4 with 16 calibration lines, noise at linear SNR 30.

    periodic=True maps the 42 patches onto the 6 patches of one wave period
    (period 192 samples)."""
    groups = periodic_groups(42, 6) if periodic else None
    return _make(2, seed, 224, 32, 6, 7, 6.0, 32, 64, 4, 16, b1=True, snr=30.0, groups=groups)


def unrolled_slices(batch: int = 8, seed: int = 0) -> List[Slice]:
    """256x256, 32 coils, os 8 (2048 samples), wave 8 cycles / +-6 rad, 64
    patches of 32, K = 80, R = 4 without calibration lines; ``batch`` phantoms
    sharing one geometry and one set of coil maps."""
    base = _make(5, seed, 256, 32, 8, 8, 6.0, 32, 80, 4, 0)
    out = [base]
    for b in range(1, batch):
        rs = _streams(5, seed * 1000 + b)
        out.append(dataclasses.replace(base, image=ellipse_phantom(256, 256, rs[_PHANTOM])))
    return out


def batch_draws(n_slices: int = 64, seed: int = 0) -> List[Slice]:
    """Uneven slices: N in {128..256 step 32}, Nc in {16, 24, 32}, os 6 or 8,
    patch length any divisor of nt in [16, 48] with 16-96 patches, K such
    that the compression factor is U(12, 20), R in {3, 4, 5} with 8
    calibration lines, wave 7 cycles / +-6 rad, one group per patch."""
    rs = _streams(4, seed)
    draw = rs[_DRAWS]
    out = []
    for i in range(n_slices):
        n = int(draw.choice([128, 160, 192, 224, 256]))
        nc = int(draw.choice([16, 24, 32]))
        os_ = int(draw.choice([6, 8]))
        nt = os_ * n
        cands = [p for p in range(16, 49) if nt % p == 0 and 16 <= nt // p <= 96]
        p = int(draw.choice(cands))
        f = float(draw.uniform(12.0, 20.0))
        k = max(1, int(round(nc * p / f)))
        r = int(draw.choice([3, 4, 5]))
        out.append(_make(4, seed * 1000 + i + 1, n, nc, os_, 7, 6.0, p, k, r, 8))
    return out


@dataclasses.dataclass
class MapSlice:
    """A slice encoded with a general modulation map (no readout PSF)."""
    geom: Geometry
    image: np.ndarray  # complex128 [ny][nx]
    coils: np.ndarray  # complex128 [nc][ny][nx]
    bmod: np.ndarray  # complex128 [nt][ny][nx] = exp(-i k_m(t, x, y))
    noise: Optional[np.ndarray]
    snr: Optional[float]


def local_b0_slice(seed: int = 0, n: int = 128, nc: int = 16, os_: int = 4, patch_len: int = 16, k: int = 16,
                   accel: int = 3, acs: int = 8, cycles: int = 4, phase_max: float = 6.0, periodic: bool = False,
                   snr: Optional[float] = None) -> MapSlice:
    """Local-B0-array slice (Section 3.1): n x n, nc receive coils, os-fold
    readout oversampling, an 8-coil local B0 array with `cycles` periods per
    readout and +-phase_max rad, patches of patch_len samples, K kept per
    group (default 16 of 256 virtual channels: 16x), R = accel with acs
    calibration lines.  periodic=True maps the patches onto those of one
    modulation period (nt / cycles samples)."""
    rs = _streams(6, seed)
    nt = os_ * n
    np_ = nt // patch_len
    per = nt // cycles
    pg = periodic_groups(np_, per // patch_len) if periodic else sequential_groups(np_)
    geom = Geometry(nx=n, ny=n, nc=nc, os=os_, patch_len=patch_len, patch_group=pg.astype(np.int32),
                    n_groups=int(pg.max()) + 1, k=k, mask=pe_mask(n, accel, acs))
    image = ellipse_phantom(n, n, rs[_PHANTOM])
    coils = gaussian_coils(n, n, nc, rs[_COILS], rs[_B1])
    bmod = local_b0_modulation(n, n, nt, rs[_DRAWS], cycles=cycles, phase_max=phase_max)
    noise = unit_noise((nc, geom.ms, nt), rs[_NOISE]) if snr is not None else None
    return MapSlice(geom, image, coils, bmod, noise, snr)


def tiny_slice(seed: int = 0, nx: int = 8, ny: int = 8, nc: int = 2, os_: int = 2,
               patch_len: int = 4, k: int = 3, accel: int = 2, acs: int = 2,
               cycles: int = 2, phase_max: float = 1.5) -> Slice:
    """A tiny slice for brute-force checks (dense matrices, per-pixel pinv)."""
    return _make(100, seed, nx, nc, os_, cycles, phase_max, patch_len, k, accel, acs) \
        if nx == ny else _make_rect(seed, nx, ny, nc, os_, patch_len, k, accel, acs, cycles, phase_max)


def _make_rect(seed, nx, ny, nc, os_, patch_len, k, accel, acs, cycles, phase_max):
    rs = _streams(101, seed)
    nt = os_ * nx
    np_ = nt // patch_len
    geom = Geometry(nx=nx, ny=ny, nc=nc, os=os_, patch_len=patch_len,
                    patch_group=sequential_groups(np_), n_groups=np_, k=k,
                    mask=pe_mask(ny, accel, acs))
    return Slice(geom, ellipse_phantom(nx, ny, rs[_PHANTOM]),
                 gaussian_coils(nx, ny, nc, rs[_COILS]), wave_psf(ny, nt, cycles, phase_max),
                 None, None, cycles, phase_max)


def orthonormal_bank(n_groups: int, k: int, nc: int, patch_len: int, rng: np.random.Generator) -> np.ndarray:
    """A random bank [G][K][nc][P] with orthonormal rows, cheap at any size:
    row r of group g is a distinct Fourier row of length Ns = nc P (random
    choice of frequencies) times random unit phases on both sides.  For
    workloads whose cost, not content, is measured."""
    ns = nc * patch_len
    j = np.arange(ns)
    out = np.empty((n_groups, k, ns), np.complex128)
    for g in range(n_groups):
        freq = rng.choice(ns, size=k, replace=False)
        row_ph = np.exp(2j * np.pi * rng.random(k))
        col_ph = np.exp(2j * np.pi * rng.random(ns))
        out[g] = row_ph[:, None] * np.exp(-2j * np.pi * np.outer(freq, j) / ns) * col_ph[None, :] / np.sqrt(ns)
    return out.reshape(n_groups, k, nc, patch_len)

