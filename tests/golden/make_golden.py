"""Writes the stored expected values of the full-size reconstruction tests.

TEST INFRASTRUCTURE.  Calls only the CPU oracle (``oracle/``) and the seeded
input generators; nothing here touches the library.  The results are the
oracle's own FP64 runs, rounded to complex64 for storage:

* ``highfield_fista50.npz`` -- the 224 x 224, 32-coil high-field slice
  (42 groups, K = 64, R = 4 + 16 ACS, SNR 30): oracle calibration (Eqs.
  6-12), compression of the acquired data (Eq. 13), lambda = 1e-3 max |W b|
  with b = E'^H S', L = 1.01 x 50 power iterations from the seeded start,
  then FISTA-50 with 3-level Haar (Section 3.4, Eq. 17); the iterate and
  the objective after every iteration.
* ``batch_largest_cg20.npz`` -- the two largest slices of the 64-slice
  uneven batch (random orthonormal banks and random data, drawn in the same
  order as the batch test), CG-20 on the normal equations (Eq. 16).
* ``unrolled_fd.npz`` -- the unrolled gradient-descent network at full size
  (256 x 256, 32 coils, os 8, 64 groups, K = 80; 10 steps
  x <- x - alpha_k E'^H E' x, i.e. zero data) on image 0: the loss
  1/2 ||x_10 - truth||^2 at x0 +- eps v for a unit direction v, eps = 1e-3,
  and their central difference, in FP64.

Run from the repository root:  python tests/golden/make_golden.py [which]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import compression as oc  # noqa: E402
from oracle import encoding as oe  # noqa: E402
from oracle import solvers as osv  # noqa: E402
from paper_2601_05418_amd import synth  # noqa: E402
from tests import helpers as H  # noqa: E402

FISTA_FILE = os.path.join(HERE, "highfield_fista50.npz")
UNROLLED_FILE = os.path.join(HERE, "unrolled_fd.npz")
BATCH_FILE = os.path.join(HERE, "batch_largest_cg20.npz")
FISTA_ITERS, LEVELS, POWER_ITERS = 50, 3, 50


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def highfield_inputs():
    """The slice (inputs rounded to complex64) and its acquired k-space
    S = E rho + noise at linear SNR 30, rounded to complex64."""
    sl = H.rounded_slice(synth.highfield_slice(0))
    g = sl.geom
    s = oe.forward_full(sl.image, sl.coils, sl.psf, g.mask, g.os)
    s = s + synth.scaled_noise(s, sl.noise, sl.snr)
    return sl, H.round64(s)


def highfield_fista():
    sl, s = highfield_inputs()
    g = sl.geom
    log("calibrate (42 groups)")
    bank, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    y = oc.compress(s, bank, g.patch_group, g.patch_len)
    args = (sl.coils, sl.psf, g.mask, g.os, bank, g.patch_group, g.patch_len)
    nrm = lambda v: oe.normal(v, *args)
    b = oe.adjoint(y, *args)
    lam = 1e-3 * float(np.max(np.abs(osv.haar_fwd(b, LEVELS))))
    log(f"lambda {lam:.6e}; power iteration")
    lip = 1.01 * osv.power_iteration(nrm, (g.ny, g.nx), POWER_ITERS, seed=0)
    log(f"L {lip:.6e}; FISTA-{FISTA_ITERS}")
    dm = osv.detail_mask((g.ny, g.nx), LEVELS)

    def objective(x):
        r = oe.forward(x, *args) - y
        return 0.5 * float(np.vdot(r, r).real) + lam * float(np.sum(np.abs(osv.haar_fwd(x, LEVELS)[dm])))

    x, objs = osv.fista(nrm, b, FISTA_ITERS, lam, lip, LEVELS, objective=objective)
    np.savez_compressed(FISTA_FILE, x=x.astype(np.complex64), lam=lam, lip=lip, obj=objs)
    log(f"wrote {FISTA_FILE}")


def batch_largest():
    slices = synth.batch_draws(64, 0)
    rng = np.random.default_rng(77)
    banks, ys = [], []
    for sl in slices:  # the batch test's draw order: bank, then data, per slice
        g = sl.geom
        banks.append(synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng))
        ys.append(H.round64(synth.unit_noise((1, g.n_patches, g.k, g.ms), rng)))
    order = sorted(range(64), key=lambda i: slices[i].geom.nc * slices[i].geom.ny * slices[i].geom.nt)
    pick = order[-2:]
    out = {"index": np.array(pick)}
    for i in pick:
        sl = H.rounded_slice(slices[i])
        g = sl.geom
        args = (sl.coils, sl.psf, g.mask, g.os, banks[i], g.patch_group, g.patch_len)
        log(f"slice {i}: {g.nx}x{g.ny}, nc {g.nc}, os {g.os}, P {g.patch_len}, K {g.k}: CG-20")
        b = oe.adjoint(ys[i][0], *args)
        x, hist = osv.cg(lambda v: oe.normal(v, *args), b, 20)
        out[f"x{i}"] = x.astype(np.complex64)
        out[f"resid{i}"] = hist
    np.savez_compressed(BATCH_FILE, **out)
    log(f"wrote {BATCH_FILE}")


def unrolled_inputs():
    """Shared by this script and the full-size unrolled test: slice 0 of the
    unrolled workload (inputs rounded to complex64), its random orthonormal
    bank, the batch of starting images x0, the unit direction v on image 0,
    and the step sizes alpha_k = c_k / L_b with L_b = max_r sum_n |c_n(r)|^2,
    an upper bound of ||E'^H E'|| (unitary DFTs, unit-modulus PSF, bank rows
    orthonormal)."""
    slices = synth.unrolled_slices(8, 0)
    sl = H.rounded_slice(slices[0])
    g = sl.geom
    rng = np.random.default_rng(43)
    bank = synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng)
    x0 = H.round64(0.1 * synth.unit_noise((8, g.ny, g.nx), rng))
    v = synth.unit_noise((g.ny, g.nx), rng)
    v = H.round64(v / np.linalg.norm(v))
    truth = H.round64(np.stack([s.image for s in slices]))
    lb = float(np.max(np.sum(np.abs(sl.coils) ** 2, axis=0)))
    alphas = np.asarray(np.linspace(0.6, 1.2, 10) / lb, np.float32).astype(np.float64)
    return sl, bank, x0, v, truth, alphas


def unrolled_fd():
    sl, bank, x0, v, truth, alphas = unrolled_inputs()
    g = sl.geom
    args = (sl.coils, sl.psf, g.mask, g.os, bank, g.patch_group, g.patch_len)
    eps = 1e-3

    def loss(x):
        for a in alphas:
            x = x - a * oe.normal(x, *args)
        return 0.5 * float(np.vdot(x - truth[0], x - truth[0]).real)

    log("unrolled network, image 0: loss at x0 + eps v")
    lp = loss(x0[0] + eps * v)
    log("unrolled network, image 0: loss at x0 - eps v")
    lm = loss(x0[0] - eps * v)
    np.savez_compressed(UNROLLED_FILE, eps=eps, loss_plus=lp, loss_minus=lm, fd=(lp - lm) / (2 * eps),
                        alphas=alphas)
    log(f"wrote {UNROLLED_FILE}: fd {(lp - lm) / (2 * eps):.9e}")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("all", "fista"):
        highfield_fista()
    if which in ("all", "batch"):
        batch_largest()
    if which in ("all", "unrolled"):
        unrolled_fd()
