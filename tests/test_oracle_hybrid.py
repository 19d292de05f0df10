"""Pins of the hybrid-space algorithm #1 oracle (oracle/hybrid.py): LSQR
against SciPy's LSQR (the same published algorithm, a library routine) and
against the least-squares solution; the decoupling into aliased sets against
the global problem (the folded model reproduces the acquired data, and the
assembled solution is the global least-squares solution)."""
import numpy as np
import scipy.sparse.linalg as sla

from oracle import compression as oc
from oracle import encoding as oe
from oracle import explicit as ox
from oracle import hybrid as oh
from oracle import solvers as osv
from paper_2601_05418_amd import synth


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_lsqr_matches_scipy_iterates():
    rng = np.random.default_rng(0)
    a = crandn(rng, (40, 17))
    b = crandn(rng, 40)
    for k in (1, 3, 8):
        x, _ = oh.lsqr(lambda v: a @ v, lambda u: a.conj().T @ u, b, k)
        ref = sla.lsqr(a, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert np.allclose(x, ref, atol=1e-10 * np.linalg.norm(ref))


def test_lsqr_converges_to_least_squares_and_reports_the_residual():
    rng = np.random.default_rng(1)
    a = crandn(rng, (30, 12))
    b = crandn(rng, 30)
    x, hist = oh.lsqr(lambda v: a @ v, lambda u: a.conj().T @ u, b, 40)
    ref = np.linalg.lstsq(a, b, rcond=None)[0]
    assert np.allclose(x, ref, atol=1e-10)
    assert abs(hist[-1] - np.linalg.norm(a @ x - b)) <= 1e-10 * np.linalg.norm(b)
    assert hist[0] == np.linalg.norm(b)


def wave_problem(accel=4):
    sl = synth.tiny_slice(0, nx=16, ny=16, nc=3, os_=2, patch_len=4, k=6)
    g = sl.geom
    mask = oh.regular_mask(g.ny, accel)
    a, _ = oc.calibrate(sl.coils, sl.psf, g.os, g.patch_len, g.patch_group, g.n_groups, g.k)
    bmod = np.repeat(sl.psf.T[:, :, None], g.nx, axis=2)
    e_c = ox.compressed_matrices(sl.coils, bmod, a, g.patch_group, g.patch_len)
    return sl, g, mask, a, e_c


def test_folded_set_models_reproduce_the_data():
    """Each set's model applied to its rows equals sqrt(R) times the
    zero-filled inverse DFT of S' = E' rho at that set's row."""
    sl, g, mask, a, e_c = wave_problem()
    rho = crandn(np.random.default_rng(2), (g.ny, g.nx))
    s = oe.forward(rho, sl.coils, sl.psf, mask, g.os, a, g.patch_group, g.patch_len)
    h = oh.set_data(s, mask, 4)
    for yr, rows in enumerate(oh.aliased_sets(g.ny, 4)):
        assert np.allclose(oh.set_model(e_c, rows, 4) @ rho[rows].reshape(-1), h[yr], atol=1e-12)


def test_assembled_solution_is_the_global_least_squares_solution():
    """Decoupled LSQR to convergence equals CG on the global normal equations
    (Eq. 16) to convergence, and its summed residual estimate is the global
    residual."""
    sl, g, mask, a, e_c = wave_problem()
    s = oe.forward(sl.image, sl.coils, sl.psf, mask, g.os, a, g.patch_group, g.patch_len)
    s = s + 0.05 * crandn(np.random.default_rng(3), s.shape)  # inconsistent data: a nonzero residual
    x1, res = oh.recon(s, e_c, mask, 4, 200)
    nrm = lambda v: oe.normal(v, sl.coils, sl.psf, mask, g.os, a, g.patch_group, g.patch_len)
    b = oe.adjoint(s, sl.coils, sl.psf, mask, g.os, a, g.patch_group, g.patch_len)
    x2, _ = osv.cg(nrm, b, 400)
    assert np.allclose(x1, x2, atol=1e-8 * np.abs(x2).max())
    r = oe.forward(x1, sl.coils, sl.psf, mask, g.os, a, g.patch_group, g.patch_len) - s
    assert abs(res[-1] - np.linalg.norm(r)) <= 1e-8 * np.linalg.norm(s)
