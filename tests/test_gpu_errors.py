"""Failure detection, forced from the host: every kernel still runs to its
normal end, and the library reports the condition through its status code.

- NaN in the data -> GPJC_E_NUMERIC from CG and from FISTA;
- an eigensolver held to zero inverse-iteration steps (its eigenvectors then
  fail the residual check) -> GPJC_E_NUMERIC from calibration;
- a group whose member patches see different modulation (Section 2.3: one
  matrix serves a group only if its patches are encoded alike) ->
  GPJC_E_INVAL at plan creation;
- FISTA's objective history (Eq. 17, wavelet form) against the oracle's.
"""
import dataclasses
import os

import numpy as np
import pytest
import torch

from oracle import compression as oc
from oracle import encoding as oe
from oracle import solvers as osv
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.complex64)).cuda()


def small_plan():
    sl = H.rounded_slice(synth.small_slice(0))
    a = H.oracle_bank(sl)[0]
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    return sl, a, plan


def test_nan_data_is_reported_by_cg_and_fista(gpu_lib):
    sl, a, plan = small_plan()
    y = np.ones(plan.data_shape(), np.complex64)
    y[0, 3, 2, 5] = np.nan
    with pytest.raises(gpjc.GpjcError) as e:
        plan.recon_cg(dev(y), 5)
    assert e.value.status == gpjc.GPJC_E_NUMERIC
    with pytest.raises(gpjc.GpjcError) as e:
        plan.recon_fista(dev(y), 5, 1e-3, 2.0)
    assert e.value.status == gpjc.GPJC_E_NUMERIC
    # the same plan still solves finite data afterwards
    ops = H.oracle_ops(sl, a)
    yf = H.round64(ops["fwd"](sl.image))
    x = plan.recon_cg(dev(yf[None]), 5)
    assert torch.isfinite(torch.view_as_real(x)).all()
    plan.recon_fista(dev(yf[None]), 5, 1e-3, 2.0)


def test_eigensolver_residual_check_is_reported(gpu_lib, monkeypatch):
    sl = H.rounded_slice(synth.small_slice(0))
    plan = gpjc.Plan.from_slice(sl)
    monkeypatch.setenv("GPJC_INVIT_ITERS", "0")
    with pytest.raises(gpjc.GpjcError) as e:
        plan.calibrate()
    assert e.value.status == gpjc.GPJC_E_NUMERIC
    assert "residual check" in str(e.value)
    monkeypatch.delenv("GPJC_INVIT_ITERS")
    eig, _ = plan.calibrate(want_eigvals=True)
    ref = H.oracle_bank(sl)[1]
    assert np.max(np.abs(eig - ref)) <= 1e-10 * ref.max()


def test_illegal_group_is_rejected(gpu_lib):
    """The small slice's wave has 5 cycles over 256 samples (period 51.2), so
    its 16 patches of 16 samples never repeat: mapping them onto 4 groups is
    illegal, and the oracle agrees."""
    sl = H.rounded_slice(synth.small_slice(0))
    pg = synth.periodic_groups(16, 4)
    assert not oc.groups_legal(sl.psf, 16, pg)
    g = dataclasses.replace(sl.geom, patch_group=pg, n_groups=4)
    with pytest.raises(gpjc.GpjcError) as e:
        gpjc.Plan.from_slice(dataclasses.replace(sl, geom=g))
    assert e.value.status == gpjc.GPJC_E_INVAL
    assert "does not share the modulation" in str(e.value)
    # a legal periodic map (period 64 samples = 4 patches) is accepted
    sp = H.rounded_slice(H.CASES["periodic"]())
    assert oc.groups_legal(sp.psf, sp.geom.patch_len, sp.geom.patch_group)
    gpjc.Plan.from_slice(sp).close()


@pytest.mark.parametrize("case", ["small", "rect"])
def test_fista_objective_history(gpu_lib, case):
    sl = H.rounded_slice(H.CASES[case]())
    g = sl.geom
    a = H.oracle_bank(sl)[0]
    plan = gpjc.Plan.from_slice(sl)
    plan.set_compression(torch.as_tensor(a).cuda())
    ops = H.oracle_ops(sl, a)
    y = H.round64(ops["fwd"](sl.image))
    b = ops["adj"](y)
    lip = osv.power_iteration(ops["nrm"], b.shape, iters=50, seed=0) * 1.01
    lam = 1e-2 * np.abs(osv.haar_fwd(b, 3)).max()
    dm = osv.detail_mask(b.shape, 3)

    def objective(x):
        r = ops["fwd"](x) - y
        return 0.5 * np.vdot(r, r).real + lam * np.sum(np.abs(osv.haar_fwd(x, 3)[dm]))

    xg, obj = plan.recon_fista(dev(y[None]), 20, lam, lip, levels=3, want_obj=True)
    xo, objo = osv.fista(ops["nrm"], b, 20, lam, lip, 3, objective=objective)
    rel = np.abs(obj - objo) / objo
    print(f"{case}: objective rel err max {rel.max():.3e}; first {objo[0]:.6e} last {objo[-1]:.6e}", flush=True)
    assert rel.max() <= 1e-5
    assert objo[-1] < objo[0]
    # the history does not change the iterate
    x2 = plan.recon_fista(dev(y[None]), 20, lam, lip, levels=3)
    assert torch.equal(xg, x2)
