"""gpjc_calibrate_static: calibration with its workspaces in the library's
static device scratch (no device allocation), against gpjc_calibrate.

Both run the same kernels with the same launch shapes on the same plan
geometry, so eigenvalues, banks and the resulting operator must agree; the
bound is the calibration parity bar (eigenvalues within 1e-10 of the largest,
projectors A^H A within 1e-9 / relative gap).  Two calls in a row, the second
on a smaller geometry, so the second reads a scratch the first has filled.
"""
import numpy as np
import pytest
import torch

from oracle import compression as oc
from paper_2601_05418_amd import gpjc, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def projector_bound(eig, k):
    lam = np.asarray(eig)
    gap = np.min((lam[:, k - 1] - lam[:, k]) / lam[:, 0]) if k < lam.shape[1] else 1.0
    return 1e-9 / max(gap, 1e-3)


@pytest.mark.parametrize("order", [("small", "periodic")])
def test_static_calibration_matches_allocating_one(gpu_lib, order):
    for case in order:  # the second geometry is smaller than the first
        sl = H.rounded_slice(H.CASES[case]())
        g = sl.geom
        ref_plan, st_plan = gpjc.Plan.from_slice(sl), gpjc.Plan.from_slice(sl)
        eig_r, bank_r = ref_plan.calibrate(want_eigvals=True, want_bank=True)
        eig_s, bank_s = st_plan.calibrate_static(want_eigvals=True, want_bank=True)
        bank_r, bank_s = host(bank_r), host(bank_s)
        same = np.array_equal(eig_r, eig_s) and np.array_equal(bank_r, bank_s)
        print(f"{case}: G {g.n_groups}, Ns {g.ns}, K {g.k}; bit-identical {same}", flush=True)
        assert np.max(np.abs(eig_s - eig_r)) <= 1e-10 * eig_r.max()
        d = np.max(np.abs(oc.projectors(bank_s) - oc.projectors(bank_r)))
        assert d <= projector_bound(eig_r, g.k)
        # the installed banks give the same operator
        x = torch.as_tensor(np.ascontiguousarray(H.round64(sl.image)[None], np.complex64)).cuda()
        a = host(ref_plan.normal(x)).astype(np.complex128)
        b = host(st_plan.normal(x)).astype(np.complex128)
        assert H.rel_l2(b, a) <= 1e-6
        ref_plan.close()
        st_plan.close()


def test_static_calibration_rejects_oversized_geometry(gpu_lib):
    """The high-field slice needs about 1.6 GB of workspace: refused before
    anything is queued, outputs untouched."""
    sl = H.rounded_slice(synth.highfield_slice(0, periodic=True))
    plan = gpjc.Plan.from_slice(sl)
    bank = torch.full((6, 64, 32, 32), 3.0 + 0j, dtype=torch.complex128, device="cuda")
    st = plan.lib.gpjc_calibrate_static(plan.handle, None, None, None, gpjc._ptr(bank))
    assert st == gpjc.GPJC_E_UNSUPPORTED
    assert b"static scratch" in plan.lib.gpjc_last_error()
    torch.cuda.synchronize()
    assert torch.all(bank == 3.0)
    plan.close()
