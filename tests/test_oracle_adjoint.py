"""Pins of the oracle's reference gradient (torch autograd through the FP64
oracle) against central finite differences of the same objective, and of the
checkpointed backward against the plain one."""
import numpy as np
import pytest
import torch

from oracle import adjoint, lbm
from oracle.params import Config
from tests import inputs

CASES = [dict(nx=24, ny=2, nz=6, model=0, re_b=400.0, cs_smag=0.1, sc_t=0.8, g_prime=1e-3),
         dict(nx=24, ny=2, nz=6, model=1, re_b=400.0, cs_smag=0.1, sc_t=0.8, g_prime=1e-3),
         dict(nx=24, ny=2, nz=6, model=2, re_b=400.0, cs_smag=0.1, sc_t=0.8, g_prime=1e-3)]


@pytest.mark.parametrize("case", CASES, ids=["cumulant", "bgk", "cumulant_fcm"])
def test_autograd_gradient_matches_central_differences(case):
    cfg = Config(**case)
    chi0 = lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 3)
    n = 30
    J, gcs, gsct, gchi = adjoint.gradient(cfg, chi0, n, k_ckpt=10)
    h = 1e-5
    fcs = (adjoint.objective(cfg, chi0, n, cs=case["cs_smag"] + h) -
           adjoint.objective(cfg, chi0, n, cs=case["cs_smag"] - h)) / (2 * h)
    fsct = (adjoint.objective(cfg, chi0, n, sct=case["sc_t"] + h) -
            adjoint.objective(cfg, chi0, n, sct=case["sc_t"] - h)) / (2 * h)
    assert abs(J - adjoint.objective(cfg, chi0, n)) < 1e-12 * max(1.0, abs(J))
    assert abs(gcs - fcs) <= 1e-5 * abs(fcs) + 1e-12
    assert abs(gsct - fsct) <= 1e-5 * abs(fsct) + 1e-12
    # direction inside the lock: a perturbation of the untouched columns ahead
    # of the front would meet the tie of the depth maximum over all-zero columns
    d = torch.from_numpy(inputs.random_field(tuple(chi0.shape), 5, -1.0, 1.0))
    d[:, :, lbm.gate_index(cfg.nx, 0.125) - 1:] = 0.0
    fd = (adjoint.objective(cfg, chi0 + h * d, n) - adjoint.objective(cfg, chi0 - h * d, n)) / (2 * h)
    ad = float((gchi * d).sum())
    assert abs(ad - fd) <= 1e-5 * abs(fd) + 1e-12


def test_checkpointed_gradient_equals_plain_gradient():
    cfg = Config(**CASES[0])
    chi0 = lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 1)
    a = adjoint.gradient(cfg, chi0, 10, k_ckpt=3)
    b = adjoint.gradient(cfg, chi0, 10, k_ckpt=100)
    assert abs(a[0] - b[0]) < 1e-14 and abs(a[1] - b[1]) < 1e-12 and abs(a[2] - b[2]) < 1e-12
    assert torch.allclose(a[3], b[3], rtol=0, atol=1e-12)
