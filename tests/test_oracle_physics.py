"""Physics sanity of the oracle itself: the slumping-phase Froude number
(Eq. 59) of the 128 x 8 x 16 lock exchange at Re_b = 1000, every model,
against the 0.37 of Table 2 (Case 2, Re_b = 1000), within 0.02.

The run is 4800 FP64 steps (t~ = 12) of the oracle: several minutes on eight
cores. It is marked slow and runs when LBM_SLOW_TESTS=1 is set; the same
check runs on the GPU's FP64 path in tests/test_gpu_physics.py.
"""
import os

import numpy as np
import pytest
import torch

from oracle import diag as odiag
from oracle import lbm as olbm
from oracle.params import Config, derive

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("LBM_SLOW_TESTS") != "1",
                                 reason="long oracle run; set LBM_SLOW_TESTS=1")]


@pytest.mark.parametrize("model", [0, 1, 2])
def test_oracle_froude_number(model):
    torch.set_num_threads(os.cpu_count() or 1)
    cfg = Config(128, 8, 16, model=model, re_b=1000.0, g_prime=1e-4)
    P = derive(cfg)
    f, phi = olbm.init_state(P, olbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 0))
    every = int(round(0.1 * P.H / P.u_b))
    n_end = int(np.ceil(10.5 * P.H / P.u_b))
    ts, xs, n = [], [], 0
    while n < n_end:
        f, phi = olbm.run(f, phi, P, every)
        n += every
        d = odiag.diagnostics(f, phi, P, n)
        ts.append(d["t_nd"])
        xs.append(d["x_f_nd"])
    fr = odiag.froude_number(ts, xs)
    print(f"oracle model {model}: Fr = {fr:.4f}", flush=True)
    assert abs(fr - 0.37) <= 0.02
