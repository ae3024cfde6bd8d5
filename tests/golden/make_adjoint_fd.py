"""Writes adjoint_fd_128x8x16.json: FP64 central finite differences of the
objective J = x_f(n) + (1/n) sum_{m=1..n} F_w(m) computed by the oracle only.

Workload: lock exchange 128 x 8 x 16, D3Q27 cumulant + D3Q7, Re_b = 1000,
C_s = 0.1, Sc_T = 1, g' = 1e-4, gate noise 1e-3 (seed 0), 500 steps.
Derivatives: d/dC_s, d/dSc_T (absolute step h = 1e-4) and directional
derivatives along chi0 directions: two seeded random directions of unit
infinity norm (tests/inputs.random_field, seeds 11 and 12, values in [-1, 1])
and two single nodes next to the gate.

Run: python tests/golden/make_adjoint_fd.py  (about 10 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint, lbm  # noqa: E402
from oracle.params import Config  # noqa: E402
from tests import inputs  # noqa: E402

CASE = dict(nx=128, ny=8, nz=16, model=0, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4)
STEPS = 500
H = 1e-4
DIR_SEEDS = (11, 12)
NODES = ((3, 2, 15), (8, 5, 16))  # (k, j, i): the two columns next to the gate (x0 = 16)


def directions(shape):
    out = []
    for s in DIR_SEEDS:
        d = inputs.random_field(shape, s, -1.0, 1.0)
        out.append(d / np.abs(d).max())
    for (k, j, i) in NODES:
        d = np.zeros(shape)
        d[k, j, i] = 1.0
        out.append(d)
    return out


def main():
    torch.set_num_threads(os.cpu_count() or 1)
    cfg = Config(**CASE)
    chi0 = lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 0)
    t0 = time.time()
    J0 = adjoint.objective(cfg, chi0, STEPS)
    res = {"case": CASE, "steps": STEPS, "h": H, "dir_seeds": list(DIR_SEEDS),
           "nodes": [list(n) for n in NODES], "J": J0}

    def fd(**kw):
        jp = adjoint.objective(cfg, kw.get("chi_p", chi0), STEPS, cs=kw.get("cs_p"), sct=kw.get("sct_p"))
        jm = adjoint.objective(cfg, kw.get("chi_m", chi0), STEPS, cs=kw.get("cs_m"), sct=kw.get("sct_m"))
        return (jp - jm) / (2 * H)

    res["dJ_dcs"] = fd(cs_p=CASE["cs_smag"] + H, cs_m=CASE["cs_smag"] - H)
    print("dJ/dC_s", res["dJ_dcs"], time.time() - t0, flush=True)
    res["dJ_dsct"] = fd(sct_p=CASE["sc_t"] + H, sct_m=CASE["sc_t"] - H)
    print("dJ/dSc_T", res["dJ_dsct"], time.time() - t0, flush=True)
    res["dJ_dchi0_dir"] = []
    for d in directions(tuple(chi0.shape)):
        dt = torch.from_numpy(d)
        v = fd(chi_p=chi0 + H * dt, chi_m=chi0 - H * dt)
        res["dJ_dchi0_dir"].append(v)
        print("dir", v, time.time() - t0, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd_128x8x16.json"), "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
