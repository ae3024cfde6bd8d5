"""Writes FP64 central finite differences of the adjoint objective
J = x_f(n) + (1/n) sum_{m=1..n} F_w(m), computed by the oracle only.

Three cases (the lock exchange, D3Q27 cumulant + D3Q7, Re_b = 1000, C_s = 0.1,
Sc_T = 1, g' = 1e-4, gate noise 1e-3 with seed 0):

* ``small`` -> adjoint_fd_128x8x16.json: 128 x 8 x 16, 500 steps.
  Derivatives d/dC_s, d/dSc_T (absolute step h = 1e-4) and directional
  derivatives along chi0 directions: two seeded random directions of unit
  infinity norm (tests/inputs.random_field, seeds 11 and 12, values in
  [-1, 1]) and two single nodes next to the gate.
  About 10 minutes on 8 cores.
* ``c3`` -> adjoint_fd_256x16x32.json: 256 x 16 x 32, 2000 steps (the size of
  the differentiated benchmark run). d/dC_s and d/dSc_T only, each from two
  2000-step runs. The five runs (J and the four shifted ones) go to parallel
  worker processes; about three hours on 8 cores.
* ``c3_chi0`` -> adjoint_fd_256x16x32_chi0.json: the same run, directional
  derivatives along two seeded random chi0 directions of unit infinity norm
  (tests/inputs.random_field, seeds 21 and 22, values in [-1, 1]); four
  2000-step runs, about two hours on 8 cores with 4 workers.

Run: python tests/golden/make_adjoint_fd.py [small|c3|c3_chi0] [workers]
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint, lbm  # noqa: E402
from oracle.params import Config  # noqa: E402
from tests import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
H = 1e-4
PHYS = dict(model=0, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4)
CASES = {
    "small": dict(grid=dict(nx=128, ny=8, nz=16), steps=500, out="adjoint_fd_128x8x16.json",
                  dir_seeds=(11, 12), nodes=((3, 2, 15), (8, 5, 16))),  # (k, j, i) next to the gate
    "c3": dict(grid=dict(nx=256, ny=16, nz=32), steps=2000, out="adjoint_fd_256x16x32.json",
               dir_seeds=(), nodes=()),
    "c3_chi0": dict(grid=dict(nx=256, ny=16, nz=32), steps=2000, out="adjoint_fd_256x16x32_chi0.json",
                    dir_seeds=(21, 22), nodes=(), params=False),
}


def directions(shape, dir_seeds, nodes):
    out = []
    for s in dir_seeds:
        d = inputs.random_field(shape, s, -1.0, 1.0)
        out.append(d / np.abs(d).max())
    for (k, j, i) in nodes:
        d = np.zeros(shape)
        d[k, j, i] = 1.0
        out.append(d)
    return out


def _objective(args):
    """One oracle run: (case kwargs, steps, C_s, Sc_T, chi0 direction or None,
    its step, threads) -> J."""
    kw, steps, cs, sct, d, hd, threads = args
    torch.set_num_threads(threads)
    cfg = Config(**kw)
    chi0 = lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 0)
    if d is not None:
        chi0 = chi0 + hd * torch.from_numpy(d)
    return adjoint.objective(cfg, chi0, steps, cs=cs, sct=sct)


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "small"
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    case = CASES[name]
    kw = dict(case["grid"], **PHYS)
    steps = case["steps"]
    cores = os.cpu_count() or 1
    threads = max(1, cores // workers)
    cs0, sct0 = kw["cs_smag"], kw["sc_t"]
    shape = (kw["nz"], kw["ny"], kw["nx"])
    dirs = directions(shape, case["dir_seeds"], case["nodes"])
    params = case.get("params", True)
    runs = []
    if params:
        runs = [(kw, steps, cs0, sct0, None, 0.0, threads),
                (kw, steps, cs0 + H, sct0, None, 0.0, threads), (kw, steps, cs0 - H, sct0, None, 0.0, threads),
                (kw, steps, cs0, sct0 + H, None, 0.0, threads), (kw, steps, cs0, sct0 - H, None, 0.0, threads)]
    for d in dirs:
        runs += [(kw, steps, cs0, sct0, d, H, threads), (kw, steps, cs0, sct0, d, -H, threads)]
    t0 = time.time()
    if workers > 1:
        with ProcessPoolExecutor(workers) as ex:
            js = list(ex.map(_objective, runs))
    else:
        js = [_objective(r) for r in runs]
    print(f"{len(runs)} runs in {time.time() - t0:.0f} s", flush=True)
    res = {"case": kw, "steps": steps, "h": H, "dir_seeds": list(case["dir_seeds"]),
           "nodes": [list(n) for n in case["nodes"]]}
    o = 0
    if params:
        res.update(J=js[0], dJ_dcs=(js[1] - js[2]) / (2 * H), dJ_dsct=(js[3] - js[4]) / (2 * H))
        o = 5
    res["dJ_dchi0_dir"] = [(js[o + 2 * i] - js[o + 1 + 2 * i]) / (2 * H) for i in range(len(dirs))]
    print(json.dumps(res), flush=True)
    with open(os.path.join(HERE, case["out"]), "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
