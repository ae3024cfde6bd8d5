"""Writes benchmark_grid_{N}steps_model{M}.json: the FP64 oracle's state of the
1024 x 64 x 128 lock exchange after N steps (100 by default), computed by the
oracle only.

Workload (the benchmark grid and physics): D3Q27 cumulant + D3Q7 (model 0)
or D3Q19 BGK + Smagorinsky + D3Q6 (model 1), Re_b = 30000, C_s = 0.1,
Sc_T = 1, g' = 1e-4, Sc = 1, lock fraction 1/8, gate noise 1e-3 with seed 0.
The oracle steps the whole grid N times (Eq. 17, 28) from the initial state
of Sec. 2.5.

Recorded:
  * diagnostics of the state at step N (mass, scalar mass, F_w of Eq. 62
    and 64, the front of Sec. 3.1, max |u|);
  * the infinity norms of delta rho = rho - 1, u_x, u_y, u_z, |u| and chi over
    the whole grid (the scales the parity test divides by);
  * rho, u and chi at sampled nodes: every combination of the x positions
    {0, 1, gate - 2 .. gate + 1, nx - 2, nx - 1}, the depths
    {0, 1, nz / 2, nz - 2, nz - 1} and the span positions {0, ny / 2, ny - 1}
    (walls, gate, periodic edges), plus 400 nodes drawn uniformly with
    numpy's generator from seed 3.

Run: python tests/golden/make_benchmark_grid_fixture.py [--steps N] [model ...]
(on 8 cores, for 100 steps: about 3.5 hours for model 0, whose collision the
oracle takes through the cumulant ring, and 6 minutes for model 1; peak memory
about 10 GB. The 1000-step fixture is made for model 1 only: about an hour.)
"""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import diag, lbm  # noqa: E402
from oracle.params import Config, derive  # noqa: E402

CASE = dict(nx=1024, ny=64, nz=128, re_b=30000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4)
SEED = 0


def sample_nodes(nx, ny, nz):
    g = nx // 8
    nodes = set()
    for i in (0, 1, g - 2, g - 1, g, g + 1, nx - 2, nx - 1):
        for k in (0, 1, nz // 2, nz - 2, nz - 1):
            for j in (0, ny // 2, ny - 1):
                nodes.add((k, j, i))
    rng = np.random.default_rng(3)
    for _ in range(400):
        nodes.add((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    return sorted(nodes)


def fixture_path(model, steps):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"benchmark_grid_{steps}steps_model{model}.json")


def main(models, steps):
    torch.set_num_threads(int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1)))
    for model in models:
        cfg = Config(model=model, **CASE)
        P = derive(cfg)
        f, phi = lbm.init_state(P, lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, SEED))
        t0 = time.time()
        for n in range(steps):
            f, phi = lbm.step(f, phi, P)
            print(f"model {model} step {n + 1}/{steps} {time.time() - t0:.0f} s", flush=True)
        d = diag.diagnostics(f, phi, P, steps)
        rho, u, chi = lbm.moments(f, phi, P)
        del f, phi
        umag = torch.sqrt((u * u).sum(0))
        nodes = sample_nodes(cfg.nx, cfg.ny, cfg.nz)
        k, j, i = (torch.tensor(c) for c in zip(*nodes))
        out = {
            "case": dict(model=model, **CASE), "steps": steps, "seed": SEED,
            "lock_fraction": 0.125, "noise_amp": 1e-3,
            "diagnostics": {key: d[key] for key in ("mass", "chi_mass", "fw", "x_front", "x_f",
                                                    "umax", "nonfinite")},
            "norms": {"drho": float((rho - 1.0).abs().max()), "ux": float(u[0].abs().max()),
                      "uy": float(u[1].abs().max()), "uz": float(u[2].abs().max()),
                      "umag": float(umag.max()), "chi": float(chi.abs().max())},
            "nodes": [list(n) for n in nodes],
            "rho": rho[k, j, i].tolist(), "ux": u[0][k, j, i].tolist(),
            "uy": u[1][k, j, i].tolist(), "uz": u[2][k, j, i].tolist(),
            "chi": chi[k, j, i].tolist(),
            "oracle_seconds": time.time() - t0,
        }
        with open(fixture_path(model, steps), "w") as fh:
            json.dump(out, fh, indent=0)
        print(f"model {model}: wrote {fixture_path(model, steps)}", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    steps = 100
    if args[:1] == ["--steps"]:
        steps, args = int(args[1]), args[2:]
    main([int(a) for a in args] or [0, 1], steps)
