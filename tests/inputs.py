"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the method: only random numbers and fixed shapes. Every
generator takes an explicit seed and returns float64 numpy arrays in the
population layout [population][z][y][x].
"""
import numpy as np

# weights are needed to place a random state near the lattice rest state; they
# are passed in by the caller (each side has its own tables)


def near_rest_state(Qf, Qs, shape, wf, ws, seed, eps=1e-3, chi_lo=0.0, chi_hi=1.0):
    """f = w (1 + eps * N(0,1)), phi = w_s * chi (1 + eps * N(0,1)) with chi
    uniform in [chi_lo, chi_hi]. shape = (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    wf = np.asarray(wf, dtype=np.float64).reshape(Qf, 1, 1, 1)
    ws = np.asarray(ws, dtype=np.float64).reshape(Qs, 1, 1, 1)
    f = wf * (1.0 + eps * rng.standard_normal((Qf,) + tuple(shape)))
    chi = rng.uniform(chi_lo, chi_hi, size=(1,) + tuple(shape))
    phi = ws * chi * (1.0 + eps * rng.standard_normal((Qs,) + tuple(shape)))
    return f, phi


def random_field(shape, seed, lo=0.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=tuple(shape))


def random_distribution_q27(n, seed):
    """n random positive distributions on {-1,0,1}^3 (27, n), each summing to 1."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.1, 1.0, size=(27, n))
    return p / p.sum(0, keepdims=True)
