"""Pins of the oracle's diagnostics (wall shear Eq. 62/64, front Sec. 3.1) and
initial condition (Sec. 2.5)."""
import os

import numpy as np
import pytest
import torch

from oracle import diag, lbm
from oracle.params import Config, derive

G = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_outputs():
    want = [int(l) for l in open(os.path.join(G, "splitmix64_seed1234567.txt")) if l.strip() and not l.startswith("#")]
    s, got = 1234567, []
    for _ in range(5):
        got.append(int(lbm.splitmix64(np.uint64(s))))
        s = (s + lbm.GOLDEN) % (1 << 64)
    assert got == want


def test_lock_exchange_initial_condition():
    cfg = Config(128, 8, 16, model=0)
    chi = lbm.chi0_lock_exchange(cfg, 0.125, 1e-3, seed=0)
    assert lbm.gate_index(128, 0.125) == 16
    assert torch.equal(chi[:, :, :15], torch.ones(16, 8, 15, dtype=torch.float64))
    assert torch.equal(chi[:, :, 17:], torch.zeros(16, 8, 111, dtype=torch.float64))
    eta15 = chi[:, :, 15] - 1.0
    eta16 = chi[:, :, 16]
    for eta in (eta15, eta16):
        assert float(eta.abs().max()) <= 1e-3
        assert float(eta.std()) > 4e-4          # uniform on [-a, a]: std a/sqrt(3)
    assert not torch.equal(eta15, eta16)
    # the noise at node (k, j, i) is a pure function of (seed, linear index)
    i, j, k = 16, 3, 5
    lin = i + 128 * (j + 8 * k)
    key = np.uint64(0) ^ np.uint64((lin * lbm.GOLDEN) % (1 << 64))
    U = int(lbm.splitmix64(key)) >> 11
    assert float(chi[k, j, i]) == 1e-3 * (2.0 * (U * 2.0 ** -53) - 1.0)
    P = derive(cfg)
    f, phi = lbm.init_state(P, chi)
    rho, u, c = lbm.moments(f, phi, P)
    assert torch.equal(c, (phi.sum(0)))
    assert float((rho - 1).abs().max()) < 1e-15
    # zero momentum: the reported velocity is the half-force shift only
    assert torch.allclose(u[2], -0.5 * P.g_prime * c / rho, atol=1e-18, rtol=0)


def _state_with_velocity(P, ux_of_z, nx=6, ny=3):
    """Equilibrium state with u_x(z) prescribed and chi = 0 (BGK model)."""
    nz = len(ux_of_z)
    from oracle import collide as C
    u = torch.zeros(3, nz * ny * nx, dtype=torch.float64)
    u[0] = torch.tensor(ux_of_z, dtype=torch.float64).repeat_interleave(ny * nx)
    f = C.feq_q19(torch.ones(nz * ny * nx, dtype=torch.float64), u, P.flow).reshape(19, nz, ny, nx)
    phi = torch.zeros(6, nz, ny, nx, dtype=torch.float64)
    return f, phi


@pytest.mark.parametrize("a,b", [(0.0, 1e-3), (2e-4, -5e-4)])
def test_wall_shear_is_exact_for_quadratic_profiles(a, b):
    """Nodes at z + 1/2 above the half-way wall: u = a z^2 + b z has wall
    slope b, so F_w = nu0 * b * N1 * N2 exactly."""
    P = derive(Config(6, 3, 5, model=1, re_b=500.0, g_prime=1e-4))
    zc = [k + 0.5 for k in range(5)]
    f, phi = _state_with_velocity(P, [a * z * z + b * z for z in zc])
    d = diag.diagnostics(f, phi, P)
    assert abs(d['fw'] - P.nu0 * b * 18) < 1e-17
    assert abs(d['fw_nd'] - d['fw'] / (P.u_b ** 2 * 25)) < 1e-20


def _chi_state(P, chi):
    nz, ny, nx = chi.shape
    f = P.flow.w[:, None, None, None].expand(P.flow.Q, nz, ny, nx).clone()
    return f, P.scal.w[:, None, None, None] * chi[None]


def test_front_linear_interpolation_and_depth_maximum():
    P = derive(Config(10, 2, 3, model=0))
    chi = torch.zeros(3, 2, 10, dtype=torch.float64)
    # column maxima m(i): 1 up to i = 4, then 0.05 at i = 5 (only at k = 2), 0.01 at i = 6
    chi[:, :, :5] = 1.0
    chi[2, :, 5] = 0.05
    chi[0, 0, 6] = 0.02            # span mean 0.01
    f, phi = _chi_state(P, chi)
    x, istar = diag.front_position(phi.sum(0))
    assert istar == 5
    want = 5 + 0.5 + (0.05 - 0.02) / (0.05 - 0.01)
    assert abs(float(x) - want) < 1e-14
    d = diag.diagnostics(f, phi, P, lock_fraction=0.2)
    assert abs(d['x_f'] - (want - 2)) < 1e-14
    assert abs(d['x_f_nd'] - (want - 2) / 3) < 1e-14


def test_front_edge_cases():
    P = derive(Config(8, 1, 2, model=0))
    chi = torch.full((2, 1, 8), 0.5, dtype=torch.float64)
    assert float(diag.front_position(chi)[0]) == 8.0          # reached the end wall
    chi = torch.zeros(2, 1, 8, dtype=torch.float64)
    assert float(diag.front_position(chi)[0]) == 0.0          # nothing above threshold
    chi[1, 0, 3] = 0.02                                        # exactly at threshold
    x, i = diag.front_position(chi)
    assert i == 3 and float(x) == 3.5
