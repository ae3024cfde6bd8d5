"""Pins of two oracle branches that the collision's other pins leave open.

1. Per-order cumulant relaxation with general rates (Eq. 55): with no force,
   every cumulant of order k >= 3 of the post-collision distribution equals
   (1 - omega_k) times the pre-collision one; the deviatoric second order
   relaxes with omega1 = 1/tau (Eq. 58) and the trace with omega_bulk towards
   3 cs^2 = 1. The cumulants on both sides are computed here from the
   populations by the textbook set-partition formula, not through the
   oracle's ring, so a swapped rate or a wrong order fails.

2. Turbulent scalar diffusivity (Eq. 25, 30, 32-35). The flow relaxation time
   actually applied is read off the output (the off-diagonal covariance of
   f / rho relaxes as C* = (1 - 1/tau_f) C in BGK and cumulant alike when no
   force acts), and so is the scalar one (the first moment about chi u
   relaxes as (1 - 1/tau_phi)). Then the diffusivities must satisfy
   D_tot = D0 + nu_T / Sc_T with D = cs_phi^2 (tau_phi - 1/2) on the scalar
   lattice (1/4 for D3Q7, 1/3 for D3Q6 and D3Q27, the second moments of their
   weights) and nu_T = (tau_f - tau0) / 3 on the flow lattice; and tau_f must
   satisfy the Smagorinsky closure nu_T = C_s^2 |S| with the strain taken from
   the pre-collision stress. A scalar conversion with the flow's cs^2, Sc_T
   multiplied instead of divided, or a closure constant off by a factor fails.
"""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import collide as C
from oracle import lattice as L
from oracle.params import Config, derive
from tests import inputs
from tests.test_oracle_cumulant import _joint_cumulant

# second moment of each scalar lattice's weights along one axis (Eq. 30's cs_phi^2)
CS2_PHI = {0: 0.25, 1: 1.0 / 3.0, 2: 1.0 / 3.0}


def _cumulants(p):
    """{(a,b,c): cumulant} of a distribution p (27 probabilities on D3Q27) for
    every exponent triple with entries <= 2 and order >= 1."""
    out = {}
    for a, b, c in itertools.product(range(3), repeat=3):
        if a + b + c >= 1:
            out[(a, b, c)] = _joint_cumulant(p, [0] * a + [1] * b + [2] * c)
    return out


@pytest.mark.parametrize("rates", [(1.3, 0.7, 1.4, 0.6, 1.9), (0.8, 1.6, 0.5, 1.2, 0.3)])
@pytest.mark.parametrize("model", [0, 2])
def test_general_rates_relax_each_order_with_its_own_rate(model, rates):
    wb, w3, w4, w5, w6 = rates
    nu = 0.05
    P = derive(Config(4, 4, 4, model=model, g_prime=0.0, re_b=1.0, nu_lu=nu, omega_bulk=wb,
                      omega3=w3, omega4=w4, omega5=w5, omega6=w6))
    w1 = 1.0 / (3.0 * nu + 0.5)
    wk = {3: w3, 4: w4, 5: w5, 6: w6}
    # far from equilibrium, so that every order carries cumulants well above rounding
    p = torch.from_numpy(inputs.random_distribution_q27(3, 41))
    rho = torch.tensor([0.93, 1.0, 1.08], dtype=torch.float64)
    f = p * rho
    phi = P.scal.w[:, None] * torch.ones(1, 3, dtype=torch.float64)
    fs, _ = C.collide(f, phi, P)
    big = 0.0
    for n in range(3):
        pre = _cumulants((f[:, n] / rho[n]).tolist())
        rs = float(fs[:, n].sum())
        assert abs(rs - float(rho[n])) < 1e-14
        post = _cumulants((fs[:, n] / rs).tolist())
        for key in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):       # no force: mean unchanged
            assert abs(post[key] - pre[key]) < 1e-14, key
        for key in ((1, 1, 0), (1, 0, 1), (0, 1, 1)):       # deviatoric, off-diagonal
            assert abs(post[key] - (1 - w1) * pre[key]) < 1e-14, key
        for a, b in (((2, 0, 0), (0, 2, 0)), ((2, 0, 0), (0, 0, 2))):  # deviatoric, normal
            assert abs((post[a] - post[b]) - (1 - w1) * (pre[a] - pre[b])) < 1e-14, (a, b)
        tr = pre[(2, 0, 0)] + pre[(0, 2, 0)] + pre[(0, 0, 2)]
        trs = post[(2, 0, 0)] + post[(0, 2, 0)] + post[(0, 0, 2)]
        assert abs(trs - ((1 - wb) * tr + wb * 1.0)) < 1e-14
        for key, v in pre.items():
            k = sum(key)
            if k >= 3:
                big = max(big, abs(v))
                assert abs(post[key] - (1 - wk[k]) * v) < 2e-14, (key, k)
    assert big > 1e-3      # the orders >= 3 were exercised


def _near_rest(model, n, seed, eps):
    qf = 19 if model == 1 else 27
    lat_f = L.D3Q19 if model == 1 else L.D3Q27
    lat_s = {0: L.D3Q7, 1: L.D3Q6, 2: L.D3Q27}[model]
    f, phi = inputs.near_rest_state(qf, lat_s.Q, (1, 1, n), lat_f.w.numpy(), lat_s.w.numpy(), seed,
                                    eps=eps, chi_lo=0.2, chi_hi=1.0)
    return torch.from_numpy(f.reshape(qf, n)), torch.from_numpy(phi.reshape(lat_s.Q, n)), lat_f, lat_s


def _covariance(f, lat):
    """rho, mean velocity j / rho and the covariance matrix (3,3,n) of f / rho."""
    c = lat.c.T
    rho = f.sum(0)
    u = (c @ f) / rho
    second = torch.einsum('aq,bq,qn->abn', c, c, f) / rho
    return rho, u, second - u[:, None] * u[None]


@pytest.mark.parametrize("sc_t", [1.0, 0.4])
@pytest.mark.parametrize("model", [0, 1, 2])
def test_turbulent_scalar_diffusivity_follows_eq35(model, sc_t):
    cs = 0.2
    nu = 0.01
    P = derive(Config(4, 4, 4, model=model, g_prime=0.0, re_b=1.0, nu_lu=nu, cs_smag=cs,
                      sc_t=sc_t, sc=0.7))
    tau0 = 3.0 * nu + 0.5
    d0 = nu / 0.7
    cs2p = CS2_PHI[model]
    tau_phi0 = 0.5 + d0 / cs2p
    f, phi, lat_f, lat_s = _near_rest(model, 24, 77, eps=0.1)
    fs, ps = C.collide(f, phi, P)
    rho, u, cov = _covariance(f, lat_f)
    rho_s, u_s, cov_s = _covariance(fs, lat_f)
    assert torch.allclose(rho_s, rho, rtol=0, atol=1e-15)
    assert torch.allclose(u_s, u, rtol=0, atol=1e-15)
    # flow relaxation time actually applied, from each off-diagonal pair
    taus = [1.0 / (1.0 - cov_s[a, b] / cov[a, b]) for a, b in ((0, 1), (0, 2), (1, 2))]
    tau_f = taus[0]
    for t in taus[1:]:
        assert torch.allclose(t, tau_f, rtol=1e-9, atol=0)
    nu_t = (tau_f - tau0) / 3.0
    assert float(nu_t.min()) > 1e-4          # the eddy viscosity is really on
    # Smagorinsky closure (standard form): nu_T = C_s^2 |S|, |S| = sqrt(2 S:S),
    # S = -Pi / (2 rho cs^2 tau_f), Pi = rho (cov - I/3) the pre-collision stress
    pi = rho * (cov - torch.eye(3, dtype=torch.float64)[:, :, None] / 3.0)
    S = -pi / (2.0 * rho * tau_f / 3.0)
    absS = torch.sqrt(2.0 * (S * S).sum((0, 1)))
    assert torch.allclose(nu_t, cs ** 2 * absS, rtol=1e-9, atol=0)
    # scalar relaxation time actually applied: first moment about chi u
    chi = phi.sum(0)
    assert torch.allclose(ps.sum(0), chi, rtol=0, atol=1e-15)
    cphi = lat_s.c.T
    flux = cphi @ phi - chi * u
    flux_s = cphi @ ps - chi * u
    tps = [1.0 / (1.0 - flux_s[a] / flux[a]) for a in range(3)]
    for t in tps[1:]:
        assert torch.allclose(t, tps[0], rtol=1e-9, atol=0)
    tau_phi = tps[0]
    # Eq. 30 on the scalar lattice, Eq. 35: D0 + nu_T / Sc_T
    assert torch.allclose(cs2p * (tau_phi - 0.5), d0 + nu_t / sc_t, rtol=1e-9, atol=0)
    assert torch.allclose((tau_phi - tau_phi0) * cs2p, (tau_f - tau0) / 3.0 / sc_t, rtol=1e-8, atol=0)


@pytest.mark.parametrize("model", [0, 1, 2])
def test_turbulent_diffusivity_in_the_printed_closure(model):
    """The same with the Smagorinsky closure as printed in Eq. 32
    (nu_T = C_s |S|): the scalar side is unchanged, only C_s enters to the
    first power."""
    cs = 0.04
    nu = 0.01
    P = derive(Config(4, 4, 4, model=model, g_prime=0.0, re_b=1.0, nu_lu=nu, cs_smag=cs,
                      sc_t=0.5, smag_paper_form=True))
    tau0 = 3.0 * nu + 0.5
    cs2p = CS2_PHI[model]
    f, phi, lat_f, lat_s = _near_rest(model, 12, 78, eps=0.1)
    fs, ps = C.collide(f, phi, P)
    rho, u, cov = _covariance(f, lat_f)
    _, _, cov_s = _covariance(fs, lat_f)
    tau_f = 1.0 / (1.0 - cov_s[0, 1] / cov[0, 1])
    nu_t = (tau_f - tau0) / 3.0
    pi = rho * (cov - torch.eye(3, dtype=torch.float64)[:, :, None] / 3.0)
    S = -pi / (2.0 * rho * tau_f / 3.0)
    absS = torch.sqrt(2.0 * (S * S).sum((0, 1)))
    assert torch.allclose(nu_t, cs * absS, rtol=1e-9, atol=0)
    chi = phi.sum(0)
    cphi = lat_s.c.T
    tau_phi = 1.0 / (1.0 - (cphi @ ps - chi * u)[2] / (cphi @ phi - chi * u)[2])
    assert torch.allclose(cs2p * (tau_phi - 0.5), nu + nu_t / 0.5, rtol=1e-9, atol=0)
