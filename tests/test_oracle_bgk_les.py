"""Pins of the oracle's BGK + Guo collision (Eq. 21-26), Smagorinsky closure
(Eq. 32-35) and scalar collision (Eq. 28-30)."""
import math

import numpy as np
import pytest
import torch

from oracle import collide as C
from oracle import lattice as L
from oracle.params import Config, derive
from tests import inputs


def _P(**kw):
    base = dict(nx=4, ny=4, nz=8, model=1, re_b=300.0, g_prime=1e-4)
    base.update(kw)
    return derive(Config(**base))


def _rand_rho_u(n, seed, umax=0.1):
    rng = np.random.default_rng(seed)
    return (torch.from_numpy(rng.uniform(0.9, 1.1, n)),
            torch.from_numpy(rng.uniform(-umax, umax, (3, n))))


def test_feq_moments():
    """sum feq = rho, sum c feq = rho u, sum c c feq = rho (I/3 + u u)."""
    rho, u = _rand_rho_u(20, 1)
    feq = C.feq_q19(rho, u, L.D3Q19)
    c = L.D3Q19.c.T
    assert torch.allclose(feq.sum(0), rho, atol=1e-15, rtol=0)
    assert torch.allclose(c @ feq, rho * u, atol=1e-15, rtol=0)
    pi = torch.einsum('aq,bq,qn->abn', c, c, feq)
    want = rho * (torch.eye(3, dtype=torch.float64)[:, :, None] / 3 + u[:, None] * u[None])
    assert torch.allclose(pi, want, atol=1e-15, rtol=0)


def test_guo_source_moments():
    """sum S = 0, sum c S = (1 - 1/2tau) F, sum c c S = (1 - 1/2tau)(u F + F u)."""
    rho, u = _rand_rho_u(20, 2)
    F = torch.from_numpy(np.random.default_rng(3).uniform(-1e-3, 1e-3, (3, 20)))
    tau = torch.full((20,), 0.8, dtype=torch.float64)
    S = C.guo_source(u, F, tau, L.D3Q19)
    c = L.D3Q19.c.T
    k = 1 - 0.5 / 0.8
    assert torch.allclose(S.sum(0), torch.zeros(20, dtype=torch.float64), atol=1e-18, rtol=0)
    assert torch.allclose(c @ S, k * F, atol=1e-18, rtol=0)
    pi = torch.einsum('aq,bq,qn->abn', c, c, S)
    assert torch.allclose(pi, k * (u[:, None] * F[None] + F[:, None] * u[None]), atol=1e-18, rtol=0)


@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_bgk_equilibrium_fixed_point_without_force(cs):
    P = _P(g_prime=0.0, nu_lu=0.05, cs_smag=cs)
    rho, u = _rand_rho_u(16, 4)
    f = C.feq_q19(rho, u, L.D3Q19)
    phi = torch.zeros(6, 16, dtype=torch.float64)
    fs, _ = C.collide(f, phi, P)
    assert torch.allclose(fs, f, atol=1e-15, rtol=0)


def test_bgk_conserves_mass_and_adds_force():
    P = _P(g_prime=2e-3, cs_smag=0.1)
    f, phi = inputs.near_rest_state(19, 6, (1, 1, 30), L.D3Q19.w.numpy(), L.D3Q6.w.numpy(), 9, eps=2e-2)
    f, phi = torch.from_numpy(f.reshape(19, 30)), torch.from_numpy(phi.reshape(6, 30))
    rho, j, chi, F, u = C.macroscopic(f, phi, P)
    fs, ps = C.collide(f, phi, P)
    assert torch.allclose(fs.sum(0), rho, atol=1e-15, rtol=0)
    assert torch.allclose(L.D3Q19.c.T @ fs, j + F, atol=1e-15, rtol=0)
    assert torch.allclose(ps.sum(0), chi, atol=1e-15, rtol=0)


def test_smagorinsky_root_satisfies_the_closure():
    """tau_f from the closed form satisfies nu_T = C_s^2 |S| with
    nu_T = (tau_f - tau0)/3, S = -Pi/(2 rho cs^2 tau_f), |S| = sqrt(2 S:S)."""
    P = _P(re_b=30000.0)
    rng = np.random.default_rng(7)
    n = 50
    A = torch.from_numpy(rng.standard_normal((3, 3, n)) * 1e-3)
    pi = A + A.transpose(0, 1)
    rho = torch.from_numpy(rng.uniform(0.95, 1.05, n))
    cs = 0.1
    tau = C.smagorinsky_tau(pi, rho, P, cs)
    S = -pi / (2 * rho * tau / 3)
    absS = torch.sqrt(2 * (S * S).sum((0, 1)))
    nu_t = (tau - P.tau0) / 3
    assert torch.allclose(nu_t, cs ** 2 * absS, rtol=1e-12, atol=0)


def test_smagorinsky_uniform_shear():
    """Pure shear du/dz = s: |S| = |s|, so nu_T = C_s^2 |s| (S_xz = s/2)."""
    P = _P(re_b=30000.0)
    s, cs, rho = 2e-3, 0.1, 1.0
    # stress consistent with the total tau: Pi_xz = -2 rho cs^2 tau S_xz; solve
    # tau = tau0 + 3 cs_smag^2 |s| directly (the closure), then build Pi from it
    tau = P.tau0 + 3 * cs ** 2 * abs(s)
    pi = torch.zeros(3, 3, 1, dtype=torch.float64)
    pi[0, 2] = pi[2, 0] = -2 * rho * (1 / 3) * tau * (s / 2)
    got = C.smagorinsky_tau(pi, torch.tensor([rho], dtype=torch.float64), P, cs)
    assert abs(float(got[0]) - tau) < 1e-15


def test_smagorinsky_printed_form():
    """The closure as printed in Eq. 32 (nu_T = C_s |S|, Delta = 1): uniform
    shear gives nu_T = C_s |s|, and the form equals the standard one at
    C_s' = sqrt(C_s)."""
    import dataclasses
    P = _P(re_b=30000.0)
    Pp = dataclasses.replace(P, cfg=dataclasses.replace(P.cfg, smag_paper_form=True))
    s, cs, rho = 2e-3, 0.03, 1.0
    tau = P.tau0 + 3 * cs * abs(s)
    pi = torch.zeros(3, 3, 1, dtype=torch.float64)
    pi[0, 2] = pi[2, 0] = -2 * rho * (1 / 3) * tau * (s / 2)
    got = C.smagorinsky_tau(pi, torch.tensor([rho], dtype=torch.float64), Pp, cs)
    assert abs(float(got[0]) - tau) < 1e-15
    rng = np.random.default_rng(8)
    A = torch.from_numpy(rng.standard_normal((3, 3, 20)) * 1e-3)
    pi = A + A.transpose(0, 1)
    r = torch.from_numpy(rng.uniform(0.95, 1.05, 20))
    assert torch.allclose(C.smagorinsky_tau(pi, r, Pp, cs), C.smagorinsky_tau(pi, r, P, cs ** 0.5),
                          rtol=1e-15, atol=0)


def test_les_off_is_bitwise_the_plain_path():
    f, phi = inputs.near_rest_state(27, 7, (1, 1, 40), L.D3Q27.w.numpy(), L.D3Q7.w.numpy(), 3, eps=1e-2)
    f, phi = torch.from_numpy(f.reshape(27, 40)), torch.from_numpy(phi.reshape(7, 40))
    for model in (0, 1):
        P = _P(model=model, cs_smag=0.0)
        if model == 1:
            ff, pp = f[:19].clone(), phi[1:].clone()
        else:
            ff, pp = f, phi
        a = C.collide(ff, pp, P)
        rho, j, chi, F, u = C.macroscopic(ff, pp, P)
        if model == 0:
            fs, tau = C.collide_cumulant(ff, rho, j, F, P, 0.0)
        else:
            fs, tau = C.collide_bgk(ff, rho, u, F, P, 0.0)
        assert torch.equal(tau, torch.full_like(rho, P.tau0))
        assert torch.equal(a[0], fs)


def test_scalar_collision_moments():
    """phi* keeps chi; the equilibrium flux is chi u (Eq. 29 with the scalar
    lattice's cs^2)."""
    for model, lat in ((0, L.D3Q7), (1, L.D3Q6)):
        P = _P(model=model)
        rng = np.random.default_rng(8)
        n = 10
        chi = torch.from_numpy(rng.uniform(0, 1, n))
        u = torch.from_numpy(rng.uniform(-0.1, 0.1, (3, n)))
        phi = lat.w[:, None] * chi[None] * (1 + 0.1 * torch.from_numpy(rng.standard_normal((lat.Q, n))))
        chi = phi.sum(0)
        tau = torch.full((n,), 0.7, dtype=torch.float64)
        ps = C.collide_scalar(phi, chi, u, tau, P)
        assert torch.allclose(ps.sum(0), chi, atol=1e-15, rtol=0)
        # with tau = 1 phi* is the equilibrium, whose flux is chi u
        ps1 = C.collide_scalar(phi, chi, u, torch.ones(n, dtype=torch.float64), P)
        assert torch.allclose(lat.c.T @ ps1, chi * u, atol=1e-15, rtol=0)


def test_parameters_follow_the_lattice_unit_scaling():
    """Sec. 2.5: U_b = sqrt(g' H), nu = U_b H / Re_b, tau = 3 nu + 1/2, and the
    paper's own convention U_b = 0.03 gives g' = 0.03^2 / N3."""
    P = derive(Config(1024, 64, 128, model=0, re_b=30000.0))
    assert math.isclose(P.u_b, math.sqrt(1e-4 * 128), rel_tol=1e-15)
    assert math.isclose(P.nu0, P.u_b * 128 / 30000.0, rel_tol=1e-15)
    assert math.isclose(P.tau0, 3 * P.nu0 + 0.5, rel_tol=1e-15)
    assert math.isclose(P.tau_phi0, 0.5 + P.nu0 * 4, rel_tol=1e-15)  # D3Q7 cs^2 = 1/4, Sc = 1
    P2 = derive(Config(1500, 100, 100, model=1, re_b=1000.0, ub_lu=0.03))
    assert math.isclose(P2.g_prime, 0.03 ** 2 / 100, rel_tol=1e-15)
    assert math.isclose(P2.u_b, 0.03, rel_tol=1e-15)
    assert math.isclose(P2.nu0, 100 * 0.03 / 1000.0, rel_tol=1e-15)
    assert math.isclose(P2.tau_phi0, 0.5 + 3 * P2.nu0, rel_tol=1e-15)
