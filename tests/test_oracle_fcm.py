"""Pins of the oracle's factorized-central-moment (FCM) scalar collision on
D3Q27 (Eq. 37-51), the scalar of the cumulant + FCM model.

* The factorization (Eq. 44-49) vanishes on product distributions whose
  one-dimensional factors have second central moment 1/3 and any mean: this
  fixes every subtraction coefficient, including the (220) reading.
* The factorization is inverted exactly.
* The product-form equilibrium chi prod_d P(c_d; u_d) is a fixed point for
  any rates; chi is conserved and the first moment relaxes with
  omega_100 = 1/tau_phi about chi u.
* With the higher rates at 1 the post-collision populations have the closed
  form chi P P P + sum_d K_d Q_d P P (derived from the moment table).
* Streaming + collision in a periodic box at rest obeys the exact discrete
  recurrences of the first and second spatial moments of chi, whose growth
  rate is 2D with D = (1/omega_100 - 1/2)/3 (Eq. 51); in a uniform flow the
  centre of mass moves exactly u0 per step.
"""
import itertools

import pytest
import torch

from oracle import collide as oc
from oracle import lbm as olbm
from oracle.lattice import D3Q27
from oracle.params import Config, derive


def _p1d(u, mean_dev=None):
    """Three-point distribution on c = -1, 0, 1 with second central moment
    1/3 about u and first central moment mean_dev (default 0): values at
    c = -1, 0, +1 (rows) for each u (columns)."""
    a = torch.zeros_like(u) if mean_dev is None else mean_dev
    # central moments about u: sum p = 1, sum (c-u) p = a, sum (c-u)^2 p = 1/3
    # -> raw: m1 = u + a, m2 = 1/3 + u^2 + 2 u a
    m1 = u + a
    m2 = 1.0 / 3.0 + u * u + 2.0 * u * a
    return torch.stack([(m2 - m1) / 2, 1.0 - m2, (m2 + m1) / 2])


def _product(chi, px, py, pz):
    c = D3Q27.c_list
    return torch.stack([chi * px[cx + 1] * py[cy + 1] * pz[cz + 1] for (cx, cy, cz) in c])


def _setup(n=64, seed=0):
    g = torch.Generator().manual_seed(seed)
    u = 0.1 * (2 * torch.rand(3, n, generator=g, dtype=torch.float64) - 1)
    chi = 0.2 + torch.rand(n, generator=g, dtype=torch.float64)
    return g, u, chi


def test_factorization_vanishes_on_products_with_variance_one_third():
    g, u, chi = _setup()
    means = 0.2 * (2 * torch.rand(3, u.shape[1], generator=g, dtype=torch.float64) - 1)
    phi = _product(chi, _p1d(u[0], means[0]), _p1d(u[1], means[1]), _p1d(u[2], means[2]))
    M = oc.fcm_factorize(oc.central_moments(phi, u, D3Q27))
    checked = 0
    for a, b, c in itertools.product(range(3), repeat=3):
        if 2 in (a, b, c):      # every pattern of Eq. 44-49
            assert torch.abs(M[a, b, c]).max() < 1e-15, (a, b, c)
            checked += 1
    assert checked == 19
    # and the moments without a 2 are the products of the factor means
    assert torch.allclose(M[1, 1, 0], chi * means[0] * means[1], atol=1e-16)
    assert torch.allclose(M[1, 1, 1], chi * means[0] * means[1] * means[2], atol=1e-16)


def test_factorization_is_inverted_exactly():
    g = torch.Generator().manual_seed(1)
    kappa = torch.rand(3, 3, 3, 50, generator=g, dtype=torch.float64)
    assert torch.allclose(oc.fcm_unfactorize(oc.fcm_factorize(kappa)), kappa, atol=1e-15, rtol=0)


def _P(cfg_kw=None):
    return derive(Config(8, 8, 8, model=2, **(cfg_kw or {})))


@pytest.mark.parametrize("tau_phi,omega_high", [(0.8, 1.0), (0.53, 1.0), (1.7, 0.6), (0.6, 1.45)])
def test_equilibrium_is_a_fixed_point(tau_phi, omega_high):
    _, u, chi = _setup(seed=2)
    phi = _product(chi, _p1d(u[0]), _p1d(u[1]), _p1d(u[2]))
    out = oc.collide_fcm(phi, chi, u, torch.full_like(chi, tau_phi), _P(), omega_high)
    assert torch.abs(out - phi).max() < 1e-15


@pytest.mark.parametrize("omega_high", [1.0, 0.7])
def test_conservation_and_first_moment_relaxation(omega_high):
    g, u, chi = _setup(seed=3)
    phi = chi * (D3Q27.w[:, None] * (1 + 0.3 * torch.rand(27, chi.shape[0], generator=g, dtype=torch.float64)))
    chi = phi.sum(0)
    tau = 0.5 + torch.rand(chi.shape[0], generator=g, dtype=torch.float64)
    out = oc.collide_fcm(phi, chi, u, tau, _P(), omega_high)
    c = D3Q27.c.T.to(torch.float64)
    assert torch.abs(out.sum(0) - chi).max() < 1e-15
    j, js = c @ phi, c @ out
    want = chi * u + (1 - 1 / tau) * (j - chi * u)
    assert torch.abs(js - want).max() < 1e-15


def test_closed_form_with_unit_higher_rates():
    g, u, chi = _setup(seed=4)
    phi = chi * (D3Q27.w[:, None] * (1 + 0.5 * torch.rand(27, chi.shape[0], generator=g, dtype=torch.float64)))
    chi = phi.sum(0)
    tau = 0.5 + torch.rand(chi.shape[0], generator=g, dtype=torch.float64)
    out = oc.collide_fcm(phi, chi, u, tau, _P(), 1.0)
    K = (1 - 1 / tau) * (D3Q27.c.T.to(torch.float64) @ phi - chi * u)
    P = [_p1d(u[d]) for d in range(3)]
    Q = [torch.stack([u[d] - 0.5, -2 * u[d], u[d] + 0.5]) for d in range(3)]
    want = _product(chi, P[0], P[1], P[2]) + _product(K[0], Q[0], P[1], P[2]) \
        + _product(K[1], P[0], Q[1], P[2]) + _product(K[2], P[0], P[1], Q[2])
    assert torch.abs(out - want).max() < 1e-15


def _box(n, u0=(0.0, 0.0, 0.0)):
    cfg = Config(n, n, n, model=2, re_b=100.0, g_prime=0.0, nu_lu=0.05, periodic_x=True,
                 periodic_z=True)
    P = derive(cfg)
    # flow: the product-form equilibrium at rho = 1 and uniform u0 (fixed point
    # of the cumulant collision; uniform, so streaming keeps it)
    u = torch.tensor(u0, dtype=torch.float64)[:, None]
    one = torch.ones(1, dtype=torch.float64)
    f1 = _product(one, _p1d(u[0]), _p1d(u[1]), _p1d(u[2]))[:, 0]
    f = f1[:, None, None, None].expand(27, n, n, n).clone()
    # scalar: a compact blob (zero outside the central 6^3 block)
    g = torch.Generator().manual_seed(5)
    chi = torch.zeros(n, n, n, dtype=torch.float64)
    s = slice(n // 2 - 3, n // 2 + 3)
    chi[s, s, s] = torch.rand(6, 6, 6, generator=g, dtype=torch.float64)
    peq = _product(chi.reshape(-1), *[_p1d(torch.full((n ** 3,), u0[d], dtype=torch.float64)) for d in range(3)])
    return P, f, peq.reshape(27, n, n, n)


def _spatial(chi, axis):
    n = chi.shape[0]
    x = torch.arange(n, dtype=torch.float64)
    shape = [1, 1, 1]
    shape[axis] = n
    return x.reshape(shape)


def test_diffusion_recurrence_gives_eq51():
    n, steps = 24, 8
    P, f, phi = _box(n)
    w = 1.0 / P.tau_phi0
    X = phi.sum().item()
    c = D3Q27.c
    xs = [_spatial(phi[0], a) for a in range(3)]
    # axis 2 of the storage is x (c_x), axis 1 is y, axis 0 is z
    comp = {2: 0, 1: 1, 0: 2}
    V = {a: (xs[a] ** 2 * phi.sum(0)).sum().item() for a in range(3)}
    S = {a: (xs[a] * (c[:, comp[a]].to(torch.float64)[:, None, None, None] * phi).sum(0)).sum().item()
         for a in range(3)}
    for _ in range(steps):
        f, phi = olbm.step(f, phi, P)
        for a in range(3):
            V[a] = V[a] + 2 * (1 - w) * S[a] + X / 3
            S[a] = (1 - w) * S[a] + X / 3
            got_v = (xs[a] ** 2 * phi.sum(0)).sum().item()
            got_s = (xs[a] * (c[:, comp[a]].to(torch.float64)[:, None, None, None] * phi).sum(0)).sum().item()
            assert abs(got_v - V[a]) < 1e-10 * V[a], (a, got_v, V[a])
            assert abs(got_s - S[a]) < 1e-10 * max(1.0, abs(S[a]))
    # asymptotic growth per step 2 D X with D = (1/w - 1/2)/3 (Eq. 51)
    D = (1 / w - 0.5) / 3
    assert abs(2 * (1 - w) * X / (3 * w) + X / 3 - 2 * D * X) < 1e-12 * X


def test_uniform_flow_carries_the_centre_of_mass():
    n, steps, u0 = 24, 6, (0.07, -0.04, 0.05)
    P, f, phi = _box(n, u0)
    X = phi.sum().item()
    xs = [_spatial(phi[0], a) for a in range(3)]
    m0 = [(xs[a] * phi.sum(0)).sum().item() for a in range(3)]
    for k in range(1, steps + 1):
        f, phi = olbm.step(f, phi, P)
        for a, d in ((2, 0), (1, 1), (0, 2)):
            got = (xs[a] * phi.sum(0)).sum().item()
            assert abs(got - (m0[a] + k * u0[d] * X)) < 1e-11 * X


@pytest.mark.parametrize("omega_high", [1.0, 0.7, 1.6])
def test_higher_moments_relax_with_their_rate(omega_high):
    """Eq. 44, 42, 43, 49 with Eq. 50, read back from the central moments of
    the output: k*_200 - chi/3 = (1 - w)(k_200 - chi/3), k*_110 = (1 - w) k_110,
    k*_111 = (1 - w) k_111, k*_222 - chi/27 = (1 - w)(k_222 - chi/27) when the
    first-order moments vanish."""
    g, u, chi = _setup(seed=6)
    phi = chi * (D3Q27.w[:, None] * (1 + 0.4 * torch.rand(27, chi.shape[0], generator=g, dtype=torch.float64)))
    chi = phi.sum(0)
    k = oc.central_moments(phi, u, D3Q27)
    tau = torch.full_like(chi, 1.0)          # omega_100 = 1: first-order moments -> 0
    ks = oc.central_moments(oc.collide_fcm(phi, chi, u, tau, _P(), omega_high), u, D3Q27)
    a = 1.0 - omega_high
    assert torch.abs(ks[1, 0, 0]).max() < 1e-15
    assert torch.abs(ks[2, 0, 0] - chi / 3 - a * (k[2, 0, 0] - chi / 3)).max() < 1e-15
    assert torch.abs(ks[0, 1, 1] - a * k[0, 1, 1]).max() < 1e-15
    assert torch.abs(ks[1, 1, 1] - a * k[1, 1, 1]).max() < 1e-15
    assert torch.abs(ks[2, 2, 2] - chi / 27 - a * (k[2, 2, 2] - chi / 27)).max() < 1e-15
    assert torch.abs(ks[2, 2, 0] - chi / 9 - a * (k[2, 2, 0] - chi / 9)).max() < 1e-15
