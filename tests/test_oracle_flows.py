"""Closed-form pins of the oracle's full time step: shear-wave and
Taylor-Green vortex decay (viscosity, Eq. 25 and 58), Poiseuille flow between half-way bounce-back walls, exact
variance growth of a diffusing scalar (Eq. 30), rest invariance, hydrostatic
balance under the Boussinesq force, conservation and span symmetry."""
import math

import numpy as np
import pytest
import torch

from oracle import collide as C
from oracle import diag, lbm
from oracle.params import Config, derive

torch.set_num_threads(min(8, torch.get_num_threads()))


def _equilibrium(P, rho, u):
    """Equilibrium populations of either model at rho (...) and u (3, ...):
    BGK uses Eq. 22; the cumulant model uses the product-form Maxwellian with
    per-axis mean u_a and central second moment 1/3."""
    shp = rho.shape
    rho_f, u_f = rho.reshape(-1), u.reshape(3, -1)
    if P.cfg.model == 1:
        f = C.feq_q19(rho_f, u_f, P.flow)
    else:
        f = torch.zeros(27, rho_f.shape[0], dtype=torch.float64)
        for q, c in enumerate(P.flow.c_list):
            v = rho_f.clone()
            for a in range(3):
                ua = u_f[a]
                v = v * ((2 / 3 - ua * ua) if c[a] == 0 else (1 / 3 + ua * ua + c[a] * ua) / 2)
            f[q] = v
    return f.reshape(P.flow.Q, *shp)


def _shear_wave_nu(model, L, tau, steps=(20, 120)):
    P = derive(Config(1, 1, L, model=model, g_prime=0.0, nu_lu=(tau - 0.5) / 3,
                      periodic_x=True, periodic_z=True))
    z = torch.arange(L, dtype=torch.float64)
    k = 2 * math.pi / L
    u = torch.zeros(3, L, 1, 1, dtype=torch.float64)
    u[0, :, 0, 0] = 0.01 * torch.sin(k * z)
    f = _equilibrium(P, torch.ones(L, 1, 1, dtype=torch.float64), u)
    phi = torch.zeros(P.scal.Q, L, 1, 1, dtype=torch.float64)
    amps = {}
    for n in range(steps[1] + 1):
        if n in steps:
            _, uu, _ = lbm.moments(f, phi, P)
            amps[n] = float((uu[0, :, 0, 0] * torch.sin(k * z)).sum() * 2 / L)
        f, phi = lbm.step(f, phi, P)
    nu_eff = -math.log(amps[steps[1]] / amps[steps[0]]) / (k * k * (steps[1] - steps[0]))
    return nu_eff, P.nu0


@pytest.mark.parametrize("model", [0, 1])
def test_shear_wave_viscosity_second_order(model):
    """nu_eff -> (tau - 1/2)/3 with an error that falls ~4x per doubling of L."""
    errs = []
    for L in (16, 32):
        nu_eff, nu = _shear_wave_nu(model, L, 0.8)
        errs.append(abs(nu_eff / nu - 1))
    assert errs[1] < 3e-3
    assert errs[0] / errs[1] > 3.0


def _taylor_green_nu(model, L, tau, steps):
    """2-D Taylor-Green vortex in the x-z plane of a periodic box,
    u = U sin(kx) cos(kz), w = -U cos(kx) sin(kz): a solution of the
    incompressible Navier-Stokes equations whose kinetic energy decays as
    exp(-4 nu k^2 t) (each velocity amplitude as exp(-2 nu k^2 t))."""
    P = derive(Config(L, 1, L, model=model, g_prime=0.0, nu_lu=(tau - 0.5) / 3,
                      periodic_x=True, periodic_z=True))
    k = 2 * math.pi / L
    x = torch.arange(L, dtype=torch.float64)
    X = x[None, None, :].expand(L, 1, L)
    Z = x[:, None, None].expand(L, 1, L)
    U = 0.01
    u = torch.zeros(3, L, 1, L, dtype=torch.float64)
    u[0] = U * torch.sin(k * X) * torch.cos(k * Z)
    u[2] = -U * torch.cos(k * X) * torch.sin(k * Z)
    # pressure of the vortex: p = rho U^2 (cos 2kx + cos 2kz) / 4, rho = 1 + 3 p
    rho = 1.0 + 3.0 * U * U * (torch.cos(2 * k * X) + torch.cos(2 * k * Z)) / 4.0
    f = _equilibrium(P, rho, u)
    phi = torch.zeros(P.scal.Q, L, 1, L, dtype=torch.float64)
    amps = {}
    for n in range(steps[1] + 1):
        if n in steps:
            _, uu, _ = lbm.moments(f, phi, P)
            amps[n] = float((uu[0] * torch.sin(k * X) * torch.cos(k * Z)).sum() * 4 / (L * L))
        f, phi = lbm.step(f, phi, P)
    nu_eff = -math.log(amps[steps[1]] / amps[steps[0]]) / (2 * k * k * (steps[1] - steps[0]))
    return nu_eff, P.nu0


@pytest.mark.parametrize("model", [0, 1])
def test_taylor_green_vortex_decay_second_order(model):
    """nu from the decay of the vortex -> (tau - 1/2)/3 (Eq. 25, 58), error
    falling about 4x per doubling of the box (time scaled diffusively)."""
    errs = []
    for L, steps in ((12, (10, 70)), (24, (40, 280))):
        nu_eff, nu = _taylor_green_nu(model, L, 0.8, steps)
        errs.append(abs(nu_eff / nu - 1))
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0


def _poiseuille(model, tau, H, steps):
    Fx = 1e-6
    P = derive(Config(1, 1, H, model=model, g_prime=0.0, nu_lu=(tau - 0.5) / 3,
                      periodic_x=True, body_force=(Fx, 0.0, 0.0)))
    zc = torch.arange(H, dtype=torch.float64) + 0.5
    exact = Fx / (2 * P.nu0) * zc * (H - zc)
    u = torch.zeros(3, H, 1, 1, dtype=torch.float64)
    u[0, :, 0, 0] = exact
    f = _equilibrium(P, torch.ones(H, 1, 1, dtype=torch.float64), u)
    phi = torch.zeros(P.scal.Q, H, 1, 1, dtype=torch.float64)
    for _ in range(steps):
        f, phi = lbm.step(f, phi, P)
    _, uu, _ = lbm.moments(f, phi, P)
    return uu[0, :, 0, 0], exact


def test_poiseuille_bgk_exact_at_magic_tau():
    """BGK with half-way bounce-back reproduces the parabola exactly at
    tau = 1/2 + sqrt(3/16)."""
    got, exact = _poiseuille(1, 0.5 + math.sqrt(3 / 16), 8, 1800)
    assert torch.allclose(got, exact, rtol=1e-9, atol=0)


@pytest.mark.parametrize("model", [0, 1])
def test_poiseuille_second_order(model):
    errs = []
    for H, steps in ((4, 300), (8, 600)):
        got, exact = _poiseuille(model, 1.0, H, steps)
        errs.append(float((got - exact).abs().max() / exact.max()))
    assert errs[1] < 0.02
    assert errs[0] / errs[1] > 3.0


@pytest.mark.parametrize("model", [0, 1, 2])
def test_scalar_variance_follows_the_exact_recurrence(model):
    """u = 0 (no force): second moment M2 of chi obeys
    M2(t+1) = M2(t) + 2(1-w) K(t) + cs^2 M0, K(t) = cs^2 M0 (1 - (1-w)^t) / w,
    so the variance grows by 2 D = 2 cs^2 (tau_phi - 1/2) per step asymptotically."""
    L = 64
    P = derive(Config(L, 1, 1, model=model, g_prime=0.0, nu_lu=0.04, sc=0.5,
                      periodic_x=True, periodic_z=True))
    x = torch.arange(L, dtype=torch.float64) - L / 2
    chi = torch.exp(-x * x / (2 * 2.0 ** 2)).reshape(1, 1, L)
    f, phi = lbm.init_state(P, chi)
    cs2 = P.scal.cs2
    w = 1 / P.tau_phi0
    M0 = float(chi.sum())

    def m2(phi):
        c = phi.sum(0)[0, 0]
        return float((x * x * c).sum())

    M2 = m2(phi)
    K = 0.0
    for t in range(80):
        f, phi = lbm.step(f, phi, P)
        M2 = M2 + 2 * (1 - w) * K + cs2 * M0
        K = (1 - w) * K + cs2 * M0
        assert abs(m2(phi) - M2) < 1e-10 * M2, t
    D = cs2 * (P.tau_phi0 - 0.5)
    slope = (2 * (1 - w) * K + cs2 * M0) / M0
    assert abs(slope - 2 * D) < 1e-12
    assert math.isclose(D, P.nu0 / 0.5, rel_tol=1e-14)


@pytest.mark.parametrize("model", [0, 1, 2])
def test_rest_state_is_invariant(model):
    """g' = 0 and arbitrary chi: the flow stays exactly at rest, chi diffuses."""
    cfg = Config(12, 3, 6, model=model, g_prime=0.0, nu_lu=0.01)
    P = derive(cfg)
    chi0 = torch.from_numpy(np.random.default_rng(0).uniform(0, 1, (6, 3, 12)))
    f, phi = lbm.init_state(P, chi0)
    w = P.flow.w[:, None, None, None]
    for _ in range(10):
        f, phi = lbm.step(f, phi, P)
    assert float((f - w).abs().max()) < 1e-15     # rounding of the generic route
    assert not torch.equal(phi.sum(0), chi0)


def test_uniform_scalar_is_invariant_without_gravity():
    cfg = Config(8, 2, 4, model=0, g_prime=0.0, nu_lu=0.01)
    P = derive(cfg)
    f, phi = lbm.init_state(P, torch.full((4, 2, 8), 0.3, dtype=torch.float64))
    for _ in range(5):
        f, phi = lbm.step(f, phi, P)
    assert float((phi.sum(0) - 0.3).abs().max()) < 1e-15


@pytest.mark.parametrize("model", [0, 1, 2])
def test_hydrostatic_balance(model):
    """Uniform chi in a closed box: the flow comes to rest and
    delta rho(z) has slope -g' chi / cs^2 = -3 g' chi."""
    g = 1e-3
    cfg = Config(4, 1, 8, model=model, g_prime=g, nu_lu=0.1)
    P = derive(cfg)
    f, phi = lbm.init_state(P, torch.ones(8, 1, 4, dtype=torch.float64))
    for _ in range(400):
        f, phi = lbm.step(f, phi, P)
    rho, u, chi = lbm.moments(f, phi, P)
    # a staggered acoustic mode of amplitude ~3e-7 decays slowly in both models;
    # an O(F) error in the force coupling leaves ~2e-4 here
    assert float(u.abs().max()) < 1e-6
    slope = (rho[1:, 0, :] - rho[:-1, 0, :])
    assert torch.allclose(slope, torch.full_like(slope, -3 * g), rtol=1e-4, atol=0)


@pytest.mark.parametrize("model", [0, 1, 2])
def test_lock_exchange_conserves_mass_and_scalar(model):
    cfg = Config(64, 4, 8, model=model, re_b=1000.0, cs_smag=0.1)
    P = derive(cfg)
    f, phi = lbm.init_state(P, lbm.chi0_lock_exchange(cfg, seed=1))
    d0 = diag.diagnostics(f, phi, P)
    for _ in range(150):
        f, phi = lbm.step(f, phi, P)
    d = diag.diagnostics(f, phi, P, 150)
    assert abs(d['mass'] - d0['mass']) / d0['mass'] < 1e-13
    assert abs(d['chi_mass'] - d0['chi_mass']) / d0['chi_mass'] < 1e-13
    assert d['nonfinite'] == 0
    assert d['x_f'] > 0.0


@pytest.mark.parametrize("model", [0, 1, 2])
def test_span_symmetry_without_noise(model):
    cfg = Config(32, 3, 8, model=model, re_b=1000.0, cs_smag=0.1)
    P = derive(cfg)
    f, phi = lbm.init_state(P, lbm.chi0_lock_exchange(cfg, amp=0.0))
    for _ in range(30):
        f, phi = lbm.step(f, phi, P)
    for j in range(1, 3):
        assert torch.equal(f[:, :, j], f[:, :, 0])
        assert torch.equal(phi[:, :, j], phi[:, :, 0])


@pytest.mark.parametrize("model", [0, 1, 2])
def test_sampled_step_equals_full_step(model):
    cfg = Config(20, 3, 6, model=model, re_b=500.0, cs_smag=0.1)
    P = derive(cfg)
    f, phi = lbm.init_state(P, lbm.chi0_lock_exchange(cfg, seed=2))
    for _ in range(3):
        f, phi = lbm.step(f, phi, P)
    f1, p1 = lbm.step(f, phi, P)
    nodes = [(0, 0, 0), (5, 2, 19), (2, 1, 2), (3, 0, 10), (0, 2, 19), (5, 0, 0)]
    sf, sp = lbm.step_at(f, phi, P, nodes)
    for m, (k, j, i) in enumerate(nodes):       # batch size changes BLAS summation order
        assert torch.allclose(sf[:, m], f1[:, k, j, i], rtol=0, atol=1e-15)
        assert torch.allclose(sp[:, m], p1[:, k, j, i], rtol=0, atol=1e-15)
