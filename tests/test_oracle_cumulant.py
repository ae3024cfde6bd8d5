"""Pins of the oracle's cumulant machinery (Eq. 54) and cumulant collision
(Eq. 55-58) against textbook definitions written out independently here."""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import collide as C
from oracle import lattice as L
from oracle import ring
from oracle.params import Config, derive
from tests import inputs

VEL = L.D3Q27.c_list


def _partitions(items):
    """All set partitions of a list (recursive, textbook)."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def _joint_cumulant(p, axes):
    """Joint cumulant of the coordinates listed in `axes` (e.g. [0,0,1]) of a
    discrete distribution p on VEL, from the moment-partition formula
    kappa = sum_pi (|pi|-1)! (-1)^(|pi|-1) prod_B E[prod_{i in B} X_i]."""
    def moment(block):
        return sum(pq * math.prod(c[a] for a in block) for pq, c in zip(p, VEL))
    tot = 0.0
    for part in _partitions(list(axes)):
        k = len(part)
        tot += math.factorial(k - 1) * (-1) ** (k - 1) * math.prod(moment(b) for b in part)
    return tot


def _moments(p):
    m = torch.zeros(3, 3, 3, 1, dtype=torch.float64)
    for a, b, c in itertools.product(range(3), repeat=3):
        m[a, b, c, 0] = sum(pq * cq[0] ** a * cq[1] ** b * cq[2] ** c for pq, cq in zip(p, VEL))
    return m


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ring_cumulants_match_partition_formula(seed):
    """Raw (non-central) moments of a random distribution; every cumulant with
    exponents <= 2 equals the set-partition formula."""
    p = inputs.random_distribution_q27(1, seed)[:, 0]
    Cr = ring.cumulants_from_moments(_moments(p))
    for a, b, c in itertools.product(range(3), repeat=3):
        if a + b + c == 0:
            continue
        want = _joint_cumulant(p, [0] * a + [1] * b + [2] * c)
        assert abs(float(Cr[a, b, c, 0]) - want) < 1e-14, (a, b, c)


def test_ring_exp_inverts_log():
    p = torch.from_numpy(inputs.random_distribution_q27(64, 7))
    m = torch.zeros(3, 3, 3, 64, dtype=torch.float64)
    for q, cq in enumerate(VEL):
        for a, b, c in itertools.product(range(3), repeat=3):
            m[a, b, c] += p[q] * cq[0] ** a * cq[1] ** b * cq[2] ** c
    back = ring.moments_from_cumulants(ring.cumulants_from_moments(m))
    assert torch.allclose(back, m, rtol=0, atol=1e-14)


def test_product_distribution_has_no_mixed_cumulants():
    rng = np.random.default_rng(3)
    px, py, pz = (rng.dirichlet(np.ones(3)) for _ in range(3))
    p = [px[c[0] + 1] * py[c[1] + 1] * pz[c[2] + 1] for c in VEL]
    Cr = ring.cumulants_from_moments(_moments(p))
    for a, b, c in itertools.product(range(3), repeat=3):
        if sum(x > 0 for x in (a, b, c)) >= 2:
            assert abs(float(Cr[a, b, c, 0])) < 1e-14


def _params(**kw):
    base = dict(nx=4, ny=4, nz=8, model=0, re_b=300.0, g_prime=1e-4)
    base.update(kw)
    return derive(Config(**base))


def _product_equilibrium(rho, u):
    """Discrete Maxwellian in product form: each axis has mean u_a and second
    central moment 1/3: p(+-1) = (1/3 + u^2 +- u)/2, p(0) = 2/3 - u^2."""
    f = torch.zeros(27, rho.shape[0], dtype=torch.float64)
    for q, c in enumerate(VEL):
        v = rho.clone()
        for a in range(3):
            ua = u[a]
            v = v * ((2.0 / 3.0 - ua * ua) if c[a] == 0 else (1.0 / 3.0 + ua * ua + c[a] * ua) / 2.0)
        f[q] = v
    return f


@pytest.mark.parametrize("rates", [(1, 1, 1, 1, 1), (1.3, 0.7, 1.4, 0.6, 1.9)])
def test_equilibrium_is_a_fixed_point(rates):
    """With F = 0 the product-form Maxwellian has equilibrium cumulants; the
    collision must return it unchanged for any relaxation rates."""
    P = _params(g_prime=0.0, re_b=1.0, nu_lu=0.05, omega_bulk=rates[0], omega3=rates[1],
                omega4=rates[2], omega5=rates[3], omega6=rates[4])
    rng = np.random.default_rng(5)
    n = 32
    rho = torch.from_numpy(rng.uniform(0.9, 1.1, n))
    u = torch.from_numpy(rng.uniform(-0.1, 0.1, (3, n)))
    f = _product_equilibrium(rho, u)
    phi = torch.zeros(7, n, dtype=torch.float64)
    fs, _ = C.collide(f, phi, P)
    assert torch.allclose(fs, f, rtol=0, atol=2e-16 * 8)


def _random_state(n, seed, eps=2e-2):
    f, phi = inputs.near_rest_state(27, 7, (1, 1, n), L.D3Q27.w.numpy(), L.D3Q7.w.numpy(), seed, eps=eps)
    return torch.from_numpy(f.reshape(27, n)), torch.from_numpy(phi.reshape(7, n))


@pytest.mark.parametrize("cs", [0.0, 0.1])
def test_cumulant_conserves_mass_and_adds_force(cs):
    P = _params(cs_smag=cs, g_prime=3e-3)
    f, phi = _random_state(50, 11)
    rho, j, chi, F, u = C.macroscopic(f, phi, P)
    fs, ps = C.collide(f, phi, P)
    c = L.D3Q27.c.T
    assert torch.allclose(fs.sum(0), rho, rtol=0, atol=1e-15)
    assert torch.allclose(c @ fs, j + F, rtol=0, atol=1e-15)
    assert torch.allclose(ps.sum(0), chi, rtol=0, atol=1e-15)


def _wick(Cs):
    """Moments of a zero-mean Gaussian with covariance entries Cs[(a,b)],
    truncated at exponent 2 per axis (Isserlis/Wick)."""
    xx, yy, zz = Cs[(0, 0)], Cs[(1, 1)], Cs[(2, 2)]
    xy, xz, yz = Cs[(0, 1)], Cs[(0, 2)], Cs[(1, 2)]
    m = {}
    m[(2, 0, 0)], m[(0, 2, 0)], m[(0, 0, 2)] = xx, yy, zz
    m[(1, 1, 0)], m[(1, 0, 1)], m[(0, 1, 1)] = xy, xz, yz
    m[(2, 2, 0)] = xx * yy + 2 * xy * xy
    m[(2, 0, 2)] = xx * zz + 2 * xz * xz
    m[(0, 2, 2)] = yy * zz + 2 * yz * yz
    m[(2, 1, 1)] = xx * yz + 2 * xy * xz
    m[(1, 2, 1)] = yy * xz + 2 * xy * yz
    m[(1, 1, 2)] = zz * xy + 2 * xz * yz
    m[(2, 2, 2)] = (xx * yy * zz + 2 * (xx * yz * yz + yy * xz * xz + zz * xy * xy)
                    + 8 * xy * xz * yz)
    return m


@pytest.mark.parametrize("cs", [0.0, 0.1])
def test_post_collision_moments_are_wick_of_relaxed_covariance(cs):
    """With omega3..6 = 1 every cumulant above second order is reset to zero,
    so the post-collision central moments about the post-collision mean
    (j + F)/rho are rho times the Gaussian (Wick) moments of the relaxed
    covariance; the pre-collision covariance is the central second moment
    about the pre-collision mean j/rho."""
    P = _params(cs_smag=cs, g_prime=3e-3, omega_bulk=1.2)
    f, phi = _random_state(40, 12)
    rho, j, chi, F, u = C.macroscopic(f, phi, P)
    k = C.central_moments(f, j / rho, L.D3Q27)
    idx = {(0, 0): (2, 0, 0), (1, 1): (0, 2, 0), (2, 2): (0, 0, 2),
           (0, 1): (1, 1, 0), (0, 2): (1, 0, 1), (1, 2): (0, 1, 1)}
    cov = {ab: k[ijk] / rho for ab, ijk in idx.items()}
    # relaxed covariance (independent restatement of the reading)
    pi = torch.zeros(3, 3, rho.shape[0], dtype=torch.float64)
    for (a, b), v in cov.items():
        pi[a, b] = pi[b, a] = rho * (v - (1 / 3 if a == b else 0))
    if cs > 0:
        Q = (pi * pi).sum((0, 1))
        tau = 0.5 * (P.tau0 + torch.sqrt(P.tau0 ** 2 + 18 * math.sqrt(2) * cs ** 2 * torch.sqrt(Q) / rho))
    else:
        tau = torch.full_like(rho, P.tau0)
    w1, w2 = 1 / tau, 1.2
    tr = cov[(0, 0)] + cov[(1, 1)] + cov[(2, 2)]
    trs = tr + w2 * (1 - tr)
    rel = {}
    for a in range(3):
        rel[(a, a)] = trs / 3 + (1 - w1) * (cov[(a, a)] - tr / 3)
    for ab in [(0, 1), (0, 2), (1, 2)]:
        rel[ab] = (1 - w1) * cov[ab]
    want = _wick(rel)
    fs, _ = C.collide(f, phi, P)
    ks = C.central_moments(fs, (j + F) / rho, L.D3Q27)
    assert torch.allclose(ks[0, 0, 0], rho, atol=1e-15, rtol=0)
    for a, b, c in itertools.product(range(3), repeat=3):
        o = a + b + c
        if o < 1:
            continue
        expect = rho * want[(a, b, c)] if (a, b, c) in want else torch.zeros_like(rho)
        assert torch.allclose(ks[a, b, c], expect, atol=2e-15, rtol=0), (a, b, c)


def _cube_symmetries():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            yield perm, signs


@pytest.mark.parametrize("model", [0, 1, 2])
def test_collision_commutes_with_the_48_cube_symmetries(model):
    """No force (g' = 0): rotating/reflecting the populations commutes with the
    collision, for general rates and LES on."""
    P = _params(model=model, g_prime=0.0, re_b=1.0, nu_lu=0.02, cs_smag=0.1,
                omega_bulk=1.1, omega3=0.9, omega4=1.2, omega5=0.8, omega6=1.3)
    lat_f, lat_s = P.flow, P.scal
    Qs = lat_s.Q
    rng = np.random.default_rng(21)
    n = 8
    f = lat_f.w[:, None] * (1 + 0.05 * torch.from_numpy(rng.standard_normal((lat_f.Q, n))))
    phi = lat_s.w[:, None] * (1 + 0.05 * torch.from_numpy(rng.standard_normal((Qs, n))))
    fs, ps = C.collide(f, phi, P)

    def perm_of(lat, perm, signs):
        out = []
        for c in lat.c_list:
            rc = tuple(signs[a] * c[perm[a]] for a in range(3))
            out.append(lat.c_list.index(rc))
        return out

    for perm, signs in _cube_symmetries():
        pf = perm_of(lat_f, perm, signs)
        pp = perm_of(lat_s, perm, signs)
        f2 = torch.empty_like(f)
        p2 = torch.empty_like(phi)
        f2[pf] = f
        p2[pp] = phi
        fs2, ps2 = C.collide(f2, p2, P)
        assert torch.allclose(fs2[pf], fs, atol=1e-15, rtol=0), (perm, signs)
        assert torch.allclose(ps2[pp], ps, atol=1e-15, rtol=0), (perm, signs)
