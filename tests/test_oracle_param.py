"""Pins of the oracle's parametrised cumulant collision (Sec. 2.3, the method
the paper's VirtualFluids runs use: third-order rates chosen for fourth-order
accurate shear diffusion, fourth-order equilibria from velocity gradients and
a limiter on the third-order relaxation).

The dispersion pins work in Fourier space on the oracle itself: the collision
is linearised about the rest state with autograd (an exact Jacobian J), and
one time step of a periodic lattice acting on a plane wave exp(i k.x) is
M(k) = diag(exp(-i k.c_q)) J (pull streaming). The hydrodynamic shear mode is
the eigenvalue lambda(k) of M(k) whose eigenvector carries the transverse
momentum; its effective viscosity is nu(k) = -ln|lambda| / |k|^2.

* Any kinetic relaxation of the stress with relaxation time
  tau = nu / cs^2 turns the shear diffusion into s + tau s^2 = -nu k^2,
  so -s / k^2 = nu (1 + 3 nu^2 k^2) for every scheme. The parametrisation
  removes every other k^2 term (the lattice and third-order ones, which are
  anisotropic). The pin: e(k) = nu(k)/nu - 1 - 3 nu^2 k^2 falls as k^4 in
  four wave orientations (axis, two face diagonals, body diagonal), while for
  the standard cumulant (every higher rate 1) it falls as k^2. A dropped
  term, a wrong coefficient or swapped rates leave a k^2 remainder.
* The gradient estimates (Chapman-Enskog, first order) are checked against
  the exact derivative of an eigenmode's velocity, for a shear and a
  longitudinal (sound) mode; the latter fixes the trace term.
"""
import math

import numpy as np
import pytest
import torch

from oracle import collide as C
from oracle import lbm as olbm
from oracle import ring
from oracle.lattice import D3Q27
from oracle.params import Config, derive

CV = D3Q27.c.numpy()


def _params(w1, w2, parametrized, limiter=0.0, model=0):
    nu = (1.0 / w1 - 0.5) / 3.0
    cfg = Config(8, 8, 8, model=model, g_prime=0.0, nu_lu=nu, omega_bulk=w2,
                 parametrized=parametrized, limiter=limiter)
    return derive(cfg), nu


def _jacobian(P):
    """Exact Jacobian of the flow collision at the rest state (no scalar)."""
    phi = torch.zeros(P.scal.Q, 1, dtype=torch.float64)

    def fn(x):
        return C.collide(x[:, None], phi, P)[0][:, 0]
    return torch.autograd.functional.jacobian(fn, D3Q27.w.clone()).numpy()


def _mode(J, kvec, dvec, pick_positive_phase=False):
    """Eigenpair of M(k) whose eigenvector has the largest momentum along
    dvec (among |lambda| > 1/2; with pick_positive_phase, Im lambda > 0)."""
    M = np.diag(np.exp(-1j * (CV @ kvec))) @ J
    ev, V = np.linalg.eig(M)
    proj = np.abs((CV @ dvec) @ V) / np.linalg.norm(V, axis=0)
    ok = np.abs(ev) > 0.5
    if pick_positive_phase:
        ok &= ev.imag > 0
    i = int(np.argmax(np.where(ok, proj, -1.0)))
    return ev[i], V[:, i]


ORIENTATIONS = {
    "axis": ((0, 1, 0), (1, 0, 0)),
    "face_yz": ((0, 1, 1), (1, 0, 0)),
    "face_xy": ((1, 1, 0), (1, -1, 0)),
    "body": ((1, 1, 1), (1, -1, 0)),
}


def _shear_errors(J, nu, kdir, udir, sizes):
    kd = np.array(kdir, float) / np.linalg.norm(kdir)
    ud = np.array(udir, float) / np.linalg.norm(udir)
    out = []
    for n in sizes:
        k = 2 * math.pi / n
        lam, _ = _mode(J, k * kd, ud)
        nu_k = -math.log(abs(lam)) / k ** 2
        out.append(abs(nu_k / nu - 1.0 - 3.0 * nu * nu * k * k))
    return out


@pytest.mark.parametrize("w1,w2", [(1.6, 1.0), (1.9, 1.0), (1.8, 1.3)])
def test_parametrized_shear_diffusion_is_fourth_order(w1, w2):
    sizes = (32, 64, 128)
    Pp, nu = _params(w1, w2, True)
    Ps, _ = _params(w1, w2, False)
    Jp, Js = _jacobian(Pp), _jacobian(Ps)
    for name, (kd, ud) in ORIENTATIONS.items():
        ep = _shear_errors(Jp, nu, kd, ud, sizes)
        es = _shear_errors(Js, nu, kd, ud, sizes)
        order_p = math.log2(ep[1] / ep[2])
        order_s = math.log2(es[1] / es[2])
        print(f"w1 {w1} w2 {w2} {name}: parametrised {ep} order {order_p:.3f}; standard order {order_s:.3f}")
        assert order_p > 3.85, (name, ep)
        assert 1.9 < order_s < 2.1, (name, es)
        assert ep[2] < 0.05 * es[2]


def test_parametrized_rates_limits():
    """At w1 -> 2 (vanishing viscosity) every third-order rate goes to 0
    (the factor w1 - 2); A and B stay finite. The rates are not symmetric
    under swapping the plus and minus combinations (they differ at w1 = 1.8)."""
    for w2 in (0.8, 1.0, 1.5):
        wp, wm, wd, A, B = C.parametrized_rates(2.0, w2)
        assert wp == 0.0 and wm == 0.0 and wd == 0.0
        assert math.isfinite(A) and math.isfinite(B)
    wp, wm, wd, _, _ = C.parametrized_rates(1.8, 1.0)
    assert abs(wp - wm) > 0.1


def _gradient_estimate(v, w1, w2):
    """Gradient estimates of the pre-collision state w + eps v to first order
    in eps (exact directional derivative; real and imaginary parts of v
    taken separately since the map is real)."""
    def est(f):
        Cm = ring.cumulants_from_moments(C.raw_moments(f[:, None], D3Q27) / f.sum())
        return torch.stack([g[0] for g in C.velocity_gradients(Cm, w1, w2)])
    res = [torch.autograd.functional.jvp(est, D3Q27.w.clone(), torch.tensor(part))[1].numpy()
           for part in (v.real.copy(), v.imag.copy())]
    return res[0] + 1j * res[1]


def _exact_gradients(v, kvec):
    """(d_x u_x, d_y u_y, d_z u_z, D_xy, D_xz, D_yz) of the plane wave
    j exp(i k.x) at x = 0 (rho = 1 at first order)."""
    j = CV.T @ v
    d = 1j * np.outer(kvec, j)                   # d[a, b] = d_a u_b
    return np.array([d[0, 0], d[1, 1], d[2, 2], d[0, 1] + d[1, 0], d[0, 2] + d[2, 0],
                     d[1, 2] + d[2, 1]])


@pytest.mark.parametrize("w1,w2", [(1.8, 1.3), (1.6, 0.8)])
def test_gradient_estimates_match_eigenmode_derivatives(w1, w2):
    P, _ = _params(w1, w2, True)
    J = _jacobian(P)
    errs = {"shear": [], "sound": []}
    for n in (32, 64, 128):
        k = 2 * math.pi / n
        for name, kvec, dvec, pos in (("shear", (0.0, k, 0.0), (1.0, 0.0, 0.0), False),
                                      ("sound", (k, 0.0, 0.0), (1.0, 0.0, 0.0), True)):
            kvec = np.array(kvec)
            _, v = _mode(J, kvec, np.array(dvec), pos)
            exact = _exact_gradients(v, kvec)
            g = _gradient_estimate(v, w1, w2)
            errs[name].append(np.linalg.norm(g - exact) / np.linalg.norm(exact))
    print(f"w1 {w1} w2 {w2}: {errs}")
    # the pre-collision non-equilibrium lags the gradient by half a step:
    # first order in k for the sound mode (frequency cs k), second for shear
    assert errs["shear"][-1] < 1e-3 and errs["sound"][-1] < 0.03
    assert errs["sound"][1] / errs["sound"][2] > 1.8
    assert errs["shear"][1] / errs["shear"][2] > 3.5


def _random_state(n=64, seed=3, amp=0.05):
    g = torch.Generator().manual_seed(seed)
    f = D3Q27.w[:, None] * (1 + amp * (2 * torch.rand(27, n, generator=g, dtype=torch.float64) - 1))
    phi = torch.rand(7, n, generator=g, dtype=torch.float64) * 0.1
    return f, phi


def _third_order_cumulants(f):
    """The seven limited third-order quantities of f: C_120 +- C_102,
    C_210 +- C_012, C_201 +- C_021 and C_111 (cumulants of f / rho)."""
    rho = f.sum(0)
    Cm = ring.cumulants_from_moments(C.raw_moments(f, D3Q27) / rho)
    out = []
    for a, b in (((1, 2, 0), (1, 0, 2)), ((2, 1, 0), (0, 1, 2)), ((2, 0, 1), (0, 2, 1))):
        out += [Cm[a] + Cm[b], Cm[a] - Cm[b]]
    return torch.stack(out + [Cm[1, 1, 1]])


def test_parametrized_collision_invariants_and_limiter_limits():
    f, phi = _random_state()
    base = dict(nx=8, ny=8, nz=8, model=0, g_prime=1e-3, nu_lu=0.02, parametrized=True)
    P0 = derive(Config(**base))
    fs0, _ = C.collide(f, phi, P0)
    # mass conserved, momentum changed by the force only (Eq. 17, 56)
    rho, j, chi, F, _ = C.macroscopic(f, phi, P0)
    c = D3Q27.c.T
    assert torch.allclose(fs0.sum(0), rho, atol=1e-14, rtol=0)
    assert torch.allclose(c @ fs0, j + F, atol=1e-14, rtol=0)
    # the rest state is a fixed point
    rest, _ = C.collide(D3Q27.w[:, None].clone(), torch.zeros(7, 1, dtype=torch.float64), P0)
    assert torch.allclose(rest[:, 0], D3Q27.w, atol=1e-15, rtol=0)
    # limiter: a huge lambda is no limiter, a tiny one resets order 3 to 0
    fs_big, _ = C.collide(f, phi, derive(Config(limiter=1e30, **base)))
    assert torch.allclose(fs_big, fs0, atol=1e-16, rtol=0)
    fs_tiny, _ = C.collide(f, phi, derive(Config(limiter=1e-30, **base)))
    assert _third_order_cumulants(fs_tiny).abs().max() < 1e-15
    # in between, each limited quantity shrinks monotonically as lambda falls
    c3 = [_third_order_cumulants(C.collide(f, phi, derive(Config(limiter=lam, **base)))[0]).abs()
          for lam in (1e-4, 1e-3, 1e-2)]
    c3_off = _third_order_cumulants(fs0).abs()
    assert (c3[0] <= c3[1] + 1e-17).all() and (c3[1] <= c3[2] + 1e-17).all()
    assert (c3[2] <= c3_off + 1e-17).all()
    # the fourth-order equilibria do not depend on the limiter
    rho0 = fs0.sum(0)
    c4 = lambda x: ring.cumulants_from_moments(C.raw_moments(x, D3Q27) / x.sum(0))[2, 2, 0]
    assert torch.allclose(c4(fs_tiny), c4(fs0), atol=1e-15, rtol=0)
    assert rho0.shape == rho.shape


def test_parametrized_lock_exchange_runs_and_conserves():
    for model in (0, 2):
        cfg = Config(24, 4, 12, model=model, re_b=2000.0, parametrized=True, limiter=0.01)
        P = derive(cfg)
        f, phi = olbm.init_state(P, olbm.chi0_lock_exchange(cfg, 0.25, 1e-3, 0))
        m0, c0 = f.sum().item(), phi.sum().item()
        for _ in range(30):
            f, phi = olbm.step(f, phi, P)
        assert torch.isfinite(f).all() and torch.isfinite(phi).all()
        assert abs(f.sum().item() - m0) < 1e-10 * m0
        assert abs(phi.sum().item() - c0) < 1e-10 * c0
