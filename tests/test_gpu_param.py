"""Parity of the parametrised cumulant (Sec. 2.3: third-order rates from
omega1 and omega_bulk, fourth-order equilibria from the velocity gradients,
third-order limiter) between the HIP library and the FP64 oracle.

Tolerances as for the other collision kinds: FP64 1e-13 on populations after
one step and 1e-10 on moments over a trajectory; FP32 2e-7 after one step
(doubled for the D3Q27 scalar) and 1e-5 on moments after 100 steps; 16-bit
storage the final rounding plus FP32 arithmetic error. The limiter is tested
off (lambda = 0), moderate (1e-2) and strong (1e-4, active at almost every
node of the random states).
"""
import numpy as np
import pytest
import torch

import paper_2112_08479_amd as pkg
from oracle import diag as odiag
from oracle import lbm as olbm
from oracle.params import Config as OConfig
from tests import inputs
from tests.gpu_helpers import both, gpu_moments, moment_errors, oracle_moments, ulp

pytestmark = pytest.mark.gpu


def _random_case(model, storage, limiter, omega_bulk=1.0, shape=(5, 3, 300), seed=11, eps=1e-2):
    kw = dict(nx=shape[2], ny=shape[1], nz=shape[0], model=model, re_b=2000.0, g_prime=1e-3,
              omega_bulk=omega_bulk, parametrized=True, limiter=limiter)
    cfg, P = both(storage, **kw)
    f, phi = inputs.near_rest_state(P.flow.Q, P.scal.Q, shape, P.flow.w.numpy(), P.scal.w.numpy(),
                                    seed, eps=eps)
    lat = pkg.Lattice(cfg)
    lat.set_populations(f, phi)
    f0, phi0 = lat.get_populations()
    lat.step(1)
    f1, phi1 = lat.get_populations()
    lat.close()
    of, ophi = olbm.step(torch.from_numpy(f0), torch.from_numpy(phi0), P)
    return P, f1, phi1, of.numpy(), ophi.numpy()


def test_derived_rates_match_the_oracle():
    from oracle.collide import parametrized_rates
    for model, re_b, wb in ((0, 1000.0, 1.0), (2, 30000.0, 1.0), (2, 300.0, 1.4)):
        cfg, P = both(pkg.F64, nx=64, ny=4, nz=16, model=model, re_b=re_b, omega_bulk=wb,
                      parametrized=True)
        d = pkg.derive_params(cfg)
        want = parametrized_rates(1.0 / P.tau0, wb)
        got = (d["w_plus"], d["w_minus"], d["w_111"], d["coef_a"], d["coef_b"])
        assert np.allclose(got, want, rtol=1e-13, atol=0), (got, want)


@pytest.mark.parametrize("limiter", [0.0, 1e-2, 1e-4])
@pytest.mark.parametrize("model", [0, 2])
@pytest.mark.parametrize("storage", [pkg.F64, pkg.F32])
def test_one_step_from_random_state(model, storage, limiter):
    P, f1, phi1, of, ophi = _random_case(model, storage, limiter)
    tol = 1e-13 if storage == pkg.F64 else 2e-7
    ef, ep = np.abs(f1 - of).max(), np.abs(phi1 - ophi).max()
    print(f"model {model} storage {storage} limiter {limiter}: {ef:.3e} {ep:.3e}", flush=True)
    assert ef < tol
    assert ep < tol * (2.0 if model == 2 else 1.0)


def test_one_step_with_bulk_rate_other_than_one():
    P, f1, phi1, of, ophi = _random_case(0, pkg.F64, 1e-2, omega_bulk=1.4)
    assert np.abs(f1 - of).max() < 1e-13 and np.abs(phi1 - ophi).max() < 1e-13


@pytest.mark.parametrize("storage,mant,mant_s", [(pkg.F16, 10, 10), (pkg.BF16_F16S, 7, 10)])
def test_one_step_16bit_storage(storage, mant, mant_s):
    # the rounded state as stored is the input of both sides
    kw = dict(nx=300, ny=3, nz=5, model=2, re_b=2000.0, g_prime=1e-3, parametrized=True, limiter=1e-2)
    cfg, P = both(storage, **kw)
    f, phi = inputs.near_rest_state(27, 27, (5, 3, 300), P.flow.w.numpy(), P.scal.w.numpy(), 12, eps=1e-2)
    lat = pkg.Lattice(cfg)
    lat.set_populations(f, phi)
    f0, phi0 = lat.get_populations()
    lat.step(1)
    f1, phi1 = lat.get_populations()
    lat.close()
    of, ophi = olbm.step(torch.from_numpy(f0), torch.from_numpy(phi0), P)
    w = P.flow.w.numpy()[:, None, None, None]
    g_got, g_want = f1 - w, of.numpy() - w
    assert np.all(np.abs(g_got - g_want) <= 0.5 * ulp(g_want, mant) + 2e-7)
    assert np.all(np.abs(phi1 - ophi.numpy()) <= 0.5 * ulp(ophi.numpy(), mant_s) + 4e-7)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 3), (4, 2, 65)])
def test_degenerate_and_ragged_grids(shape):
    kw = dict(nx=shape[2], ny=shape[1], nz=shape[0], model=2, re_b=50.0, g_prime=1e-3,
              parametrized=True, limiter=1e-3)
    cfg, P = both(pkg.F64, **kw)
    f, phi = inputs.near_rest_state(27, 27, shape, P.flow.w.numpy(), P.scal.w.numpy(), 4, eps=1e-2)
    lat = pkg.Lattice(cfg)
    lat.set_populations(f, phi)
    lat.step(1)
    f1, phi1 = lat.get_populations()
    lat.close()
    of, ophi = olbm.step(torch.from_numpy(f), torch.from_numpy(phi), P)
    assert np.abs(f1 - of.numpy()).max() < 1e-13
    assert np.abs(phi1 - ophi.numpy()).max() < 1e-13


@pytest.mark.parametrize("storage", [pkg.F64, pkg.F32])
def test_rest_state_stays_exactly_at_rest(storage):
    cfg, P = both(storage, nx=70, ny=3, nz=5, model=2, parametrized=True, limiter=1e-2)
    lat = pkg.Lattice(cfg)
    lat.init_from_field(torch.zeros(5, 3, 70, dtype=torch.float64, device="cuda"))
    lat.step(25)
    f, phi = lat.get_populations()
    lat.close()
    assert np.array_equal(f, np.broadcast_to(P.flow.w.numpy()[:, None, None, None], f.shape))
    assert not phi.any()


C0P = dict(nx=128, ny=8, nz=16, re_b=1000.0, parametrized=True, limiter=1e-2)
_cache = {}


def _oracle_trajectory(model, P, steps):
    if model not in _cache:
        torch.set_num_threads(max(1, min(16, torch.get_num_threads())))
        f, phi = olbm.init_state(P, olbm.chi0_lock_exchange(OConfig(128, 8, 16), 0.125, 1e-3, 0))
        out, n = {}, 0
        for s in steps:
            while n < s:
                f, phi = olbm.step(f, phi, P)
                n += 1
            out[s] = (oracle_moments(f, phi, P), odiag.diagnostics(f, phi, P, s))
        _cache[model] = out
    return _cache[model]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("model", [0, 2])
def test_lock_exchange_fp64_200_steps(model):
    """128 x 8 x 16 lock exchange, Re_b = 1000, limiter 1e-2: moments within
    1e-10 of the oracle's, front and masses within 1e-9."""
    cfg, P = both(pkg.F64, model=model, **C0P)
    steps = (1, 10, 100, 200)
    ref = _oracle_trajectory(model, P, steps)
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    n = 0
    for s in steps:
        lat.step(s - n)
        n = s
        errs = moment_errors(gpu_moments(lat), ref[s][0])
        print(f"model {model} step {s} errors {errs}", flush=True)
        assert max(errs.values()) < 1e-10, (s, errs)
        d, od = lat.diagnostics(), ref[s][1]
        for k in ("mass", "chi_mass", "x_front", "x_f"):
            assert abs(d[k] - od[k]) <= 1e-9 * max(1.0, abs(od[k])), (s, k, d[k], od[k])
    lat.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("model", [0, 2])
def test_lock_exchange_fp32_100_steps(model):
    cfg, P = both(pkg.F32, model=model, **C0P)
    ref = _oracle_trajectory(model, P, (1, 10, 100, 200))
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    lat.step(100)
    errs = moment_errors(gpu_moments(lat), ref[100][0])
    lat.close()
    print(f"fp32 model {model} errors {errs}", flush=True)
    assert max(errs.values()) < 1e-5, errs


def test_parametrised_differs_from_the_standard_cumulant():
    """The switch reaches the kernel: after 50 steps the parametrised run
    differs from the standard one by far more than rounding."""
    out = []
    for par in (False, True):
        lat = pkg.Lattice(pkg.Config(128, 8, 16, model=2, storage=pkg.F64, re_b=1000.0,
                                     parametrized=par, limiter=1e-2 if par else 0.0))
        lat.init_lock_exchange(0.125, 1e-3, 0)
        lat.step(50)
        out.append(gpu_moments(lat))
        lat.close()
    diff = moment_errors(out[1], out[0])
    assert max(diff["ux"], diff["uz"]) > 1e-6, diff
