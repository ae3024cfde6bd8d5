"""Wall shear stress export and the physics of the lock exchange on the GPU.

* lbm_wall_shear against the oracle's tau_w field (Eq. 62 with the half-way
  wall) on the same stored state, FP64 and FP32, a ragged row length; its sum
  is the F_w of the diagnostics (Eq. 64).
* The slumping-phase Froude number (Eq. 59) of the 128 x 8 x 16 lock
  exchange at Re_b = 1000 (FP64, every model; the FP64 path is tied to the
  oracle step by step by the parity tests): within 0.02 of the 0.37 that
  Table 2 gives for Re_b = 1000 (Case 2), i.e. about the 5 % band of the
  errors Table 2 reports for the paper's own codes. (Measured: 0.369 and
  0.370 here; 0.367-0.370 on grids up to 1024 x 64 x 128 in FP32.)
"""
import numpy as np
import pytest
import torch

import paper_2112_08479_amd as pkg
from oracle import diag as odiag
from oracle import lbm as olbm
from paper_2112_08479_amd import analysis
from tests import inputs
from tests.gpu_helpers import both

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("storage,tol", [(pkg.F64, 1e-13), (pkg.F32, 1e-6)], ids=["f64", "f32"])
def test_wall_shear_matches_oracle(model, storage, tol):
    shape = (6, 3, 300)
    cfg, P = both(storage, nx=shape[2], ny=shape[1], nz=shape[0], model=model, re_b=2000.0,
                  g_prime=1e-3)
    f, phi = inputs.near_rest_state(P.flow.Q, P.scal.Q, shape, P.flow.w.numpy(), P.scal.w.numpy(),
                                    5, eps=1e-2)
    lat = pkg.Lattice(cfg)
    lat.set_populations(f, phi)
    f0, phi0 = lat.get_populations()
    tau, bar = lat.wall_shear(pkg.OUT_F64)
    tau32, bar32 = lat.wall_shear(pkg.OUT_F32)
    d = lat.diagnostics()
    torch.cuda.synchronize()
    _, u, _ = olbm.moments(torch.from_numpy(f0), torch.from_numpy(phi0), P)
    otau, obar = odiag.wall_shear(u, P)
    otau, obar = otau.numpy(), obar.numpy()
    scale = np.abs(otau).max()
    assert np.abs(tau.cpu().numpy() - otau).max() <= tol * scale
    assert np.abs(bar.cpu().numpy() - obar).max() <= tol * scale
    assert np.abs(tau32.cpu().numpy() - otau).max() <= 1e-6 * scale
    # Eq. 64: the diagnostics' F_w is the wall sum of the same field
    assert abs(analysis.friction_force(tau.cpu().numpy()) - d["fw"]) <= 1e-12 * scale * tau.numel()
    lat.close()


def test_wall_shear_error_paths():
    lat = pkg.Lattice(pkg.Config(64, 2, 1, storage=pkg.F32))
    lat.init_lock_exchange()
    with pytest.raises(pkg.LBMError) as e:
        lat.wall_shear()
    assert e.value.code == pkg.LBM_EINVAL
    lat.close()
    lat = pkg.Lattice(pkg.Config(64, 2, 4, storage=pkg.F32))
    with pytest.raises(pkg.LBMError) as e:
        lat.wall_shear()
    assert e.value.code == pkg.LBM_ESTATE
    lat.close()


def _front_series(cfg, t_end=10.5, dt=0.1):
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    ub, H = lat.params["u_b"], cfg.nz
    every = max(1, int(round(dt * H / ub)))
    n_end = int(np.ceil(t_end * H / ub))
    ts, xs, n = [], [], 0
    while n < n_end:
        lat.step(every)
        n += every
        d = lat.diagnostics()
        ts.append(d["t_nd"])
        xs.append(d["x_f_nd"])
    lat.close()
    return np.array(ts), np.array(xs)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("model", [0, 1, 2])
def test_froude_number_of_the_slumping_phase(model):
    cfg = pkg.Config(128, 8, 16, model=model, storage=pkg.F64, re_b=1000.0, g_prime=1e-4)
    t, x = _front_series(cfg)
    fr = analysis.froude_number(t, x)
    print(f"model {model}: Fr = {fr:.4f} (Table 2, Re_b = 1000: 0.37)", flush=True)
    assert abs(fr - 0.37) <= 0.02
    # Past the start-up the front only advances, and it is still in the
    # channel at t~ = 10. (In the first few tenths of t~ the scalar, relaxed
    # at tau_phi close to 1/2, carries start-up oscillations of the step in
    # chi nearly ballistically ahead of the gate, and they cross the 0.02
    # threshold briefly.)
    late = t >= 1.0
    assert np.all(np.diff(x[late]) >= -1e-9)
    assert x[-1] < 7.0


# Table 2 (Froude number of the slumping phase): Re_b 5000 -> 0.42 (DNS, Cases 4
# and 5), 10000 -> 0.42 (experiment, Case 6), 30000 -> 0.44 (experiment, Case 8)
# (model, Re_b, C_s, parametrised cumulant with limiter 1e-2, Table 2 value)
FR_CASES = [(0, 5000.0, 0.0, False, 0.42), (1, 10000.0, 0.1, False, 0.42),
            (0, 30000.0, 0.1, False, 0.44), (2, 30000.0, 0.1, False, 0.44),
            (2, 30000.0, 0.0, True, 0.44), (0, 5000.0, 0.0, True, 0.42)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("model,re_b,cs,par,fr_ref", FR_CASES,
                         ids=["cumulant-5000", "bgk-10000-les", "cumulant-30000-les", "fcm-30000-les",
                              "fcm-30000-parametrised", "cumulant-5000-parametrised"])
def test_froude_number_across_reynolds_numbers(model, re_b, cs, par, fr_ref):
    """1024 x 64 x 128 (128 nodes over the depth), FP32, to t~ = 10.5: the
    slumping-phase Froude number within 0.02 of Table 2's value for the same
    Re_b (about the 5 % band of the errors Table 2 reports for the paper's own
    codes). The parametrised cases run without a sub-grid model, as the
    paper's VirtualFluids runs do. Measured: 0.413, 0.426, 0.436, 0.445,
    0.446, 0.411."""
    cfg = pkg.Config(1024, 64, 128, model=model, storage=pkg.F32, re_b=re_b, g_prime=1e-4,
                     cs_smag=cs, sc_t=1.0, parametrized=par, limiter=1e-2 if par else 0.0)
    t, x = _front_series(cfg)
    fr = analysis.froude_number(t, x)
    print(f"model {model} Re_b {re_b} C_s {cs}: Fr = {fr:.4f} (Table 2: {fr_ref})", flush=True)
    assert abs(fr - fr_ref) <= 0.02


@pytest.mark.timeout(300)
def test_bgk_model_at_re30000_with_the_printed_closure():
    """Model 2 (D3Q19 BGK + Smagorinsky + D3Q6) at Re_b = 30000 on 1024 x 64 x
    128, FP32, with the Smagorinsky closure as printed in Eq. 32 (nu_T =
    C_s |S|) and the paper's C_s = 0.03 and Sc_T = C_s (Sec. 2.3.1): the run
    stays finite to t~ = 10.5 (about 12 000 steps) and its slumping-phase
    Froude number is within 0.02 of Table 2's 0.44 for Re_b = 30000 (Case 8,
    experiment), the band of the other Froude tests. (Measured: 0.421. With C_s = 0.1 in the standard form and
    Sc_T = 1 the D3Q6 scalar, relaxed at tau_phi close to 1/2, goes unstable
    near t~ = 5.6.)"""
    cfg = pkg.Config(1024, 64, 128, model=1, storage=pkg.F32, re_b=30000.0, g_prime=1e-4,
                     cs_smag=0.03, sc_t=0.03, smag_paper_form=True)
    t, x = _front_series(cfg)
    assert t[-1] >= 10.5
    fr = analysis.froude_number(t, x)
    print(f"model 1 Re_b 30000, printed closure C_s = Sc_T = 0.03: Fr = {fr:.4f} (Table 2: 0.44)",
          flush=True)
    assert abs(fr - 0.44) <= 0.02
