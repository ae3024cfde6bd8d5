"""The hand-written adjoint (lbm_adjoint_run) against the oracle.

* 64 x 4 x 8, 200 steps, checkpoints every 50: J, dJ/dC_s, dJ/dSc_T and the
  field dJ/dchi0 against torch autograd through the FP64 oracle, every model,
  the Smagorinsky closure as printed, and the parametrised cumulant with the
  limiter; FP64 storage to 1e-8 (relative to the largest entry), FP32 to 1e-3.
* 128 x 8 x 16, 500 steps (cumulant, Re_b 1000, C_s 0.1, Sc_T 1): against the
  oracle's FP64 central differences stored in tests/golden (written by
  tests/golden/make_adjoint_fd.py, which calls only the oracle): FP64 to 1e-5,
  FP32 to 1e-3 relative.
* 256 x 16 x 32, 2000 steps, checkpoints every 100 (the benchmark adjoint):
  dJ/dC_s, dJ/dSc_T and two chi0 directions against the oracle's FP64
  central differences at that size (tests/golden/adjoint_fd_256x16x32.json
  and adjoint_fd_256x16x32_chi0.json, same script), FP64 to 1e-5 and FP32 to
  1e-3 relative; and the adjoint gradient against central differences
  (h = 1e-4) of the library's own FP64 forward map to 1e-3 relative.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
import torch

import paper_2112_08479_amd as pkg
from oracle import adjoint as oadj
from oracle import lbm as olbm
from oracle.params import Config as OConfig
from tests import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_128x8x16.json")
GOLDEN_C3 = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_256x16x32.json")
GOLDEN_C3_CHI0 = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_256x16x32_chi0.json")


def _gpu_grad(kw, storage, chi0, n, k, w_front=1.0, w_fw=1.0):
    cfg = pkg.Config(storage=storage, **kw)
    lat = pkg.Lattice(cfg)
    lat.init_from_field(chi0.to("cuda"), 0.125)
    J, dcs, dsct, g = lat.adjoint_run(n, k, w_front, w_fw)
    torch.cuda.synchronize()
    out = (J, dcs, dsct, g.cpu().numpy())
    lat.close()
    return out


TINY = [dict(nx=64, ny=4, nz=8, model=0, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4),
        dict(nx=64, ny=4, nz=8, model=1, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4),
        dict(nx=64, ny=4, nz=8, model=2, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4),
        # the Smagorinsky closure as printed (C_s to the first power), the paper's C_s
        dict(nx=64, ny=4, nz=8, model=0, re_b=1000.0, cs_smag=0.03, sc_t=1.0, g_prime=1e-4,
             smag_paper_form=True),
        # the parametrised cumulant without the LES, limiter active at most nodes
        dict(nx=64, ny=4, nz=8, model=2, re_b=1000.0, cs_smag=0.0, sc_t=1.0, g_prime=1e-4,
             parametrized=True, limiter=1e-4),
        dict(nx=64, ny=4, nz=8, model=0, re_b=1000.0, cs_smag=0.0, sc_t=1.0, g_prime=1e-4,
             parametrized=True, limiter=1e-2)]
_ref = {}


def _oracle_ref(i):
    if i not in _ref:
        torch.set_num_threads(max(1, min(16, torch.get_num_threads())))
        kw = TINY[i]
        cfg = OConfig(**kw)
        chi0 = olbm.chi0_lock_exchange(cfg, 0.125, 1e-3, 0)
        _ref[i] = (chi0, oadj.gradient(cfg, chi0, 200, k_ckpt=50))
    return _ref[i]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("i", [0, 1, 2, 3, 4, 5], ids=["cumulant", "bgk", "cumulant_fcm", "cumulant_printed_smag",
                                               "parametrised_fcm", "parametrised_cumulant"])
@pytest.mark.parametrize("storage,tol", [(pkg.F64, 1e-8), (pkg.F32, 1e-3)], ids=["f64", "f32"])
def test_adjoint_matches_oracle_autograd(i, storage, tol):
    chi0, (J, gcs, gsct, gchi) = _oracle_ref(i)
    gJ, gdcs, gdsct, ggchi = _gpu_grad(TINY[i], storage, chi0, 200, 50)
    gchi = gchi.numpy()
    scale = np.abs(gchi).max()
    print(f"model {i} storage {storage}: J {gJ} vs {J}; dCs {gdcs} vs {gcs}; dSct {gdsct} vs {gsct}; "
          f"dchi0 max err {np.abs(ggchi - gchi).max() / scale:.3e}", flush=True)
    assert abs(gJ - J) <= tol * abs(J)
    assert abs(gdcs - gcs) <= tol * abs(gcs)
    assert abs(gdsct - gsct) <= tol * abs(gsct) + 1e-12
    assert np.abs(ggchi - gchi).max() <= tol * scale


def test_checkpoint_interval_does_not_change_the_gradient():
    """Recomputed states are bitwise the forward pass's, so every checkpoint
    interval gives the same bits: one segment (60, 1000), two (30: the second
    stream recomputes only segment 0), three (20), a ragged last segment (7),
    and a checkpoint at every step (1: nothing to recompute)."""
    kw = TINY[0]
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 2)
    ref = _gpu_grad(kw, pkg.F32, chi0, 60, 60)
    for k in (7, 30, 20, 1, 1000):
        x = _gpu_grad(kw, pkg.F32, chi0, 60, k)
        assert x[0] == ref[0] and x[1] == ref[1] and x[2] == ref[2], k
        assert np.array_equal(x[3], ref[3]), k


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage,tol", [(pkg.F64, 1e-5), (pkg.F32, 1e-3)], ids=["f64", "f32"])
def test_adjoint_matches_oracle_finite_differences(storage, tol):
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    kw = ref["case"]
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 0)
    J, dcs, dsct, g = _gpu_grad(kw, storage, chi0, ref["steps"], 100)
    dirs = []
    for s in ref["dir_seeds"]:
        d = inputs.random_field(tuple(chi0.shape), s, -1.0, 1.0)
        dirs.append(d / np.abs(d).max())
    for (k, j, i) in ref["nodes"]:
        d = np.zeros(tuple(chi0.shape))
        d[k, j, i] = 1.0
        dirs.append(d)
    got = [float((g * d).sum()) for d in dirs]
    print(f"storage {storage}: J {J} vs {ref['J']}; dCs {dcs} vs {ref['dJ_dcs']}; dSct {dsct} vs "
          f"{ref['dJ_dsct']}; dirs {got} vs {ref['dJ_dchi0_dir']}", flush=True)
    # J itself: FP64 forward to 1e-6, FP32 forward (500 steps) to 1e-5
    assert abs(J - ref["J"]) <= (1e-6 if storage == pkg.F64 else 1e-5) * abs(ref["J"])
    assert abs(dcs - ref["dJ_dcs"]) <= tol * abs(ref["dJ_dcs"])
    assert abs(dsct - ref["dJ_dsct"]) <= tol * abs(ref["dJ_dsct"])
    for a, b in zip(got, ref["dJ_dchi0_dir"]):
        assert abs(a - b) <= tol * abs(b) + 1e-9 * max(abs(x) for x in ref["dJ_dchi0_dir"])


def _gpu_J(kw, chi0, n, cs=None, sct=None):
    kw = dict(kw)
    if cs is not None:
        kw["cs_smag"] = cs
    if sct is not None:
        kw["sc_t"] = sct
    return _gpu_grad(kw, pkg.F64, chi0, n, n)[0]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage,tol", [(pkg.F64, 1e-5), (pkg.F32, 1e-3)], ids=["f64", "f32"])
def test_full_size_adjoint_matches_oracle_finite_differences(storage, tol):
    with open(GOLDEN_C3) as fh:
        ref = json.load(fh)
    kw = ref["case"]
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 0)
    J, dcs, dsct, _ = _gpu_grad(kw, storage, chi0, ref["steps"], 100)
    print(f"storage {storage}: J {J} vs {ref['J']}; dCs {dcs} vs {ref['dJ_dcs']}; dSct {dsct} vs "
          f"{ref['dJ_dsct']}", flush=True)
    # J itself: FP64 forward to 1e-9, FP32 forward (2000 steps) to 1e-5
    assert abs(J - ref["J"]) <= (1e-9 if storage == pkg.F64 else 1e-5) * abs(ref["J"])
    assert abs(dcs - ref["dJ_dcs"]) <= tol * abs(ref["dJ_dcs"])
    assert abs(dsct - ref["dJ_dsct"]) <= tol * abs(ref["dJ_dsct"])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage,tol", [(pkg.F64, 1e-5), (pkg.F32, 1e-3)], ids=["f64", "f32"])
def test_full_size_adjoint_chi0_directions_match_oracle_finite_differences(storage, tol):
    with open(GOLDEN_C3_CHI0) as fh:
        ref = json.load(fh)
    kw = ref["case"]
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 0)
    _, _, _, g = _gpu_grad(kw, storage, chi0, ref["steps"], 100)
    got = []
    for s in ref["dir_seeds"]:
        d = inputs.random_field(tuple(chi0.shape), s, -1.0, 1.0)
        got.append(float((g * (d / np.abs(d).max())).sum()))
    print(f"storage {storage}: dirs {got} vs {ref['dJ_dchi0_dir']}", flush=True)
    for a, b in zip(got, ref["dJ_dchi0_dir"]):
        assert abs(a - b) <= tol * abs(b)


@pytest.mark.timeout(900)
def test_full_size_adjoint_equals_derivative_of_the_forward_map():
    kw = dict(nx=256, ny=16, nz=32, model=0, re_b=1000.0, cs_smag=0.1, sc_t=1.0, g_prime=1e-4)
    n, h = 2000, 1e-4
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 0)
    J, dcs, dsct, g = _gpu_grad(kw, pkg.F32, chi0, n, 100)
    fcs = (_gpu_J(kw, chi0, n, cs=0.1 + h) - _gpu_J(kw, chi0, n, cs=0.1 - h)) / (2 * h)
    fsct = (_gpu_J(kw, chi0, n, sct=1.0 + h) - _gpu_J(kw, chi0, n, sct=1.0 - h)) / (2 * h)
    rows = [("C_s", dcs, fcs), ("Sc_T", dsct, fsct)]
    for s in (21, 22):
        d = inputs.random_field(tuple(chi0.shape), s, -1.0, 1.0)
        d = torch.from_numpy(d / np.abs(d).max())
        fd = (_gpu_J(kw, chi0 + h * d, n) - _gpu_J(kw, chi0 - h * d, n)) / (2 * h)
        rows.append((f"chi0 dir {s}", float((g * d.numpy()).sum()), fd))
    for name, a, b in rows:
        print(f"{name}: adjoint {a:.8e}  fd {b:.8e}  rel {abs(a - b) / abs(b):.2e}", flush=True)
    for name, a, b in rows:
        assert abs(a - b) <= 1e-3 * abs(b), name


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kw", [
    dict(nx=70, ny=3, nz=6, model=0, cs_smag=0.1),            # ragged x tail, one node per thread
    dict(nx=1024, ny=64, nz=128, model=0, cs_smag=0.1),       # two nodes per thread
    dict(nx=1024, ny=64, nz=128, model=1, cs_smag=0.1),       # BGK, two nodes per thread
    dict(nx=200, ny=5, nz=9, model=2, cs_smag=0.0),           # FCM scalar
    dict(nx=1024, ny=64, nz=128, model=0, cs_smag=0.0, parametrized=True, limiter=1e-2),
], ids=["ragged", "npt2", "bgk_npt2", "fcm", "parametrised_npt2"])
def test_fused_wall_friction_sums_match_the_diagnostics(kw):
    """The adjoint's forward pass sums F_w inside the step kernel; with
    w_front = 0, J is the mean of F_w(m), m = 1..n. It must equal the mean of
    the diagnostics kernel's F_w over a plain run of the same steps (FP64:
    only the order of the sums and the compiler's contractions differ)."""
    n = 30
    cfg = pkg.Config(storage=pkg.F64, re_b=1000.0, g_prime=1e-4, sc_t=1.0, **kw)
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    J = lat.adjoint_run(n, 7, 0.0, 1.0)[0]
    lat.close()
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    fws, umax = [], 0.0
    for _ in range(n):
        lat.step(1)
        d = lat.diagnostics()
        fws.append(d["fw"])
        umax = max(umax, d["umax"])
    nu0 = lat.params["nu0"]
    lat.close()
    scale = nu0 * 3.0 * umax * cfg.nx * cfg.ny
    print(f"{kw}: J {J:.15e} mean F_w {np.mean(fws):.15e} scale {scale:.3e}", flush=True)
    assert abs(J - np.mean(fws)) <= 1e-11 * scale


def test_autograd_function_returns_the_library_gradient():
    kw = TINY[0]
    chi0 = olbm.chi0_lock_exchange(OConfig(**kw), 0.125, 1e-3, 4).to("cuda").requires_grad_(True)
    cs = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    sct = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    cfg = pkg.Config(storage=pkg.F64, **kw)
    J = pkg.lock_exchange_objective(chi0, cs, sct, cfg, 40, 10)
    (3.0 * J).backward()
    ref = _gpu_grad(kw, pkg.F64, chi0.detach().cpu(), 40, 10)
    assert abs(float(J) - ref[0]) < 1e-12 * abs(ref[0])
    assert abs(float(cs.grad) - 3 * ref[1]) <= 1e-12 * abs(ref[1])
    assert abs(float(sct.grad) - 3 * ref[2]) <= 1e-12 * abs(ref[2]) + 1e-15
    assert np.allclose(chi0.grad.cpu().numpy(), 3 * ref[3], rtol=0, atol=1e-12 * np.abs(ref[3]).max())


def test_adjoint_error_paths():
    kw = dict(TINY[0])
    lat = pkg.Lattice(pkg.Config(storage=pkg.F32, **kw))
    lat.init_lock_exchange()
    lat.step(1)
    with pytest.raises(pkg.LBMError) as e:
        lat.adjoint_run(10, 5)
    assert e.value.code == pkg.LBM_ESTATE
    for bad in (dict(storage=pkg.F16), dict(storage=pkg.F32, omega4=1.2)):
        c = pkg.Config(**{**kw, **bad})
        assert pkg.lib().lbm_adjoint_workspace_bytes(c.c(), 10, 5) == 0
