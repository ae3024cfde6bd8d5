"""Shared helpers of the GPU parity tests: build both sides from one set of
keyword arguments and compare moments the way the tests report them."""
import numpy as np
import torch

import paper_2112_08479_amd as pkg
from oracle import lbm as olbm
from oracle.params import Config as OConfig
from oracle.params import derive

ORACLE_KEYS = ("nx", "ny", "nz", "model", "re_b", "sc", "g_prime", "ub_lu", "cs_smag", "sc_t",
               "omega_bulk", "omega3", "omega4", "omega5", "omega6", "parametrized", "limiter",
               "smag_paper_form")


def both(storage, **kw):
    cfg = pkg.Config(storage=storage, **kw)
    P = derive(OConfig(**{k: v for k, v in kw.items() if k in ORACLE_KEYS}))
    return cfg, P


def oracle_moments(f, phi, P):
    rho, u, chi = olbm.moments(f, phi, P)
    return {"rho": rho.numpy(), "ux": u[0].numpy(), "uy": u[1].numpy(), "uz": u[2].numpy(),
            "chi": chi.numpy()}


def gpu_moments(lat):
    m = lat.moments(pkg.OUT_F64)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in m.items()}


def component_errors(got, want):
    """Infinity-norm error of each field against that field's own infinity norm
    (the plain per-component figure the tests print beside moment_errors)."""
    out = {}
    for k in ("rho", "ux", "uy", "uz", "chi"):
        ref = want[k] - 1.0 if k == "rho" else want[k]
        scale = np.abs(ref).max()
        out[k] = float(np.abs(got[k] - want[k]).max() / scale) if scale > 0 else float(np.abs(got[k] - want[k]).max())
    return out


def moment_errors(got, want):
    """Infinity-norm error of each field relative to the oracle field's
    infinity norm: delta rho = rho - 1 for the density, chi, and for every
    velocity component the velocity magnitude's infinity norm (a component
    that is itself ~0, e.g. the span velocity of an almost two-dimensional
    start, would otherwise divide rounding noise by rounding noise)."""
    out = {}
    umax = np.sqrt(want["ux"] ** 2 + want["uy"] ** 2 + want["uz"] ** 2).max()
    for k in ("rho", "ux", "uy", "uz", "chi"):
        ref = want[k] - 1.0 if k == "rho" else want[k]
        scale = umax if k in ("ux", "uy", "uz") else np.abs(ref).max()
        out[k] = float(np.abs(got[k] - want[k]).max() / scale) if scale > 0 else float(np.abs(got[k] - want[k]).max())
    return out


def ulp(v, mant_bits):
    """Spacing of a float format with `mant_bits` explicit mantissa bits at |v|."""
    a = np.maximum(np.abs(v), 2.0 ** -14)
    return 2.0 ** (np.floor(np.log2(a)) - mant_bits)
