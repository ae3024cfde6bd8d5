"""Objective of the differentiation form and its reference gradients (oracle;
test infrastructure only).

J = w_front * x_f(n_end) + w_fw * (1/n_end) * sum_{n=1..n_end} F_w(n), with
x_f the front position and F_w the bottom-wall friction force of the
pre-collision state at step n (diag.py; Sec. 3.1, Eq. 62, 64), for a run of
n_end steps from the lock-exchange state whose scalar populations are
w_phi chi0 (f = w). Parameters: the Smagorinsky constant C_s, the turbulent
Schmidt number Sc_T and the field chi0.

gradient(): reverse mode by torch autograd through the FP64 oracle, with the
run split into segments of k steps whose forward is recomputed in the backward
pass (torch.utils.checkpoint). Non-smooth points take the branch autograd
takes: the zero subgradient of sqrt(Q) at Q = 0 (collide.smagorinsky_tau),
the first maximum over depth for the front, the active i*.
objective(): the same J without gradients, for central finite differences.
"""
import torch
from torch.utils.checkpoint import checkpoint

from . import diag, lbm
from .params import derive


def _run(chi0, cs, sct, P, n_end, w_front, w_fw, k_ckpt, lock_fraction):
    f, phi = lbm.init_state(P, chi0)
    acc = {"fw": chi0.sum() * 0.0}

    def seg(f, phi, cs, sct, nsteps):
        fw = f.sum() * 0.0
        for _ in range(nsteps):
            f, phi = lbm.step(f, phi, P, cs, sct)
            _, u, _ = lbm.moments(f, phi, P)
            fw = fw + diag.wall_friction(u, P)
        return f, phi, fw

    n = 0
    while n < n_end:
        k = min(k_ckpt, n_end - n)
        if torch.is_grad_enabled() and k_ckpt < n_end:
            f, phi, fw = checkpoint(seg, f, phi, cs, sct, k, use_reentrant=False)
        else:
            f, phi, fw = seg(f, phi, cs, sct, k)
        acc["fw"] = acc["fw"] + fw
        n += k
    _, _, chi = lbm.moments(f, phi, P)
    x_front, _ = diag.front_position(chi)
    x0 = lbm.gate_index(P.cfg.nx, lock_fraction)
    return w_front * (x_front - x0) + w_fw * acc["fw"] / n_end


def objective(cfg, chi0, n_end, cs=None, sct=None, w_front=1.0, w_fw=1.0, lock_fraction=0.125):
    P = derive(cfg)
    cs = cfg.cs_smag if cs is None else cs
    sct = cfg.sc_t if sct is None else sct
    with torch.no_grad():
        return float(_run(chi0, cs, sct, P, n_end, w_front, w_fw, n_end + 1, lock_fraction))


def gradient(cfg, chi0, n_end, w_front=1.0, w_fw=1.0, k_ckpt=100, lock_fraction=0.125):
    """Returns (J, dJ/dC_s, dJ/dSc_T, dJ/dchi0 tensor)."""
    P = derive(cfg)
    cs = torch.tensor(cfg.cs_smag, dtype=torch.float64, requires_grad=True)
    sct = torch.tensor(cfg.sc_t, dtype=torch.float64, requires_grad=True)
    chi = chi0.clone().requires_grad_(True)
    J = _run(chi, cs, sct, P, n_end, w_front, w_fw, k_ckpt, lock_fraction)
    gcs, gsct, gchi = torch.autograd.grad(J, (cs, sct, chi), allow_unused=True)
    z = torch.zeros((), dtype=torch.float64)
    return (float(J.detach()), float(gcs if gcs is not None else z), float(gsct if gsct is not None else z),
            gchi if gchi is not None else torch.zeros_like(chi0))
