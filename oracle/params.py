"""Lattice-unit parameters of a lock-exchange run (oracle; test infrastructure).

Sec. 2.5 fixes the scaling: the depth H is resolved by N3 nodes; with half-way
bounce-back walls at z = 0 and z = N3 the depth is exactly N3 lattice units.
The buoyancy velocity is U_b = sqrt(g' H) and the buoyancy Reynolds number
Re_b = U_b H / nu (Eq. 12-14). The relaxation time follows from Eq. 25
(nu = cs^2 (tau - 1/2), cs^2 = 1/3) and the scalar relaxation time from Eq. 30
(D = cs_phi^2 (tau_phi - 1/2)) with D = nu / Sc.

Reading: g' is given in lattice units. When ``ub_lu`` > 0 the paper's own
convention U_b = 0.03 LU is used instead, i.e. g' = ub_lu^2 / N3.

Non-dimensional time is t~ = n U_b / H and lengths in units of H are x / N3.
"""
import math
from dataclasses import dataclass, field

from .lattice import D3Q6, D3Q7, D3Q19, D3Q27

CUMULANT27_Q7 = 0
BGK19_SMAG_Q6 = 1
CUMULANT27_FCM27 = 2        # D3Q27 cumulant flow, D3Q27 factorized-central-moment scalar


@dataclass
class Config:
    nx: int
    ny: int
    nz: int
    model: int = CUMULANT27_Q7
    re_b: float = 1000.0
    sc: float = 1.0
    g_prime: float = 1e-4
    ub_lu: float = 0.0
    cs_smag: float = 0.0
    sc_t: float = 1.0
    omega_bulk: float = 1.0
    omega3: float = 1.0
    omega4: float = 1.0
    omega5: float = 1.0
    omega6: float = 1.0
    # parametrised cumulant (Sec. 2.3, VirtualFluids): third-order rates and
    # fourth-order equilibria from omega1 and omega_bulk; limiter lambda of the
    # third-order relaxation, 0 = no limiter
    parametrized: bool = False
    limiter: float = 0.0
    # Smagorinsky closure as printed in Eq. 32, nu_T = C_s Delta^2 |S| (C_s
    # enters to the first power); default: the standard (C_s Delta)^2 |S|
    smag_paper_form: bool = False
    # oracle-only switches for the closed-form checks (the product has walls)
    periodic_x: bool = False
    periodic_z: bool = False
    body_force: tuple = field(default=(0.0, 0.0, 0.0))
    nu_lu: float = 0.0          # > 0: use this viscosity instead of U_b H / Re_b


@dataclass
class Params:
    cfg: Config
    flow: object
    scal: object
    H: float
    g_prime: float
    u_b: float
    nu0: float
    tau0: float
    d0: float
    tau_phi0: float


def derive(cfg: Config) -> Params:
    flow = D3Q19 if cfg.model == BGK19_SMAG_Q6 else D3Q27
    scal = {CUMULANT27_Q7: D3Q7, BGK19_SMAG_Q6: D3Q6, CUMULANT27_FCM27: D3Q27}[cfg.model]
    H = float(cfg.nz)
    g = cfg.ub_lu ** 2 / H if cfg.ub_lu > 0 else cfg.g_prime
    u_b = math.sqrt(g * H)
    nu0 = cfg.nu_lu if cfg.nu_lu > 0 else u_b * H / cfg.re_b
    tau0 = nu0 / flow.cs2 + 0.5
    d0 = nu0 / cfg.sc
    tau_phi0 = 0.5 + d0 / scal.cs2
    return Params(cfg, flow, scal, H, g, u_b, nu0, tau0, d0, tau_phi0)
